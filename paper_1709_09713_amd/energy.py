"""Energy to solution on the GPU: socket power sampled while the work runs,
integrated over the run.

The paper's headline metric is energy (power sampled while the solver
runs, integrated over the run, and compared between algorithm classes;
performance section).  Here AMD SMI's current socket power is sampled about
every 10 ms on a host thread while the region runs, and integrated with the
trapezoid rule; the board's accumulated-energy counter, which advances only
about once per second, is read at the same time and gives an independent
mean power over the whole counter intervals that fall inside the region.
If AMD SMI is not usable in the process, ``EnergyMeter.available`` is False
and ``reason`` says why; nothing else changes.
"""
from __future__ import annotations

import threading
import time

import torch


class EnergyMeter:
    def __init__(self, device_index: int = 0, sample_interval_s: float = 0.01):
        self.available = False
        self.reason = ""
        self.interval = sample_interval_s
        self._smi = None
        self._h = None
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            handles = amdsmi.amdsmi_get_processor_handles()
            if not handles:
                raise RuntimeError("no GPU handles")
            self._h = handles[min(device_index, len(handles) - 1)]
            self._smi = amdsmi
            e = amdsmi.amdsmi_get_energy_count(self._h)
            if not e["counter_resolution"]:
                raise RuntimeError("energy counter has zero resolution")
            self.available = True
        except Exception as exc:  # the meter is optional: report why
            self.reason = f"{type(exc).__name__}: {exc}"

    def energy_j(self) -> float:
        e = self._smi.amdsmi_get_energy_count(self._h)
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6

    def power_w(self):
        p = self._smi.amdsmi_get_power_info(self._h)
        v = p.get("current_socket_power")
        if v in (None, "N/A"):
            v = p.get("average_socket_power")
        return None if v in (None, "N/A") else float(v)

    def _counter(self):
        e = self._smi.amdsmi_get_energy_count(self._h)
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6, e["timestamp"]

    def measure(self, fn, *, min_seconds: float = 1.0):
        """Run fn() (which queues GPU work) repeatedly until at least
        min_seconds have passed, wait for the device, and return {calls,
        seconds, joules, joules_per_call, mean_watts, samples,
        counter_watts}.  joules integrates the sampled power over the run;
        counter_watts is the energy counter's mean power between its first
        and last update inside the run (None if it advanced fewer than two
        times)."""
        if not self.available:
            raise RuntimeError(f"energy counter unavailable: {self.reason}")
        samples = []      # (host time, watts, counter joules, counter timestamp)
        stop = threading.Event()

        def sampler():
            while not stop.is_set():
                w = self.power_w()
                ej, ts = self._counter()
                samples.append((time.perf_counter(), w, ej, ts))
                stop.wait(self.interval)

        torch.cuda.synchronize()
        th = threading.Thread(target=sampler, daemon=True)
        th.start()
        time.sleep(2 * self.interval)
        t0 = time.perf_counter()
        calls = 0
        while True:
            fn()
            calls += 1
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if t1 - t0 >= min_seconds:
                break
        time.sleep(2 * self.interval)
        stop.set()
        th.join()
        sec = t1 - t0
        pw = [(t, w) for t, w, _, _ in samples if w is not None]
        joules = 0.0
        for (ta, wa), (tb, wb) in zip(pw, pw[1:]):
            lo, hi = max(ta, t0), min(tb, t1)
            if hi > lo:   # trapezoid on the part of [ta, tb] inside the run
                wl = wa + (wb - wa) * (lo - ta) / (tb - ta)
                wh = wa + (wb - wa) * (hi - ta) / (tb - ta)
                joules += 0.5 * (wl + wh) * (hi - lo)
        inside = [(ej, ts) for t, _, ej, ts in samples if t0 <= t <= t1]
        updates = []
        for ej, ts in inside:
            if not updates or ts != updates[-1][1]:
                updates.append((ej, ts))
        counter_watts = None
        if len(updates) >= 3:   # two whole counter intervals inside the run
            (e_a, ts_a), (e_b, ts_b) = updates[1], updates[-1]
            if ts_b > ts_a:
                counter_watts = (e_b - e_a) / ((ts_b - ts_a) * 1e-9)
        return {"calls": calls, "seconds": sec, "joules": joules, "joules_per_call": joules / calls,
                "mean_watts": joules / sec if sec > 0 else None,
                "samples": sum(1 for t, _ in pw if t0 <= t <= t1),
                "counter_watts": counter_watts}
