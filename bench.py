"""Benchmark: RK-stage grid-point updates/s of the fused FP64 residual + RK3
path on the 512^3 Taylor-Green vortex (Re = 1600, Pr = 0.71, M = 0.1,
gamma = 1.4, dt = 4.23125e-4), one MI355X.

A step is one full RK3 time step (three fused stage launches, the
diagnostics of the step's input state computed inside the first stage, and
the small fixed-order diagnostics reduction).  Inputs are resident in HBM
before the timed region; timing uses HIP events on the stream the kernels
run on, bracketed by device synchronisation.

Prints one JSON line.  Extra keys: ``roofline`` (dominant kernel: the fused
stage kernel; with the achievable ceiling of its access pattern measured by
``ns_stage_stream``), ``cpu_baseline`` (the FP64 oracle on the host cores:
one residual evaluation of the 512^3 state, plus the 16^3 workload in full,
a 256^3 step, single-thread rates and per-size rates for the batched and
serving mixes), ``variants`` (the 256^3 TGV in every class and precision,
the 512^3 stored and intermediate-storage classes, FP32 storage at 512^3,
the evaluation-order study and a 512x512x64 slab), ``tgv512_errors`` (the
512^3 x 50-step workload in FP64 and FP32 storage against stored oracle
samples), ``batched`` (64 independent TGV instances of mixed sizes, FP32
storage, autotuned launch shapes, against the same instances solved one
after another in FP64), ``serving`` (Poisson request streams through the
continuous-batching server over three seeds, p50/p99 latency and
throughput, against sequential FP64 solves, and runs at the measured
sustainable rate) and ``energy`` (energy to solution per step and per
update of the fused and stored classes).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import torch  # noqa: E402

import paper_1709_09713_amd as ns  # noqa: E402
import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per grid point per RK step (three stages): the
# fused FP64 path reads/writes 5-field sets of 40 B: stage 1 reads Q^n and
# writes the next stage input and the accumulator (120 B), stage 2 reads two
# and writes two (160 B), stage 3 reads two and writes the state (120 B).
BYTES_PER_POINT_STEP = {"fp64": 400.0, "fp32": 320.0}


# Sources of the fused stage kernel: traffic counters recorded for another
# version of them are not reported.
FUSED_SOURCES = ("paper_1709_09713_amd/csrc/ns_fused.hip", "paper_1709_09713_amd/csrc/ns_split.hip",
                 "paper_1709_09713_amd/csrc/ns_common.hpp")


def fused_source_hash():
    h = hashlib.sha256()
    for rel in FUSED_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class Run:
    def __init__(self, n, algo, prec, reynolds=1600.0, mach=0.1):
        shape = (n, n, n) if isinstance(n, int) else tuple(n)
        self.n = n
        self.points = shape[0] * shape[1] * shape[2]
        self.p = ns.make_params(shape, reynolds=reynolds, mach=mach)
        self.algo = ns.ALGOS[algo]
        self.prec = ns.PRECS[prec]
        self.state = torch.empty((5, shape[2], shape[1], shape[0]), dtype=torch.float64, device="cuda")
        wb = ns.ns_workspace_bytes(self.p, self.algo, self.prec)
        self.work = torch.empty(wb, dtype=torch.uint8, device="cuda")
        self.dt = synth.stable_dt(max(shape), mach)
        self.stream = torch.cuda.current_stream()
        ns.tgv_init(self.p, self.state, self.stream)

    def steps(self, k, diag=None):
        ns.rk3_step(self.p, self.algo, self.prec, self.dt, k, self.state, self.work,
                    diag_dev=diag, stream=self.stream)

    def time_steps(self, k, warmup, with_diag=True, chunks=1):
        """Time exactly k steps (HIP events on the launch stream, device
        synchronised on both sides).  With chunks > 1 (dividing k), events
        are also recorded at the chunk boundaries inside the timed region;
        the per-chunk times come back in self.chunk_ms."""
        diag = torch.zeros((max(k, warmup, 1), 8), dtype=torch.float64, device="cuda") if with_diag else None
        if warmup:
            self.steps(warmup, diag)
        torch.cuda.synchronize()
        if k % chunks:
            chunks = 1
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(chunks + 1)]
        t0 = time.perf_counter()
        ev[0].record(self.stream)
        per = k // chunks
        for c in range(chunks):
            d = diag[c * per:] if diag is not None else None
            self.steps(per, d)
            ev[c + 1].record(self.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev[0].elapsed_time(ev[-1])
        self.chunk_ms = [ev[c].elapsed_time(ev[c + 1]) for c in range(chunks)]
        return ms, wall, diag

    def free(self):
        del self.state, self.work
        torch.cuda.empty_cache()


def copy_bandwidth_gbps(nbytes=1 << 31, reps=5):
    """Device-to-device copy bandwidth (read + write bytes per second) of
    a plain torch copy of nbytes: what a simple streaming kernel reaches on
    this device, beside the 8 TB/s data-sheet peak."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / best / 1e9


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


ORACLE_CHILD_TIMEOUT_S = 300


def _oracle_child(code):
    """Run `code` (which prints one number) in a child interpreter with one
    OpenMP thread; None if it fails."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                             text=True, timeout=ORACLE_CHILD_TIMEOUT_S, check=True)
        return float(out.stdout.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError):
        return None


def cpu_baseline(n):
    """The FP64 oracle as it stands, on this host's cores.

    Headline sample: one evaluation of the residual over the whole n^3 TGV
    state (the residual is nearly all of an RK stage's oracle work; the
    pointwise update is left out), as updates/s.  Beside it: the 16^3 x 10
    workload in full (all threads and one thread), one RK3 step of the 256^3
    TGV on all threads and the residual at 2^20 sampled points of it on one
    thread, and one RK3 step per grid size of the batched / serving mixes,
    from which the oracle's time for the 64-instance batch (seed 0) and for
    a stratified sample of at least 16 requests of the serving stream is
    projected.  The recorded times of the full 256^3 x 100 and 512^3 x 50
    oracle runs behind the stored samples are added as found."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    out = {"unit": "updates/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model()}
    ph = oracle.Physics(n=(n, n, n))
    Q = oracle.tgv_init(ph)
    t0 = time.perf_counter()
    oracle.residual(ph, Q)
    sec = time.perf_counter() - t0
    del Q
    out["value"] = n ** 3 / sec
    out["sample"] = (f"one residual evaluation (one RK stage without its pointwise update) over "
                     f"the whole {n}^3 TGV state (FP64 C oracle, OpenMP over z-planes, {threads} "
                     f"threads), {sec:.1f} s")
    log(f"bench cpu: {n}^3 residual {sec:.1f} s")

    # the 16^3 x 10-step workload in full
    ph16 = oracle.Physics(n=(16, 16, 16))
    q16 = oracle.tgv_init(ph16)
    t0 = time.perf_counter()
    oracle.rk3(ph16, q16, 3.385e-3, 10)
    out["tgv16_10steps"] = {"all_threads_updates_per_s": 16 ** 3 * 30 / (time.perf_counter() - t0)}
    out["tgv16_10steps"]["single_thread_updates_per_s"] = _oracle_child(
        "import time, oracle; ph = oracle.Physics(n=(16, 16, 16)); Q = oracle.tgv_init(ph); "
        "t = time.perf_counter(); oracle.rk3(ph, Q, 3.385e-3, 10); "
        "print(16 ** 3 * 30 / (time.perf_counter() - t))")

    # 256^3: one RK3 step on all threads, residual at sampled points on one
    ph256 = oracle.Physics(n=(256, 256, 256))
    q256 = oracle.tgv_init(ph256)
    t0 = time.perf_counter()
    oracle.rk3(ph256, q256, synth.stable_dt(256, 0.1), 1)
    sec256 = time.perf_counter() - t0
    del q256
    out["tgv256_one_step"] = {"all_threads_updates_per_s": 256 ** 3 * 3 / sec256,
                              "seconds": sec256}
    out["tgv256_one_step"]["single_thread_updates_per_s"] = _oracle_child(
        "import time, oracle, synth; ph = oracle.Physics(n=(256, 256, 256)); Q = oracle.tgv_init(ph); "
        "pts = synth.sample_points((256, 256, 256), 1 << 20, seed=3); "
        "t = time.perf_counter(); oracle.residual_points(ph, Q, pts); "
        "print(pts.size / (time.perf_counter() - t))")
    out["tgv256_one_step"]["single_thread_sample"] = (
        "residual at 2^20 sampled points of the 256^3 TGV state on one thread (includes one "
        "pass of primitives over the whole grid)")
    log(f"bench cpu: 256^3 step {sec256:.1f} s")

    # one RK3 step per grid size of the batched / serving mixes
    rate = {}
    for m in synth.SERVE_SIZES:
        phm = oracle.Physics(n=(m, m, m))
        qm = oracle.tgv_init(phm)
        t0 = time.perf_counter()
        oracle.rk3(phm, qm, synth.stable_dt(m, 0.1), 1)
        rate[m] = m ** 3 * 3 / (time.perf_counter() - t0)
    out["per_size_updates_per_s"] = {str(m): r for m, r in rate.items()}
    insts = synth.batch_instances(0, 64, steps=200)
    sec_b = sum(i["n"] ** 3 * 3 * i["steps"] / rate[i["n"]] for i in insts)
    out["batched_seed0_projected"] = {
        "seconds": sec_b,
        "updates_per_s": sum(i["n"] ** 3 * 3 * i["steps"] for i in insts) / sec_b,
        "method": "every instance's N^3 x 3 x steps at the measured rate of its grid size"}
    reqs = synth.poisson_requests(0, SERVE_REQUESTS, rate_hz=50.0)
    sample = []
    for m in synth.SERVE_SIZES:             # stratified by grid size, arrival order
        sample += [r for r in reqs if r["n"] == m][:3]
    sample = sorted(sample, key=lambda r: r["rid"])      # 21 requests (>= 16)
    solve = [r["n"] ** 3 * 3 * r["steps"] / rate[r["n"]] for r in sample]
    out["serving_sample_projected"] = {
        "requests": len(sample), "rids": [r["rid"] for r in sample],
        "median_solve_seconds": float(sorted(solve)[len(solve) // 2]),
        "max_solve_seconds": float(max(solve)),
        "updates_per_s": sum(r["n"] ** 3 * 3 * r["steps"] for r in sample) / sum(solve),
        "method": "up to 3 requests of each grid size from the seed-0 stream, each request's "
                  "solve time at the measured rate of its grid size"}
    # the full 256^3 x 100 and 512^3 x 50 oracle runs, made once by
    # tests/golden/make_tgv_oracle_samples.py on the machine that wrote the
    # stored samples (not this host): their recorded time and thread count
    full = {}
    for fn, fs in ((256, 100), (512, 50)):
        z = golden(fn, fs)
        if z is not None:
            sec = float(z["oracle_seconds"])
            full[f"tgv{fn}_{fs}steps"] = {"seconds": sec, "threads": int(z["oracle_threads"]),
                                          "updates_per_s": fn ** 3 * 3 * fs / sec}
    out["full_runs_of_stored_samples"] = full
    out["paper_context_24core_ivy_bridge"] = {"BL": 2.07e7, "SN": 4.58e7}
    log(f"bench cpu: baseline {out['value']:.3e} updates/s on {threads} threads")
    return out


def stage_ceiling(n, reps=10):
    """The stage kernels' achievable HBM ceiling: ns_stage_stream moves the
    algorithmic bytes of each FP64 stage over the same buffers without the
    residual.  Returns GB/s per stage and for a whole step (400 B/point over
    the sum of the three stage times), HIP events on the launch stream."""
    p = ns.make_params(n)
    state = torch.zeros((5, n, n, n), dtype=torch.float64, device="cuda")
    work = torch.zeros(ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP64), dtype=torch.uint8,
                       device="cuda")
    stream = torch.cuda.current_stream()
    bytes_stage = {1: 120.0, 2: 160.0, 3: 120.0}
    ms = {}
    for stage in (1, 2, 3):
        for _ in range(2):
            ns.ns_stage_stream(p, stage, state, work, stream=stream)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ns.ns_stage_stream(p, stage, state, work, stream=stream)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms[stage] = sorted(times)[len(times) // 2]
    del state, work
    torch.cuda.empty_cache()
    pts = n ** 3
    out = {f"stage{k}_gbps": bytes_stage[k] * pts / (ms[k] * 1e-3) / 1e9 for k in ms}
    out["step_gbps"] = 400.0 * pts / (sum(ms.values()) * 1e-3) / 1e9
    out["stage_ms"] = ms
    return out


def golden(n, steps):
    path = os.path.join(ROOT, "tests", "golden", f"tgv{n}_{steps}steps_oracle.npz")
    if not os.path.exists(path):
        return None
    import numpy as np
    return np.load(path, allow_pickle=False)


def tgv512_errors(n=512, steps=50):
    """The 512^3 TGV (Re 1600, M 0.1) advanced `steps` steps with the fused
    kernel in FP64 and in FP32 storage.  Error of each against the FP64
    oracle: per field max|x - x_ref| / max|x_ref| (the momentum components
    sharing the momentum vector's scale) at the points stored by
    tests/golden/make_tgv_oracle_samples.py, which ran the oracle for these
    50 steps (max|x_ref| over the whole oracle state).  Without that file,
    FP32 storage is compared with the FP64 path instead, and says so."""
    import numpy as np
    p = ns.make_params(n)
    dt = synth.stable_dt(n, 0.1)
    z = golden(n, steps)
    out = {"n": n, "steps": steps, "dt": dt}
    host = {}
    for prec in ("fp64", "fp32"):
        st = torch.empty((5, n, n, n), dtype=torch.float64, device="cuda")
        wk = torch.empty(ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.PRECS[prec]),
                         dtype=torch.uint8, device="cuda")
        ns.tgv_init(p, st)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ns.rk3_step(p, ns.NS_ALGO_FUSED, ns.PRECS[prec], dt, steps, st, wk)
        e1.record()
        torch.cuda.synchronize()
        out[f"{prec}_updates_per_s"] = n ** 3 * 3 * steps / (e0.elapsed_time(e1) * 1e-3)
        if z is not None:
            pts = torch.as_tensor(z["points"], device="cuda")
            host[prec] = st.reshape(5, -1)[:, pts].cpu().numpy().T
        else:
            host[prec] = st.cpu().numpy().reshape(5, -1).T
        del st, wk
        torch.cuda.empty_cache()
    if z is not None:
        scale = [float(x) for x in z["field_max"]]
        ref = z["values"]
        out["reference"] = (f"FP64 oracle, {steps} steps, at {z['points'].size} stored points "
                            "(random, the 8 corners, full x-, y- and z-lines); scale = max|x| of "
                            "the whole oracle state")
    else:
        ref = host["fp64"]
        scale = [float(abs(ref[:, v]).max()) for v in range(5)]
        out["reference"] = "fused FP64 GPU path (no stored oracle samples found)"
    mom = max(scale[1:4])
    scale[1:4] = [mom] * 3
    for prec in ("fp64", "fp32"):
        if z is None and prec == "fp64":
            continue
        err = [float(np.abs(host[prec][:, v] - ref[:, v]).max() / scale[v]) for v in range(5)]
        out[f"{prec}_rel_error_per_field"] = err
        out[f"{prec}_rel_error_max"] = max(err)
        log(f"bench 512^3 x{steps}: {prec} rel error {max(err):.2e} ({out['reference'][:20]})")
    return out


def batched(tuner, seed=0, count=64, steps=200):
    """64 independent TGV instances (N from {32,48,64,96,128}, Re ~ U[400,
    3200], M ~ U[0.05, 0.4]), `steps` RK3 steps each: one batch in FP32
    storage with autotuned launch shapes, the same batch in FP64, and the
    instances solved one after another with rk3_step in FP64."""
    insts = synth.batch_instances(seed, count, steps=steps)
    upd = sum(i["n"] ** 3 * 3 * i["steps"] for i in insts)
    out = {"instances": count, "seed": seed, "steps": steps, "updates": upd,
           "total_points": sum(i["n"] ** 3 for i in insts)}
    stream = torch.cuda.current_stream()
    for prec, graphs in (("fp32", False), ("fp64", False), ("fp32", True)):
        b = ns.Batch(count, prec, nstreams=3, graphs=graphs)
        for i in insts:
            tile, zc = tuner.lookup(i["n"], prec)
            b.add(i["n"], reynolds=i["reynolds"], mach=i["mach"], dt=i["dt"], steps=i["steps"],
                  tile=tile, zchunk=zc, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        b.step(steps, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        b.close()
        key = f"batch_{prec}" + ("_graphs" if graphs else "")
        out[key] = {"updates_per_s": upd / (ms * 1e-3), "ms": ms, "wall_s": wall}
        log(f"bench batched {key}: {upd / (ms * 1e-3):.3e} updates/s")
    runs = []
    for i in insts:
        p = ns.make_params(i["n"], reynolds=i["reynolds"], mach=i["mach"])
        st = torch.empty((5, i["n"], i["n"], i["n"]), dtype=torch.float64, device="cuda")
        wk = torch.empty(ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP64),
                         dtype=torch.uint8, device="cuda")
        ns.tgv_init(p, st, stream)
        runs.append((p, st, wk, i))
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for p, st, wk, i in runs:
        ns.rk3_step(p, ns.NS_ALGO_FUSED, ns.NS_FP64, i["dt"], i["steps"], st, wk, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del runs
    torch.cuda.empty_cache()
    out["sequential_fp64"] = {"updates_per_s": upd / (ms * 1e-3), "ms": ms}
    out["batch_fp32_over_sequential_fp64"] = (out["batch_fp32"]["updates_per_s"]
                                              / out["sequential_fp64"]["updates_per_s"])
    log(f"bench sequential fp64: {upd / (ms * 1e-3):.3e} updates/s")
    return out


def energy(n):
    """Energy to solution of the fused and stored FP64 classes (and FP32
    storage) on the n^3 TGV: the board energy counter around a run of
    at least 2.5 seconds per variant."""
    from paper_1709_09713_amd.energy import EnergyMeter
    meter = EnergyMeter()
    if not meter.available:
        return {"available": False, "reason": meter.reason}
    out = {"available": True, "method": "AMD SMI current socket power sampled every ~10 ms, "
           "trapezoid integral over >= 2.5 s of back-to-back steps; counter_watts = the board "
           "energy counter's mean power over its whole update intervals inside the run",
           "n": n}
    for algo, prec, k in (("fused", "fp64", 100), ("fused", "fp32", 100), ("some", "fp64", 20),
                          ("stored", "fp64", 10)):
        r = Run(n, algo, prec)
        r.steps(2)
        m = meter.measure(lambda: r.steps(k), min_seconds=2.5)
        r.free()
        steps = k * m["calls"]
        upd = n ** 3 * 3 * steps
        out[f"{algo}_{prec}"] = dict(m, steps=steps, joules_per_step=m["joules"] / steps,
                                     nanojoules_per_update=m["joules"] / upd * 1e9,
                                     updates_per_s=upd / m["seconds"])
        log(f"bench energy {algo} {prec}: {m['joules'] / steps:.3f} J/step, {m['mean_watts']:.0f} W")
    out["stored_over_fused_energy_fp64"] = (out["stored_fp64"]["joules_per_step"]
                                            / out["fused_fp64"]["joules_per_step"])
    return out


SERVE_REQUESTS = 200
SERVE_SEEDS = (0, 1, 2)


def _mean_request_updates(sizes=synth.SERVE_SIZES, steps=(100, 1000)):
    """Expected N^3 x 3 x steps of one request of the serving distribution."""
    mean_pts = sum(m ** 3 for m in sizes) / len(sizes)
    return mean_pts * 3 * (steps[0] + steps[1]) / 2.0


def serving(tuner, seeds=SERVE_SEEDS, count=SERVE_REQUESTS, rate=50.0):
    """Poisson arrivals (mean gap 1/rate s); N from {32,...,192}, Re, M as
    above, steps ~ U{100..1000}; `count` requests per seed.  The
    continuous-batching server in FP32 storage against sequential
    first-come-first-served FP64 solves of the same requests.  The offered
    load exceeds what the device sustains, so these latencies are mostly
    queueing; the highest sustained rate is then measured: the server runs
    fresh streams at 0.75, 0.9 and 1.0 of the rate its measured capacity predicts,
    and a rate counts as sustained if the backlog at the last arrival stays
    within two batches of members and the last quarter's mean latency within
    twice the first quarter's."""
    from paper_1709_09713_amd.serve import Server, serve_sequential
    out = {"requests_per_seed": count, "rate_hz": rate, "seeds": {}}
    cap = []
    srv = None
    for seed in seeds:
        reqs = synth.poisson_requests(seed, count, rate_hz=rate)
        for n in sorted({r["n"] for r in reqs}):
            tuner.lookup(n, "fp32")
        torch.cuda.synchronize()
        srv = Server("fp32", max_instances=4, nstreams=3, quantum=25, tuner=tuner)
        _, s32 = srv.run(reqs)
        torch.cuda.empty_cache()
        _, s64 = serve_sequential(reqs, "fp64")
        torch.cuda.empty_cache()
        offered = sum(r["n"] ** 3 * 3 * r["steps"] for r in reqs) / (reqs[-1]["arrival"] or 1.0)
        cap.append(s32["updates_per_s"])
        out["seeds"][str(seed)] = {"continuous_batching_fp32": s32, "sequential_fp64": s64,
                                   "throughput_ratio": s32["updates_per_s"] / s64["updates_per_s"],
                                   "offered_updates_per_s": offered,
                                   "offered_over_capacity": offered / s32["updates_per_s"]}
        log(f"bench serving seed {seed}: fp32 p50 {s32['p50_latency_s']:.2f} s p99 "
            f"{s32['p99_latency_s']:.2f} s {s32['updates_per_s']:.3e} updates/s; sequential fp64 "
            f"{s64['updates_per_s']:.3e}")
    ratios = [v["throughput_ratio"] for v in out["seeds"].values()]
    out["mean_throughput_ratio"] = sum(ratios) / len(ratios)
    out["hbm_budget_bytes"] = srv.hbm_budget
    out["max_instances"] = srv.max_instances
    out["quantum_steps"] = srv.quantum
    capacity = sum(cap) / len(cap)
    wbar = _mean_request_updates()
    predicted = capacity / wbar
    out["capacity_updates_per_s"] = capacity
    out["predicted_sustainable_rate_hz"] = predicted
    runs = []
    for frac in (0.75, 0.9, 1.0):
        r_hz = frac * predicted
        reqs = synth.poisson_requests(100, count, rate_hz=r_hz)
        torch.cuda.synchronize()
        srv = Server("fp32", max_instances=4, nstreams=3, quantum=25, tuner=tuner)
        _, st = srv.run(reqs)
        torch.cuda.empty_cache()
        ok = (st["backlog_at_last_arrival"] <= 2 * srv.max_instances
              and (st["latency_last_over_first_quarter"] or 0.0) < 2.0)
        runs.append({"rate_hz": r_hz, "fraction_of_predicted": frac, "sustained": ok,
                     "seed": 100, **st})
        log(f"bench serving at {r_hz:.2f} req/s: p50 {st['p50_latency_s']:.2f} s p99 "
            f"{st['p99_latency_s']:.2f} s backlog {st['backlog_at_last_arrival']} "
            f"sustained={ok}")
    out["measured_rate_runs"] = runs
    good = [r for r in runs if r["sustained"]]
    out["sustainable_rate_hz"] = max(r["rate_hz"] for r in good) if good else None
    out["error_bound_fp32_vs_fp64_oracle"] = 1e-5
    return out


def timed_variant(vn, va, vp, vk, warm=2):
    log(f"bench variant: {vn} {va} {vp} x{vk}")
    r = Run(vn, va, vp)
    vms, _, _ = r.time_steps(vk, warm)
    pts = r.points
    r.free()
    return {"updates_per_s": pts * 3 * vk / (vms * 1e-3), "ms_per_step": vms / vk, "steps": vk}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--algo", default="fused", choices=list(ns.ALGOS))
    ap.add_argument("--precision", default="fp64", choices=list(ns.PRECS))
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-energy", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=SERVE_REQUESTS)
    ap.add_argument("--traffic-json", default=None)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                          "(multi-GPU slab decomposition is a design, not an implementation)"}))
        sys.exit(2)
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)

    n, K, W = args.n, args.steps, args.warmup
    traffic_json = args.traffic_json or os.path.join(
        ROOT, "profiles", f"fused_{args.precision}_{n}_traffic.json")
    log(f"bench: TGV {n}^3 {args.algo} {args.precision}, steps={K} warmup={W}")
    run = Run(n, args.algo, args.precision)
    ms, wall, diag = run.time_steps(K, W, chunks=5)
    upd = n ** 3 * 3 * K
    value = upd / (ms * 1e-3)
    ms_step = ms / K
    chunk_steps = K // len(run.chunk_ms)
    chunk_ms_step = sorted(c / chunk_steps for c in run.chunk_ms)
    repeats = {"chunks": len(run.chunk_ms), "steps_each": chunk_steps,
               "median_ms_per_step": chunk_ms_step[len(chunk_ms_step) // 2],
               "min_ms_per_step": chunk_ms_step[0], "max_ms_per_step": chunk_ms_step[-1]}
    d = diag[:K].cpu().numpy()
    ke = float(d[K - 1, 5])
    # kinetic-energy budget of the TGV: -dKE/dt from the per-step series
    # (central difference) beside the dissipation eps = 2 Omega / Re
    budget = None
    if K >= 3:
        dke = -(d[K - 1, 5] - d[K - 3, 5]) / (2.0 * run.dt)
        eps = float(d[K - 2, 7])
        budget = {"step": K - 2, "minus_dKE_dt": float(dke), "epsilon": eps,
                  "ratio": float(dke / eps) if eps else None}
    run_dt = run.dt
    run.free()
    log(f"bench: {ms_step:.3f} ms/step, {value:.4e} updates/s (wall {wall:.3f} s)")

    # Dominant kernel: the fused stage kernel (3 launches per step; the
    # per-step diagnostics reduction is a one-block kernel of a few us and is
    # included in the time, so the figure is conservative).
    roofline = None
    if args.algo == "fused":
        bps = BYTES_PER_POINT_STEP[args.precision]
        per_launch_bytes = bps / 3.0 * n ** 3
        avg_launch_s = ms * 1e-3 / (3 * K)
        achieved = per_launch_bytes / avg_launch_s / 1e9
        traffic = None
        if os.path.exists(traffic_json):
            with open(traffic_json) as f:
                t = json.load(f)
            if (t.get("n") == n and t.get("precision") == args.precision
                    and t.get("source_sha256") == fused_source_hash()):
                traffic = t.get("bytes_per_launch")
        copy_gbps = copy_bandwidth_gbps()
        ceil = stage_ceiling(n) if args.precision == "fp64" else None
        log(f"bench: device copy {copy_gbps:.0f} GB/s; stage kernel {achieved:.0f} GB/s algorithmic"
            + (f"; stage-pattern ceiling {ceil['step_gbps']:.0f} GB/s" if ceil else ""))
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "copy_gbps": round(copy_gbps, 1), "frac_of_copy": round(achieved / copy_gbps, 4),
                    "bytes_per_launch_algorithmic": per_launch_bytes,
                    "avg_launch_us": round(avg_launch_s * 1e6, 2)}
        if ceil:
            roofline["achievable_gbps"] = round(ceil["step_gbps"], 1)
            roofline["frac_of_achievable"] = round(achieved / ceil["step_gbps"], 4)
            roofline["achievable_detail"] = ceil

    variants = {}
    if not args.no_variants:
        for (vn, va, vp, vk) in ((256, "fused", "fp64", 40), (256, "fused", "fp32", 40),
                                 (256, "stored", "fp64", 10), (256, "some", "fp64", 20),
                                 (512, "fused", "fp32", 20), (512, "stored", "fp64", 3),
                                 (512, "some", "fp64", 5)):
            if (vn, va, vp) == (n, args.algo, args.precision):
                continue
            variants[f"{va}_{vp}_{vn}"] = timed_variant(vn, va, vp, vk)
        # evaluation-order study: the same kernels with the in-plane terms
        # grouped by derivative direction instead of by equation
        for vp, tile in (("fp64", 4), ("fp32", 0)):
            ns.ns_set_fused_config(tile, 0)
            ns.ns_set_fused_order(1)
            try:
                v = timed_variant(256, "fused", vp, 40)
            finally:
                ns.ns_set_fused_order(0)
                ns.ns_set_fused_config(-1, 0)
            variants[f"fused_{vp}_256_order_by_direction"] = dict(v, tile=tile)
        # one GPU's share of a 512^3 grid in 8 z-slabs, at its real shape
        variants["fused_fp64_slab_512x512x64"] = timed_variant((512, 512, 64), "fused", "fp64", 40)
        f512 = value if (n, args.algo, args.precision) == (512, "fused", "fp64") else None
        if f512:
            variants["fused_over_stored_512"] = f512 / variants["stored_fp64_512"]["updates_per_s"]
            variants["fused_over_some_512"] = f512 / variants["some_fp64_512"]["updates_per_s"]
        variants["fused_over_stored_256"] = (variants["fused_fp64_256"]["updates_per_s"]
                                             / variants["stored_fp64_256"]["updates_per_s"])

    errs = None
    if not args.no_variants:
        log("bench: 512^3 x 50 errors against the oracle")
        errs = tgv512_errors()

    batch_out = serve_out = None
    if not (args.no_batched and args.no_serving):
        from paper_1709_09713_amd.autotune import Autotuner
        tuner = Autotuner()
        if not args.no_batched:
            per_seed = []
            for seed in (0, 1, 2):
                log(f"bench: batched 64 instances, seed {seed}")
                per_seed.append(batched(tuner, seed=seed))
            batch_out = dict(per_seed[0])
            batch_out["seeds"] = {
                str(b["seed"]): {"batch_fp32": b["batch_fp32"]["updates_per_s"],
                                 "batch_fp32_graphs": b["batch_fp32_graphs"]["updates_per_s"],
                                 "batch_fp64": b["batch_fp64"]["updates_per_s"],
                                 "sequential_fp64": b["sequential_fp64"]["updates_per_s"],
                                 "ratio": b["batch_fp32_over_sequential_fp64"]}
                for b in per_seed}
            batch_out["mean_batch_fp32_over_sequential_fp64"] = (
                sum(b["batch_fp32_over_sequential_fp64"] for b in per_seed) / len(per_seed))
        if not args.no_serving:
            log(f"bench: serving {args.serve_requests} requests x {len(SERVE_SEEDS)} seeds")
            serve_out = serving(tuner, count=args.serve_requests)
        tuned = {k: {"tile": v["tile"], "zchunk": v["zchunk"], "ms_per_step": v["ms_per_step"],
                     "default_ms_per_step": v["default_ms_per_step"]}
                 for k, v in tuner.table.items()}
        (batch_out if batch_out is not None else serve_out)["autotuned"] = tuned

    energy_out = None
    if not args.no_energy:
        log("bench: energy to solution")
        energy_out = energy(256)

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(n)

    out = {
        "metric": "RK-stage grid-point updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-store/f64-acc",
        "data": "synthetic (analytic Taylor-Green vortex initial state)",
        "config": {"workload": f"Taylor-Green vortex {n}^3, Re=1600, Pr=0.71, M=0.1, gamma=1.4, "
                               f"dt={run_dt:g}, {args.algo} {args.precision}",
                   "n": n, "algo": args.algo, "precision": args.precision,
                   "tile_zchunk": list(ns.ns_get_fused_config(ns.make_params(n),
                                                              ns.PRECS[args.precision]))},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
        "tgv512_errors": errs,
        "batched": batch_out,
        "serving": serve_out,
        "energy": energy_out,
        "repeats": repeats,
        "kinetic_energy_last_step": ke,
        "tgv_energy_budget": budget,
        "paper_context": "paper (other hardware, 256^3 TGV): best K40c SN2 ~1.14e8, 24-core Ivy "
                         "Bridge SN 4.58e7 updates/s (derived from its runtimes); "
                         "on-the-fly ~2x faster than stored derivatives",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
