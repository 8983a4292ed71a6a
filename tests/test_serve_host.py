"""Host logic of the continuous-batching server, on the CPU: a fake device
backend stands in for the GPU (members advance on the host), and the
scheduler's admission (first come first served, by free slot and HBM
footprint), quantum accounting, retirement and latency bookkeeping are
checked."""
import pytest

from paper_1709_09713_amd.serve import Server, summarize


class FakeEvent:
    def query(self):
        return True

    def synchronize(self):
        pass


class FakeBatch:
    def __init__(self, max_instances, footprint, log):
        self.max_instances = max_instances
        self.footprint = footprint
        self.members = {}
        self.log = log

    def add(self, n, *, reynolds, mach, dt, steps, tile=-1, zchunk=0, stream=None):
        slot = next(i for i in range(self.max_instances) if i not in self.members)
        self.members[slot] = {"n": n, "steps": steps, "done": 0, "rid": len(self.log["admitted"])}
        self.log["admitted"].append(n)
        self.log["max_active"] = max(self.log["max_active"], len(self.members))
        used = sum(self.footprint(m["n"]) for m in self.members.values())
        self.log["max_used"] = max(self.log["max_used"], used)
        return slot

    def step(self, q, stream=None):
        self.log["quanta"].append(q)
        for m in self.members.values():
            m["done"] += min(q, m["steps"] - m["done"])

    def remove(self, slot):
        m = self.members.pop(slot)
        return ("params", m, "work")

    def close(self):
        pass


class FakeBackend:
    def __init__(self, max_instances):
        self.max_instances = max_instances
        self.log = {"admitted": [], "max_active": 0, "max_used": 0, "quanta": []}

    def stream(self):
        return "stream"

    def side_stream(self):
        return "side"

    def batch(self):
        return FakeBatch(self.max_instances, self.footprint, self.log)

    def event(self, stream):
        return FakeEvent()

    def diagnostics(self, p, state, work, side, ev):
        return {"status": 0, "steps_done": state["done"], "n": state["n"]}

    def footprint(self, n):
        return n ** 3

    def free_bytes(self):
        return 1 << 40

    def host_state(self, state):
        return dict(state)


def reqs(spec, gap=0.002):
    return [dict(rid=i, arrival=gap * i, n=n, reynolds=1000.0, mach=0.1, dt=1e-3, steps=st)
            for i, (n, st) in enumerate(spec)]


def test_every_request_runs_exactly_its_steps_in_fifo_order():
    spec = [(32, 7), (48, 30), (16, 3), (64, 12), (32, 1), (40, 25), (16, 60)]
    be = FakeBackend(3)
    res, summ = Server("fp32", max_instances=3, quantum=5, backend=be).run(reqs(spec))
    assert [r.rid for r in res] == list(range(len(spec)))
    for r, (n, st) in zip(res, spec):
        assert r.diag["steps_done"] == st and r.diag["n"] == n
        assert r.finished >= r.admitted >= r.arrival
    # first come first served: admitted in arrival order
    assert be.log["admitted"] == [n for n, _ in spec]
    assert [r.admitted for r in res] == sorted(r.admitted for r in res)
    assert be.log["max_active"] <= 3
    assert all(0 < q <= 5 for q in be.log["quanta"])
    assert summ["requests"] == len(spec) and summ["p50_latency_s"] <= summ["p99_latency_s"]


def test_admission_respects_the_hbm_budget():
    spec = [(40, 10), (40, 10), (40, 10), (20, 5), (40, 4)]
    be = FakeBackend(8)
    budget = 2 * 40 ** 3 + 20 ** 3 // 2     # room for two 40^3 members at a time
    res, _ = Server("fp32", max_instances=8, hbm_budget=budget, quantum=4, backend=be).run(reqs(spec))
    assert len(res) == len(spec)
    assert be.log["max_used"] <= budget
    # FIFO: the small request may not overtake the third large one
    assert be.log["admitted"] == [40, 40, 40, 20, 40]


def test_request_larger_than_budget_is_rejected():
    with pytest.raises(ValueError):
        Server("fp32", max_instances=2, hbm_budget=1000, backend=FakeBackend(2)).run(reqs([(16, 2)]))


def test_quanta_stop_at_the_next_completion():
    # with quantum 100 the loop still cuts at each member's own budget
    be = FakeBackend(4)
    Server("fp32", max_instances=4, quantum=100, backend=be).run(reqs([(16, 9), (16, 20), (16, 4)], gap=0.0))
    assert be.log["quanta"][0] == 4
    assert sum(be.log["quanta"]) == 20


def test_summary_statistics():
    class R:
        def __init__(self, n, steps, lat, arrival):
            self.n, self.steps, self.latency, self.arrival = n, steps, lat, arrival
            self.finished = arrival + lat
    rs = [R(10, 2, 1.0, 0.0), R(10, 2, 3.0, 0.5), R(10, 2, 2.0, 1.0)]
    s = summarize(rs, 0.0, 4.0)
    assert s["p50_latency_s"] == 2.0 and s["mean_latency_s"] == 2.0
    assert s["updates_per_s"] == 3 * 10 ** 3 * 3 * 2 / 4.0
    # unfinished when the last request arrived (t = 1.0): the ones finishing
    # at 3.5 and 3.0
    assert s["backlog_at_last_arrival"] == 2
    assert s["latency_last_over_first_quarter"] == 2.0


def test_summary_flags_a_growing_queue():
    """A queue that grows: each arrival waits for all earlier ones, so the
    latency climbs and work is left over at the last arrival."""
    class R:
        def __init__(self, k):
            self.n, self.steps, self.arrival = 8, 1, 0.1 * k
            self.finished = 0.3 * (k + 1)
            self.latency = self.finished - self.arrival
    s = summarize([R(k) for k in range(40)], 0.0, 12.0)
    assert s["backlog_at_last_arrival"] > 8
    assert s["latency_last_over_first_quarter"] > 2.0


def test_no_requests():
    res, summ = Server("fp32", max_instances=2, backend=FakeBackend(2)).run([])
    assert res == [] and summ["requests"] == 0
