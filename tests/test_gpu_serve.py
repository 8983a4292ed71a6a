"""Continuous-batching serving loop on the GPU: requests that arrive while
others run are admitted by slot and HBM footprint, every result equals the
same request served alone (bit for bit) and the oracle within the FP32
bound; the sequential FP64 comparison matches the oracle to 1e-12; the
autotuner picks a valid launch shape and its choice keeps parity."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    import paper_1709_09713_amd as ns
    assert torch.cuda.is_available()
    ns.ns_set_fused_config(-1, 0)
    return ns


def rel(a, b):
    scale = [np.abs(b[v]).max() for v in range(5)]
    scale[1:4] = [max(scale[1:4])] * 3
    return [float(np.abs(a[v] - b[v]).max() / scale[v]) for v in range(5)]


def requests():
    spec = [(16, 1600.0, 0.1, 3.385e-3, 9), (24, 800.0, 0.3, 2e-3, 4),
            (20, 2000.0, 0.05, 1e-3, 12), (32, 500.0, 0.2, 2e-3, 6),
            (16, 3000.0, 0.4, 1e-3, 3), (28, 1200.0, 0.15, 1.5e-3, 7)]
    return [dict(rid=i, arrival=0.003 * i, n=n, reynolds=re, mach=m, dt=dt, steps=st)
            for i, (n, re, m, dt, st) in enumerate(spec)]


def want(req):
    n = (req["n"],) * 3
    ph = oracle.Physics(n=n, reynolds=req["reynolds"], mach=req["mach"])
    return oracle.rk3(ph, oracle.tgv_init(ph), req["dt"], req["steps"])


def test_server_mix_equals_alone_and_oracle(ns):
    from paper_1709_09713_amd.batch import Batch
    from paper_1709_09713_amd.serve import Server
    reqs = requests()
    # budget for about two of the larger members: admission must queue
    budget = 2 * Batch.footprint(32, "fp32")
    srv = Server("fp32", max_instances=3, hbm_budget=budget, nstreams=2, quantum=3,
                 keep_states=True)
    print("serve mix", flush=True)
    res, summ = srv.run(reqs)
    assert [r.rid for r in res] == list(range(len(reqs)))
    assert summ["requests"] == len(reqs)
    assert 0 < summ["p50_latency_s"] <= summ["p99_latency_s"]
    for r, q in zip(res, reqs):
        assert r.finished >= r.admitted >= q["arrival"]
        assert r.diag["status"] == ns.NS_OK
        print(f"  request {q['rid']} {q['n']}^3: alone", flush=True)
        alone, _ = Server("fp32", max_instances=1, nstreams=1, keep_states=True).run(
            [dict(q, arrival=0.0)])
        assert np.array_equal(r.state, alone[0].state), q["rid"]
        e = max(rel(r.state, want(q)))
        assert 1e-12 < e < 1e-5, (q["rid"], e)
        ph = oracle.Physics(n=(q["n"],) * 3, reynolds=q["reynolds"], mach=q["mach"])
        d = oracle.diagnostics(ph, r.state)
        assert r.diag["kinetic_energy"] == pytest.approx(d["kinetic_energy"], rel=1e-12)


def test_sequential_fp64_matches_oracle(ns):
    from paper_1709_09713_amd.serve import serve_sequential
    reqs = requests()[:3]
    print("serve sequential", flush=True)
    res, summ = serve_sequential(reqs, "fp64", keep_states=True)
    assert summ["requests"] == 3
    for r, q in zip(res, reqs):
        assert max(rel(r.state, want(q))) < 1e-12


def test_autotuner_choice_keeps_parity(ns, tmp_path):
    from paper_1709_09713_amd.autotune import Autotuner
    from paper_1709_09713_amd.serve import Server
    cache = str(tmp_path / "tune.json")
    tuner = Autotuner(cache, tiles=(0, 4, 6), zchunks=(0, 6), steps=2, reps=2)
    print("autotune 24^3 fp32", flush=True)
    tile, zc = tuner.lookup(24, "fp32")
    assert tile in (0, 4, 6) and zc in (0, 6)
    again = Autotuner(cache)
    assert again.lookup(24, "fp32") == (tile, zc)          # cached, no re-tune
    reqs = [r for r in requests() if r["n"] == 24]
    res, _ = Server("fp32", max_instances=2, nstreams=1, tuner=again, keep_states=True).run(reqs)
    for r, q in zip(res, reqs):
        assert max(rel(r.state, want(q))) < 1e-5
