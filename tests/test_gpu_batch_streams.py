"""Batched execution (ns_batch_*) on the GPU: members with different grids,
Reynolds and Mach numbers, time steps, step budgets and launch shapes match
the oracle; a member gives identical bits alone and in a mix and on any
number of internal streams; members join and leave between steps."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL32 = 1e-5


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


def oracle_run(n, re, mach, dt, steps):
    ph = oracle.Physics(n=tuple(n), reynolds=re, mach=mach)
    return oracle.rk3(ph, oracle.tgv_init(ph), dt, steps)


# (grid, Re, M, dt, steps, tile)
SPECS = [((16, 16, 16), 1600.0, 0.1, 3.385e-3, 4, -1),
         ((24, 20, 18), 800.0, 0.3, 2e-3, 3, 4),
         ((37, 21, 13), 2000.0, 0.05, 1e-3, 5, 2),
         ((20, 28, 17), 1200.0, 0.2, 1.5e-3, 2, 10)]


@pytest.mark.parametrize("nstreams", [1, 4])
def test_members_match_oracle_fp64(ns, nstreams):
    print(f"batch fp64 nstreams={nstreams}", flush=True)
    b = ns.Batch(8, "fp64", nstreams=nstreams)
    slots = [b.add(n, reynolds=re, mach=m, dt=dt, steps=st, tile=t)
             for (n, re, m, dt, st, t) in SPECS]
    b.step(7)            # more steps than any budget: members stop at their own
    torch.cuda.synchronize()
    left, done, _ = b.poll()
    for slot, (n, re, m, dt, st, _) in zip(slots, SPECS):
        assert left[slot] == 0 and done[slot] == st
        got = b.members[slot][1].cpu().numpy()
        e = rel(got, oracle_run(n, re, m, dt, st))
        print(f"  member {n}: rel={max(e):.2e}", flush=True)
        assert max(e) < TOL, e
    assert b.info() == (8, len(SPECS), nstreams)
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_alone_and_in_mix_are_bitwise_identical(ns, prec):
    print(f"batch alone-vs-mix {prec}", flush=True)
    n, re, m, dt, st = (32, 32, 32), 1000.0, 0.2, synth.stable_dt(32, 0.2), 6
    alone = ns.Batch(1, prec, nstreams=1)
    s = alone.add(n, reynolds=re, mach=m, dt=dt, steps=st)
    alone.step(st)
    torch.cuda.synchronize()
    A = alone.members[s][1].cpu().numpy()
    alone.close()

    mix = ns.Batch(8, prec, nstreams=4)
    mix.add((48, 48, 48), reynolds=3000.0, mach=0.4, dt=synth.stable_dt(48, 0.4), steps=9)
    mix.add((24, 24, 24), reynolds=500.0, mach=0.07, dt=synth.stable_dt(24, 0.07), steps=2)
    s2 = mix.add(n, reynolds=re, mach=m, dt=dt, steps=st)
    mix.add((40, 32, 36), reynolds=1200.0, mach=0.15, dt=1e-3, steps=12)
    mix.step(12)
    torch.cuda.synchronize()
    B = mix.members[s2][1].cpu().numpy()
    mix.close()
    assert np.array_equal(A, B)
    # and the same bits as a plain rk3_step solve
    sol = ns.Solver(n, reynolds=re, mach=m, precision=prec).init_tgv()
    sol.step(dt, st)
    torch.cuda.synchronize()
    assert np.array_equal(sol.state.cpu().numpy(), A)
    e = rel(A, oracle_run(n, re, m, dt, st))
    print(f"  rel vs oracle {max(e):.2e}", flush=True)
    assert max(e) < (TOL if prec == "fp64" else TOL32), e


def test_membership_changes_between_steps(ns):
    """Solves join and leave at step boundaries while others keep running;
    the final states match the oracle with each member's own step count."""
    print("batch membership", flush=True)
    b = ns.Batch(4, "fp64", nstreams=2)
    X = ((20, 20, 20), 1600.0, 0.1, 2e-3, 6)
    Y = ((16, 24, 20), 900.0, 0.2, 1.5e-3, 3)
    Z = ((24, 16, 16), 2500.0, 0.3, 1e-3, 2)
    sx = b.add(X[0], reynolds=X[1], mach=X[2], dt=X[3], steps=X[4])
    sy = b.add(Y[0], reynolds=Y[1], mach=Y[2], dt=Y[3], steps=Y[4])
    b.step(2)
    sz = b.add(Z[0], reynolds=Z[1], mach=Z[2], dt=Z[3], steps=Z[4])
    b.step(1)
    left, done, _ = b.poll()
    assert (left[sx], left[sy], left[sz]) == (3, 0, 1)
    _, ystate, _ = b.remove(sy)            # Y finished: retire it
    b.step(5)
    torch.cuda.synchronize()
    left, done, _ = b.poll()
    assert left[sy] == -1 and done[sx] == 6 and done[sz] == 2
    for slot, spec in ((sx, X), (sz, Z)):
        got = b.members[slot][1].cpu().numpy()
        assert max(rel(got, oracle_run(*spec))) < TOL
    assert max(rel(ystate.cpu().numpy(), oracle_run(*Y))) < TOL
    b.close()


def test_per_step_diagnostics(ns):
    print("batch diagnostics", flush=True)
    b = ns.Batch(4, "fp64", nstreams=2, diagnostics=True)
    specs = [((16, 16, 16), 1600.0, 0.1, 3.385e-3, 3), ((24, 24, 24), 700.0, 0.2, 2e-3, 3)]
    slots = [b.add(n, reynolds=re, mach=m, dt=dt, steps=st) for (n, re, m, dt, st) in specs]
    b.step(3)
    _, _, diag = b.poll(torch.cuda.current_stream())
    for slot, (n, re, m, dt, st) in zip(slots, specs):
        ph = oracle.Physics(n=n, reynolds=re, mach=m)
        want = oracle.diagnostics(ph, oracle_run(n, re, m, dt, st - 1))   # start of last step
        for k in oracle.DIAG_NAMES:
            if k.startswith("momentum"):
                assert abs(diag[slot][k]) < 1e-11
            else:
                assert diag[slot][k] == pytest.approx(want[k], rel=1e-12)
    b.close()


def test_fp32_members_error_bound(ns):
    print("batch fp32 error", flush=True)
    b = ns.Batch(4, "fp32", nstreams=4)
    specs = [((32, 32, 32), 1600.0, 0.1, 3.385e-3, 20), ((48, 40, 32), 400.0, 0.4, 1.5e-3, 15)]
    slots = [b.add(n, reynolds=re, mach=m, dt=dt, steps=st) for (n, re, m, dt, st) in specs]
    b.step(20)
    torch.cuda.synchronize()
    for slot, spec in zip(slots, specs):
        e = rel(b.members[slot][1].cpu().numpy(), oracle_run(*spec))
        print(f"  member {spec[0]}: rel per field {['%.2e' % x for x in e]}", flush=True)
        assert 1e-12 < max(e) < TOL32, e
    b.close()


def test_rejects_bad_members(ns):
    b = ns.Batch(1, "fp64", nstreams=1)
    s = b.add((16, 16, 16), reynolds=1600.0, mach=0.1, dt=1e-3, steps=1)
    with pytest.raises(ns.NativeError) as e:
        b.add((16, 16, 16), reynolds=1600.0, mach=0.1, dt=1e-3, steps=1)   # no free slot
    assert e.value.status == ns.NS_ERR_WORKSPACE
    with pytest.raises(ns.NativeError):
        b.remove(3)
    _, state, work = b.members[s]
    b.close()
    b2 = ns.Batch(2, "fp64", nstreams=1)
    p = ns.make_params(16)
    ns.ns_batch_add(b2.handle, p, 1e-3, 1, state, work)
    with pytest.raises(ns.NativeError) as e:            # same buffers twice
        ns.ns_batch_add(b2.handle, p, 1e-3, 1, state, work)
    assert e.value.status == ns.NS_ERR_ARG
    with pytest.raises(ns.NativeError) as e:            # bad launch tile
        ns.ns_batch_add(b2.handle, p, 1e-3, 1, state, work, tile=11)
    assert e.value.status == ns.NS_ERR_ARG
    b2.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replays_match_eager(ns, prec):
    """Steps replayed from captured graphs equal the eager steps bit for bit
    after every replay, with the program's own eager work between replays;
    a member running out of steps forces a new capture."""
    print(f"batch graphs vs eager {prec}", flush=True)
    specs = [((16, 16, 16), 1600.0, 0.1, 3.385e-3, 40),
             ((24, 20, 18), 800.0, 0.3, 2e-3, 40),
             ((20, 28, 17), 1200.0, 0.2, 1.5e-3, 28)]
    eager = ns.Batch(4, prec, nstreams=2, diagnostics=True)
    graph = ns.Batch(4, prec, nstreams=2, diagnostics=True, graphs=True)
    se = [eager.add(n, reynolds=re, mach=m, dt=dt, steps=st) for n, re, m, dt, st in specs]
    sg = [graph.add(n, reynolds=re, mach=m, dt=dt, steps=st) for n, re, m, dt, st in specs]
    for chunk in range(5):          # one graph of 8 steps per call
        eager.step(8)
        graph.step(8)
        torch.cuda.synchronize()
        busy = torch.ones(1 << 20, dtype=torch.float64, device="cuda").mul_(2.0).sum()
        assert float(busy) == 2.0 * (1 << 20)
        for a, b in zip(se, sg):
            assert torch.equal(eager.members[a][1], graph.members[b][1]), (chunk, a)
        le, de, diag_e = eager.poll()
        lg, dg, diag_g = graph.poll()
        assert le == lg and de == dg
        for a, b in zip(se, sg):
            assert diag_e[a] == diag_g[b], (chunk, a)
    left, done, _ = graph.poll()
    assert [done[s] for s in sg] == [st for *_, st in specs]
    if prec == "fp64":
        for s, (n, re, m, dt, st) in zip(sg, specs):
            e = rel(graph.members[s][1].cpu().numpy(), oracle_run(n, re, m, dt, st))
            assert max(e) < TOL, e
    eager.close()
    graph.close()
