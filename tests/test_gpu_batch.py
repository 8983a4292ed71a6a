"""Tests of the persistent-kernel form of batched execution (one fused launch
per RK stage over a device-resident tile list of all members, the step
captured in a hipGraph).

That form took a GPU memory-access fault on its first run (the FP64 member
test with the 32x8 tile) and no cause could be shown on the CPU: host-side
tables, tile lists and every global and LDS address of the kernel were
checked in bounds by emulation.  The persistent kernel and its graph were
therefore removed from the library, and batching now runs the validated
per-solve launches on several streams (tests/test_gpu_batch_streams.py).
These tests stay as the record of that form and are skipped: they use its
API (tile-list capacity, one tile shape per batch) and must not run until a
persistent kernel with a shown fix exists."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="persistent-kernel batch removed after an unexplained "
                                      "GPU memory fault; see the module docstring")]

TOL = 1e-12


@pytest.fixture(scope="module")
def ns():
    import paper_1709_09713_amd as ns
    assert torch.cuda.is_available()
    return ns


def rel(a, b):
    scale = [np.abs(b[v]).max() for v in range(5)]
    scale[1:4] = [max(scale[1:4])] * 3
    return [float(np.abs(a[v] - b[v]).max() / scale[v]) for v in range(5)]


def oracle_run(n, re, mach, dt, steps):
    ph = oracle.Physics(n=tuple(n), reynolds=re, mach=mach)
    return oracle.rk3(ph, oracle.tgv_init(ph), dt, steps)


SPECS = [((16, 16, 16), 1600.0, 0.1, 3.385e-3, 4),
         ((24, 20, 18), 800.0, 0.3, 2e-3, 3),
         ((37, 21, 13), 2000.0, 0.05, 1e-3, 5)]


@pytest.mark.parametrize("tile", [0, 4])
def test_batch_members_match_oracle_fp64(ns, tile):
    b = ns.Batch(8, 1 << 14, "fp64", tile=tile)
    slots = [b.add(n, reynolds=re, mach=m, dt=dt, steps=st) for (n, re, m, dt, st) in SPECS]
    b.step(7)            # more replays than any budget: members stop at their own
    torch.cuda.synchronize()
    left, done, _ = b.poll()
    for slot, (n, re, m, dt, st) in zip(slots, SPECS):
        assert left[slot] == 0 and done[slot] == st
        got = b.members[slot][1].cpu().numpy()
        e = rel(got, oracle_run(n, re, m, dt, st))
        print(f"batch tile {tile} member {n}: rel={max(e):.2e}", flush=True)
        assert max(e) < TOL, e
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_alone_and_in_mix_are_bitwise_identical(ns, prec):
    n, re, m, dt, st = (32, 32, 32), 1000.0, 0.2, synth.stable_dt(32, 0.2), 6
    alone = ns.Batch(4, 1 << 14, prec, tile=0)
    s = alone.add(n, reynolds=re, mach=m, dt=dt, steps=st)
    alone.step(st)
    torch.cuda.synchronize()
    A = alone.members[s][1].cpu().numpy()
    alone.close()

    mix = ns.Batch(8, 1 << 15, prec, tile=0)
    mix.add((48, 48, 48), reynolds=3000.0, mach=0.4, dt=synth.stable_dt(48, 0.4), steps=9)
    mix.add((24, 24, 24), reynolds=500.0, mach=0.07, dt=synth.stable_dt(24, 0.07), steps=2)
    s2 = mix.add(n, reynolds=re, mach=m, dt=dt, steps=st)
    mix.add((40, 32, 36), reynolds=1200.0, mach=0.15, dt=1e-3, steps=12)
    mix.step(12)
    torch.cuda.synchronize()
    B = mix.members[s2][1].cpu().numpy()
    mix.close()
    assert np.array_equal(A, B)
    # and the result is the physics, not a no-op
    e = rel(A, oracle_run(n, re, m, dt, st))
    assert max(e) < (TOL if prec == "fp64" else 1e-5), e


def test_membership_changes_between_replays(ns):
    """Solves join and leave at step boundaries while others keep running;
    every replay of the captured graph is checked through the final states
    against the oracle with each member's own step count."""
    b = ns.Batch(4, 1 << 14, "fp64", tile=4)
    X = ((20, 20, 20), 1600.0, 0.1, 2e-3, 6)
    Y = ((16, 24, 20), 900.0, 0.2, 1.5e-3, 3)
    Z = ((24, 16, 16), 2500.0, 0.3, 1e-3, 2)
    sx = b.add(X[0], reynolds=X[1], mach=X[2], dt=X[3], steps=X[4])
    sy = b.add(Y[0], reynolds=Y[1], mach=Y[2], dt=Y[3], steps=Y[4])
    b.step(2)
    sz = b.add(Z[0], reynolds=Z[1], mach=Z[2], dt=Z[3], steps=Z[4])
    b.step(1)
    torch.cuda.synchronize()
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


def test_batch_per_step_diagnostics(ns):
    b = ns.Batch(4, 1 << 14, "fp64", tile=0, diagnostics=True)
    specs = [((16, 16, 16), 1600.0, 0.1, 3.385e-3, 3), ((24, 24, 24), 700.0, 0.2, 2e-3, 3)]
    slots = [b.add(n, reynolds=re, mach=m, dt=dt, steps=st) for (n, re, m, dt, st) in specs]
    b.step(3)
    torch.cuda.synchronize()
    _, _, diag = b.poll()
    for slot, (n, re, m, dt, st) in zip(slots, specs):
        ph = oracle.Physics(n=n, reynolds=re, mach=m)
        want = oracle.diagnostics(ph, oracle_run(n, re, m, dt, st - 1))   # start of last step
        for k in oracle.DIAG_NAMES:
            if k.startswith("momentum"):
                assert abs(diag[slot][k]) < 1e-11
            else:
                assert diag[slot][k] == pytest.approx(want[k], rel=1e-12)
    b.close()


def test_batch_fp32_error_bound(ns):
    b = ns.Batch(4, 1 << 15, "fp32", tile=0)
    specs = [((32, 32, 32), 1600.0, 0.1, 3.385e-3, 20), ((48, 40, 32), 400.0, 0.4, 1.5e-3, 15)]
    slots = [b.add(n, reynolds=re, mach=m, dt=dt, steps=st) for (n, re, m, dt, st) in specs]
    b.step(20)
    torch.cuda.synchronize()
    for slot, spec in zip(slots, specs):
        e = rel(b.members[slot][1].cpu().numpy(), oracle_run(*spec))
        print(f"batch fp32 member {spec[0]}: rel per field {['%.2e' % x for x in e]}", flush=True)
        assert 1e-12 < max(e) < 1e-5, e
    b.close()


def test_batch_rejects_bad_members(ns):
    b = ns.Batch(1, 64, "fp64", tile=0)
    with pytest.raises(ns.NativeError):
        b.add((128, 128, 128), reynolds=1600.0, mach=0.1, dt=1e-3, steps=1)   # too many tiles
    b.add((16, 16, 16), reynolds=1600.0, mach=0.1, dt=1e-3, steps=1)
    with pytest.raises(ns.NativeError):
        b.add((16, 16, 16), reynolds=1600.0, mach=0.1, dt=1e-3, steps=1)   # no free slot
    with pytest.raises(ns.NativeError):
        b.remove(3)
    b.close()
    assert math.isfinite(1.0)
