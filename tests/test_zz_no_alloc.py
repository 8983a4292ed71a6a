"""rk3_step_noalloc: rk3_step of the fused class with the library's static
device workspace, for callers that cannot allocate.  Called through the C
ABI and checked against rk3_step (same kernels, so bit for bit) and against
the FP64 oracle, on two calls in a row, the second with a smaller grid."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    import paper_1709_09713_amd as ns
    assert torch.cuda.is_available()
    return ns


def run_both(ns, n, prec, steps, seed, re=800.0, mach=0.3, dt=2e-3):
    p = ns.make_params(n, reynolds=re, mach=mach)
    Q0 = synth.random_state(n[::-1], seed=seed)
    ref = torch.as_tensor(Q0, device="cuda")
    work = torch.empty(ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, prec), dtype=torch.uint8,
                       device="cuda")
    dref = torch.zeros((steps, 8), dtype=torch.float64, device="cuda")
    ns.rk3_step(p, ns.NS_ALGO_FUSED, prec, dt, steps, ref, work, diag_dev=dref)
    got = torch.as_tensor(Q0, device="cuda")
    dgot = torch.zeros((steps, 8), dtype=torch.float64, device="cuda")
    ns.rk3_step_noalloc(p, prec, dt, steps, got, diag_dev=dgot)
    torch.cuda.synchronize()
    return Q0, p, ref.cpu().numpy(), got.cpu().numpy(), dref.cpu().numpy(), dgot.cpu().numpy()


def test_noalloc_matches_rk3_step_on_two_calls(ns):
    """FP64 then FP32 storage; in each precision a ragged 40x36x28 grid and
    then a smaller 24x20x18 one, so the second call reuses the array left by
    the first with a different layout."""
    for prec in (ns.NS_FP64, ns.NS_FP32_STORE):
        for n, steps, seed in (((40, 36, 28), 3, 11), ((24, 20, 18), 2, 12)):
            print(f"noalloc prec={prec} n={n} steps={steps}", flush=True)
            Q0, p, ref, got, dref, dgot = run_both(ns, n, prec, steps, seed)
            assert np.array_equal(got, ref), (prec, n)
            assert np.array_equal(dgot, dref), (prec, n)
            if prec == ns.NS_FP64:
                ph = oracle.Physics(n=n, reynolds=800.0, mach=0.3)
                want = oracle.rk3(ph, Q0, 2e-3, steps)
                sc = [np.abs(want[v]).max() for v in range(5)]
                sc[1:4] = [max(sc[1:4])] * 3
                e = max(float(np.abs(got[v] - want[v]).max() / sc[v]) for v in range(5))
                assert e < 1e-12, e


def test_noalloc_limit(ns):
    """A grid whose workspace exceeds the static array is refused; the
    largest cube that fits runs."""
    limit = ns.ns_noalloc_scratch_bytes()
    big = ns.make_params(96)
    assert ns.ns_workspace_bytes(big, ns.NS_ALGO_FUSED, ns.NS_FP64) > limit
    Q = torch.zeros((5, 96, 96, 96), dtype=torch.float64, device="cuda")
    with pytest.raises(ns.NativeError) as e:
        ns.rk3_step_noalloc(big, ns.NS_FP64, 1e-3, 1, Q)
    assert e.value.status == ns.NS_ERR_WORKSPACE
    n = 80
    p = ns.make_params(n)
    assert ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP64) <= limit
    Q = torch.empty((5, n, n, n), dtype=torch.float64, device="cuda")
    ns.tgv_init(p, Q)
    ref = Q.clone()
    work = torch.empty(ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP64), dtype=torch.uint8,
                       device="cuda")
    dt = synth.stable_dt(n, 0.1)
    ns.rk3_step(p, ns.NS_ALGO_FUSED, ns.NS_FP64, dt, 2, ref, work)
    ns.rk3_step_noalloc(p, ns.NS_FP64, dt, 2, Q)
    torch.cuda.synchronize()
    assert torch.equal(Q, ref)
