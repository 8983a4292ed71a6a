"""The stage-pattern ceiling kernel (ns_stage_stream) moves every byte it is
measured for: after stages 1, 2 and 3 each element of the state holds the
update written in the header, bit for bit, for even and odd element counts
and for counts large enough that lanes take more than one chunk."""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    import paper_1709_09713_amd as ns
    assert torch.cuda.is_available()
    return ns


@pytest.mark.parametrize("n", [(16, 12, 10), (15, 13, 11), (128, 128, 128)])
def test_three_stages_apply_the_stated_update(ns, n):
    print(f"stage stream n={n}", flush=True)
    p = ns.make_params(n)
    q0 = torch.from_numpy(synth.random_state(n[::-1], seed=5)).cuda().contiguous()
    state = q0.clone()
    work = torch.zeros(ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP64), dtype=torch.uint8,
                       device="cuda")
    for stage in (1, 2, 3):
        ns.ns_stage_stream(p, stage, state, work)
    torch.cuda.synchronize()
    # the same sequence in torch: products by 1/2 and 1/4 are exact, so
    # each step rounds once, as the kernel's multiply-add does
    s1 = q0 + 0.5 * q0
    acc = q0 + 0.25 * q0
    s2 = acc + 0.5 * s1
    acc = acc + 0.25 * s1
    want = acc + 0.5 * s2
    assert torch.equal(state, want)
