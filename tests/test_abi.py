"""The C-ABI library loads, exports every symbol include/ns_tgv.h declares,
and validates its arguments before touching the device (CPU only: none of
these calls reaches a kernel)."""
import math
import os
import re
import subprocess

import pytest

import paper_1709_09713_amd as ns
from paper_1709_09713_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ns_tgv.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ("tgv_init", "ns_residual", "rk3_step", "diagnostics",
                 "ns_state_bytes", "ns_workspace_bytes", "ns_status_string"):
        assert name in fns
    assert tuple(fns) == nat.EXPORTS


def test_library_exports_every_declared_symbol():
    out = subprocess.check_output(["nm", "-D", "--defined-only", nat.LIB_PATH]).decode()
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in header_functions():
        assert name in syms, name
        assert getattr(ns.lib(), name) is not None


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert ns.status_string(code).startswith("NS_")


def test_sizes():
    p = ns.make_params(16)
    assert ns.ns_state_bytes(p) == 5 * 16 ** 3 * 8
    wf = ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP64)
    w32 = ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP32_STORE)
    ws = ns.ns_workspace_bytes(p, ns.NS_ALGO_STORED, ns.NS_FP64)
    assert wf >= 3 * 5 * 16 ** 3 * 8          # accumulator + two stage buffers
    assert 5 * 16 ** 3 * 16 <= w32 < wf        # float stage buffers
    assert ws >= wf + 85 * 16 ** 3 * 8         # residual + 80 work arrays
    assert ns.ns_workspace_bytes(p, ns.NS_ALGO_STORED, ns.NS_FP32_STORE) == 0
    wr = ns.ns_workspace_bytes(p, ns.NS_ALGO_SOME, ns.NS_FP64)
    assert wr >= wf + 9 * 16 ** 3 * 8 and wr < ws   # nine gradient arrays
    assert ns.ns_workspace_bytes(p, ns.NS_ALGO_SOME, ns.NS_FP32_STORE) == 0
    assert ns.ns_workspace_bytes(p, 7, ns.NS_FP64) == 0
    p2 = ns.make_params((5, 6, 7))
    assert ns.ns_state_bytes(p2) == 5 * 5 * 6 * 7 * 8


@pytest.mark.parametrize("field,value,code", [
    ("n", (4, 16, 16), ns.NS_ERR_SHAPE),
    ("n", (16, 2049, 16), ns.NS_ERR_SHAPE),
    ("n", (2048, 2048, 2048), ns.NS_ERR_SHAPE),
    ("gamma", 1.0, ns.NS_ERR_ARG),
    ("gamma", float("nan"), ns.NS_ERR_ARG),
    ("mach", 0.0, ns.NS_ERR_ARG),
    ("prandtl", -1.0, ns.NS_ERR_ARG),
    ("reynolds", float("nan"), ns.NS_ERR_ARG),
    ("reynolds", -5.0, ns.NS_ERR_ARG),
    ("length", (0.0, 1.0, 1.0), ns.NS_ERR_ARG),
])
def test_bad_params_rejected_before_any_launch(field, value, code):
    kw = dict(n=16)
    if field == "n":
        kw["n"] = value
    elif field == "length":
        kw["length"] = value
    else:
        kw[field] = value
    p = ns.make_params(**kw)
    assert ns.ns_state_bytes(p) == 0
    # a bogus but non-null device pointer: validation must fail first
    with pytest.raises(ns.NativeError) as e:
        ns.tgv_init(p, 0x1000)
    assert e.value.status == code
    with pytest.raises(ns.NativeError) as e:
        ns.rk3_step(p, ns.NS_ALGO_FUSED, ns.NS_FP64, 1e-3, 1, 0x1000, 0x1000, 1 << 40)
    assert e.value.status == code


def test_inviscid_is_valid():
    p = ns.make_params(16, reynolds=math.inf)
    assert ns.ns_state_bytes(p) > 0


def test_rk3_argument_checks():
    p = ns.make_params(16)
    wb = ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP64)
    cases = [
        (dict(dt=0.0), ns.NS_ERR_ARG),
        (dict(dt=float("inf")), ns.NS_ERR_ARG),
        (dict(nsteps=-1), ns.NS_ERR_ARG),
        (dict(state=None), ns.NS_ERR_ARG),
        (dict(work_bytes=wb - 1), ns.NS_ERR_WORKSPACE),
        (dict(work=0x1010), ns.NS_ERR_WORKSPACE),          # misaligned
        (dict(algo=ns.NS_ALGO_STORED, prec=ns.NS_FP32_STORE), ns.NS_ERR_UNSUPPORTED),
        (dict(algo=ns.NS_ALGO_SOME, prec=ns.NS_FP32_STORE), ns.NS_ERR_UNSUPPORTED),
        (dict(algo=3), ns.NS_ERR_ARG),
        (dict(prec=5), ns.NS_ERR_ARG),
    ]
    for over, code in cases:
        a = dict(algo=ns.NS_ALGO_FUSED, prec=ns.NS_FP64, dt=1e-3, nsteps=1, state=0x1000,
                 work=0x100000, work_bytes=wb)
        a.update(over)
        with pytest.raises(ns.NativeError) as e:
            ns.rk3_step(p, a["algo"], a["prec"], a["dt"], a["nsteps"], a["state"], a["work"],
                        a["work_bytes"])
        assert e.value.status == code, over


def test_residual_rejects_overlap_and_small_work():
    p = ns.make_params(16)
    with pytest.raises(ns.NativeError) as e:
        ns.ns_residual(p, ns.NS_ALGO_FUSED, 0x100000, 0x100000 + 8)
    assert e.value.status == ns.NS_ERR_ARG
    with pytest.raises(ns.NativeError) as e:
        ns.ns_residual(p, ns.NS_ALGO_STORED, 0x100000, 0x10000000, 0x20000000, 1024)
    assert e.value.status == ns.NS_ERR_WORKSPACE


def test_fused_config_validation():
    with pytest.raises(ns.NativeError):
        ns.ns_set_fused_config(len(ns.TILES), 0)
    with pytest.raises(ns.NativeError):
        ns.ns_set_fused_config(0, -1)
    p = ns.make_params(64)
    ns.ns_set_fused_config(1, 8)
    assert ns.ns_get_fused_config(p) == (1, 8)
    ns.ns_set_fused_config(-1, 0)
    t, z = ns.ns_get_fused_config(p)
    assert t in ns.TILES and 1 <= z <= 64
    # the default chunk divides the z extent into chunks of equal length
    p256 = ns.make_params(256)
    t, z = ns.ns_get_fused_config(p256)
    assert 256 % z == 0
    t32, _ = ns.ns_get_fused_config(p, ns.NS_FP32_STORE)
    assert t32 in ns.TILES


def test_package_has_no_cpu_fallback():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_1709_09713_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in src, fn


def test_batch_create_validates_before_touching_the_device():
    # (max_instances, precision, nstreams, with_diagnostics)
    for args in ((0, 0, 1, 0), (4097, 0, 1, 0), (4, 5, 1, 0), (4, 0, 0, 0), (4, 0, 9, 0)):
        with pytest.raises(ns.NativeError) as e:
            ns.ns_batch_create(*args)
        assert e.value.status == ns.NS_ERR_ARG


def test_batch_calls_reject_null_handle():
    import ctypes
    L = ns.lib()
    assert L.ns_batch_step(None, 1, None) == ns.NS_ERR_ARG
    assert L.ns_batch_set_graphs(None, 1) == ns.NS_ERR_ARG
    assert L.ns_batch_remove(None, 0) == ns.NS_ERR_ARG
    assert L.ns_batch_destroy(None) == ns.NS_ERR_ARG
    assert L.ns_batch_poll(None, None, None, None, None) == ns.NS_ERR_ARG
    assert L.ns_batch_info(None, None, None, None) == ns.NS_ERR_ARG
    slot = ctypes.c_int32()
    assert L.ns_batch_add(None, None, ctypes.byref(slot)) == ns.NS_ERR_ARG
    assert L.ns_batch_create(1, 0, 1, 0, None) == ns.NS_ERR_ARG


def test_instance_struct_matches_header():
    """ns_instance field order and offsets agree between the header and the
    ctypes binding (the struct crosses the ABI by pointer)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\} ns_instance;", text).group(1)
    names = re.findall(r"(\w+)\s*;", body)
    assert tuple(names) == tuple(f for f, _ in nat.ns_instance._fields_)
    assert nat.ns_instance.tile.offset == nat.ns_instance.steps.offset + 4
    assert nat.ns_instance.state.offset % 8 == 0


def test_fused_order_validation():
    assert ns.ns_get_fused_order() == 0
    with pytest.raises(ns.NativeError) as e:
        ns.ns_set_fused_order(2)
    assert e.value.status == ns.NS_ERR_ARG
    p = ns.make_params(16)
    wb = ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP64)
    try:
        ns.ns_set_fused_order(1)
        assert ns.ns_get_fused_order() == 1
        ns.ns_set_fused_config(1, 0)            # 16x16: order 1 is not compiled for it
        with pytest.raises(ns.NativeError) as e:
            ns.rk3_step(p, ns.NS_ALGO_FUSED, ns.NS_FP64, 1e-3, 1, 0x1000, 0x100000, wb)
        assert e.value.status == ns.NS_ERR_UNSUPPORTED
    finally:
        ns.ns_set_fused_config(-1, 0)
        ns.ns_set_fused_order(0)


def test_c_abi_rejects_misaligned_pointers():
    """State, Q and R must be 16-byte aligned (pairs of doubles are loaded
    with one access) and per-step diagnostics records 8-byte aligned; the
    check comes before any enqueue."""
    p = ns.make_params(16)
    wb = ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP64)
    calls = [
        lambda: ns.tgv_init(p, 0x1008),
        lambda: ns.rk3_step(p, ns.NS_ALGO_FUSED, ns.NS_FP64, 1e-3, 1, 0x1008, 0x100000, wb),
        lambda: ns.rk3_step(p, ns.NS_ALGO_FUSED, ns.NS_FP64, 1e-3, 1, 0x1000, 0x100000, wb,
                            diag_dev=0x2004),
        lambda: ns.ns_residual(p, ns.NS_ALGO_FUSED, 0x100008, 0x10000000),
        lambda: ns.ns_residual(p, ns.NS_ALGO_FUSED, 0x100000, 0x10000008),
        lambda: ns.diagnostics(p, 0x1008, 0x100000, wb),
    ]
    for i, call in enumerate(calls):
        with pytest.raises(ns.NativeError) as e:
            call()
        assert e.value.status == ns.NS_ERR_ARG, i


def test_binding_rejects_bad_tensors_before_the_library():
    """The Python binding refuses tensors the kernels would read or write
    past: wrong dtype, not contiguous, too small, or not on a GPU."""
    import torch
    p = ns.make_params(16)
    n5 = 5 * 16 ** 3
    wb = ns.ns_workspace_bytes(p, ns.NS_ALGO_FUSED, ns.NS_FP64)
    good_work = 0x100000
    bad_states = [
        torch.zeros(n5, dtype=torch.float32),                  # dtype
        torch.zeros((2 * n5,), dtype=torch.float64)[::2],      # not contiguous
        torch.zeros(n5 - 1, dtype=torch.float64),              # too small
        torch.zeros(n5, dtype=torch.float64),                  # host memory
    ]
    for st in bad_states:
        with pytest.raises(ns.NativeError) as e:
            ns.rk3_step(p, ns.NS_ALGO_FUSED, ns.NS_FP64, 1e-3, 1, st, good_work, wb)
        assert e.value.status == ns.NS_ERR_ARG
        with pytest.raises(ns.NativeError):
            ns.tgv_init(p, st)
        with pytest.raises(ns.NativeError):
            ns.ns_residual(p, ns.NS_ALGO_FUSED, st, 0x10000000)
        with pytest.raises(ns.NativeError):
            ns.diagnostics(p, st, good_work, wb)
    # workspace smaller than the bytes claimed for it, per-step diagnostics
    # with fewer records than steps
    with pytest.raises(ns.NativeError):
        ns.rk3_step(p, ns.NS_ALGO_FUSED, ns.NS_FP64, 1e-3, 1, 0x1000,
                    torch.zeros(16, dtype=torch.uint8), wb)
    with pytest.raises(ns.NativeError):
        ns.rk3_step(p, ns.NS_ALGO_FUSED, ns.NS_FP64, 1e-3, 3, 0x1000, good_work, wb,
                    diag_dev=torch.zeros((2, 8), dtype=torch.float64))


def test_launch_settings_are_per_thread():
    """ns_set_fused_config / ns_set_fused_order apply to the calling thread
    only: two threads with different settings, interleaved, each see their
    own, and the main thread keeps the default."""
    import threading
    p = ns.make_params(64)
    default = ns.ns_get_fused_config(p)
    barrier = threading.Barrier(2)
    seen = {}

    def worker(name, tile, zchunk, order):
        ns.ns_set_fused_config(tile, zchunk)
        ns.ns_set_fused_order(order)
        got = []
        for _ in range(50):
            barrier.wait()
            got.append((ns.ns_get_fused_config(p), ns.ns_get_fused_order()))
        seen[name] = got
        ns.ns_set_fused_config(-1, 0)
        ns.ns_set_fused_order(0)

    ts = [threading.Thread(target=worker, args=("a", 4, 6, 1)),
          threading.Thread(target=worker, args=("b", 9, 11, 0))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert set(seen["a"]) == {((4, 6), 1)}
    assert set(seen["b"]) == {((9, 11), 0)}
    assert ns.ns_get_fused_config(p) == default
    assert ns.ns_get_fused_order() == 0


def test_noalloc_validates_before_touching_the_device():
    """rk3_step_noalloc rejects arguments, and grids whose workspace exceeds
    its static array, before any device call."""
    limit = ns.ns_noalloc_scratch_bytes()
    assert limit == 64 << 20
    big = ns.make_params(128)
    assert ns.ns_workspace_bytes(big, ns.NS_ALGO_FUSED, ns.NS_FP64) > limit
    cases = [
        (big, ns.NS_FP64, 1e-3, 1, 0x1000, ns.NS_ERR_WORKSPACE),
        (ns.make_params(4), ns.NS_FP64, 1e-3, 1, 0x1000, ns.NS_ERR_SHAPE),
        (ns.make_params(16), 7, 1e-3, 1, 0x1000, ns.NS_ERR_ARG),
        (ns.make_params(16), ns.NS_FP64, 1e-3, 1, 0x1008, ns.NS_ERR_ARG),
        (ns.make_params(16), ns.NS_FP64, 0.0, 1, 0x1000, ns.NS_ERR_ARG),
        (ns.make_params(16), ns.NS_FP64, 1e-3, -1, 0x1000, ns.NS_ERR_ARG),
    ]
    for p, prec, dt, k, st, code in cases:
        with pytest.raises(ns.NativeError) as e:
            ns.rk3_step_noalloc(p, prec, dt, k, st)
        assert e.value.status == code, (p.n[:], prec, dt, k)
    # zero steps: nothing to do, nothing touched
    ns.rk3_step_noalloc(ns.make_params(16), ns.NS_FP64, 1e-3, 0, 0x1000)
