"""ctypes binding of ``libns_tgv.so`` (the C ABI declared in
``include/ns_tgv.h``).  Argument marshalling only: every step of the
residual / RK3 path runs in the HIP kernels of the library.

Device buffers are passed as raw device addresses (``int``) or as torch CUDA
tensors (their ``data_ptr()``); PyTorch is used for device memory and streams
only.  There is no CPU fallback: if the library is missing, loading fails
with an error that says how to build it.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libns_tgv.so")

NS_OK = 0
NS_ERR_ARG = -1
NS_ERR_SHAPE = -2
NS_ERR_WORKSPACE = -3
NS_ERR_DEVICE = -4
NS_ERR_NONFINITE = -5
NS_ERR_NOMEM = -6
NS_ERR_UNSUPPORTED = -7

NS_ALGO_STORED = 0
NS_ALGO_FUSED = 1
NS_ALGO_SOME = 2
NS_FP64 = 0
NS_FP32_STORE = 1

ALGOS = {"stored": NS_ALGO_STORED, "fused": NS_ALGO_FUSED, "some": NS_ALGO_SOME}
PRECS = {"fp64": NS_FP64, "fp32": NS_FP32_STORE}

# tile code -> (BX, BY) column tile of one block; codes 8-10 run two threads
# per column (momentum in one wave group; mass, energy and the viscous terms in the other)
TILES = {0: (32, 8), 1: (16, 16), 2: (64, 4), 3: (32, 16), 4: (16, 8), 5: (32, 4),
         6: (16, 4), 7: (8, 8), 8: (16, 8), 9: (32, 8), 10: (16, 4)}


class ns_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("length", ctypes.c_double * 3),
                ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("reynolds", ctypes.c_double), ("mach", ctypes.c_double)]


class ns_diag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
                ("energy", ctypes.c_double), ("kinetic_energy", ctypes.c_double),
                ("enstrophy", ctypes.c_double), ("dissipation", ctypes.c_double)]

    def as_dict(self):
        return {"mass": self.mass, "momentum_x": self.momentum[0],
                "momentum_y": self.momentum[1], "momentum_z": self.momentum[2],
                "energy": self.energy, "kinetic_energy": self.kinetic_energy,
                "enstrophy": self.enstrophy, "dissipation": self.dissipation}


DIAG_NAMES = ("mass", "momentum_x", "momentum_y", "momentum_z", "energy",
              "kinetic_energy", "enstrophy", "dissipation")

class ns_instance(ctypes.Structure):
    _fields_ = [("p", ns_params), ("dt", ctypes.c_double), ("steps", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("zchunk", ctypes.c_int32), ("state", ctypes.c_void_p),
                ("work", ctypes.c_void_p), ("work_bytes", ctypes.c_size_t)]


# Exported C symbols, in header order.
EXPORTS = ("ns_status_string", "ns_state_bytes", "ns_workspace_bytes",
           "tgv_init", "ns_residual", "rk3_step", "rk3_step_noalloc", "ns_noalloc_scratch_bytes",
           "diagnostics", "ns_stage_stream",
           "ns_set_fused_config", "ns_get_fused_config", "ns_set_fused_order",
           "ns_get_fused_order",
           "ns_batch_create", "ns_batch_destroy", "ns_batch_add", "ns_batch_remove",
           "ns_batch_step", "ns_batch_set_graphs", "ns_batch_poll", "ns_batch_info")


_STATUS_TEXT = {NS_ERR_ARG: "NS_ERR_ARG: invalid argument"}


class NativeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        text = _STATUS_TEXT.get(status) if _lib is None else None
        super().__init__(f"{where}: {text or status_string(status)} ({status})")


_lib = None


def lib():
    """The loaded library (ctypes.CDLL); raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'` "
                "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(ns_params)
        vp, sz, i32, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
        L.ns_status_string.restype = ctypes.c_char_p
        L.ns_status_string.argtypes = [ctypes.c_int]
        L.ns_state_bytes.restype = sz
        L.ns_state_bytes.argtypes = [P]
        L.ns_workspace_bytes.restype = sz
        L.ns_workspace_bytes.argtypes = [P, ctypes.c_int, ctypes.c_int]
        L.tgv_init.restype = ctypes.c_int
        L.tgv_init.argtypes = [P, vp, vp]
        L.ns_residual.restype = ctypes.c_int
        L.ns_residual.argtypes = [P, ctypes.c_int, vp, vp, vp, sz, vp]
        L.rk3_step.restype = ctypes.c_int
        L.rk3_step.argtypes = [P, ctypes.c_int, ctypes.c_int, d, i32, vp, vp, sz, vp, vp]
        L.rk3_step_noalloc.restype = ctypes.c_int
        L.rk3_step_noalloc.argtypes = [P, ctypes.c_int, d, i32, vp, vp, vp]
        L.ns_noalloc_scratch_bytes.restype = sz
        L.ns_noalloc_scratch_bytes.argtypes = []
        L.diagnostics.restype = ctypes.c_int
        L.diagnostics.argtypes = [P, vp, ctypes.POINTER(ns_diag), vp, sz, vp]
        L.ns_stage_stream.restype = ctypes.c_int
        L.ns_stage_stream.argtypes = [P, i32, vp, vp, sz, vp]
        L.ns_set_fused_config.restype = ctypes.c_int
        L.ns_set_fused_config.argtypes = [i32, i32]
        L.ns_get_fused_config.restype = ctypes.c_int
        L.ns_get_fused_config.argtypes = [P, ctypes.c_int, ctypes.POINTER(i32),
                                          ctypes.POINTER(i32)]
        L.ns_set_fused_order.restype = ctypes.c_int
        L.ns_set_fused_order.argtypes = [i32]
        L.ns_get_fused_order.restype = i32
        L.ns_get_fused_order.argtypes = []
        pi32 = ctypes.POINTER(i32)
        for f, args in (("ns_batch_create", [i32, ctypes.c_int, i32, i32, ctypes.POINTER(vp)]),
                        ("ns_batch_destroy", [vp]),
                        ("ns_batch_add", [vp, ctypes.POINTER(ns_instance), pi32]),
                        ("ns_batch_remove", [vp, i32]),
                        ("ns_batch_step", [vp, i32, vp]),
                        ("ns_batch_set_graphs", [vp, i32]),
                        ("ns_batch_poll", [vp, pi32, pi32, ctypes.POINTER(ns_diag), vp]),
                        ("ns_batch_info", [vp, pi32, pi32, pi32])):
            getattr(L, f).restype = ctypes.c_int
            getattr(L, f).argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().ns_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != NS_OK:
        raise NativeError(status, where)


def make_params(n, length=None, gamma=1.4, prandtl=0.71, reynolds=1600.0,
                mach=0.1) -> ns_params:
    if isinstance(n, int):
        n = (n, n, n)
    if length is None:
        length = (2 * math.pi,) * 3
    p = ns_params()
    p.n[:] = [int(x) for x in n]
    p.length[:] = [float(x) for x in length]
    p.gamma, p.prandtl, p.reynolds, p.mach = (float(gamma), float(prandtl),
                                              float(reynolds), float(mach))
    return p


def _ptr(x, where: str = "buffer", dtype: str | None = None, min_bytes: int = 0) -> int | None:
    """Device address of x: an int is taken as a raw device address (the C
    side still checks null and alignment); a tensor must be a contiguous CUDA
    tensor of ``dtype`` (e.g. "float64") holding at least ``min_bytes`` bytes,
    else NativeError(NS_ERR_ARG) is raised before anything reaches the
    library."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not hasattr(x, "data_ptr"):
        raise NativeError(NS_ERR_ARG, f"{where}: expected a device tensor or an address")
    if dtype is not None and str(x.dtype) != "torch." + dtype:
        raise NativeError(NS_ERR_ARG, f"{where}: dtype {x.dtype}, expected {dtype}")
    if not x.is_contiguous():
        raise NativeError(NS_ERR_ARG, f"{where}: tensor is not contiguous")
    nbytes = x.numel() * x.element_size()
    if nbytes < min_bytes:
        raise NativeError(NS_ERR_ARG, f"{where}: {nbytes} bytes, needs {min_bytes}")
    if x.device.type != "cuda":
        raise NativeError(NS_ERR_ARG, f"{where}: tensor on {x.device}, expected a CUDA device")
    return x.data_ptr()


def _nbytes(x) -> int:
    return x.numel() * x.element_size()


def _stream(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def ns_state_bytes(p: ns_params) -> int:
    return lib().ns_state_bytes(ctypes.byref(p))


def ns_workspace_bytes(p: ns_params, algo: int, prec: int = NS_FP64) -> int:
    return lib().ns_workspace_bytes(ctypes.byref(p), int(algo), int(prec))


def tgv_init(p: ns_params, state, stream=None):
    st = _ptr(state, "tgv_init state", "float64", ns_state_bytes(p))
    _check(lib().tgv_init(ctypes.byref(p), st, _stream(stream)), "tgv_init")


def ns_residual(p: ns_params, algo: int, Q, R, work=None, work_bytes: int = 0,
                stream=None):
    if work is not None and work_bytes == 0 and not isinstance(work, int):
        work_bytes = _nbytes(work)
    sb = ns_state_bytes(p)
    q = _ptr(Q, "ns_residual Q", "float64", sb)
    r = _ptr(R, "ns_residual R", "float64", sb)
    w = _ptr(work, "ns_residual work", None, work_bytes)
    _check(lib().ns_residual(ctypes.byref(p), int(algo), q, r, w, work_bytes, _stream(stream)),
           "ns_residual")


def rk3_step(p: ns_params, algo: int, prec: int, dt: float, nsteps: int, state,
             work, work_bytes: int = 0, diag_dev=None, stream=None):
    if work_bytes == 0 and work is not None and not isinstance(work, int):
        work_bytes = _nbytes(work)
    st = _ptr(state, "rk3_step state", "float64", ns_state_bytes(p))
    w = _ptr(work, "rk3_step work", None, work_bytes)
    d = _ptr(diag_dev, "rk3_step diag_dev", "float64", 64 * max(int(nsteps), 0))
    _check(lib().rk3_step(ctypes.byref(p), int(algo), int(prec), float(dt), int(nsteps),
                          st, w, work_bytes, d, _stream(stream)), "rk3_step")


def rk3_step_noalloc(p: ns_params, prec: int, dt: float, nsteps: int, state, diag_dev=None,
                     stream=None):
    """rk3_step of the fused class with the library's static device
    workspace (for callers that cannot allocate)."""
    st = _ptr(state, "rk3_step_noalloc state", "float64", ns_state_bytes(p))
    d = _ptr(diag_dev, "rk3_step_noalloc diag_dev", "float64", 64 * max(int(nsteps), 0))
    _check(lib().rk3_step_noalloc(ctypes.byref(p), int(prec), float(dt), int(nsteps), st, d,
                                  _stream(stream)), "rk3_step_noalloc")


def ns_noalloc_scratch_bytes() -> int:
    return int(lib().ns_noalloc_scratch_bytes())


def diagnostics(p: ns_params, state, work, work_bytes: int = 0, stream=None) -> dict:
    if work_bytes == 0 and work is not None and not isinstance(work, int):
        work_bytes = _nbytes(work)
    sp = _ptr(state, "diagnostics state", "float64", ns_state_bytes(p))
    w = _ptr(work, "diagnostics work", None, work_bytes)
    out = ns_diag()
    st = lib().diagnostics(ctypes.byref(p), sp, ctypes.byref(out), w, work_bytes, _stream(stream))
    if st not in (NS_OK, NS_ERR_NONFINITE):
        _check(st, "diagnostics")
    d = out.as_dict()
    d["status"] = st
    return d


def ns_stage_stream(p: ns_params, stage: int, state, work, work_bytes: int = 0, stream=None):
    """The bytes of fused RK stage `stage` without the residual (the memory
    system's ceiling for the stage kernel); overwrites state and work."""
    if work_bytes == 0 and work is not None and not isinstance(work, int):
        work_bytes = _nbytes(work)
    st = _ptr(state, "ns_stage_stream state", "float64", ns_state_bytes(p))
    w = _ptr(work, "ns_stage_stream work", None, work_bytes)
    _check(lib().ns_stage_stream(ctypes.byref(p), int(stage), st, w, work_bytes, _stream(stream)),
           "ns_stage_stream")


def ns_set_fused_config(tile: int, zchunk: int = 0):
    _check(lib().ns_set_fused_config(int(tile), int(zchunk)), "ns_set_fused_config")


def ns_get_fused_config(p: ns_params, prec: int = NS_FP64):
    t, z = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().ns_get_fused_config(ctypes.byref(p), int(prec), ctypes.byref(t),
                                     ctypes.byref(z)), "ns_get_fused_config")
    return t.value, z.value


def ns_set_fused_order(order: int):
    _check(lib().ns_set_fused_order(int(order)), "ns_set_fused_order")


def ns_get_fused_order() -> int:
    return int(lib().ns_get_fused_order())


# ---------------------------------------------------------------------------
# Batched execution (ns_batch_*)

def ns_batch_create(max_instances: int, prec: int, nstreams: int = 3,
                    with_diagnostics: bool = False) -> int:
    h = ctypes.c_void_p()
    _check(lib().ns_batch_create(int(max_instances), int(prec), int(nstreams),
                                 1 if with_diagnostics else 0, ctypes.byref(h)), "ns_batch_create")
    return h.value


def ns_batch_destroy(handle: int):
    _check(lib().ns_batch_destroy(handle), "ns_batch_destroy")


def ns_batch_add(handle: int, p: ns_params, dt: float, steps: int, state, work,
                 work_bytes: int = 0, tile: int = -1, zchunk: int = 0) -> int:
    if work_bytes == 0 and not isinstance(work, int):
        work_bytes = _nbytes(work)
    st = _ptr(state, "ns_batch_add state", "float64", ns_state_bytes(p))
    w = _ptr(work, "ns_batch_add work", None, work_bytes)
    inst = ns_instance(p, float(dt), int(steps), int(tile), int(zchunk), st, w, work_bytes)
    slot = ctypes.c_int32()
    _check(lib().ns_batch_add(handle, ctypes.byref(inst), ctypes.byref(slot)), "ns_batch_add")
    return slot.value


def ns_batch_remove(handle: int, slot: int):
    _check(lib().ns_batch_remove(handle, int(slot)), "ns_batch_remove")


def ns_batch_step(handle: int, nsteps: int, stream=None):
    _check(lib().ns_batch_step(handle, int(nsteps), _stream(stream)), "ns_batch_step")


def ns_batch_set_graphs(handle: int, enable: bool):
    _check(lib().ns_batch_set_graphs(handle, 1 if enable else 0), "ns_batch_set_graphs")


def ns_batch_info(handle: int):
    """(max_instances, active members, internal streams)."""
    m, a, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().ns_batch_info(handle, ctypes.byref(m), ctypes.byref(a), ctypes.byref(s)),
           "ns_batch_info")
    return m.value, a.value, s.value


def ns_batch_poll(handle: int, max_instances: int, with_diag: bool = False, stream=None):
    """(steps_left list, steps_done list, diag list of dicts or None)."""
    left = (ctypes.c_int32 * max_instances)()
    done = (ctypes.c_int32 * max_instances)()
    diag = (ns_diag * max_instances)() if with_diag else None
    _check(lib().ns_batch_poll(handle, left, done, diag, _stream(stream)), "ns_batch_poll")
    return (list(left), list(done), [d.as_dict() for d in diag] if with_diag else None)
