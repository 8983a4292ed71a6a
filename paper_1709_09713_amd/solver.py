"""One solve held in device memory: state + workspace (torch tensors used
as plain device buffers) driven through the C ABI."""
from __future__ import annotations

import torch

from . import _native as nat


class Solver:
    """A periodic TGV solve on the current CUDA (HIP) device.

    algo: "fused", "stored" or "some" (intermediate storage: nine
    velocity-gradient arrays); precision: "fp64" or "fp32" (FP32 storage of
    the stage inputs, fused class only).
    """

    def __init__(self, n, *, reynolds=1600.0, mach=0.1, gamma=1.4, prandtl=0.71,
                 length=None, algo="fused", precision="fp64", device="cuda"):
        self.params = nat.make_params(n, length, gamma, prandtl, reynolds, mach)
        self.algo = nat.ALGOS[algo]
        self.prec = nat.PRECS[precision]
        nx, ny, nz = self.params.n
        self.shape = (5, nz, ny, nx)
        self.device = torch.device(device)
        self.state = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        wb = nat.ns_workspace_bytes(self.params, self.algo, self.prec)
        if wb == 0:
            raise nat.NativeError(nat.NS_ERR_UNSUPPORTED, "Solver workspace")
        self.work = torch.empty(wb, dtype=torch.uint8, device=self.device)

    def init_tgv(self, stream=None):
        nat.tgv_init(self.params, self.state, stream)
        return self

    def set_state(self, Q):
        self.state.copy_(torch.as_tensor(Q, dtype=torch.float64))
        return self

    def step(self, dt: float, nsteps: int = 1, diag=None, stream=None):
        """Advance nsteps RK3 steps; diag: optional float64 device tensor of
        shape (nsteps, 8) receiving the per-step diagnostics."""
        nat.rk3_step(self.params, self.algo, self.prec, dt, nsteps, self.state, self.work,
                     diag_dev=diag, stream=stream)
        return self

    def residual(self, Q=None, stream=None):
        Q = self.state if Q is None else Q
        R = torch.empty_like(Q)
        nat.ns_residual(self.params, self.algo, Q, R, self.work, stream=stream)
        return R

    def diagnostics(self, stream=None) -> dict:
        return nat.diagnostics(self.params, self.state, self.work, stream=stream)
