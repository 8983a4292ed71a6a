"""A batch of independent solves held on the device, driven through the
ns_batch_* C ABI: each member runs the fused-class RK3 launches of rk3_step
under its own launch shape, members spread over a few internal HIP streams
so small grids overlap.  Each member's state and workspace are torch tensors
used as plain device buffers (caller-owned, kept alive here while the member
is in the batch)."""
from __future__ import annotations

import torch

from . import _native as nat


class Batch:
    def __init__(self, max_instances: int, precision: str = "fp32", nstreams: int = 3,
                 diagnostics: bool = False, graphs: bool = False, device="cuda"):
        self.prec = nat.PRECS[precision]
        self.precision = precision
        self.max_instances = max_instances
        self.diag = diagnostics
        self.device = torch.device(device)
        self.handle = nat.ns_batch_create(max_instances, self.prec, nstreams, diagnostics)
        self.members = {}   # slot -> (params, state, work)
        if graphs:
            self.set_graphs(True)

    def set_graphs(self, enable: bool):
        """Replay later steps through captured HIP graphs (bit-identical)."""
        nat.ns_batch_set_graphs(self.handle, enable)

    @staticmethod
    def footprint(n, precision: str) -> int:
        """Device bytes one member holds: state plus fused workspace."""
        p = nat.make_params(n)
        return nat.ns_state_bytes(p) + nat.ns_workspace_bytes(p, nat.NS_ALGO_FUSED,
                                                              nat.PRECS[precision])

    def add(self, n, *, reynolds, mach, dt, steps, state=None, init_tgv=True, tile=-1, zchunk=0,
            gamma=1.4, prandtl=0.71, length=None, stream=None):
        """Admit a solve.  With init_tgv the Taylor-Green state is written on
        `stream` (the stream later passed to step), else `state` (a
        (5, nz, ny, nx) float64 device tensor) is the initial state."""
        p = nat.make_params(n, length, gamma, prandtl, reynolds, mach)
        nx, ny, nz = p.n
        if state is None:
            state = torch.empty((5, nz, ny, nx), dtype=torch.float64, device=self.device)
        work = torch.empty(nat.ns_workspace_bytes(p, nat.NS_ALGO_FUSED, self.prec),
                           dtype=torch.uint8, device=self.device)
        if init_tgv:
            nat.tgv_init(p, state, stream)
        slot = nat.ns_batch_add(self.handle, p, dt, steps, state, work, tile=tile, zchunk=zchunk)
        self.members[slot] = (p, state, work)
        return slot

    def remove(self, slot):
        """Retire a slot; returns (params, state, work) of the member."""
        nat.ns_batch_remove(self.handle, slot)
        return self.members.pop(slot)

    def step(self, nsteps=1, stream=None):
        nat.ns_batch_step(self.handle, nsteps, stream)

    def poll(self, stream=None):
        return nat.ns_batch_poll(self.handle, self.max_instances, self.diag, stream)

    def info(self):
        return nat.ns_batch_info(self.handle)

    def close(self):
        if self.handle:
            nat.ns_batch_destroy(self.handle)
            self.handle = None
            self.members.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
