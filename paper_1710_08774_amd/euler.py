"""Split Godunov time stepping on top of the fused chains.

Per step: the x sweep reads smax (the CFL reduction of the current state)
and derives dt = cfl/smax in its prologue; the y sweep uses the same dt and
writes the reduction of its updated state into the other smax slot, which the
next step reads.  dt never leaves the device, so a run of steps needs no
host synchronisation and can be captured in a HIP graph.  State buffers
ping-pong between two sets of four planes (rho, rho u, rho v, E).
"""
from __future__ import annotations

import torch

from . import hfav as H


class EulerStepper:
    """fused_step=True runs each step as ONE chain (both sweeps; the
    two-sweep kernel keeps the x-swept state on chip); otherwise one chain
    per sweep.  in_place=True keeps ONE state: each sweep's goals are
    declared over its axioms (hfav_chain_alias) and written over them."""

    def __init__(self, nx, ny, dtype=torch.float64, gamma=1.4, cfl=0.5, niter=10,
                 bc=H.BC_PERIODIC, mode=H.MODE_FUSED, precision=H.PREC_NATIVE,
                 config_source=H.CONFIG_DEFAULT, forced_x=None, forced_y=None, device="cuda",
                 fused_step=False, forced_xy=None, in_place=False):
        if in_place and fused_step:
            raise ValueError("in-place execution runs one chain per sweep")
        self.nx, self.ny = nx, ny
        self.in_place = in_place
        self.dtype = dtype
        cd = H.F64 if dtype == torch.float64 else H.F32
        if cd == H.F32 and precision == H.PREC_NATIVE:
            precision = H.PREC_F32_F64ACC
        self.device = device
        self.smax_chain = H.Chain(H.smax_spec(gamma, cd))
        self.smax_chain.plan((nx, ny), (bc, bc), mode=H.MODE_AUTO)
        self.cx = H.Chain(H.euler_sweep_spec(0, gamma, niter, cfl, "smax", False, cd))
        self.cy = H.Chain(H.euler_sweep_spec(1, gamma, niter, cfl, "smax", True, cd))
        if in_place:
            for ch in (self.cx, self.cy):
                for g, a in zip(H.EULER_GOALS, H.EULER_AXIOMS):
                    ch.alias(g, a)
        fx = H.CONFIG_FORCED if forced_x is not None else config_source
        fy = H.CONFIG_FORCED if forced_y is not None else config_source
        self.ix = self.cx.plan((nx, ny), (bc, bc), mode=mode, precision=precision, config_source=fx,
                               forced=forced_x)
        self.iy = self.cy.plan((nx, ny), (bc, bc), mode=mode, precision=precision, config_source=fy,
                               forced=forced_y)
        self.cxy = self.ixy = None
        if fused_step:
            self.cxy = H.Chain(H.euler_step_spec(gamma, niter, cfl, "smax", True, cd))
            fxy = H.CONFIG_FORCED if forced_xy is not None else config_source
            self.ixy = self.cxy.plan((nx, ny), (bc, bc), mode=mode, precision=precision, config_source=fxy,
                                     forced=forced_xy)
        if in_place:
            u = torch.empty((4, ny, nx), dtype=dtype, device=device)
            self.U = [u, u]          # both sweeps read and write the one state
        else:
            self.U = [torch.empty((4, ny, nx), dtype=dtype, device=device) for _ in range(2)]
        self.smax = torch.zeros(2, dtype=torch.float64, device=device)
        ws = max(self.ix.workspace_bytes, self.iy.workspace_bytes,
                 self.ixy.workspace_bytes if self.ixy is not None else 0)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=device) if ws else None
        self.cur = 0
        self.slot = 0
        self._calls = {}

    def footprint_bytes(self):
        """Device bytes of the state buffers and the workspace."""
        states = 1 if self.in_place else 2
        return states * self.U[0].numel() * self.U[0].element_size() + (self.ws.numel() if self.ws is not None else 0)

    def load(self, U):
        self.U[0].copy_(torch.as_tensor(U, dtype=self.dtype))
        self.cur = 0
        self.slot = 0
        self.smax_chain.execute(list(self.U[0]), [self.smax[0]])

    def _bound(self, kind):
        """The execute of sweep `kind` ("x", "y" or "xy") for the current
        state and dt slot, its buffers checked once (Chain.bind)."""
        key = (kind, self.cur, self.slot)
        call = self._calls.get(key)
        if call is None or call.stale():
            a, b = self.U[self.cur], self.U[1 - self.cur]
            s0, s1 = self.smax[self.slot], self.smax[1 - self.slot]
            if kind == "xy":
                call = self.cxy.bind([a[0], a[1], a[2], a[3], s0], [b[0], b[1], b[2], b[3], s1], self.ws)
            elif kind == "x":
                call = self.cx.bind([a[0], a[1], a[2], a[3], s0], [b[0], b[1], b[2], b[3]], self.ws)
            else:
                call = self.cy.bind([b[0], b[1], b[2], b[3], s0], [a[0], a[1], a[2], a[3], s1], self.ws)
            self._calls[key] = call
        return call

    def step(self, n=1):
        for _ in range(n):
            if self.cxy is not None:
                self._bound("xy")()
                self.cur = 1 - self.cur
            else:
                self._bound("x")()
                self._bound("y")()
            self.slot = 1 - self.slot

    def sweep_x(self):
        self._bound("x")()

    def sweep_y(self):
        self._bound("y")()

    def state(self):
        return self.U[self.cur]

    def dt(self, cfl=0.5):
        return cfl / float(self.smax[self.slot])


class EulerBatchStepper:
    """Many independent grids advanced together by the persistent batched
    sweeps.  Fields are packed: plane q of grid g is U[q, off_g : off_g +
    nx_g*ny_g] (row-major (ny_g, nx_g)).  Each grid has its own dt and CFL
    slot.  `capture(steps)` records `steps` (even) steps into a HIP graph.

    fused_step=True runs each step as ONE chain (both sweeps) planned for
    the batch: one persistent launch per step whose y items wait for their
    grid's x items, the x-swept state in the workspace; otherwise one
    persistent launch per sweep."""

    def __init__(self, sizes, dtype=torch.float64, gamma=1.4, cfl=0.5, niter=10, bc=H.BC_PERIODIC,
                 precision=H.PREC_NATIVE, config_source=H.CONFIG_DEFAULT, forced_y=None, device="cuda",
                 forced_x=None, fused_step=False, forced_xy=None):
        self.sizes = [(int(a), int(b)) for a, b in sizes]
        self.dtype = dtype
        cd = H.F64 if dtype == torch.float64 else H.F32
        if cd == H.F32 and precision == H.PREC_NATIVE:
            precision = H.PREC_F32_F64ACC
        self.n = len(self.sizes)
        self.smax_chain = H.Chain(H.smax_spec(gamma, cd))
        self.smax_chain.plan_batch(self.sizes, (bc, bc))
        self.cx = H.Chain(H.euler_sweep_spec(0, gamma, niter, cfl, "smax", False, cd))
        self.cy = H.Chain(H.euler_sweep_spec(1, gamma, niter, cfl, "smax", True, cd))
        src_x = H.CONFIG_FORCED if forced_x is not None else config_source
        self.ix = self.cx.plan_batch(self.sizes, (bc, bc), precision=precision, config_source=src_x,
                                     forced=forced_x)
        src_y = H.CONFIG_FORCED if forced_y is not None else config_source
        self.iy = self.cy.plan_batch(self.sizes, (bc, bc), precision=precision, config_source=src_y,
                                     forced=forced_y)
        self.cxy = self.ixy = None
        if fused_step:
            self.cxy = H.Chain(H.euler_step_spec(gamma, niter, cfl, "smax", True, cd))
            src = H.CONFIG_FORCED if forced_xy is not None else config_source
            self.ixy = self.cxy.plan_batch(self.sizes, (bc, bc), precision=precision, config_source=src,
                                           forced=forced_xy)
        self.off = [self.cx.batch_offset(g) for g in range(self.n)]
        self.total = self.off[-1] + self.sizes[-1][0] * self.sizes[-1][1]
        self.U = [torch.empty((4, self.total), dtype=dtype, device=device) for _ in range(2)]
        self.smax = torch.zeros((2, self.n), dtype=torch.float64, device=device)
        ws = self.ixy.workspace_bytes if self.ixy is not None else 0
        self.ws = torch.empty(ws, dtype=torch.uint8, device=device) if ws else None
        self.cur = 0
        self.slot = 0
        self.graph = None
        self._calls = {}

    def cells(self):
        return sum(a * b for a, b in self.sizes)

    def y_segments(self):
        """Segment length of every grid's batched y sweep (from the plan)."""
        return self.cy.plan_json()["batch"]["y_seg"]

    def load(self, states):
        host = torch.empty((4, self.total), dtype=self.dtype)
        for g, U in enumerate(states):
            nx, ny = self.sizes[g]
            host[:, self.off[g]:self.off[g] + nx * ny] = torch.as_tensor(U, dtype=self.dtype).reshape(4, -1)
        self.U[0].copy_(host)
        self.cur = 0
        self.slot = 0
        self.smax_chain.execute(list(self.U[0]), [self.smax[0]])

    def _bound(self, kind):
        key = (kind, self.cur, self.slot)
        call = self._calls.get(key)
        if call is None or call.stale():
            a, b = self.U[self.cur], self.U[1 - self.cur]
            s0, s1 = self.smax[self.slot], self.smax[1 - self.slot]
            if kind == "xy":
                call = self.cxy.bind([a[0], a[1], a[2], a[3], s0], [b[0], b[1], b[2], b[3], s1], self.ws)
            elif kind == "x":
                call = self.cx.bind([a[0], a[1], a[2], a[3], s0], [b[0], b[1], b[2], b[3]])
            else:
                call = self.cy.bind([b[0], b[1], b[2], b[3], s0], [a[0], a[1], a[2], a[3], s1])
            self._calls[key] = call
        return call

    def step(self, n=1):
        for _ in range(n):
            if self.cxy is not None:
                self._bound("xy")()
                self.cur = 1 - self.cur
            else:
                self._bound("x")()
                self._bound("y")()
            self.slot = 1 - self.slot

    def step_status(self):
        """Status word of the last one-launch step (synchronises): 0, or bit
        0 set when a y item gave up waiting for its grid's x items (its
        cells are then not updated and its grid's CFL slot holds NaN)."""
        if self.ws is None:
            return 0
        torch.cuda.synchronize()
        return int(self.ws[:4].cpu().view(torch.int32)[0])

    def capture(self, steps):
        """Record `steps` steps (an even number, so the dt slots line up on
        every replay) into a HIP graph."""
        assert steps % 2 == 0
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        slot0, cur0 = self.slot, self.cur
        with torch.cuda.graph(g, stream=side):
            self.step(steps)
        self.slot, self.cur = slot0, cur0
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def grid(self, g):
        nx, ny = self.sizes[g]
        return self.U[self.cur][:, self.off[g]:self.off[g] + nx * ny].reshape(4, ny, nx)
