"""Gradient of a time-averaged body torque through the PSM hot path.

Objective (one body): J = sum_t w(t) * a . T(t), T the torque of eq. (11) on
the body about its centre, a the rotation axis, w the window weights (e.g.
1/200 on the last 200 of 800 steps).  Parameters: a time-invariant offset
field dB added to the solid fraction (B_eff = B_map(t) + dB) and the rotation
rate Omega, which enters the solid velocity u_s = V + Omega a x (x - X).
Frozen-B convention: the mapping B_map(t) follows the prescribed motion and
is not differentiated (it is piecewise constant in the angle).

Reverse mode keeps the forward trajectory in one of two ways.  sqrt(T)
checkpointing: the forward keeps the lattice every L steps (L even, so
checkpoints sit in the standard in-place layout); the backward recomputes each
segment, storing its L states (copies of the PDF buffer) and the solid
fractions B(t) the recompute mapped, then runs L adjoint steps
(psm_adjoint_step, one HIP kernel per step) from the last to the first with
each step's stored B(t) put back (no second mapping).  Whole trajectory (when
T states and T copies of B fit the memory budget, e.g. the 128^3 FP32 rotor's
800 steps in about 136 GB of HBM): the forward stores every state and B(t)
itself and the backward runs the adjoint steps only, with no recompute.  Both
feed the adjoint step the same states and fractions, so their results are
bit-identical.  All arithmetic and copies run in the library's kernels; torch
only owns the buffers.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _capi as capi
from . import sim
from ._capi import check, lib


class TorqueAdjoint:
    def __init__(self, wl, steps: int, weights, storage=None, segment: int | None = None, device="cuda",
                 store_all: bool | None = None, memory_budget: int | None = None):
        """``store_all``: keep the whole trajectory (True), checkpoint every
        ``segment`` steps (False), or decide by size (None: the whole
        trajectory if it needs at most ``memory_budget`` bytes, default half
        of the device's free memory)."""
        if len(wl.bodies) != 1:
            raise ValueError("the torque objective takes exactly one body")
        self.wl = wl
        self.steps = int(steps)
        self.weights = [float(w) for w in weights]
        if len(self.weights) != self.steps:
            raise ValueError("one weight per step")
        self.field = sim.Field(wl, storage=storage, slots=1, device=device, map_ahead=False)
        self.q, self.N = wl.q, wl.n_cells
        # adjoint buffers: the PDF buffer's layout, adjoint-precision elements
        self.aelems = self.field.pdf.numel()
        L = segment or int(math.ceil(math.sqrt(self.steps)))
        self.L = max(2, L + (L & 1))
        self.adt = torch.float64 if self.field.storage == "f64" else torch.float32
        self.body = wl.bodies[0]
        self.axis = (C.c_double * 3)(*self.body.motion.axis)
        self.device = device
        self._ckpt = {}
        self._ckpt_pool = []
        self._store = None
        self._bstore = None
        self.omega = self.body.motion.omega
        need = self.steps * (self.field.pdf.numel() * self.field.pdf.element_size() + self.field.bbuf.numel())
        if store_all is None:
            budget = memory_budget if memory_budget is not None else torch.cuda.mem_get_info(device)[0] // 2
            store_all = need <= budget
        self.store_all = bool(store_all)
        self.trajectory_bytes = need if self.store_all else 0
        self._states = []
        self._bst = []
        self.dB = None
        self.ft = torch.zeros((self.steps, 6), dtype=torch.float64, device=device)

    # -- poses: mapping from the prescribed motion, u_s from the rate --------
    def _poses(self, t):
        pm = self.field.poses(t)
        pu = (capi.psm_body * 1)()
        C.memmove(C.byref(pu), C.byref(pm), C.sizeof(capi.psm_body))
        pu[0].W = (C.c_double * 3)(*[self.omega * a for a in self.body.motion.axis])
        return pm, pu

    def _step(self, t, ft=None):
        pm, pu = self._poses(t)
        f = self.field
        check(lib.psm_step(f.handle, pm, pu, f._geom_ptrs, 1, int(t),
                           C.c_void_p(ft.data_ptr()) if ft is not None else None, sim._stream()), "psm_step")
        return pu

    def _set_offset(self, dB):
        self.dB = None if dB is None else dB.detach().to(device=self.device, dtype=torch.float32).contiguous()
        ptr = C.c_void_p(self.dB.data_ptr()) if self.dB is not None else None
        check(lib.psm_set_fraction_offset(self.field.handle, ptr), "psm_set_fraction_offset")

    def forward(self, dB=None, omega=None, f0=None) -> float:
        """Run the steps from rest (or the deviation state f0, (q, N) in the
        library's direction order) and return J; keeps the checkpoints."""
        self.omega = self.body.motion.omega if omega is None else float(omega)
        self._set_offset(dB)
        self.field.reset()
        if f0 is not None:
            self.field.load_pdf_std(f0)
        self._ckpt = {}
        if self.store_all:
            f = self.field
            while len(self._states) < self.steps:
                self._states.append(torch.empty_like(f.pdf))
                self._bst.append(torch.empty_like(f.bbuf))
            for t in range(self.steps):
                sim.stream_copy(f.pdf, self._states[t])
                self._step(t, ft=self.ft[t])
                sim.stream_copy(f.bbuf, self._bst[t])
        else:
            nck = (self.steps + self.L - 1) // self.L
            while len(self._ckpt_pool) < nck:
                self._ckpt_pool.append(torch.empty_like(self.field.pdf))
            for t in range(self.steps):
                if t % self.L == 0:
                    ck = self._ckpt_pool[t // self.L]
                    sim.stream_copy(self.field.pdf, ck)
                    self._ckpt[t] = ck
                self._step(t, ft=self.ft[t])
        a = torch.tensor(list(self.body.motion.axis), dtype=torch.float64, device=self.device)
        w = torch.tensor(self.weights, dtype=torch.float64, device=self.device)
        return float((w * (self.ft[:, 3:] @ a)).sum().item())

    def backward(self):
        """(dJ/d dB (N,), dJ/dOmega, dJ/d f0 (q, N)) for the last forward."""
        q, N = self.q, self.N
        f = self.field
        if not self.store_all and (self._store is None or len(self._store) < self.L):
            self._store = [torch.empty_like(f.pdf) for _ in range(self.L)]
            self._bstore = [torch.empty_like(f.bbuf) for _ in range(self.L)]
        ahat = [torch.zeros(self.aelems, dtype=self.adt, device=self.device),
                torch.empty(self.aelems, dtype=self.adt, device=self.device)]
        gB = torch.zeros(N, dtype=self.adt, device=self.device)
        gW = torch.zeros(1, dtype=torch.float64, device=self.device)
        stream = sim._stream()

        def adjoint_step(t, state, bstore):
            pm, pu = self._poses(t)
            sim.stream_copy(bstore, f.bbuf)
            check(lib.psm_adjoint_step(f.handle, C.c_void_p(state.data_ptr()), t, C.c_void_p(ahat[0].data_ptr()),
                                       C.c_void_p(ahat[1].data_ptr()), C.c_void_p(gB.data_ptr()), pu, self.axis,
                                       self.weights[t], stream), "psm_adjoint_step")
            check(lib.psm_adjoint_omega(f.handle, C.c_void_p(gW.data_ptr()), stream), "psm_adjoint_omega")
            ahat.reverse()

        if self.store_all:
            for t in range(self.steps - 1, -1, -1):
                adjoint_step(t, self._states[t], self._bst[t])
        for s0 in sorted(self._ckpt.keys(), reverse=True):
            s1 = min(s0 + self.L, self.steps)
            # B is put back from the store below, outside the mapping's
            # bookkeeping: restart the mapping from a cleared field
            f.reset()
            sim.stream_copy(self._ckpt[s0], f.pdf)
            for t in range(s0, s1):
                sim.stream_copy(f.pdf, self._store[t - s0])
                self._step(t)
                sim.stream_copy(f.bbuf, self._bstore[t - s0])
            for t in range(s1 - 1, s0 - 1, -1):
                adjoint_step(t, self._store[t - s0], self._bstore[t - s0])
        gF = torch.empty((q, N), dtype=self.adt, device=self.device)
        check(lib.psm_adjoint_gather(f.handle, C.c_void_p(ahat[0].data_ptr()), C.c_void_p(gF.data_ptr()), stream),
              "psm_adjoint_gather")
        return gB, float(gW.item()), gF


class PSMTorque(torch.autograd.Function):
    """J = PSMTorque.apply(dB, omega, objective): forward runs the steps,
    backward returns dJ/d dB and dJ/domega from the adjoint sweep."""

    @staticmethod
    def forward(ctx, dB, omega, objective: TorqueAdjoint):
        use_dB = dB is not None and bool(torch.any(dB != 0))
        J = objective.forward(dB=dB if use_dB else None, omega=float(omega))
        ctx.objective = objective
        ctx.dB_meta = (dB.shape, dB.dtype, dB.device) if dB is not None else None
        ctx.omega_meta = (omega.dtype, omega.device) if torch.is_tensor(omega) else None
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        gB, gW, _ = ctx.objective.backward()
        g = gJ.item()
        dB_grad = None
        if ctx.dB_meta is not None:
            shape, dtype, dev = ctx.dB_meta
            dB_grad = (gB * g).to(dtype=dtype, device=dev).reshape(shape)
        om_grad = None
        if ctx.omega_meta is not None:
            om_grad = torch.tensor(gW * g, dtype=ctx.omega_meta[0], device=ctx.omega_meta[1])
        return dB_grad, om_grad, None
