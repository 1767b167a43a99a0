"""Thin driver over the C ABI: torch owns device memory and streams.

``Field`` allocates the caller-owned buffers of one lattice as torch tensors,
creates the library handle and its geometry fields, and calls the per-step
entry points (geometry_map_step, psm_stream_collide, body_force_torque) on
torch's current stream.  Nothing here computes any part of the method.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _capi as capi
from ._capi import check, lib

FACE = {"periodic": capi.PSM_PERIODIC, "wall": capi.PSM_WALL, "inlet": capi.PSM_INLET, "outlet": capi.PSM_OUTLET}
STORAGE = {"f64": (capi.PSM_F64, torch.float64), "f32": (capi.PSM_F32, torch.float32),
           "f16": (capi.PSM_F16, torch.float16)}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def lattice(q: int):
    c = np.zeros(3 * q, dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    o = np.zeros(q, dtype=np.int32)
    check(lib.psm_lattice(q, c.ctypes.data_as(C.POINTER(C.c_int32)), w.ctypes.data_as(C.POINTER(C.c_double)),
                          o.ctypes.data_as(C.POINTER(C.c_int32))), "psm_lattice")
    return c.reshape(q, 3), w, o


def make_config(wl, storage=None, psm=True, slots=None, max_bodies=None, map_ahead=False) -> capi.psm_config:
    cfg = capi.psm_config()
    cfg.nx, cfg.ny, cfg.nz, cfg.q = wl.nx, wl.ny, wl.nz, wl.q
    cfg.storage = STORAGE[storage or wl.storage][0]
    cfg.psm = 1 if psm else 0
    cfg.sc = wl.sc
    cfg.b_form = wl.b_form
    cfg.slots = slots or wl.slots
    cfg.max_bodies = max_bodies or max(1, len(wl.bodies))
    cfg.bc = (C.c_int32 * 6)(*[FACE[b] for b in wl.bc])
    cfg.tau = wl.tau
    cfg.magic = wl.magic
    cfg.force = (C.c_double * 3)(*wl.force)
    cfg.u_in = (C.c_double * 3)(*wl.u_in)
    cfg.collision = {"trt": capi.PSM_COLL_TRT, "cumulant": capi.PSM_COLL_CUMULANT}[getattr(wl, "collision", "trt")]
    cfg.map_reading = getattr(wl, "map_reading", 0)
    cfg.layout = {"soa": capi.PSM_LAYOUT_SOA, "blocked": capi.PSM_LAYOUT_BLOCKED}[getattr(wl, "layout", "soa")]
    cfg.block_rows = getattr(wl, "block_rows", 0)
    cfg.map_ahead = 1 if (map_ahead and psm) else 0
    return cfg


def required_bytes(cfg, which) -> int:
    n = C.c_size_t()
    check(lib.psm_required_bytes(C.byref(cfg), which, C.byref(n)), "psm_required_bytes")
    return n.value


def body_pose(motion, t: int) -> capi.psm_body:
    m = capi.psm_motion()
    m.axis = (C.c_double * 3)(*motion.axis)
    m.theta0 = motion.theta0
    m.omega = motion.omega
    m.x0 = (C.c_double * 3)(*motion.x0)
    m.v = (C.c_double * 3)(*motion.v)
    b = capi.psm_body()
    check(lib.psm_body_pose(C.byref(m), int(t), C.byref(b)), "psm_body_pose")
    return b


class Geometry:
    """Body-frame geometry field in a caller-owned (torch) device buffer."""

    def __init__(self, shape, s: int, device="cuda"):
        dp = C.POINTER(C.c_double)
        mmin = (C.c_int32 * 3)()
        dims = (C.c_int32 * 3)()
        nbytes = C.c_size_t()
        self.handle = C.c_void_p()
        if shape.kind == "mesh":
            v = np.ascontiguousarray(shape.mesh.verts, dtype=np.float64)
            t = np.ascontiguousarray(shape.mesh.tris, dtype=np.int32)
            check(lib.psm_geometry_box(-1, None, v.ctypes.data_as(dp), v.shape[0], s, mmin, dims, C.byref(nbytes)),
                  "psm_geometry_box")
            self.buf = torch.empty(max(16, nbytes.value), dtype=torch.uint8, device=device)
            check(lib.geometry_field_create(v.ctypes.data_as(dp), v.shape[0], t.ctypes.data_as(C.POINTER(C.c_int32)),
                                            t.shape[0], s, C.c_void_p(self.buf.data_ptr()), nbytes.value, _stream(),
                                            C.byref(self.handle)), "geometry_field_create")
        else:
            kind = capi.PSM_SHAPE_ELLIPSOID if shape.kind == "ellipsoid" else capi.PSM_SHAPE_CUBE
            p = np.zeros(3)
            p[: len(shape.params)] = shape.params
            check(lib.psm_geometry_box(kind, p.ctypes.data_as(dp), None, 0, s, mmin, dims, C.byref(nbytes)),
                  "psm_geometry_box")
            self.buf = torch.empty(max(16, nbytes.value), dtype=torch.uint8, device=device)
            check(lib.geometry_field_create_analytic(kind, p.ctypes.data_as(dp), s, C.c_void_p(self.buf.data_ptr()),
                                                     nbytes.value, _stream(), C.byref(self.handle)),
                  "geometry_field_create_analytic")
        self.mmin = tuple(mmin)
        self.dims = tuple(dims)
        self.s = s

    def __del__(self, _lib=lib, _vp=C.c_void_p):
        # bound at definition: module globals may already be gone at exit
        if getattr(self, "handle", None) and self.handle.value:
            _lib.geometry_field_destroy(self.handle)
            self.handle = _vp()


# PSM_OPT_CONCURRENT of new fields (None: the library's default)
CONCURRENT_DEFAULT = None
# map_ahead of new PSM fields when not given: Field.step then maps the next
# step on the field's mapping stream during this one (prescribed motion)
MAP_AHEAD_DEFAULT = True


class Field:
    """One lattice on the current device; ``wl`` is a psm_inputs.Workload."""

    def __init__(self, wl, storage=None, psm=True, slots=None, max_bodies=None, device="cuda", remap_every_step=True,
                 fused=True, noalloc=False, concurrent=None, map_ahead=None):
        """``noalloc``: create the handle with pdf_field_create_noalloc (the
        library's static work area instead of a caller work buffer).
        ``concurrent``: PSM_OPT_CONCURRENT (None: CONCURRENT_DEFAULT).
        ``map_ahead``: two sets of fractions and psm_step_ahead in step()
        (None: MAP_AHEAD_DEFAULT)."""
        self.wl = wl
        self.storage = storage or wl.storage
        self.map_ahead = bool(psm) and bool(MAP_AHEAD_DEFAULT if map_ahead is None else map_ahead)
        self.cfg = make_config(wl, self.storage, psm, slots, max_bodies, self.map_ahead)
        self.q = wl.q
        self.N = wl.n_cells
        self.dtype = STORAGE[self.storage][1]
        pb = required_bytes(self.cfg, capi.PSM_BUF_PDF)
        st = C.c_int64()
        check(lib.psm_pdf_stride(C.byref(self.cfg), C.byref(st)), "psm_pdf_stride")
        self.dstride = st.value
        bb = required_bytes(self.cfg, capi.PSM_BUF_B)
        wb = required_bytes(self.cfg, capi.PSM_BUF_WORK)
        self.pdf = torch.empty(pb // self.dtype.itemsize, dtype=self.dtype, device=device)
        self.bbuf = torch.empty(max(16, bb), dtype=torch.uint8, device=device) if bb else None
        self.handle = C.c_void_p()
        if noalloc:
            self.work = None
            check(lib.pdf_field_create_noalloc(C.byref(self.cfg), C.c_void_p(self.pdf.data_ptr()), pb,
                                               C.c_void_p(self.bbuf.data_ptr()) if bb else None, bb, _stream(),
                                               C.byref(self.handle)), "pdf_field_create_noalloc")
        else:
            self.work = torch.empty(wb, dtype=torch.uint8, device=device)
            check(lib.pdf_field_create(C.byref(self.cfg), C.c_void_p(self.pdf.data_ptr()), pb,
                                       C.c_void_p(self.bbuf.data_ptr()) if bb else None, bb,
                                       C.c_void_p(self.work.data_ptr()), wb, _stream(), C.byref(self.handle)),
                  "pdf_field_create")
        conc = CONCURRENT_DEFAULT if concurrent is None else concurrent
        if conc is not None:
            check(lib.psm_set_option(self.handle, capi.PSM_OPT_CONCURRENT, int(bool(conc))), "psm_set_option")
        self.psm = bool(psm)
        self.bodies = list(wl.bodies) if psm else []
        self.geoms = [Geometry(b.shape, b.s, device) for b in self.bodies]
        self._geom_ptrs = (C.c_void_p * max(1, len(self.geoms)))(*[g.handle.value for g in self.geoms])
        self.nb = len(self.bodies)
        self.remap_every_step = remap_every_step
        self.fused = fused  # one psm_step call per step
        self._mapped_once = False
        self.ft = torch.zeros((max(1, self.nb), 6), dtype=torch.float64, device=device)
        self.reset()

    # -- buffers ---------------------------------------------------------
    def pdf_view(self):
        """(q, N) view of the stored deviations f_k - w_k (library direction
        order) of a SoA field; rows are psm_pdf_stride elements apart in the
        buffer.  Blocked fields have no such view: use pdf_std / load_pdf_std."""
        if self.cfg.layout != capi.PSM_LAYOUT_SOA:
            raise ValueError("a blocked PDF buffer has no (q, N) view; use pdf_std() / load_pdf_std()")
        return self.pdf.as_strided((self.q, self.N), (self.dstride, 1))

    def pdf_std(self, out=None):
        """The stored slots as a (q, N) tensor in the standard layout
        (psm_pdf_gather; a copy, either layout)."""
        out = torch.empty((self.q, self.N), dtype=self.dtype, device=self.pdf.device) if out is None else out
        assert out.is_contiguous() and out.dtype == self.dtype and tuple(out.shape) == (self.q, self.N)
        check(lib.psm_pdf_gather(self.handle, C.c_void_p(out.data_ptr()), _stream()), "psm_pdf_gather")
        return out

    def load_pdf_std(self, src):
        """Set the stored slots from a (q, N) tensor in the standard layout
        (psm_pdf_scatter; either layout)."""
        src = src.to(device=self.pdf.device, dtype=self.dtype).contiguous()
        assert tuple(src.shape) == (self.q, self.N)
        check(lib.psm_pdf_scatter(self.handle, C.c_void_p(src.data_ptr()), _stream()), "psm_pdf_scatter")
        torch.cuda.current_stream().synchronize()

    def b_view(self):
        """(slots, N) float32 solid fractions and (N,) uint8 body ids."""
        n = self.N
        s = self.cfg.slots
        b0, meta_p = C.c_void_p(), C.c_void_p()
        check(lib.psm_fractions(self.handle, C.byref(b0), None, C.byref(meta_p)), "psm_fractions")
        o = b0.value - self.bbuf.data_ptr()  # the set the last step used (map_ahead: one of two)
        B = self.bbuf[o: o + 4 * n * s].view(torch.float32).view(s, n)
        m = meta_p.value - self.bbuf.data_ptr()
        meta = self.bbuf[m: m + n]
        return B, meta

    def reset(self):
        check(lib.psm_field_reset(self.handle, _stream()), "psm_field_reset")
        self._mapped_once = False

    def set_option(self, opt, value):
        check(lib.psm_set_option(self.handle, opt, int(value)), "psm_set_option")

    # -- one step --------------------------------------------------------
    def poses(self, t: int, motions=None):
        ms = motions or [b.motion for b in self.bodies]
        arr = (capi.psm_body * max(1, len(ms)))(*[body_pose(m, t) for m in ms])
        return arr

    def map(self, t: int, poses=None):
        poses = poses if poses is not None else self.poses(t)
        check(lib.geometry_map_step(self.handle, poses, self._geom_ptrs, self.nb, _stream()), "geometry_map_step")
        self._mapped_once = True

    def collide(self, t: int, poses=None):
        poses = poses if poses is not None else self.poses(t)
        check(lib.psm_stream_collide(self.handle, poses, self.nb, int(t), _stream()), "psm_stream_collide")

    def step(self, t: int, poses=None, ft=None):
        """Map B(t) (every step, or once for static scenes) and advance from t
        to t+1; with ``ft`` (a (n_bodies, 6) float64 device tensor) also sum the
        force/torque of the step into it."""
        if self.nb and self.fused and self.map_ahead and self.remap_every_step and poses is None:
            poses, nxt = self.poses(t), self.poses(t + 1)
            check(lib.psm_step_ahead(self.handle, poses, poses, nxt, self._geom_ptrs, self.nb, int(t),
                                     C.c_void_p(ft.data_ptr()) if ft is not None else None, _stream()),
                  "psm_step_ahead")
            self._mapped_once = True
            return
        poses = poses if poses is not None else (self.poses(t) if self.nb else None)
        if self.nb and self.fused and (self.remap_every_step or not self._mapped_once):
            check(lib.psm_step(self.handle, poses, poses, self._geom_ptrs, self.nb, int(t),
                               C.c_void_p(ft.data_ptr()) if ft is not None else None, _stream()), "psm_step")
            self._mapped_once = True
            return
        if self.nb and (self.remap_every_step or not self._mapped_once):
            self.map(t, poses)
        self.collide(t, poses)
        if ft is not None and self.nb:
            self.force_torque(out=ft)

    def coupled_step(self, t: int, states, ft_host=None):
        """One two-way coupled step (psm_coupled_step): ``states`` is a ctypes
        array of capi.psm_rigid (one per body), advanced in place; returns the
        step's F/T as a (n_bodies, 6) numpy array."""
        if ft_host is None:
            if getattr(self, "_ft_pinned", None) is None:
                self._ft_pinned = torch.zeros((max(1, self.nb), 6), dtype=torch.float64, pin_memory=True)
            ft_host = self._ft_pinned.numpy()
        check(lib.psm_coupled_step(self.handle, states, self._geom_ptrs, self.nb, int(t),
                                   C.c_void_p(self.ft.data_ptr()), ft_host.ctypes.data_as(C.POINTER(C.c_double)),
                                   _stream()), "psm_coupled_step")
        return ft_host[: self.nb].copy()

    def set_obstacle(self, solid):
        """Static no-slip obstacle of a plain-LBM field: ``solid`` is an (N,)
        uint8 device tensor (1 = obstacle cell), None removes it.  Returns the
        number of fluid cells next to the obstacle."""
        nn = C.c_int64()
        if solid is None:
            check(lib.lbm_set_obstacle(self.handle, None, None, 0, C.byref(nn), _stream()), "lbm_set_obstacle")
            self.obst = None
            return 0
        assert solid.dtype == torch.uint8 and solid.numel() == self.N and solid.is_contiguous()
        ob = required_bytes(self.cfg, capi.PSM_BUF_OBSTACLE)
        self.obst = torch.empty(ob, dtype=torch.uint8, device=self.pdf.device)
        check(lib.lbm_set_obstacle(self.handle, C.c_void_p(solid.data_ptr()), C.c_void_p(self.obst.data_ptr()), ob,
                                   C.byref(nn), _stream()), "lbm_set_obstacle")
        return nn.value

    def force_torque(self, out=None):
        out = self.ft if out is None else out
        check(lib.body_force_torque(self.handle, self.nb, C.c_void_p(out.data_ptr()), _stream()), "body_force_torque")
        return out[: self.nb]

    # -- diagnostics -----------------------------------------------------
    def mass(self, t: int):
        out = torch.empty(1, dtype=torch.float64, device=self.pdf.device)
        check(lib.psm_mass_fp64(self.handle, int(t), C.c_void_p(out.data_ptr()), _stream()), "psm_mass_fp64")
        return out

    def macroscopic(self, t: int):
        rho = torch.empty(self.N, dtype=torch.float64, device=self.pdf.device)
        u = torch.empty((self.N, 3), dtype=torch.float64, device=self.pdf.device)
        check(lib.psm_macroscopic(self.handle, int(t), C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr()),
                                  _stream()), "psm_macroscopic")
        return rho, u

    def error_flags(self):
        out = torch.zeros(4, dtype=torch.int32, device=self.pdf.device)
        check(lib.psm_error_flags(self.handle, C.c_void_p(out.data_ptr()), _stream()), "psm_error_flags")
        return out

    def __del__(self, _lib=lib, _vp=C.c_void_p):
        if getattr(self, "handle", None) and self.handle.value:
            _lib.pdf_field_destroy(self.handle)
            self.handle = _vp()


def rigid_states(rigids, average=True):
    """ctypes array of capi.psm_rigid at rest from dicts (m, I, F_ext, X0);
    average: advance with the mean hydrodynamic F/T of the last two steps."""
    arr = (capi.psm_rigid * len(rigids))()
    for s, r in zip(arr, rigids):
        s.average = 1 if average else 0
        s.m = r["m"]
        s.I = (C.c_double * 3)(*r["I"])
        s.F_ext = (C.c_double * 3)(*r["F_ext"])
        s.X = (C.c_double * 3)(*r["X0"])
        s.R = (C.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    return arr


def voxelize_obstacle(wl, t: int = 0, device="cuda"):
    """(N,) uint8 obstacle flags of the workload's bodies at step t: a cell is
    an obstacle cell when its centre lies inside a body (the mapping with one
    sample per cell, s = 0)."""
    import dataclasses

    wl0 = dataclasses.replace(wl, bodies=[dataclasses.replace(b, s=0) for b in wl.bodies])
    f = Field(wl0, storage="f32", psm=True, device=device)
    f.map(t)
    B, _ = f.b_view()
    solid = (B.sum(0) > 0).to(torch.uint8).contiguous()
    torch.cuda.synchronize()
    del f
    return solid


def stream_copy(src: torch.Tensor, dst: torch.Tensor):
    check(lib.psm_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                              src.numel() * src.element_size(), _stream()), "psm_stream_copy")
