"""FP64 CPU oracle for the PSM hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps ``liboracle.so`` (plain C, see ``oracle.c``) with
ctypes and numpy; it shares no code with the HIP path and never imports it.

The oracle works on full distribution functions f (not deviations) in FP64,
with a two-buffer pull streaming scheme.  PDF arrays are direction-major,
``f[i, n]`` with n = x + nx*(y + ny*z) and the oracle's own direction order
(:func:`lattice`).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FACE = {"periodic": 0, "wall": 1, "inlet": 2, "outlet": 3}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP64, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fno-builtin-sin", "-fno-builtin-cos", os.path.join(_HERE, "oracle.c"), "-lm", "-o", _LIB_PATH + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Config(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("q", C.c_int),
                ("tau", C.c_double), ("magic", C.c_double), ("force", C.c_double * 3),
                ("bc", C.c_int * 6), ("u_in", C.c_double * 3), ("sc", C.c_int), ("psm", C.c_int),
                ("collision", C.c_int)]


class Pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("X", C.c_double * 3), ("V", C.c_double * 3), ("W", C.c_double * 3)]


class Geom(C.Structure):
    _fields_ = [("kind", C.c_int), ("p", C.c_double * 3), ("s", C.c_int), ("mmin", C.c_int * 3),
                ("dims", C.c_int * 3), ("inside", C.c_void_p), ("r_bound", C.c_double),
                ("verts", C.c_void_p), ("tris", C.c_void_p), ("nt", C.c_longlong)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.or_lattice.argtypes = [C.c_int, C.POINTER(C.c_int), dp, C.POINTER(C.c_int)]
        L.or_feq.argtypes = [C.c_int, C.c_double, dp, dp]
        L.or_feq.restype = None
        L.or_pose_at.argtypes = [dp, C.c_double, C.c_double, dp, dp, C.c_longlong, C.POINTER(Pose)]
        L.or_pose_at.restype = None
        L.or_collide_cell.argtypes = [C.POINTER(Config), dp, C.c_int, dp, dp, dp, dp]
        L.or_step.argtypes = [C.POINTER(Config), dp, dp, C.c_int, dp, C.POINTER(Pose), dp]
        L.or_step_obstacle.argtypes = [C.POINTER(Config), dp, dp, C.POINTER(C.c_ubyte)]
        L.or_macro.argtypes = [C.POINTER(Config), dp, dp, dp]
        L.or_macro.restype = None
        L.or_mass.argtypes = [C.POINTER(Config), dp]
        L.or_mass.restype = C.c_double
        L.or_geom_inside.argtypes = [C.POINTER(Geom), C.c_longlong, C.c_longlong, C.c_longlong]
        L.or_map_cell.argtypes = [C.POINTER(Geom), C.POINTER(Pose), C.c_int, C.c_int, C.c_int]
        L.or_map_cell.restype = C.c_double
        L.or_map_cell_block.argtypes = [C.POINTER(Geom), C.POINTER(Pose), C.c_int, C.c_int, C.c_int]
        L.or_map_cell_block.restype = C.c_double
        L.or_map.argtypes = [C.POINTER(Config), C.POINTER(Geom), C.POINTER(Pose), C.c_int, C.c_int, dp]
        L.or_b_from_eps.argtypes = [C.c_double, C.c_double, C.c_int]
        L.or_b_from_eps.restype = C.c_float
        L.or_winding.argtypes = [dp, C.POINTER(C.c_int), C.c_longlong, dp]
        L.or_winding.restype = C.c_double
        L.or_voxelize.argtypes = [dp, C.POINTER(C.c_int), C.c_longlong, C.c_int, C.POINTER(C.c_int),
                                  C.POINTER(C.c_int), C.POINTER(C.c_ubyte)]
        L.or_update_cell.argtypes = [C.POINTER(Config), C.c_int, C.c_int, C.c_int, dp, C.c_int, dp,
                                     C.POINTER(Pose), dp]
        L.or_adjoint_step.argtypes = [C.POINTER(Config), dp, dp, dp, dp, C.POINTER(Pose), dp, C.c_double, dp, dp]
        L.or_mesh_volume.argtypes = [dp, C.POINTER(C.c_int), C.c_longlong]
        L.or_mesh_volume.restype = C.c_double
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = None
        L.or_threads.argtypes = []
        L.or_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int))


# ----------------------------------------------------------------------------
def lattice(q: int):
    """(c (q,3) int, w (q,) float64, opp (q,) int) in the oracle's order."""
    c = np.zeros(q * 3, dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    opp = np.zeros(q, dtype=np.int32)
    if lib().or_lattice(q, _ip(c), _dp(w), _ip(opp)) != 0:
        raise ValueError(q)
    return c.reshape(q, 3), w, opp


def feq(q: int, rho: float, u) -> np.ndarray:
    out = np.zeros(q)
    u = np.asarray(u, dtype=np.float64)
    lib().or_feq(q, rho, _dp(u), _dp(out))
    return out


def make_config(wl=None, **kw) -> Config:
    """or_config from a psm_inputs.Workload (or keyword overrides)."""
    d = {}
    if wl is not None:
        d = dict(nx=wl.nx, ny=wl.ny, nz=wl.nz, q=wl.q, tau=wl.tau, magic=wl.magic, force=wl.force,
                 bc=wl.bc, u_in=wl.u_in, sc=wl.sc, psm=1, collision=getattr(wl, "collision", "trt"))
    d.update(kw)
    cfg = Config()
    cfg.nx, cfg.ny, cfg.nz, cfg.q = d["nx"], d["ny"], d["nz"], d["q"]
    cfg.tau, cfg.magic = d["tau"], d.get("magic", 3.0 / 16.0)
    cfg.force = (C.c_double * 3)(*d.get("force", (0, 0, 0)))
    cfg.bc = (C.c_int * 6)(*[FACE[b] if isinstance(b, str) else int(b) for b in d.get("bc", ("periodic",) * 6)])
    cfg.u_in = (C.c_double * 3)(*d.get("u_in", (0, 0, 0)))
    cfg.sc = d.get("sc", 1)
    cfg.psm = d.get("psm", 1)
    coll = d.get("collision", "trt")
    cfg.collision = {"trt": 0, "cumulant": 1}[coll] if isinstance(coll, str) else int(coll)
    return cfg


def pose_at(motion, t: int) -> Pose:
    p = Pose()
    ax = np.asarray(motion.axis, dtype=np.float64)
    x0 = np.asarray(motion.x0, dtype=np.float64)
    v = np.asarray(motion.v, dtype=np.float64)
    lib().or_pose_at(_dp(ax), float(motion.theta0), float(motion.omega), _dp(x0), _dp(v), int(t), C.byref(p))
    return p


def pose_arrays(p: Pose):
    return (np.array(p.R[:]).reshape(3, 3), np.array(p.X[:]), np.array(p.V[:]), np.array(p.W[:]))


def collide_cell(cfg: Config, fin, B=(), us=()):
    q = cfg.q
    fin = np.ascontiguousarray(fin, dtype=np.float64)
    ns = len(B)
    Bv = np.ascontiguousarray(np.asarray(B, dtype=np.float64).reshape(-1) if ns else np.zeros(1))
    uv = np.ascontiguousarray(np.asarray(us, dtype=np.float64).reshape(-1) if ns else np.zeros(3))
    fo = np.zeros(q)
    dF = np.zeros(6)
    if lib().or_collide_cell(C.byref(cfg), _dp(fin), ns, _dp(Bv), _dp(uv), _dp(fo), _dp(dF)) != 0:
        raise RuntimeError("or_collide_cell")
    return fo, dF[: 3 * ns].reshape(ns, 3)


def step(cfg: Config, f: np.ndarray, B: np.ndarray | None, poses) -> np.ndarray:
    """Advance f (q, N) in place by one step; returns F/T (nb, 6) on each body."""
    nb = 0 if B is None else B.shape[0]
    fpost = np.empty_like(f)
    Bv = np.ascontiguousarray(B if nb else np.zeros((1, 1)), dtype=np.float64)
    P = (Pose * max(1, nb))(*poses) if nb else (Pose * 1)()
    ft = np.zeros((max(1, nb), 6))
    r = lib().or_step(C.byref(cfg), _dp(f), _dp(fpost), nb, _dp(Bv), P, _dp(ft))
    if r != 0:
        raise RuntimeError(f"or_step failed ({r})")
    return ft[:nb]


def step_obstacle(cfg: Config, f: np.ndarray, solid: np.ndarray) -> None:
    """Advance f (q, N) in place by one plain-LBM step with static no-slip
    obstacle cells (solid[n] != 0): halfway bounce-back on every link from a
    fluid cell into an obstacle cell; obstacle cells keep their values (the
    LBM variant of the paper's node-level benchmark, section V)."""
    fpost = np.empty_like(f)
    sm = np.ascontiguousarray(solid, dtype=np.uint8)
    assert sm.size == f.shape[1]
    r = lib().or_step_obstacle(C.byref(cfg), _dp(f), _dp(fpost), sm.ctypes.data_as(C.POINTER(C.c_ubyte)))
    if r != 0:
        raise RuntimeError(f"or_step_obstacle failed ({r})")


def rodrigues(axis, angle) -> np.ndarray:
    """Rotation matrix by `angle` about the unit `axis`."""
    a = np.asarray(axis, dtype=np.float64)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return math.cos(angle) * np.eye(3) + (1.0 - math.cos(angle)) * np.outer(a, a) + math.sin(angle) * K


def rigid_advance(st: dict, ft, dt: float = 1.0) -> None:
    """One step of a free rigid body under the hydrodynamic force / torque
    ft = (F, T) of the step (force on the body, torque about X) and the
    constant external force F_ext: semi-implicit Euler, V then X, W then R
    (Newton and Euler's equations written in the lab frame with
    I_lab = R diag(I) R^T, the orientation rotated by dt|W| about W).  With
    st["average"], the mean of this step's and the previous step's
    hydrodynamic F/T drives the step."""
    ft_step = np.asarray(ft, dtype=np.float64)
    ft = 0.5 * (ft_step + st["ft_prev"]) if st["average"] else ft_step
    st["ft_prev"] = ft_step.copy()
    st["V"] = st["V"] + dt * (ft[:3] + np.asarray(st["F_ext"])) / st["m"]
    st["X"] = st["X"] + dt * st["V"]
    R = st["R"]
    I_lab = R @ np.diag(np.asarray(st["I"], dtype=np.float64)) @ R.T
    W = st["W"]
    st["W"] = W + dt * np.linalg.solve(I_lab, ft[3:] - np.cross(W, I_lab @ W))
    th = dt * float(np.linalg.norm(st["W"]))
    if th > 0.0:
        st["R"] = rodrigues(st["W"] * dt / th, th) @ R


def rigid_pose(st: dict) -> Pose:
    p = Pose()
    p.R = (C.c_double * 9)(*np.asarray(st["R"], dtype=np.float64).ravel())
    p.X = (C.c_double * 3)(*st["X"])
    p.V = (C.c_double * 3)(*st["V"])
    p.W = (C.c_double * 3)(*st["W"])
    return p


def rigid_state(rigid: dict, average: bool = True) -> dict:
    """Rest state of a rigid body: dict(m, I, F_ext, X0) -> state dict
    (average: drive each step with the mean hydrodynamic F/T of the last two
    steps)."""
    return {"m": float(rigid["m"]), "I": tuple(rigid["I"]), "F_ext": tuple(rigid["F_ext"]),
            "X": np.asarray(rigid["X0"], dtype=np.float64), "V": np.zeros(3), "R": np.eye(3), "W": np.zeros(3),
            "ft_prev": np.zeros(6), "average": bool(average)}


def coupled_run(wl, states, steps: int, f0: np.ndarray | None = None):
    """Two-way coupled steps (section IV's freely settling sphere): per step,
    map B from the states' poses, collide / stream with their velocities, then
    advance every state with the step's F/T.  Returns (f, trajectory) with one
    record per step: the state used for the step and the step's F/T."""
    cfg = make_config(wl)
    c, w, _ = lattice(wl.q)
    f = np.repeat(w[:, None], wl.n_cells, axis=1).copy() if f0 is None else np.ascontiguousarray(f0, dtype=np.float64)
    geoms = [OracleGeometry(b.shape, b.s) for b in wl.bodies]
    traj = []
    for _ in range(steps):
        poses = [rigid_pose(s) for s in states]
        B = np.stack([map_body(cfg, g, p, wl.b_form, wl.map_reading) for g, p in zip(geoms, poses)])
        rec = [{"X": s["X"].copy(), "V": s["V"].copy(), "W": s["W"].copy(), "R": s["R"].copy()} for s in states]
        ft = step(cfg, f, B, poses)
        for s, r, fb in zip(states, rec, ft):
            r["ft"] = fb.copy()
            rigid_advance(s, fb)
        traj.append(rec)
    return f, traj


def macro(cfg: Config, f: np.ndarray):
    N = f.shape[1]
    rho = np.empty(N)
    u = np.empty((N, 3))
    lib().or_macro(C.byref(cfg), _dp(f), _dp(rho), _dp(u))
    return rho, u


def mass(cfg: Config, f: np.ndarray) -> float:
    return lib().or_mass(C.byref(cfg), _dp(f))


# ----------------------------------------------------------------------------
# geometry
class OracleGeometry:
    """Geometry lattice of one body: analytic (ellipsoid/cube) or voxelised mesh."""

    def __init__(self, shape, s: int, lazy: bool = False):
        self.s = s
        self._keep = None
        g = Geom()
        g.s = s
        if shape.kind == "ellipsoid":
            g.kind = 0
            g.p = (C.c_double * 3)(*shape.params)
            g.r_bound = float(max(shape.params))
        elif shape.kind == "cube":
            g.kind = 1
            g.p = (C.c_double * 3)(shape.params[0], 0, 0)
            g.r_bound = float(shape.params[0]) * 3 ** 0.5
        elif shape.kind == "mesh" and lazy:
            # winding number evaluated at each queried lattice centre
            v = np.ascontiguousarray(shape.mesh.verts, dtype=np.float64)
            t = np.ascontiguousarray(shape.mesh.tris, dtype=np.int32)
            self._keep = (v, t)
            g.kind = 3
            g.verts = v.ctypes.data_as(C.c_void_p)
            g.tris = t.ctypes.data_as(C.c_void_p)
            g.nt = t.shape[0]
            g.r_bound = float(np.linalg.norm(v, axis=1).max()) + 1e-9
        elif shape.kind == "mesh":
            v = np.ascontiguousarray(shape.mesh.verts, dtype=np.float64)
            t = np.ascontiguousarray(shape.mesh.tris, dtype=np.int32)
            h = 2.0 ** -s
            lo = np.floor(v.min(axis=0) / h).astype(np.int64) - 2
            hi = np.floor(v.max(axis=0) / h).astype(np.int64) + 2
            dims = (hi - lo + 1).astype(np.int32)
            inside = voxelize(v, t, s, lo.astype(np.int32), dims)
            self._keep = inside
            g.kind = 2
            g.mmin = (C.c_int * 3)(*[int(x) for x in lo])
            g.dims = (C.c_int * 3)(*[int(x) for x in dims])
            g.inside = inside.ctypes.data_as(C.c_void_p)
            # farthest box corner from the body origin
            g.r_bound = float(np.linalg.norm(np.maximum(np.abs(lo), np.abs(hi + 1)) * h))
        else:
            raise ValueError(shape.kind)
        self.g = g

    def inside(self, m):
        m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
        return np.array([lib().or_geom_inside(C.byref(self.g), int(a), int(b), int(c)) for a, b, c in m], dtype=bool)


def map_body(cfg: Config, geom: OracleGeometry, pose: Pose, b_form: int = 0, reading: int = 0) -> np.ndarray:
    """Dense B of one body (section III).  reading 0: every sub-sample of a
    cell rotated to the body frame; reading 1: the cell centre rotated, the
    axis-aligned block of geometry cells around it averaged."""
    N = cfg.nx * cfg.ny * cfg.nz
    out = np.zeros(N)
    if lib().or_map(C.byref(cfg), C.byref(geom.g), C.byref(pose), int(b_form), int(reading), _dp(out)) != 0:
        raise ValueError(f"mapping reading {reading}")
    return out


def map_cell(geom: OracleGeometry, pose: Pose, ix: int, iy: int, iz: int, reading: int = 0) -> float:
    if reading:
        return lib().or_map_cell_block(C.byref(geom.g), C.byref(pose), ix, iy, iz)
    return lib().or_map_cell(C.byref(geom.g), C.byref(pose), ix, iy, iz)


def b_from_eps(eps: float, tau: float, b_form: int) -> float:
    return float(lib().or_b_from_eps(eps, tau, b_form))


def winding(verts, tris, p) -> float:
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    return lib().or_winding(_dp(v), _ip(t), t.shape[0], _dp(np.asarray(p, dtype=np.float64)))


def voxelize(verts, tris, s, mmin, dims) -> np.ndarray:
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    mmin = np.ascontiguousarray(mmin, dtype=np.int32)
    dims = np.ascontiguousarray(dims, dtype=np.int32)
    out = np.zeros(int(np.prod(dims.astype(np.int64))), dtype=np.uint8)
    lib().or_voxelize(_dp(v), _ip(t), t.shape[0], int(s), _ip(mmin), _ip(dims),
                      out.ctypes.data_as(C.POINTER(C.c_ubyte)))
    return out


def set_threads(n: int) -> None:
    """Thread count of the oracle's parallel loops (timing only)."""
    lib().or_set_threads(int(n))


def threads() -> int:
    return int(lib().or_threads())


def mesh_volume(verts, tris) -> float:
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    return lib().or_mesh_volume(_dp(v), _ip(t), t.shape[0])


# ----------------------------------------------------------------------------
class Run:
    """Time loop of a workload in the oracle: per step, map B(t) from the poses
    at t, then collide/stream step t (B(t), u_s(t)); records F/T(t)."""

    def __init__(self, wl, f0: np.ndarray | None = None, b_form=None):
        self.wl = wl
        self.cfg = make_config(wl)
        self.b_form = wl.b_form if b_form is None else b_form
        q = wl.q
        c, w, opp = lattice(q)
        self.c, self.w, self.opp = c, w, opp
        N = wl.n_cells
        if f0 is None:
            self.f = np.repeat(w[:, None], N, axis=1).copy()
        else:
            self.f = np.ascontiguousarray(f0, dtype=np.float64)
        self.geoms = [OracleGeometry(b.shape, b.s) for b in wl.bodies]
        self.t = 0
        self.B = np.zeros((len(wl.bodies), N))
        self.ft = []
        self._static_done = False

    def map(self, t):
        for k, (b, g) in enumerate(zip(self.wl.bodies, self.geoms)):
            self.B[k] = map_body(self.cfg, g, pose_at(b.motion, t), self.b_form, self.wl.map_reading)

    def advance(self, steps: int, remap: bool = True):
        for _ in range(steps):
            poses = [pose_at(b.motion, self.t) for b in self.wl.bodies]
            if self.wl.bodies and (remap or not self._static_done):
                self.map(self.t)
                self._static_done = True
            ft = step(self.cfg, self.f, self.B if self.wl.bodies else None, poses)
            self.ft.append(ft)
            self.t += 1
        return self

    def macro(self):
        return macro(self.cfg, self.f)

    def mass(self):
        return mass(self.cfg, self.f)


def update_cell(cfg: Config, x: int, y: int, z: int, nbr: np.ndarray, Bn: np.ndarray, poses) -> np.ndarray:
    """One-step update of cell (x,y,z) from its 3x3x3 pre-step neighbourhood
    ``nbr`` (27, q) and solid fractions ``Bn`` (27, nb) (x fastest order)."""
    q = cfg.q
    nb = Bn.shape[1] if Bn is not None and Bn.ndim == 2 else 0
    out = np.zeros(q)
    nbr = np.ascontiguousarray(nbr, dtype=np.float64)
    Bv = np.ascontiguousarray(Bn if nb else np.zeros((27, 1)), dtype=np.float64)
    P = (Pose * max(1, nb))(*poses) if nb else (Pose * 1)()
    r = lib().or_update_cell(C.byref(cfg), x, y, z, _dp(nbr), nb, _dp(Bv), P, _dp(out))
    if r != 0:
        raise RuntimeError(f"or_update_cell failed ({r})")
    return out


def sampled_steps(wl, cells, f_at, geoms, steps: int, b_form: int = 0, t0: int = 0):
    """f(t0 + steps) at the given cells, computed one cell at a time.

    ``f_at(xyz (m,3)) -> (m, q)`` gives the full f at t0 for any cells (the
    seeded generator); ``geoms`` are OracleGeometry objects of the bodies.
    The dependence cone of each cell (radius ``steps``) is evaluated
    recursively with or_update_cell; solid fractions come from or_map_cell.
    """
    cfg = make_config(wl)
    n3 = np.array([wl.nx, wl.ny, wl.nz])
    per = np.array([wl.bc[0] == "periodic", wl.bc[2] == "periodic", wl.bc[4] == "periodic"])
    offs = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    cache = {}

    def nbrs(c):
        p = c + offs
        p = np.where(per, p % n3, p)
        inside = np.all((p >= 0) & (p < n3), axis=1)
        return p, inside

    bcache = {}

    def B_at(c, t):
        key = (int(c[0]), int(c[1]), int(c[2]), t)
        if key not in bcache:
            poses = [pose_at(b.motion, t) for b in wl.bodies]
            bcache[key] = np.array([b_from_eps(map_cell(g, P, *map(int, c), reading=wl.map_reading), wl.tau, b_form)
                                    for g, P in zip(geoms, poses)])
        return bcache[key]

    def value(c, t):
        key = (int(c[0]), int(c[1]), int(c[2]), t)
        if key in cache:
            return cache[key]
        if t == t0:
            v = f_at(np.asarray([c]))[0]
        else:
            p, inside = nbrs(np.asarray(c))
            nbr = np.zeros((27, wl.q))
            Bn = np.zeros((27, max(1, len(wl.bodies))))
            for j in range(27):
                if inside[j]:
                    nbr[j] = value(p[j], t - 1)
                    if wl.bodies:
                        Bn[j] = B_at(p[j], t - 1)
            poses = [pose_at(b.motion, t - 1) for b in wl.bodies]
            v = update_cell(cfg, int(c[0]), int(c[1]), int(c[2]), nbr, Bn if wl.bodies else None, poses)
        cache[key] = v
        return v

    return np.array([value(np.asarray(c), t0 + steps) for c in cells])


# ----------------------------------------------------------------------------
# torque objective and its discrete adjoint (frozen solid fractions)
def _pose_with_rate(motion, t, omega_us):
    """Pose at t from the prescribed motion (drives the mapping); the solid
    velocity uses the rate ``omega_us`` instead when given."""
    p = pose_at(motion, t)
    if omega_us is not None:
        p.W = (C.c_double * 3)(*[omega_us * a for a in motion.axis])
    return p


def torque_forward(wl, f0, steps, weights, dB=None, omega_us=None, keep_states=False, geom=None, sums=None):
    """J = sum_t weights[t] * a . T_0(t) for the single body of ``wl``, with
    B_eff = B_map(t) + dB and u_s from ``omega_us`` (mapping from the motion).
    ``geom``: the body's OracleGeometry when already built; ``sums``: a dict
    that receives sum(B_map(t)) per step."""
    cfg = make_config(wl)
    body = wl.bodies[0]
    geom = OracleGeometry(body.shape, body.s) if geom is None else geom
    f = np.ascontiguousarray(f0, dtype=np.float64).copy()
    axis = np.asarray(body.motion.axis, dtype=np.float64)
    J = 0.0
    states, Bs = [], []
    for t in range(steps):
        B = map_body(cfg, geom, pose_at(body.motion, t), wl.b_form, wl.map_reading)
        if sums is not None:
            sums[t] = float(B.sum())
        if dB is not None:
            B = B + dB
        if keep_states:
            states.append(f.copy())
            Bs.append(B.copy())
        ft = step(cfg, f, B[None, :].copy(), [_pose_with_rate(body.motion, t, omega_us)])
        J += weights[t] * float(axis @ ft[0, 3:])
    return J, f, states, Bs


def torque_adjoint(wl, f0, steps, weights, dB=None, omega_us=None):
    """(J, dJ/dB (N,), dJ/domega, dJ/df0 (q,N)) by the oracle's adjoint steps."""
    cfg = make_config(wl)
    body = wl.bodies[0]
    J, _, states, Bs = torque_forward(wl, f0, steps, weights, dB, omega_us, keep_states=True)
    q, N = f0.shape
    axis = np.ascontiguousarray(body.motion.axis, dtype=np.float64)
    gnext = np.zeros((q, N))
    g = np.zeros((q, N))
    dJdB = np.zeros(N)
    dJdW = np.zeros(1)
    for t in range(steps - 1, -1, -1):
        pose = _pose_with_rate(body.motion, t, omega_us)
        r = lib().or_adjoint_step(C.byref(cfg), _dp(states[t]), _dp(gnext), _dp(g), _dp(Bs[t]), C.byref(pose),
                                  _dp(axis), float(weights[t]), _dp(dJdB), _dp(dJdW))
        if r != 0:
            raise RuntimeError("or_adjoint_step failed")
        gnext, g = g, gnext
    return J, dJdB, float(dJdW[0]), gnext
