"""Seeded synthetic inputs for the PSM hot path.

This module is the only code shared by the HIP path's callers and by the
test-side FP64 oracle.  It holds no arithmetic of the method itself: it only
produces inputs (random lattice states, random solid fractions, triangle
meshes, motion parameters and the workload descriptions).

Random values come from one counter-based generator so that any element can be
recomputed on its own (numpy, on the host, for sampled cells) or for a whole
field at once (torch, on the device).  The generator is Chris Wellons'
"lowbias32" integer hash, x ^= x>>16; x *= 0x7feb352d; x ^= x>>15;
x *= 0x846ca68b; x ^= x>>16 (all mod 2^32), chained over
(stream, seed, high word, low word) of a 64-bit element counter.

Workloads mirror the paper's node-level scenes (section V.A: one block of 256^3
cells per GPU, rotating geometry in a small part of the domain) and its
counter-rotating open rotor (section III, fig. CROR), with procedural meshes
standing in for the CROR / bunny meshes, which are not available.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK32 = 0xFFFFFFFF

# ----------------------------------------------------------------------------
# counter-based generator
# ----------------------------------------------------------------------------


def _lowbias32_np(x):
    x = np.asarray(x, dtype=np.uint64) & np.uint64(MASK32)
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x7FEB352D)) & np.uint64(MASK32)
    x ^= x >> np.uint64(15)
    x = (x * np.uint64(0x846CA68B)) & np.uint64(MASK32)
    x ^= x >> np.uint64(16)
    return x


def _lowbias32_torch(x):
    # x: int64 tensor holding values in [0, 2^32).  int64 products wrap mod
    # 2^64, so the low 32 bits after masking equal the uint32 product.
    x = x & MASK32
    x = x ^ (x >> 16)
    x = (x * 0x7FEB352D) & MASK32
    x = x ^ (x >> 15)
    x = (x * 0x846CA68B) & MASK32
    x = x ^ (x >> 16)
    return x


def _key(seed: int, stream: int) -> int:
    k = _lowbias32_np(np.uint64(stream & MASK32))
    k = _lowbias32_np(np.uint64(int(k) ^ (seed & MASK32)))
    return int(k)


def counter_u32(seed: int, stream: int, idx):
    """uint32 random word for each 64-bit element counter in ``idx`` (numpy)."""
    idx = np.asarray(idx, dtype=np.int64)
    k = np.uint64(_key(seed, stream))
    hi = (idx >> 32).astype(np.uint64)
    lo = (idx & MASK32).astype(np.uint64)
    h = _lowbias32_np(hi ^ k)
    return _lowbias32_np(lo ^ h)


def counter_u32_torch(seed: int, stream: int, idx):
    """Same words as :func:`counter_u32` for an int64 torch tensor ``idx``."""
    k = _key(seed, stream)
    hi = idx >> 32
    lo = idx & MASK32
    h = _lowbias32_torch(hi ^ k)
    return _lowbias32_torch(lo ^ h)


# Random PDF deviations are multiples of 2^-17 in [-512, 511] * 2^-17, exactly
# representable in binary16, binary32 and binary64.
DEV_SCALE = 2.0 ** -17


def pdf_deviation(seed: int, q: int, n_cells: int, k, cell):
    """Random deviation delta f_k(cell) (float64, exact in fp16) - numpy, sampled.

    ``k`` and ``cell`` broadcast; the element counter is k*n_cells + cell, the
    position of the value in a direction-major (SoA) array.
    """
    k = np.asarray(k, dtype=np.int64)
    cell = np.asarray(cell, dtype=np.int64)
    h = counter_u32(seed, 1, k * np.int64(n_cells) + cell)
    return ((h >> np.uint64(22)).astype(np.int64) - 512).astype(np.float64) * DEV_SCALE


def pdf_deviation_full(seed: int, q: int, n_cells: int):
    """Whole (q, n_cells) float64 deviation array (numpy)."""
    out = np.empty((q, n_cells), dtype=np.float64)
    cells = np.arange(n_cells, dtype=np.int64)
    for k in range(q):
        out[k] = pdf_deviation(seed, q, n_cells, k, cells)
    return out


def pdf_deviation_torch(seed: int, q: int, n_cells: int, k: int, device, dtype, chunk=1 << 26):
    """Deviation values of direction ``k`` for all cells, as a torch tensor."""
    import torch

    out = torch.empty(n_cells, dtype=dtype, device=device)
    for a in range(0, n_cells, chunk):
        b = min(n_cells, a + chunk)
        idx = torch.arange(a, b, dtype=torch.int64, device=device) + k * n_cells
        h = counter_u32_torch(seed, 1, idx)
        v = ((h >> 22) - 512).to(torch.float64) * DEV_SCALE
        out[a:b] = v.to(dtype)
    return out


def random_fractions(seed: int, n_cells: int, levels: int = 64, p_zero=0.35, p_one=0.25, stream=2):
    """Random solid fractions in {0, 1/levels, ..., 1}: many exact 0 and 1 values."""
    cells = np.arange(n_cells, dtype=np.int64)
    h = counter_u32(seed, stream, cells).astype(np.float64) / 2.0**32
    g = counter_u32(seed, stream + 100, cells).astype(np.int64) % (levels - 1)
    b = (g + 1).astype(np.float64) / levels
    b[h < p_zero] = 0.0
    b[(h >= p_zero) & (h < p_zero + p_one)] = 1.0
    return b


def random_obstacle(seed: int, n_cells: int, p_solid: float = 0.2, stream=4):
    """uint8 obstacle flags (1 = obstacle cell) with probability p_solid."""
    h = counter_u32(seed, stream, np.arange(n_cells, dtype=np.int64)).astype(np.float64) / 2.0**32
    return (h < p_solid).astype(np.uint8)


def random_unit(seed: int, n: int, stream=3):
    """n uniform doubles in [0,1) (multiples of 2^-32)."""
    return counter_u32(seed, stream, np.arange(n, dtype=np.int64)).astype(np.float64) / 2.0**32


# ----------------------------------------------------------------------------
# procedural meshes (body frame; watertight, outward oriented components)
# ----------------------------------------------------------------------------


@dataclass
class Mesh:
    verts: np.ndarray  # (nv, 3) float64
    tris: np.ndarray   # (nt, 3) int32

    @property
    def n_tris(self):
        return int(self.tris.shape[0])

    def bounds(self):
        return self.verts.min(axis=0), self.verts.max(axis=0)


def _signed_volume(v, t):
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def _orient_outward(v, t):
    if _signed_volume(v, t) < 0:
        t = t[:, [0, 2, 1]]
    return t


def _merge(parts):
    vs, ts, off = [], [], 0
    for v, t in parts:
        vs.append(v)
        ts.append(t + off)
        off += v.shape[0]
    return Mesh(np.concatenate(vs).astype(np.float64), np.concatenate(ts).astype(np.int32))


def _loft(rings, cap=True):
    """Close a sequence of rings (each (m,3)) into a tube with fan caps."""
    rings = [np.asarray(r, dtype=np.float64) for r in rings]
    m = rings[0].shape[0]
    v = np.concatenate(rings)
    tris = []
    for j in range(len(rings) - 1):
        a0, b0 = j * m, (j + 1) * m
        for i in range(m):
            i1 = (i + 1) % m
            tris.append((a0 + i, a0 + i1, b0 + i1))
            tris.append((a0 + i, b0 + i1, b0 + i))
    if cap:
        c0 = rings[0].mean(axis=0)
        c1 = rings[-1].mean(axis=0)
        n0 = v.shape[0]
        v = np.concatenate([v, c0[None], c1[None]])
        last = (len(rings) - 1) * m
        for i in range(m):
            i1 = (i + 1) % m
            tris.append((n0, i1, i))
            tris.append((n0 + 1, last + i, last + i1))
    t = np.asarray(tris, dtype=np.int64)
    return v, _orient_outward(v, t)


def ellipsoid_mesh(a, b, c, n_lat=24, n_lon=48, center=(0.0, 0.0, 0.0), phase=0.0):
    """UV-ellipsoid surface with semi-axes (a, b, c) along body x, y, z."""
    rings = []
    for i in range(1, n_lat):
        th = math.pi * i / n_lat
        ph = np.linspace(0, 2 * math.pi, n_lon, endpoint=False) + phase
        x = a * math.cos(th) * np.ones_like(ph)
        y = b * math.sin(th) * np.cos(ph)
        z = c * math.sin(th) * np.sin(ph)
        rings.append(np.stack([x, y, z], axis=1))
    v = np.concatenate(rings + [np.array([[a, 0, 0], [-a, 0, 0]], dtype=np.float64)])
    m = n_lon
    tris = []
    for j in range(len(rings) - 1):
        a0, b0 = j * m, (j + 1) * m
        for i in range(m):
            i1 = (i + 1) % m
            tris.append((a0 + i, a0 + i1, b0 + i1))
            tris.append((a0 + i, b0 + i1, b0 + i))
    top, bot = v.shape[0] - 2, v.shape[0] - 1
    last = (len(rings) - 1) * m
    for i in range(m):
        i1 = (i + 1) % m
        tris.append((top, i1, i))
        tris.append((bot, last + i, last + i1))
    t = _orient_outward(v, np.asarray(tris, dtype=np.int64))
    return Mesh(v + np.asarray(center, dtype=np.float64), t.astype(np.int32))


def cube_mesh(half):
    h = float(half)
    v = np.array([[x, y, z] for z in (-h, h) for y in (-h, h) for x in (-h, h)], dtype=np.float64)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    t = []
    for a, b, c, d in quads:
        t += [(a, b, c), (a, c, d)]
    return Mesh(v, _orient_outward(v, np.asarray(t, dtype=np.int64)).astype(np.int32))


def _naca_thickness(xi, t):
    return 5.0 * t * (0.2969 * np.sqrt(xi) - 0.1260 * xi - 0.3516 * xi**2 + 0.2843 * xi**3 - 0.1015 * xi**4)


@dataclass
class RotorSpec:
    n_blades: int
    radius: float
    hub_radius: float
    hub_length: float
    chord_root: float
    chord_tip: float
    pitch_root_deg: float = 50.0
    pitch_tip_deg: float = 20.0
    thickness: float = 0.12
    n_chord: int = 60
    n_span: int = 60
    n_hub: int = 64
    gap: float = 0.3
    seed: int = 0
    jitter: float = 0.05
    handed: int = 1  # +1 / -1 mirrors the blade pitch (counter-rotating rotors)


def rotor_mesh(spec: RotorSpec) -> Mesh:
    """Procedural bladed rotor, axis along body x, centred at the origin.

    Blades are symmetric NACA-00xx-like sections lofted from the hub to the tip
    with linear chord taper and linear twist; chord and pitch get a seeded
    per-blade jitter.  Hub and blades are disjoint closed surfaces (gap between
    hub surface and blade root), so the solid is their plain union.
    """
    rng = np.random.default_rng(spec.seed)
    parts = []
    # hub cylinder along x
    ph = np.linspace(0, 2 * math.pi, spec.n_hub, endpoint=False)
    rings = []
    for x in (-spec.hub_length / 2, spec.hub_length / 2):
        rings.append(np.stack([np.full_like(ph, x), spec.hub_radius * np.cos(ph), spec.hub_radius * np.sin(ph)], 1))
    parts.append(_loft(rings))
    m = np.arange(spec.n_chord + 1)
    xi = 0.5 * (1 - np.cos(np.pi * m / spec.n_chord))
    r0 = spec.hub_radius + spec.gap
    for kb in range(spec.n_blades):
        phi = 2 * math.pi * kb / spec.n_blades
        e_r = np.array([0.0, math.cos(phi), math.sin(phi)])
        e_t = np.array([0.0, -math.sin(phi), math.cos(phi)])
        e_x = np.array([1.0, 0.0, 0.0])
        cf = 1.0 + spec.jitter * rng.uniform(-1, 1)
        dpitch = math.radians(2.0) * rng.uniform(-1, 1)
        rings = []
        for j in range(spec.n_span + 1):
            eta = j / spec.n_span
            r = r0 + (spec.radius - r0) * eta
            c = (spec.chord_root + (spec.chord_tip - spec.chord_root) * eta) * cf
            beta = spec.handed * (math.radians(spec.pitch_root_deg + (spec.pitch_tip_deg - spec.pitch_root_deg) * eta) + dpitch)
            d_c = math.cos(beta) * e_t + math.sin(beta) * e_x
            d_n = -math.sin(beta) * e_t + math.cos(beta) * e_x
            yt = _naca_thickness(xi, spec.thickness) * c
            # ring: LE, upper surface to TE, lower surface back (TE has finite thickness)
            s_xi = np.concatenate([xi[:1], xi[1:], xi[1:][::-1]])
            s_y = np.concatenate([yt[:1], yt[1:], -yt[1:][::-1]])
            pts = r * e_r[None] + ((s_xi - 0.25) * c)[:, None] * d_c[None] + s_y[:, None] * d_n[None]
            rings.append(pts)
        parts.append(_loft(rings))
    return _merge(parts)


def mesh_signed_volume(mesh: Mesh) -> float:
    return _signed_volume(mesh.verts, mesh.tris.astype(np.int64))


# ----------------------------------------------------------------------------
# motion and workloads
# ----------------------------------------------------------------------------


@dataclass
class Motion:
    """Prescribed rigid motion: theta(t) = theta0 + omega*t about ``axis`` through X0 + V*t."""
    axis: tuple = (0.0, 0.0, 1.0)
    theta0: float = 0.0
    omega: float = 0.0
    x0: tuple = (0.0, 0.0, 0.0)
    v: tuple = (0.0, 0.0, 0.0)


@dataclass
class Shape:
    kind: str                 # "ellipsoid" (analytic, incl. sphere), "cube" (analytic), "mesh"
    params: tuple = ()        # ellipsoid: (a, b, c); cube: (half,)
    mesh: Mesh | None = None


@dataclass
class Body:
    shape: Shape
    motion: Motion
    s: int = 2                # supersampling depth: 2^s sub-cells per axis


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    q: int = 19
    storage: str = "f32"      # f64 / f32 / f16
    tau: float = 0.8
    magic: float = 3.0 / 16.0
    force: tuple = (0.0, 0.0, 0.0)
    bc: tuple = ("periodic",) * 6   # -x,+x,-y,+y,-z,+z
    u_in: tuple = (0.0, 0.0, 0.0)
    sc: int = 1
    b_form: int = 0
    slots: int = 1
    steps: int = 100
    bodies: list = field(default_factory=list)
    collision: str = "trt"    # "trt" or "cumulant" (D3Q27, no body force)
    map_reading: int = 0      # 0: every sub-sample rotated; 1: centre rotated, axis-aligned block
    layout: str = "soa"       # PDF buffer layout: "soa" or "blocked"
    block_rows: int = 0       # rows per block of the blocked layout (0: the library's choice)

    @property
    def n_cells(self):
        return self.nx * self.ny * self.nz


def _channel_bc():
    return ("inlet", "outlet", "wall", "wall", "wall", "wall")


def workload_sphere32(storage="f64"):
    """32^3 periodic box, static sphere r=6 at the centre, body force 1e-6 along x."""
    sph = Body(Shape("ellipsoid", (6.0, 6.0, 6.0)), Motion(x0=(16.0, 16.0, 16.0)), s=2)
    return Workload("sphere32_periodic_d3q19", 32, 32, 32, 19, storage, 0.8, 3 / 16, (1e-6, 0, 0),
                    ("periodic",) * 6, (0, 0, 0), 1, 0, 1, 200, [sph])


def workload_settling_sphere(nx=135, ny=135, nz=216, r=10.0, storage="f32", steps=4000, tau=0.575,
                             rho_s=1.16, g=7.4e-4, s=2, z0=None):
    """A sphere released from rest near the top of a closed box (no-slip walls on
    every face; the settling-sphere setup of section IV, 135 x 135 x 216 cells),
    SRT (TRT with Lambda = (tau - 1/2)^2), SC2.  Returns (workload, rigid) with
    rigid = dict(m, I, F_ext, X0): mass rho_s V, moments 2/5 m r^2, gravity
    minus buoyancy (rho_s - 1) V g along -z (fluid density 1)."""
    z0 = nz - 2.0 * r if z0 is None else z0
    X0 = (nx / 2.0, ny / 2.0, z0)
    sph = Body(Shape("ellipsoid", (r, r, r)), Motion(x0=X0), s=s)
    wl = Workload(f"settling_sphere_{nx}x{ny}x{nz}_r{r:g}", nx, ny, nz, 19, storage, tau, (tau - 0.5) ** 2,
                  (0.0, 0.0, 0.0), ("wall",) * 6, (0.0, 0.0, 0.0), 2, 0, 1, steps, [sph])
    vol = 4.0 / 3.0 * math.pi * r ** 3
    m = rho_s * vol
    rigid = dict(m=m, I=(0.4 * m * r * r,) * 3, F_ext=(0.0, 0.0, -(rho_s - 1.0) * vol * g), X0=X0)
    return wl, rigid


def workload_ellipsoid_channel(n=256, storage="f32", steps=2000, scale=1.0, s=3):
    """n^3 channel (inlet -x u=0.05, outlet +x, walls y,z), rotating ellipsoid about z."""
    a, b, c = 40.0 * scale, 20.0 * scale, 10.0 * scale
    ell = Body(Shape("ellipsoid", (round(a), round(b), round(c))),
               Motion(axis=(0, 0, 1), omega=1e-3, x0=(n / 2, n / 2, n / 2)), s=s)
    return Workload(f"ellipsoid_channel_{n}^3_d3q19", n, n, n, 19, storage, 0.8, 3 / 16, (0, 0, 0),
                    _channel_bc(), (0.05, 0, 0), 1, 0, 1, steps, [ell])


def cror_rotors(radius, n_blades, hub_len, n_chord, n_span, seed, centers, omegas, s=2, n_hub=64):
    bodies = []
    for i, (cx, om) in enumerate(zip(centers, omegas)):
        spec = RotorSpec(n_blades=n_blades, radius=radius, hub_radius=0.25 * radius, hub_length=hub_len,
                         chord_root=0.30 * radius, chord_tip=0.15 * radius, n_chord=n_chord, n_span=n_span,
                         n_hub=n_hub, seed=seed * 10 + i, handed=1 if om >= 0 else -1,
                         gap=max(0.3, 0.01 * radius))
        bodies.append(Body(Shape("mesh", (), rotor_mesh(spec)),
                           Motion(axis=(1, 0, 0), omega=om, x0=cx), s=s))
    return bodies


def workload_cror(nx=768, ny=384, nz=384, storage="f32", steps=1000, radius=120.0, s=2,
                  n_chord=60, n_span=60):
    """Counter-rotating pair of 8-blade rotors, D3Q27, inflow 0.05 along x."""
    yc, zc = ny / 2, nz / 2
    bodies = cror_rotors(radius, 8, 0.42 * radius, n_chord, n_span, 3,
                         [(nx / 3, yc, zc), (nx / 3 + 0.667 * radius, yc, zc)], [2e-3, -2e-3], s=s)
    return Workload(f"cror_{nx}x{ny}x{nz}_d3q27", nx, ny, nz, 27, storage, 0.6, 3 / 16, (0, 0, 0),
                    ("inlet", "outlet", "periodic", "periodic", "periodic", "periodic"), (0.05, 0, 0),
                    1, 0, 1, steps, bodies)


def workload_rotor_box(n=256, storage="f32", steps=1000, radius=120.0, s=2, n_chord=60, n_span=60):
    """One 8-blade rotor of radius 120 filling an n^3 box (the rotor-heavy
    scenario beside the small-body channel), D3Q19, inflow 0.05 along x."""
    c = n / 2
    bodies = cror_rotors(radius, 8, 0.42 * radius, n_chord, n_span, 3, [(c, c, c)], [2e-3], s=s)
    return Workload(f"rotor_box_{n}^3_d3q19", n, n, n, 19, storage, 0.8, 3 / 16, (0, 0, 0),
                    ("inlet", "outlet", "periodic", "periodic", "periodic", "periodic"), (0.05, 0, 0),
                    1, 0, 1, steps, bodies)


def workload_adjoint_rotor(n=128, steps=800, radius=40.0, s=2, n_chord=50, n_span=50, storage="f32"):
    """Single 4-blade rotor in an n^3 box, inflow 0.04 along x, periodic y, z."""
    c = n / 2
    bodies = cror_rotors(radius, 4, 0.5 * radius, n_chord, n_span, 4, [(c, c, c)], [1e-3], s=s)
    return Workload(f"rotor_adjoint_{n}^3_d3q19", n, n, n, 19, storage, 0.8, 3 / 16, (0, 0, 0),
                    ("inlet", "outlet", "periodic", "periodic", "periodic", "periodic"), (0.04, 0, 0),
                    1, 0, 1, steps, bodies)


def workload_capacity(n=1024, steps=500, radius=300.0, s=2, n_chord=100, n_span=100):
    """1024^3 in-place FP32 run with two counter-rotating 6-blade rotors."""
    c = n / 2
    bodies = cror_rotors(radius, 6, 0.333 * radius, n_chord, n_span, 5,
                         [(0.35 * n, c, c), (0.35 * n + 0.5 * radius, c, c)], [5e-4, -5e-4], s=s)
    return Workload(f"capacity_{n}^3_d3q19", n, n, n, 19, "f32", 0.8, 3 / 16, (0, 0, 0),
                    ("inlet", "outlet", "periodic", "periodic", "periodic", "periodic"), (0.05, 0, 0),
                    1, 0, 1, steps, bodies)


# ----------------------------------------------------------------------------
# random lattice states keyed by velocity (independent of any direction order)
# ----------------------------------------------------------------------------
def velocity_code(c) -> int:
    """Base-3 code (cx+1) + 3(cy+1) + 9(cz+1) in [0, 27) of a lattice velocity."""
    return int(c[0] + 1) + 3 * int(c[1] + 1) + 9 * int(c[2] + 1)


def random_state(seed: int, velocities, n_cells: int, cells, amp: float = 8.0):
    """delta f (len(cells), q) for the given velocities (q,3): exact in fp16 when
    ``amp`` is a power of two up to 8 (values are multiples of amp * 2^-17)."""
    cells = np.asarray(cells, dtype=np.int64)
    out = np.empty((cells.shape[0], len(velocities)))
    for j, c in enumerate(velocities):
        out[:, j] = pdf_deviation(seed, 27, n_cells, velocity_code(c), cells) * amp
    return out


def random_state_torch(seed: int, c, n_cells: int, device, dtype, amp: float = 8.0):
    """Whole (q, n_cells) delta f for the velocities c (q,3) as a torch tensor."""
    import torch

    out = torch.empty((len(c), n_cells), dtype=dtype, device=device)
    for k, ck in enumerate(c):
        out[k] = pdf_deviation_torch(seed, 27, n_cells, velocity_code(ck), device, torch.float64) .mul_(amp).to(dtype)
    return out
