"""Host-side checks of the C ABI (no GPU): exported symbols, sizes, argument
validation, lattice table, kinematics and the host voxeliser, each against the
oracle or a closed form."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import psm_inputs as pi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def capi():
    from paper_2502_20049_amd import _capi

    return _capi


@pytest.fixture(scope="module")
def sim():
    from paper_2502_20049_amd import sim

    return sim


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "psm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_library_exports_every_declared_symbol(capi):
    decl = _declared_functions()
    assert len(decl) >= 20
    for name in decl:
        assert hasattr(capi.lib, name), name
    assert sorted(decl) == sorted(capi.EXPORTS)


def _cfg(sim, **kw):
    wl = pi.Workload("t", 40, 30, 20, bodies=[])
    for k, v in kw.items():
        setattr(wl, k, v)
    return sim.make_config(wl, max_bodies=2)


def test_required_bytes(capi, sim):
    cfg = _cfg(sim)
    N = 40 * 30 * 20
    def stride(sz):  # N padded to a 4 KiB multiple plus 4 KiB, in elements
        return ((N * sz + 4095) // 4096 * 4096 + 4096) // sz

    st = C.c_int64()
    assert capi.lib.psm_pdf_stride(C.byref(cfg), C.byref(st)) == 0 and st.value == stride(4)
    assert sim.required_bytes(cfg, capi.PSM_BUF_PDF) == 19 * stride(4) * 4
    assert sim.required_bytes(cfg, capi.PSM_BUF_B) == N * 4 + N
    cfg.slots = 2
    assert sim.required_bytes(cfg, capi.PSM_BUF_B) == 2 * N * 4 + N
    # two sets of fractions, the second 256-byte aligned
    cfg.map_ahead = 1
    assert sim.required_bytes(cfg, capi.PSM_BUF_B) == 2 * ((2 * N * 4 + N + 255) // 256 * 256)
    cfg.map_ahead = 0
    cfg.q, cfg.storage = 27, capi.PSM_F16
    assert sim.required_bytes(cfg, capi.PSM_BUF_PDF) == 27 * stride(2) * 2
    assert sim.required_bytes(cfg, capi.PSM_BUF_OBSTACLE) == 0
    cfg.psm = 0
    assert sim.required_bytes(cfg, capi.PSM_BUF_B) == 0
    assert sim.required_bytes(cfg, capi.PSM_BUF_WORK) > 256
    # header + class bytes padded to 256 + one 8-byte list entry per cell
    assert sim.required_bytes(cfg, capi.PSM_BUF_OBSTACLE) == 256 + ((N + 255) // 256) * 256 + 8 * N


def test_noalloc_rejects_lattices_beyond_the_static_area(capi, sim):
    """pdf_field_create_noalloc refuses (PSM_ESIZE, before any device call)
    a lattice whose fixed part of the work area exceeds the static array."""
    cfg = _cfg(sim, nx=1024, ny=1024, nz=520)
    h = C.c_void_p()
    assert capi.lib.pdf_field_create_noalloc(C.byref(cfg), None, 0, None, 0, None, C.byref(h)) == capi.PSM_ESIZE
    assert "static" in capi.last_error() and not h.value
    assert capi.lib.pdf_field_create_noalloc(None, None, 0, None, 0, None, C.byref(h)) == capi.PSM_EINVAL


@pytest.mark.parametrize("field,value,code", [
    ("q", 15, -1), ("storage", 7, -1), ("sc", 4, -1), ("slots", 3, -1), ("tau", 0.5, -1),
    ("b_form", 2, -1), ("max_bodies", 9, -1), ("nx", 0, -1), ("map_reading", 2, -1), ("map_reading", -1, -1),
    ("layout", 2, -1), ("block_rows", 4, -1), ("map_ahead", 2, -1), ("map_ahead", -1, -1),
])
def test_config_validation(capi, sim, field, value, code):
    cfg = _cfg(sim)
    setattr(cfg, field, value)
    n = C.c_size_t()
    assert capi.lib.psm_required_bytes(C.byref(cfg), 0, C.byref(n)) == code
    assert capi.last_error()


def test_cumulant_config_validation(capi, sim):
    """The cumulant collision is D3Q27 without body force; other values of
    `collision` are invalid."""
    n = C.c_size_t()
    cfg = _cfg(sim)
    cfg.q, cfg.collision = 27, capi.PSM_COLL_CUMULANT
    assert capi.lib.psm_required_bytes(C.byref(cfg), 0, C.byref(n)) == capi.PSM_OK
    cfg.q = 19
    assert capi.lib.psm_required_bytes(C.byref(cfg), 0, C.byref(n)) == capi.PSM_EUNSUP
    cfg.q = 27
    cfg.force[0] = 1e-5
    assert capi.lib.psm_required_bytes(C.byref(cfg), 0, C.byref(n)) == capi.PSM_EUNSUP
    cfg.force[0] = 0.0
    cfg.collision = 2
    assert capi.lib.psm_required_bytes(C.byref(cfg), 0, C.byref(n)) == capi.PSM_EINVAL


def test_unpaired_periodic_face_rejected(capi, sim):
    cfg = _cfg(sim)
    cfg.bc[0] = capi.PSM_PERIODIC
    cfg.bc[1] = capi.PSM_WALL
    n = C.c_size_t()
    assert capi.lib.psm_required_bytes(C.byref(cfg), 0, C.byref(n)) == capi.PSM_EINVAL


def test_create_rejects_bad_buffers(capi, sim):
    cfg = _cfg(sim)
    h = C.c_void_p()
    need = sim.required_bytes(cfg, capi.PSM_BUF_PDF)
    # null buffers and undersized buffers are rejected before any device access
    assert capi.lib.pdf_field_create(C.byref(cfg), None, need, None, 0, None, 0, None, C.byref(h)) == capi.PSM_EINVAL
    fake = C.c_void_p(1 << 20)  # never dereferenced: size checks fail first
    assert capi.lib.pdf_field_create(C.byref(cfg), fake, need - 1, fake, 1 << 30, fake, 1 << 30, None,
                                     C.byref(h)) == capi.PSM_ESIZE
    assert capi.lib.pdf_field_destroy(None) == capi.PSM_EINVAL


def test_lattice_matches_oracle_set(orc, sim):
    for q in (19, 27):
        c, w, o = sim.lattice(q)
        oc, ow, oo = orc.lattice(q)
        # same velocity set and weights, in a different order
        key = {tuple(v): wv for v, wv in zip(oc, ow)}
        assert len(key) == q
        for v, wv in zip(c, w):
            assert key[tuple(v)] == wv
        assert np.all(c[o] == -c)
        assert c[0].tolist() == [0, 0, 0]


def test_body_pose_bit_identical_to_oracle(orc, sim):
    rng = np.random.default_rng(1)
    for trial in range(20):
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        m = pi.Motion(axis=tuple(ax), theta0=float(rng.uniform(-3, 3)), omega=float(rng.uniform(-0.01, 0.01)),
                      x0=tuple(rng.uniform(0, 100, 3)), v=tuple(rng.uniform(-0.1, 0.1, 3)))
        for t in (0, 1, 17, 799, 123456):
            a = sim.body_pose(m, t)
            b = orc.pose_at(m, t)
            assert list(a.R) == list(b.R) and list(a.X) == list(b.X)
            assert list(a.V) == list(b.V) and list(a.W) == list(b.W)


def _box(capi, shape, s, mesh=None):
    dp = C.POINTER(C.c_double)
    mmin = (C.c_int32 * 3)()
    dims = (C.c_int32 * 3)()
    nb = C.c_size_t()
    if mesh is not None:
        v = np.ascontiguousarray(mesh.verts)
        assert capi.lib.psm_geometry_box(-1, None, v.ctypes.data_as(dp), v.shape[0], s, mmin, dims, C.byref(nb)) == 0
    else:
        p = np.zeros(3)
        p[: len(shape[1])] = shape[1]
        assert capi.lib.psm_geometry_box(shape[0], p.ctypes.data_as(dp), None, 0, s, mmin, dims, C.byref(nb)) == 0
    return np.array(mmin), np.array(dims)


def _unpack(bits, dims):
    wx = (dims[0] + 31) // 32
    w = bits.reshape(dims[2], dims[1], wx)
    out = np.zeros((dims[2], dims[1], wx * 32), dtype=np.uint8)
    for b in range(32):
        out[:, :, b::32] = (w >> np.uint32(b)) & 1
    return out[:, :, : dims[0]]


def test_analytic_fill_matches_oracle(capi, orc):
    for shape, params, s in [(capi.PSM_SHAPE_ELLIPSOID, (5.0, 3.0, 2.0), 2), (capi.PSM_SHAPE_ELLIPSOID, (6.0, 6.0, 6.0), 1),
                             (capi.PSM_SHAPE_CUBE, (2.5,), 3)]:
        mmin, dims = _box(capi, (shape, params), s)
        wx = (dims[0] + 31) // 32
        bits = np.zeros(wx * dims[1] * dims[2], dtype=np.uint32)
        p = np.zeros(3)
        p[: len(params)] = params
        assert capi.lib.psm_analytic_host(shape, p.ctypes.data_as(C.POINTER(C.c_double)), s,
                                          (C.c_int32 * 3)(*mmin), (C.c_int32 * 3)(*dims),
                                          bits.ctypes.data_as(C.POINTER(C.c_uint32))) == 0
        got = _unpack(bits, dims)
        g = orc.OracleGeometry(pi.Shape("ellipsoid" if shape == 0 else "cube", params), s)
        mz, my, mx = np.meshgrid(*[np.arange(mmin[a], mmin[a] + dims[a]) for a in (2, 1, 0)], indexing="ij")
        ref = g.inside(np.stack([mx.ravel(), my.ravel(), mz.ravel()], 1)).reshape(got.shape)
        assert np.array_equal(got.astype(bool), ref)
        # one LBM cell of padding around the shape: the border planes are empty
        assert got[0].sum() == 0 and got[-1].sum() == 0 and got[:, :, 0].sum() == 0


@pytest.mark.parametrize("which", ["rotor", "ellipsoid", "cube"])
def test_voxeliser_matches_winding_number(capi, orc, which):
    if which == "rotor":
        mesh = pi.rotor_mesh(pi.RotorSpec(n_blades=3, radius=5.0, hub_radius=1.25, hub_length=2.5, chord_root=1.5,
                                          chord_tip=0.75, n_chord=8, n_span=5, n_hub=16, seed=3))
        s = 2
    elif which == "ellipsoid":
        mesh = pi.ellipsoid_mesh(4.0, 2.5, 1.75, n_lat=10, n_lon=20, phase=0.1)
        s = 2
    else:
        mesh = pi.cube_mesh(1.3)
        s = 3
    mmin, dims = _box(capi, None, s, mesh)
    wx = (dims[0] + 31) // 32
    bits = np.zeros(wx * dims[1] * dims[2], dtype=np.uint32)
    v = np.ascontiguousarray(mesh.verts)
    t = np.ascontiguousarray(mesh.tris)
    assert capi.lib.psm_voxelize_host(v.ctypes.data_as(C.POINTER(C.c_double)), v.shape[0],
                                      t.ctypes.data_as(C.POINTER(C.c_int32)), t.shape[0], s,
                                      (C.c_int32 * 3)(*mmin), (C.c_int32 * 3)(*dims),
                                      bits.ctypes.data_as(C.POINTER(C.c_uint32))) == 0
    got = _unpack(bits, dims).astype(bool)
    ref = orc.voxelize(v, t, s, mmin.astype(np.int32), dims.astype(np.int32)).reshape(got.shape).astype(bool)
    assert got.sum() > 50
    assert np.array_equal(got, ref), int((got != ref).sum())


def test_rigid_advance_matches_oracle(capi, orc):
    """The library's host integrator (psm_rigid_advance) against the oracle's
    over 40 steps of an asymmetric body with random force / torque."""
    import ctypes as C

    import numpy as np

    import psm_inputs as pi

    rg = dict(m=7.0, I=(2.0, 3.5, 5.0), F_ext=(0.0, 0.0, -0.3), X0=(4.0, 5.0, 6.0))
    st = orc.rigid_state(rg, average=True)
    s = capi.psm_rigid()
    s.average = 1
    s.m, s.I, s.F_ext, s.X = rg["m"], (C.c_double * 3)(*rg["I"]), (C.c_double * 3)(*rg["F_ext"]), \
        (C.c_double * 3)(*rg["X0"])
    s.R = (C.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    ft_all = (pi.random_unit(17, 40 * 6) - 0.5) * 0.2
    for k in range(40):
        ft = np.ascontiguousarray(ft_all[6 * k: 6 * k + 6])
        assert capi.lib.psm_rigid_advance(C.byref(s), ft.ctypes.data_as(C.POINTER(C.c_double)), 1.0) == 0
        orc.rigid_advance(st, ft)
    assert np.allclose(np.array(s.X), st["X"], rtol=0, atol=1e-12)
    assert np.allclose(np.array(s.V), st["V"], rtol=0, atol=1e-13)
    assert np.allclose(np.array(s.W), st["W"], rtol=0, atol=1e-13)
    assert np.allclose(np.array(s.R).reshape(3, 3), st["R"], rtol=0, atol=1e-12)
    body = capi.psm_body()
    assert capi.lib.psm_rigid_body(C.byref(s), C.byref(body)) == 0
    assert np.array_equal(np.array(body.X), np.array(s.X)) and np.array_equal(np.array(body.W), np.array(s.W))
    bad = capi.psm_rigid()
    assert capi.lib.psm_rigid_advance(C.byref(bad), ft.ctypes.data_as(C.POINTER(C.c_double)), 1.0) == capi.PSM_EINVAL


def test_new_entry_points_reject_null_arguments(capi, sim):
    """Host-side argument checks of the obstacle, coupling and layout calls
    (no device access)."""
    cfg = _cfg(sim)
    st = C.c_int64()
    assert capi.lib.psm_pdf_stride(None, C.byref(st)) == capi.PSM_EINVAL
    assert capi.lib.psm_pdf_stride(C.byref(cfg), None) == capi.PSM_EINVAL
    assert capi.lib.lbm_set_obstacle(None, None, None, 0, None, None) == capi.PSM_EINVAL
    assert capi.lib.psm_coupled_step(None, None, None, 1, 0, None, None, None) == capi.PSM_EINVAL
    assert capi.lib.psm_rigid_body(None, None) == capi.PSM_EINVAL
    s = capi.psm_rigid()
    assert capi.lib.psm_rigid_advance(C.byref(s), None, 1.0) == capi.PSM_EINVAL
    assert capi.lib.psm_step_ahead(None, None, None, None, None, 1, 0, None, None) == capi.PSM_EINVAL
    assert capi.lib.psm_adjoint_gather(None, None, None, None) == capi.PSM_EINVAL
    assert capi.lib.psm_fractions(None, None, None, None) == capi.PSM_EINVAL
    # map_ahead needs a PSM field
    cfg.psm, cfg.map_ahead = 0, 1
    n = C.c_size_t()
    assert capi.lib.psm_required_bytes(C.byref(cfg), 0, C.byref(n)) == capi.PSM_EINVAL
    assert "map_ahead" in capi.last_error()


@pytest.mark.parametrize("shape,storage,rows", [((70, 22, 13), 1, 0), ((256, 256, 256), 1, 0), ((256, 8, 8), 2, 0),
                                                ((1024, 4, 4), 0, 0), ((70, 22, 13), 1, 8), ((5, 3, 2), 2, 8)])
def test_blocked_layout_sizes(capi, sim, shape, storage, rows):
    """psm_pdf_layout and the PDF buffer size agree: blocks of RB rows (a
    power of two; by default RB*nx*sizeof <= 16 KiB), q*RB*nx elements
    each, the last block padded."""
    cfg = _cfg(sim)
    cfg.nx, cfg.ny, cfg.nz = shape
    cfg.storage = storage
    cfg.layout = capi.PSM_LAYOUT_BLOCKED
    cfg.block_rows = rows
    rb, ds, bs = C.c_int32(), C.c_int64(), C.c_int64()
    assert capi.lib.psm_pdf_layout(C.byref(cfg), C.byref(rb), C.byref(ds), C.byref(bs)) == 0
    nx, ny, nz = shape
    sz = {0: 8, 1: 4, 2: 2}[storage]
    RB = rb.value
    assert RB & (RB - 1) == 0
    if rows:
        assert RB == rows
    else:
        assert RB == 1 or RB * nx * sz <= 16384
        assert 2 * RB > ny * nz or 2 * RB * nx * sz > 16384
    assert ds.value == RB * nx and bs.value == cfg.q * RB * nx
    n = C.c_size_t()
    assert capi.lib.psm_required_bytes(C.byref(cfg), capi.PSM_BUF_PDF, C.byref(n)) == 0
    assert n.value == -(-(ny * nz) // RB) * bs.value * sz
    st = C.c_int64()
    assert capi.lib.psm_pdf_stride(C.byref(cfg), C.byref(st)) == 0 and st.value == ds.value
