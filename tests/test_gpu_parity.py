"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (error of f, lattice units) follow from the arithmetic:
FP64 storage/arithmetic: a few ulp of O(1) sums over two steps -> 1e-13;
FP32: arithmetic rounding ~6e-8 relative on O(1) terms (rho, 1 - B) over two
steps -> 2e-6; FP16 storage: each store rounds delta f to half an ulp,
2^-11 |delta f|; the first step's roundings of all Q neighbours feed the
second collision, so max |err| <= 4 * 2^-11 max |delta f| + 2e-6.  Solid
fractions and body ids must match bit for bit.  Test meshes avoid vertices
or faces on sample centres (no on-surface ties between the two voxelisers).
"""
import sys

import numpy as np
import pytest

import psm_inputs as pi

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 2e-6, "f16": 6e-5}
TOL_FT = {"f64": 1e-12, "f32": 2e-5, "f16": 5e-4}


@pytest.fixture(scope="module")
def sim():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2502_20049_amd import sim as s

    return s


@pytest.fixture(scope="module")
def gc():
    import gpu_common

    return gpu_common


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


BCS = {
    "periodic": ("periodic",) * 6,
    "channel": ("inlet", "outlet", "wall", "wall", "wall", "wall"),
    "box": ("wall",) * 6,
    "mixed": ("inlet", "outlet", "periodic", "periodic", "wall", "wall"),
    "zpipe": ("periodic", "periodic", "wall", "wall", "inlet", "outlet"),
}


def _workload(q, storage, bc, sc=1, two=False, s=2, force=(0, 0, 0), nx=70, ny=22, nz=13, b_form=0):
    bodies = [pi.Body(pi.Shape("ellipsoid", (9.0, 5.0, 4.0)),
                      pi.Motion(axis=(0.0, 0.6, 0.8), theta0=0.3, omega=0.05, x0=(31.0, 11.0, 6.0)), s=s)]
    if two:
        bodies.append(pi.Body(pi.Shape("ellipsoid", (4.0, 4.0, 4.0)),
                              pi.Motion(axis=(0, 0, 1), omega=-0.1, x0=(39.0, 12.0, 7.0), v=(0.2, 0.0, 0.0)), s=1))
    return pi.Workload(f"small_{q}_{storage}_{bc}", nx, ny, nz, q, storage, 0.8, 3 / 16, force, BCS[bc],
                       (0.04, 0.01, -0.02), sc, b_form, 2 if two else 1, 2, bodies)


def _two_step_compare(orc, sim, gc, wl, seed=5, general=False, solid_grid=0):
    import torch

    torch.manual_seed(0)
    f = sim.Field(wl)
    if general:
        f.set_option(1, 1)
    if solid_grid:
        f.set_option(8, solid_grid)  # PSM_OPT_SOLID_GRID
    gc.load_random_state(f, seed)
    run = orc.Run(wl, f0=gc.oracle_state(orc, wl, seed))
    out = {}
    for t in range(2):
        f.step(t)
        if not wl.bodies:
            run.advance(1)
            continue
        ftg = f.force_torque().cpu().numpy().copy()
        torch.cuda.synchronize()
        Bg = gc.gpu_B_per_body(f, len(wl.bodies))
        run.advance(1)
        assert np.array_equal(Bg, run.B), f"B mismatch at t={t}: {(Bg != run.B).sum()} cells"
        fto = run.ft[-1]
        scale = max(1e-12, np.abs(fto).max())
        err = np.abs(ftg - fto).max() / scale
        _say(f"  t={t} F/T rel err {err:.2e}")
        assert err < TOL_FT[wl.storage], (ftg, fto)
    g = gc.gpu_state_oracle_order(f, orc, sim)
    err = np.abs(g - run.f).max()
    _say(f"  {wl.name}: max |f_gpu - f_oracle| = {err:.3e}")
    if wl.storage == "f16":
        _, ow, _ = orc.lattice(wl.q)
        bound = 4 * 2.0 ** -11 * np.abs(run.f - ow[:, None]).max() + 2e-6
        assert err <= bound, (err, bound)
    else:
        assert err < TOL[wl.storage]
    flags = f.error_flags().cpu().numpy()
    assert flags[0] == 0
    out["f"] = f
    return out


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("bc", list(BCS))
def test_two_steps_parity(orc, sim, gc, q, storage, bc):
    _say(f"[two_steps] q={q} storage={storage} bc={bc}")
    wl = _workload(q, storage, bc)
    _two_step_compare(orc, sim, gc, wl)


@pytest.mark.parametrize("bc", ["channel", "mixed"])
@pytest.mark.parametrize("q", [19, 27])
def test_block_reading_two_steps_parity(orc, sim, gc, q, bc):
    """The block reading of the mapping (centre rotated, axis-aligned block)
    feeding two PSM steps: B bit-exact, f and F/T against the oracle."""
    import dataclasses

    wl = dataclasses.replace(_workload(q, "f32", bc, two=True, s=2), map_reading=1)
    _say(f"[two steps, block reading] q={q} bc={bc}")
    _two_step_compare(orc, sim, gc, wl)


@pytest.mark.parametrize("grid", [1, 2])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("q", [19, 27])
def test_solid_kernel_few_workgroups(orc, sim, gc, q, storage, grid):
    """The solid kernel capped at 1 or 2 workgroups (PSM_OPT_SOLID_GRID), two
    overlapping bodies: each workgroup walks several groups of chunks and
    carries the cells short of a whole round of 256 over to the next group.
    PDFs, B and F/T against the oracle."""
    _say(f"[solid_grid] q={q} {storage} grid={grid}")
    wl = _workload(q, storage, "mixed", two=True, force=(1e-5, 0.0, 0.0))
    _two_step_compare(orc, sim, gc, wl, solid_grid=grid)


def test_solid_grid_option_pdfs_bitwise(sim, gc):
    """The 192^3 channel (a few hundred chunks of 256 cells): the solid kernel
    capped at 3 workgroups gives the same PDF bits as the default grid, and
    F/T equal to FP64 rounding of the other grouping; out-of-range values are
    refused."""
    import ctypes as C

    import torch
    from paper_2502_20049_amd import _capi as capi

    wl = pi.workload_ellipsoid_channel(n=192, storage="f32", steps=4, s=3)
    res = []
    for grid in (0, 3):
        f = sim.Field(wl)
        f.set_option(8, grid)
        gc.load_random_state(f, 2)
        fts = []
        for t in range(4):
            ft = torch.zeros((1, 6), dtype=torch.float64, device="cuda")
            f.step(t, ft=ft)
            fts.append(ft)
        torch.cuda.synchronize()
        res.append((f.pdf_view().clone(), torch.stack(fts)))
    assert torch.equal(res[0][0], res[1][0])
    d = (res[0][1] - res[1][1]).abs().max().item() / res[0][1].abs().max().item()
    _say(f"[solid_grid 192] F/T rel diff {d:.1e}")
    assert d < 1e-12
    for bad in (-1, 4097):
        assert capi.lib.psm_set_option(f.handle, 8, bad) == capi.PSM_EINVAL


@pytest.mark.parametrize("sc", [1, 2, 3])
@pytest.mark.parametrize("q", [19, 27])
def test_solid_operators_two_bodies_force(orc, sim, gc, sc, q):
    """SC1/SC2/SC3, two overlapping moving bodies (two slots, one translating),
    Guo body force, tau-weighted B (eq. 6) for SC2."""
    _say(f"[solid_ops] q={q} sc={sc}")
    wl = _workload(q, "f64", "mixed", sc=sc, two=True, force=(1e-4, -5e-5, 2e-5), b_form=1 if sc == 2 else 0)
    _two_step_compare(orc, sim, gc, wl)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_fast_path_bitwise_equals_general_path(orc, sim, gc, storage):
    import torch

    _say(f"[fast_vs_general] {storage}")
    wl = _workload(19, storage, "mixed", two=True)
    res = []
    for general in (False, True):
        f = sim.Field(wl)
        f.set_option(1, 1 if general else 0)
        gc.load_random_state(f, 9)
        for t in range(4):
            f.step(t)
        torch.cuda.synchronize()
        res.append(f.pdf_view().clone())
    assert torch.equal(res[0], res[1])


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("bc", ["periodic", "channel", "box", "zpipe"])
def test_cumulant_two_steps_parity(orc, sim, gc, storage, bc):
    """Cumulant fluid collision (D3Q27, no body force) with the PSM blend of a
    moving body, two steps against the oracle."""
    _say(f"[cumulant] storage={storage} bc={bc}")
    wl = _workload(27, storage, bc)
    wl.collision = "cumulant"
    _two_step_compare(orc, sim, gc, wl)


@pytest.mark.parametrize("sc", [1, 2, 3])
def test_cumulant_two_bodies(orc, sim, gc, sc):
    _say(f"[cumulant two bodies] sc={sc}")
    wl = _workload(27, "f64", "mixed", sc=sc, two=True)
    wl.collision = "cumulant"
    _two_step_compare(orc, sim, gc, wl)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_cumulant_fast_path_bitwise_equals_general_path(sim, gc, storage):
    """nx = 128 (FP16 odd steps take the paired kernel) and four steps: the
    row kernels give the same bits as the per-cell general path."""
    import torch

    _say(f"[cumulant fast_vs_general] {storage}")
    wl = _workload(27, storage, "mixed", two=True, nx=128, ny=20, nz=14)
    wl.collision = "cumulant"
    res = []
    for general in (False, True):
        f = sim.Field(wl)
        f.set_option(1, 1 if general else 0)
        gc.load_random_state(f, 9)
        for t in range(4):
            f.step(t)
        torch.cuda.synchronize()
        res.append(f.pdf_view().clone())
    assert torch.equal(res[0], res[1])


@pytest.mark.parametrize("case", ["two_bodies_mixed", "channel_96", "channel_192", "plain_static", "q27_channel",
                                  "f16_rows_128", "general_path"])
def test_psm_step_equals_separate_calls(sim, gc, case):
    """psm_step against geometry_map_step + psm_stream_collide +
    body_force_torque called one by one: bit-identical PDFs, fractions and
    F/T (channel_192: more solid workgroups than the 256 threads of the F/T
    sum)."""
    import torch

    _say(f"[psm_step] {case}")
    if case == "two_bodies_mixed":
        wl, steps = _workload(19, "f32", "mixed", two=True, nx=96, ny=40, nz=36), 6
    elif case == "channel_96":
        wl, steps = pi.workload_ellipsoid_channel(n=96, storage="f32", steps=8, scale=0.4, s=2), 8
        wl.bodies[0].motion.omega = 0.02
    elif case == "channel_192":
        wl, steps = pi.workload_ellipsoid_channel(n=192, storage="f32", steps=4, s=3), 4
    elif case == "q27_channel":  # face-row launch on both parities
        wl, steps = _workload(27, "f32", "channel", two=True), 4
    elif case == "f16_rows_128":  # paired odd-step kernel, then the face rows
        wl, steps = _workload(19, "f16", "channel", two=True, nx=128, ny=24, nz=20), 4
    elif case == "general_path":  # no row kernels: the separate reduction
        wl, steps = _workload(19, "f32", "mixed", two=True), 4
    else:
        wl, steps = pi.workload_sphere32(storage="f32"), 4
    res = []
    for fused in (False, True):
        f = sim.Field(wl, fused=fused, remap_every_step=case != "plain_static")
        if case == "general_path":
            f.set_option(1, 1)  # PSM_OPT_GENERAL_PATH
        gc.load_random_state(f, 11)
        fts = []
        for t in range(steps):
            ft = torch.zeros((max(1, f.nb), 6), dtype=torch.float64, device="cuda")
            f.step(t, ft=ft)
            fts.append(ft)
        torch.cuda.synchronize()
        B, meta = f.b_view()
        res.append((f.pdf_view().clone(), B.clone(), meta.clone(), torch.stack(fts)))
    for other in res[1:]:
        for a, b in zip(res[0], other):
            assert torch.equal(a, b)


@pytest.mark.parametrize("nx", [256, 300])
@pytest.mark.parametrize("bc", ["channel", "periodic"])
@pytest.mark.parametrize("storage", ["f16", "f32"])
def test_wide_rows(orc, sim, gc, nx, bc, storage):
    """Rows of full 64/128-cell segments (and a partial one at nx = 300), with
    a body in the row: two steps against the oracle, then four steps of the
    fast path against the general path bit for bit."""
    import torch

    _say(f"[wide rows] nx={nx} {bc} {storage}")
    body = pi.Body(pi.Shape("ellipsoid", (9.0, 4.0, 3.0)),
                   pi.Motion(axis=(0.0, 0.6, 0.8), theta0=0.3, omega=0.05, x0=(130.0, 5.0, 4.0)), s=2)
    wl = pi.Workload(f"wide_{nx}_{bc}_{storage}", nx, 10, 8, 19, storage, 0.8, 3 / 16, (1e-5, 0, 0), BCS[bc],
                     (0.04, 0.01, -0.02), 1, 0, 1, 2, [body])
    _two_step_compare(orc, sim, gc, wl)
    res = []
    for general in (False, True):
        f = sim.Field(wl)
        f.set_option(1, 1 if general else 0)
        gc.load_random_state(f, 13)
        for t in range(4):
            f.step(t)
        torch.cuda.synchronize()
        res.append(f.pdf_view().clone())
    assert torch.equal(res[0], res[1])


DEGENERATE = [
    ((5, 1, 1), "periodic", False), ((40, 1, 6), "channel", False), ((40, 6, 1), "mixed", False),
    ((40, 2, 2), "box", False), ((70, 3, 3), "channel", True), ((1, 8, 8), "box", False),
    ((2, 9, 7), "zpipe", False), ((33, 17, 5), "channel", True),
]


@pytest.mark.parametrize("shape,bc,body", DEGENERATE)
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_degenerate_domains(orc, sim, gc, shape, bc, body, storage):
    """Slab, line and single-column lattices (no interior rows, rows shorter
    than a wave, a single cell per row, both x faces on one cell), with and
    without a body: two steps against the oracle, then the fast path against
    the general path bit for bit."""
    import torch

    nx, ny, nz = shape
    _say(f"[degenerate] {shape} {bc} body={body} {storage}")
    bodies = []
    if body:
        bodies = [pi.Body(pi.Shape("ellipsoid", (5.0, 2.5, 1.5)),
                          pi.Motion(axis=(0.0, 0.0, 1.0), theta0=0.4, omega=0.07, x0=(nx / 2, ny / 2, nz / 2)), s=2)]
    wl = pi.Workload(f"deg_{nx}x{ny}x{nz}_{bc}", nx, ny, nz, 19, storage, 0.8, 3 / 16, (1e-5, 2e-6, 0), BCS[bc],
                     (0.04, 0.01, -0.02), 1, 0, 1, 2, bodies)
    _two_step_compare(orc, sim, gc, wl)
    res = []
    for general in (False, True):
        f = sim.Field(wl)
        f.set_option(1, 1 if general else 0)
        gc.load_random_state(f, 17)
        for t in range(4):
            f.step(t)
        torch.cuda.synchronize()
        res.append(f.pdf_view().clone())
    assert torch.equal(res[0], res[1])


def test_bodies_outside_or_across_the_domain(orc, sim, gc):
    """A body entirely outside the lattice (empty swept box) and one cut by
    the domain faces."""
    _say("[bodies outside]")
    bodies = [pi.Body(pi.Shape("ellipsoid", (4.0, 3.0, 2.0)), pi.Motion(axis=(0, 0, 1), omega=0.1,
                                                                     x0=(-30.0, 5.0, 5.0)), s=1),
              pi.Body(pi.Shape("cube", (3.0,)), pi.Motion(axis=(0.6, 0.8, 0.0), omega=-0.2, x0=(1.0, 0.5, 6.0)),
                      s=2)]
    wl = pi.Workload("outside", 24, 12, 10, 19, "f64", 0.8, 3 / 16, (0, 0, 0), BCS["box"], (0.03, 0, 0), 1, 0, 2,
                     2, bodies)
    _two_step_compare(orc, sim, gc, wl)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_eight_bodies(orc, sim, gc, storage):
    """The most bodies a field takes (8): spheres, ellipsoids and cubes,
    moving and spinning, two pairs overlapping (two slots), one body partly
    outside the lattice, SC2 with a body force; B per body bit for bit, F/T of
    every body and the PDFs against the oracle over two steps."""
    _say(f"[eight bodies] {storage}")
    shapes = [pi.Shape("ellipsoid", (4.0, 3.0, 2.5)), pi.Shape("ellipsoid", (2.5, 2.5, 2.5)),
              pi.Shape("cube", (2.6,)), pi.Shape("ellipsoid", (3.5, 2.0, 2.0))]
    centres = [(8.0, 8.0, 7.0), (12.5, 9.0, 8.0), (24.0, 10.0, 9.0), (36.0, 14.0, 12.0),
               (47.0, 10.0, 8.5), (49.5, 12.0, 10.0), (60.0, 9.0, 11.0), (70.5, 20.0, 9.0)]
    bodies = []
    for i, x0 in enumerate(centres):
        axis = ((0.0, 0.0, 1.0), (0.6, 0.8, 0.0), (0.0, 1.0, 0.0), (0.48, 0.6, 0.64))[i % 4]
        bodies.append(pi.Body(shapes[i % 4], pi.Motion(axis=axis, theta0=0.1 * i, omega=0.05 * (i - 3.5),
                                                         x0=x0, v=(0.02 * (i % 3), -0.01 * (i % 2), 0.0)),
                              s=1 + (i % 3)))
    wl = pi.Workload(f"eight_{storage}", 72, 22, 19, 19, storage, 0.8, 3 / 16, (2e-5, 0.0, -1e-5), BCS["mixed"],
                     (0.04, 0.0, 0.0), 2, 0, 2, 2, bodies)
    _two_step_compare(orc, sim, gc, wl)


def test_xcd_remap_bitwise_identical(sim, gc):
    import torch

    wl = _workload(19, "f32", "channel")
    res = []
    for remap in (0, 1):
        f = sim.Field(wl)
        f.set_option(2, remap)
        gc.load_random_state(f, 3)
        for t in range(2):
            f.step(t)
        ft = f.force_torque().clone()
        torch.cuda.synchronize()
        res.append((f.pdf_view().clone(), ft))
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])


@pytest.mark.parametrize("s,cap,reading", [(0, None, 0), (1, None, 0), (2, None, 0), (3, None, 0), (2, 0, 0),
                                           (3, 0, 0), (2, 5, 0), (3, 5, 0), (0, None, 1), (1, None, 1),
                                           (2, None, 1), (3, None, 1), (3, 5, 1)])
def test_mapping_bit_exact(orc, sim, gc, s, cap, reading):
    """B(t) of rotating analytic and mesh bodies, two slots, random poses.
    cap: capacity of the surface-cell list sampled by the second mapping
    kernel (None: the default; 0: no list; 5: most cells overflow it).
    reading 0: every sub-sample rotated; 1: the centre rotated and the
    axis-aligned block averaged (section III, both readings)."""
    import torch

    _say(f"[mapping] s={s} list cap={cap} reading={reading}")
    rotor = pi.rotor_mesh(pi.RotorSpec(n_blades=3, radius=7.0, hub_radius=1.75, hub_length=3.1, chord_root=2.1,
                                       chord_tip=1.05, n_chord=8, n_span=6, n_hub=16, seed=7))
    bodies = [pi.Body(pi.Shape("mesh", (), rotor), pi.Motion(axis=(1, 0, 0), theta0=0.2, omega=0.37,
                                                              x0=(16.0, 15.0, 14.0)), s=s),
              pi.Body(pi.Shape("cube", (3.0,)), pi.Motion(axis=(0.48, 0.6, 0.64), theta0=1.0, omega=-0.3,
                                                          x0=(22.5, 13.0, 15.5), v=(0.3, -0.1, 0.2)), s=s),
              pi.Body(pi.Shape("ellipsoid", (4.0, 3.0, 2.0)), pi.Motion(axis=(0, 1, 0), omega=0.7,
                                                                       x0=(8.0, 20.0, 9.0)), s=max(0, s - 1))]
    wl = pi.Workload("map", 33, 30, 28, 19, "f32", 0.8, 3 / 16, (0, 0, 0), ("periodic",) * 6, (0, 0, 0), 1, 0, 2, 3,
                     bodies, map_reading=reading)
    f = sim.Field(wl, max_bodies=3)
    if cap is not None:
        f.set_option(4, cap)
    run = orc.Run(wl)
    for t in (0, 1, 2, 5):
        f.map(t)
        torch.cuda.synchronize()
        Bg = gc.gpu_B_per_body(f, 3)
        run.map(t)
        diff = (Bg != run.B).sum()
        _say(f"  t={t}: sum B = {Bg.sum(axis=1)}, mismatches {diff}")
        assert diff == 0
        assert f.error_flags().cpu().numpy()[0] == 0


def test_three_bodies_in_two_slots_flags_error(sim):
    import torch

    bodies = [pi.Body(pi.Shape("ellipsoid", (4.0, 4.0, 4.0)), pi.Motion(x0=(10.0 + d, 10.0, 10.0)), s=1)
              for d in (0.0, 1.0, 2.0)]
    wl = pi.Workload("three", 24, 20, 20, 19, "f32", 0.8, 3 / 16, (0, 0, 0), ("periodic",) * 6, (0, 0, 0), 1, 0, 2, 1,
                     bodies)
    f = sim.Field(wl, max_bodies=3)
    f.map(0)
    torch.cuda.synchronize()
    assert f.error_flags().cpu().numpy()[0] & 1
    wl2 = pi.Workload("two", 24, 20, 20, 19, "f32", 0.8, 3 / 16, (0, 0, 0), ("periodic",) * 6, (0, 0, 0), 1, 0, 2, 1,
                      bodies[:2])
    f2 = sim.Field(wl2)
    f2.map(0)
    torch.cuda.synchronize()
    assert f2.error_flags().cpu().numpy()[0] == 0


def test_sphere32_periodic_fp64_trajectory(orc, sim, gc):
    """32^3 periodic box, static sphere r=6 (s=2), force 1e-6 along x, FP64,
    200 steps: drag series, velocity field and exact mass conservation."""
    import torch

    _say("[sphere32] 200 steps")
    wl = pi.workload_sphere32()
    f = sim.Field(wl, remap_every_step=False)
    run = orc.Run(wl)
    m0 = f.mass(0).item()
    drag_g = []
    for t in range(wl.steps):
        f.step(t)
        drag_g.append(f.force_torque().cpu().numpy().copy())
    torch.cuda.synchronize()
    run.advance(wl.steps, remap=False)
    drag_g = np.array(drag_g)[:, 0]
    drag_o = np.array(run.ft)[:, 0]
    rel = np.abs(drag_g[:, 0] - drag_o[:, 0]).max() / np.abs(drag_o[:, 0]).max()
    _say(f"  drag rel err {rel:.2e}; final drag {drag_o[-1, 0]:.6e}")
    assert rel < 1e-10
    # symmetric body centred on a lattice corner, force along x: no torque, no lift
    assert np.abs(drag_g[:, 3:]).max() < 1e-12 * np.abs(drag_o[:, 0]).max()
    assert np.abs(drag_g[:, 1:3]).max() < 1e-12 * np.abs(drag_o[:, 0]).max()
    m1 = f.mass(wl.steps).item()
    assert abs(m1 - m0) / m0 < 1e-13 and abs(m0 - wl.n_cells) < 1e-9
    rho_g, u_g = f.macroscopic(wl.steps)
    rho_o, u_o = run.macro()
    u_g = u_g.cpu().numpy()
    relu = np.linalg.norm(u_g - u_o) / np.linalg.norm(u_o)
    _say(f"  u rel L2 {relu:.2e}, mass drift {abs(m1 - m0) / m0:.2e}")
    assert relu < 1e-10


def test_ellipsoid_channel_fp32_trajectory(orc, sim, gc):
    """Reduced copy of the rotating-ellipsoid channel (64^3, semi-axes 10,5,3
    (integer-scaled), s=3, inlet 0.05, FP32 storage) for 200 steps against the
    FP64 oracle: velocity rel. L2 <= 1e-5 and torque <= 1e-4 (the targets for
    FP32 storage)."""
    import torch

    _say("[ellipsoid channel 64^3] 200 steps")
    wl = pi.workload_ellipsoid_channel(n=64, storage="f32", steps=200, scale=0.25, s=3)
    wl.bodies[0].motion.omega = 4e-3
    f = sim.Field(wl)
    run = orc.Run(wl)
    ftg = []
    for t in range(wl.steps):
        f.step(t)
        ftg.append(f.force_torque().cpu().numpy().copy())
    torch.cuda.synchronize()
    run.advance(wl.steps)
    rho_g, u_g = f.macroscopic(wl.steps)
    rho_o, u_o = run.macro()
    relu = np.linalg.norm(u_g.cpu().numpy() - u_o) / np.linalg.norm(u_o)
    ftg = np.array(ftg)[:, 0]
    fto = np.array(run.ft)[:, 0]
    Tz_g, Tz_o = ftg[:, 5], fto[:, 5]
    relT = np.abs(Tz_g - Tz_o).max() / np.abs(Tz_o).max()
    relJ = abs(Tz_g[-50:].mean() - Tz_o[-50:].mean()) / abs(Tz_o[-50:].mean())
    _say(f"  u rel L2 {relu:.2e}; torque series rel {relT:.2e}; window mean rel {relJ:.2e}")
    assert relu < 1e-5
    assert relT < 1e-4 and relJ < 1e-4


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_channel_accuracy_vs_fp64_oracle(orc, sim, storage):
    """Reduced rotating-ellipsoid channel (48^3, s = 3, 100 steps): FP32 and
    FP16 deviation storage against the FP64 oracle, velocity rel. L2 and the
    torque series (targets: FP32 1e-5 / 1e-4; FP16 storage rounds each stored
    deviation to 11 bits: 5e-4 / 1e-4)."""
    import torch

    wl = pi.workload_ellipsoid_channel(n=48, storage=storage, steps=100, scale=0.25, s=3)
    wl.bodies[0].motion.omega = 4e-3
    run = orc.Run(wl).advance(wl.steps)
    _, uo = run.macro()
    Tz_o = np.array(run.ft)[:, 0, 5]
    f = sim.Field(wl)
    tz = []
    for t in range(wl.steps):
        f.step(t)
        tz.append(f.force_torque()[0, 5].item())
    _, ug = f.macroscopic(wl.steps)
    torch.cuda.synchronize()
    ug = ug.cpu().numpy()
    relu = float(np.linalg.norm(ug - uo) / np.linalg.norm(uo))
    relT = float(np.abs(np.array(tz) - Tz_o).max() / np.abs(Tz_o).max())
    _say(f"[accuracy] {storage}: u rel L2 {relu:.2e}, torque rel max {relT:.2e}")
    if storage == "f32":
        assert relu < 1e-5 and relT < 1e-4
    else:
        assert relu < 5e-4 and relT < 1e-4
