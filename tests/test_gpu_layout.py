"""The blocked PDF layout (psm_config.layout = PSM_LAYOUT_BLOCKED) against the
SoA layout and the oracle.

Only the addresses differ between the layouts: every kernel runs the same
arithmetic in the same order, so results must be bit-identical to the SoA
field's (PDFs in the standard layout, B, force/torque, macroscopic fields,
mass), and the oracle parity of the SoA tests carries over with the same
tolerances.  Lattices cover blocks cut short at the end of the rows, row
lengths that are and are not multiples of 128 (the paired FP16 odd step),
every face rule, both collision models, two-body overlap, static obstacles,
the general path and the adjoint.
"""
import dataclasses
import sys

import numpy as np
import pytest

import psm_inputs as pi

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def _blocked(wl, rows=0):
    return dataclasses.replace(wl, layout="blocked", block_rows=rows)


def _layout_numbers(sim, wl):
    import ctypes as C

    from paper_2502_20049_amd import _capi as capi

    cfg = sim.make_config(wl)
    rb, ds, bs = C.c_int32(), C.c_int64(), C.c_int64()
    capi.check(capi.lib.psm_pdf_layout(C.byref(cfg), C.byref(rb), C.byref(ds), C.byref(bs)), "psm_pdf_layout")
    return rb.value, ds.value, bs.value


@pytest.mark.parametrize("shape", [(70, 22, 13), (256, 8, 8), (300, 5, 7), (1, 1, 1), (4097, 2, 3)])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_gather_scatter_round_trip(sim, shape, storage):
    """Scatter then gather gives the array back bit for bit, and the blocked
    buffer holds each element where psm_pdf_layout says."""
    import torch

    nx, ny, nz = shape
    wl = pi.Workload("rt", nx, ny, nz, 19, storage, 0.8, 3 / 16, (0, 0, 0), ("periodic",) * 6, (0, 0, 0), 1, 0, 1, 1,
                     [], layout="blocked")
    f = sim.Field(wl, psm=False)
    q, N = 19, wl.n_cells
    src = torch.arange(q * N, device="cuda", dtype=torch.float64).remainder(2039.0).mul(0.25).sub(250.0)
    src = src.to(f.dtype).view(q, N)
    f.load_pdf_std(src)
    back = f.pdf_std()
    torch.cuda.synchronize()
    assert torch.equal(back, src)
    rb, ds, bs = _layout_numbers(sim, wl)
    assert rb >= 1 and (rb & (rb - 1)) == 0 and (rb * nx * f.dtype.itemsize <= 16384 or rb == 1)
    assert ds == rb * nx and bs == q * ds
    buf = f.pdf
    rng = np.random.default_rng(0)
    for _ in range(50):
        k, n = int(rng.integers(q)), int(rng.integers(N))
        x, r = n % nx, n // nx
        e = (r // rb) * bs + k * ds + (r % rb) * nx + x
        assert buf[e].item() == src[k, n].item()


def _run_pair(sim, gc, wl, steps, seed=3, setup=None, collect_ft=True, rows=0):
    """The same steps on a SoA and a blocked field (rows per block: `rows`,
    0 for the library's choice) from one seeded state: returns the two
    result dicts."""
    import torch

    out = []
    for w in (wl, _blocked(wl, rows)):
        f = sim.Field(w)
        if setup:
            setup(f)
        gc.load_random_state(f, seed)
        fts = []
        for t in range(steps):
            f.step(t)
            if collect_ft and f.nb:
                fts.append(f.force_torque().clone())
        torch.cuda.synchronize()
        r = {"pdf": f.pdf_std().clone(), "ft": torch.stack(fts) if fts else None,
             "mass": f.mass(steps).item()}
        rho, u = f.macroscopic(steps)
        r["rho"], r["u"] = rho.clone(), u.clone()
        if f.nb:
            B, meta = f.b_view()
            r["B"], r["meta"] = B.clone(), meta.clone()
        r["flags"] = f.error_flags().cpu().numpy()[0]
        out.append(r)
        del f
    return out


def _assert_same(a, b):
    import torch

    for key in a:
        if a[key] is None:
            assert b[key] is None
        elif isinstance(a[key], float):
            assert a[key] == b[key], key
        elif isinstance(a[key], np.integer) or isinstance(a[key], int):
            assert a[key] == b[key] == 0, key
        else:
            assert torch.equal(a[key], b[key]), key


CASES = {
    # name: (workload builder, steps)
    "channel_q19_f32": (lambda: _small(19, "f32", ("inlet", "outlet", "wall", "wall", "wall", "wall")), 4),
    "channel_q19_f16_h2": (lambda: _small(19, "f16", ("inlet", "outlet", "wall", "wall", "wall", "wall"), nx=128), 4),
    "mixed_q19_f64": (lambda: _small(19, "f64", ("inlet", "outlet", "periodic", "periodic", "wall", "wall")), 3),
    "zpipe_q27_f32": (lambda: _small(27, "f32", ("periodic", "periodic", "wall", "wall", "inlet", "outlet")), 4),
    "box_q27_f16_h2": (lambda: _small(27, "f16", ("wall",) * 6, nx=256), 4),
    "periodic_q19_f32_two_sc2": (lambda: _small(19, "f32", ("periodic",) * 6, two=True, sc=2), 4),
    "periodic_q27_f32_two_sc3": (lambda: _small(27, "f32", ("periodic",) * 6, two=True, sc=3), 3),
    "cumulant_q27_f16": (lambda: dataclasses.replace(_small(27, "f16", ("inlet", "outlet", "wall", "wall", "periodic",
                                                                         "periodic"), nx=128), collision="cumulant"), 4),
    "forced_q19_f32_eq6": (lambda: dataclasses.replace(_small(19, "f32", ("periodic",) * 6, force=(2e-5, 0, 1e-5)),
                                                       b_form=1), 4),
    "wide_300_q19_f16": (lambda: _small(19, "f16", ("inlet", "outlet", "wall", "wall", "wall", "wall"), nx=300), 4),
}


def _small(q, storage, bc, nx=70, ny=22, nz=13, two=False, sc=1, force=(0, 0, 0)):
    bodies = [pi.Body(pi.Shape("ellipsoid", (9.0, 5.0, 4.0)),
                      pi.Motion(axis=(0.0, 0.6, 0.8), theta0=0.3, omega=0.05, x0=(31.0, 11.0, 6.0)), s=2)]
    if two:
        bodies.append(pi.Body(pi.Shape("ellipsoid", (4.0, 4.0, 4.0)),
                              pi.Motion(axis=(0, 0, 1), omega=-0.1, x0=(39.0, 12.0, 7.0), v=(0.2, 0.0, 0.0)), s=1))
    return pi.Workload(f"lay_{q}_{storage}_{nx}", nx, ny, nz, q, storage, 0.8, 3 / 16, force, bc, (0.04, 0.01, -0.02),
                       sc, 0, 2 if two else 1, 4, bodies)


@pytest.mark.parametrize("case", list(CASES))
def test_blocked_bitwise_equals_soa(sim, gc, case):
    build, steps = CASES[case]
    wl = build()
    _say(f"[layout] {case}: {steps} steps")
    a, b = _run_pair(sim, gc, wl, steps)
    _assert_same(a, b)


@pytest.mark.parametrize("rows", [1, 2, 8, 64, 512])
def test_blocked_rows_per_block(sim, gc, rows):
    """Explicit rows per block, from one row to more rows than the lattice
    has (one partly used block): bit-identical to SoA on the FP16 channel
    (paired odd steps) and the FP32 box with two bodies."""
    for wl in (_small(19, "f16", ("inlet", "outlet", "wall", "wall", "wall", "wall"), nx=128),
               _small(27, "f32", ("wall",) * 6, two=True, sc=2)):
        a, b = _run_pair(sim, gc, wl, 4, rows=rows)
        _assert_same(a, b)


def test_blocked_general_path_and_obstacle(sim, gc):
    """The general per-cell path (option) and a plain-LBM field with a static
    obstacle: blocked equal to SoA bit for bit."""
    import torch

    wl = _small(19, "f32", ("inlet", "outlet", "wall", "wall", "wall", "wall"))
    a, b = _run_pair(sim, gc, wl, 4, setup=lambda f: f.set_option(1, 1))
    _assert_same(a, b)
    wp = dataclasses.replace(wl, bodies=[], bc=("periodic",) * 6, u_in=(0.0, 0.0, 0.0))
    solid = torch.zeros(wp.n_cells, dtype=torch.uint8, device="cuda")
    sv = solid.view(wp.nz, wp.ny, wp.nx)
    sv[3:9, 6:15, 20:40] = 1
    out = []
    for w in (wp, _blocked(wp)):
        f = sim.Field(w, psm=False)
        gc.load_random_state(f, 6)
        f.set_obstacle(solid)
        for t in range(4):
            f.step(t)
        torch.cuda.synchronize()
        out.append((f.pdf_std().clone(), f.mass(4).item()))
    assert torch.equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_blocked_two_steps_parity_vs_oracle(orc, sim, gc):
    """Blocked fields against the FP64 oracle, element by element (the SoA
    tests' tolerances): D3Q19/27, FP32/FP16, channel faces."""
    import test_gpu_parity as tp

    for q in (19, 27):
        for storage in ("f32", "f16"):
            wl = _blocked(tp._workload(q, storage, "channel", two=True))
            _say(f"[layout vs oracle] q={q} {storage}")
            tp._two_step_compare(orc, sim, gc, wl)


def test_blocked_adjoint_equals_soa(sim):
    """The adjoint sweep on a blocked field (forward states gathered to the
    standard layout) gives the SoA field's J and gradients bit for bit."""
    import torch

    from paper_2502_20049_amd import adjoint

    wl = pi.workload_adjoint_rotor(n=32, steps=24, radius=10.0, s=2, n_chord=8, n_span=8)
    w = np.zeros(24)
    w[-8:] = 1.0 / 8
    res = []
    for ww in (wl, _blocked(wl)):
        obj = adjoint.TorqueAdjoint(ww, 24, w, segment=6)
        J = obj.forward()
        gB, gW, gF = obj.backward()
        torch.cuda.synchronize()
        res.append((J, gB.clone(), gW, gF.clone()))
    assert res[0][0] == res[1][0] and res[0][2] == res[1][2]
    assert torch.equal(res[0][1], res[1][1]) and torch.equal(res[0][3], res[1][3])


def test_blocked_channel_256_full_size_equals_soa(sim, gc):
    """The benchmark lattice (256^3 channel, rotating ellipsoid, s = 3) in both
    layouts, four steps from a seeded state, FP32 and FP16: bit-identical."""
    import torch

    for storage in ("f32", "f16"):
        wl = pi.workload_ellipsoid_channel(256, storage, steps=4, s=3)
        _say(f"[layout] 256^3 channel {storage}")
        a, b = _run_pair(sim, gc, wl, 4, seed=7)
        _assert_same(a, b)
        del a, b
        torch.cuda.empty_cache()


@pytest.mark.parametrize("case", ["channel_q19_f32", "channel_q19_f16_h2", "zpipe_q27_f32", "periodic_q19_f32_two_sc2",
                                  "cumulant_q27_f16"])
def test_second_stream_bitwise_equals_one_stream(sim, gc, case):
    """The solid-cell, F/T and face-row launches on the field's second stream
    (the default) against every launch on the caller's stream: the same PDFs,
    F/T, B and mass bit for bit, over whole psm_step calls."""
    from paper_2502_20049_amd import _capi as capi

    build, steps = CASES[case]
    wl = _blocked(build())
    _say(f"[second stream] {case}: {steps} steps")
    a, b = _run_pair_option(sim, gc, wl, steps, capi.PSM_OPT_CONCURRENT)
    _assert_same(a, b)


def _run_pair_option(sim, gc, wl, steps, opt, seed=5):
    """The same steps with option `opt` at 1 and at 0, from one seeded state."""
    import torch

    out = []
    for v in (1, 0):
        f = sim.Field(wl)
        f.set_option(opt, v)
        gc.load_random_state(f, seed)
        fts = []
        ftb = torch.zeros((max(1, f.nb), 6), dtype=torch.float64, device="cuda")
        for t in range(steps):
            # the step's own F/T sum (psm_step), and body_force_torque after it
            f.step(t, ft=ftb if f.nb else None)
            if f.nb:
                fts.append(ftb[: f.nb].clone())
                fts.append(f.force_torque().clone())
        torch.cuda.synchronize()
        r = {"pdf": f.pdf_std().clone(), "ft": torch.stack(fts) if fts else None, "mass": f.mass(steps).item()}
        if f.nb:
            B, meta = f.b_view()
            r["B"], r["meta"] = B.clone(), meta.clone()
        r["flags"] = f.error_flags().cpu().numpy()[0]
        out.append(r)
        del f
    return out


def _run_steps_ahead(sim, gc, wl, steps, ahead, seed=9, plain_steps=()):
    """Steps 0..steps-1 through Field.step on a field with or without
    map_ahead (psm_step_ahead / psm_step), from one seeded state; the steps in
    `plain_steps` go through psm_step (explicit poses) on either field."""
    import torch

    f = sim.Field(wl, map_ahead=ahead)
    gc.load_random_state(f, seed)
    fts = []
    ftb = torch.zeros((max(1, f.nb), 6), dtype=torch.float64, device="cuda")
    for t in range(steps):
        if t in plain_steps:
            f.step(t, poses=f.poses(t), ft=ftb)
        else:
            f.step(t, ft=ftb)
        fts.append(ftb[: f.nb].clone())
    torch.cuda.synchronize()
    B, meta = f.b_view()
    r = {"pdf": f.pdf_std().clone(), "ft": torch.stack(fts), "mass": f.mass(steps).item(), "B": B.clone(),
         "meta": meta.clone(), "flags": f.error_flags().cpu().numpy()[0]}
    del f
    return r


@pytest.mark.parametrize("case", ["channel_q19_f32", "channel_q19_f16_h2", "zpipe_q27_f32", "periodic_q19_f32_two_sc2",
                                  "periodic_q27_f32_two_sc3", "cumulant_q27_f16", "wide_300_q19_f16"])
def test_map_ahead_bitwise_equals_psm_step(sim, gc, case):
    """psm_step_ahead (the next step mapped into the second set of fractions
    on the mapping stream during this step) against psm_step on a one-set
    field: PDFs, the step's F/T, the last step's B and body ids, mass and
    error flags bit for bit, including a psm_step in the middle of the run
    (the next psm_step_ahead maps its own step first)."""
    build, steps = CASES[case]
    wl = _blocked(build())
    steps = max(steps, 6)
    _say(f"[map ahead] {case}: {steps} steps")
    ref = _run_steps_ahead(sim, gc, wl, steps, False)
    a = _run_steps_ahead(sim, gc, wl, steps, True)
    _assert_same(ref, a)
    b = _run_steps_ahead(sim, gc, wl, steps, True, plain_steps=(3,))
    _assert_same(ref, b)


def test_map_ahead_refused_without_second_set(sim):
    """psm_step_ahead on a field with one set of fractions: PSM_EUNSUP."""
    from paper_2502_20049_amd import _capi as capi

    wl = _small(19, "f32", ("periodic",) * 6)
    f = sim.Field(wl, map_ahead=False)
    p0, p1 = f.poses(0), f.poses(1)
    r = capi.lib.psm_step_ahead(f.handle, p0, p0, p1, f._geom_ptrs, f.nb, 0, None, None)
    assert r == capi.PSM_EUNSUP and "map_ahead" in capi.last_error()
    g = sim.Field(wl, map_ahead=True)
    assert capi.lib.psm_step_ahead(g.handle, p0, p0, None, g._geom_ptrs, g.nb, 0, None, None) == capi.PSM_EINVAL
    assert g.bbuf.numel() >= 2 * (wl.n_cells * 5)


def test_map_ahead_reset_clears_both_sets(sim, gc):
    """After an even number of psm_step_ahead calls the second set of
    fractions is the current one; psm_field_reset clears the whole fractions
    buffer (both sets) and makes the first set current again; the next run
    equals a fresh field's bit for bit."""
    import torch

    wl = _blocked(_small(19, "f32", ("periodic",) * 6, two=True, sc=2))
    f = sim.Field(wl, map_ahead=True)
    for t in range(2):
        f.step(t)
    f.reset()
    torch.cuda.synchronize()
    assert int(f.bbuf.count_nonzero().item()) == 0
    B, _ = f.b_view()
    assert B.data_ptr() == f.bbuf.data_ptr()
    gc.load_random_state(f, 4)
    for t in range(3):
        f.step(t)
    torch.cuda.synchronize()
    g = sim.Field(wl, map_ahead=True)
    gc.load_random_state(g, 4)
    for t in range(3):
        g.step(t)
    torch.cuda.synchronize()
    assert torch.equal(f.pdf_std(), g.pdf_std())
    assert torch.equal(f.b_view()[0], g.b_view()[0])
