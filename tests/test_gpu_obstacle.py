"""GPU parity of the static no-slip obstacle (plain LBM, ``lbm_set_obstacle``)
against the FP64 oracle's ``step_obstacle``, through the C ABI.

Tolerances as for the other parity tests (error of f after an even number of
steps, lattice units): FP64 1e-13 per two steps, FP32 2e-6, FP16 storage
6e-5.  Obstacle cells must keep their values bit for bit.
"""
import sys

import numpy as np
import pytest

import psm_inputs as pi

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 2e-6, "f16": 6e-5}

BCS = {
    "periodic": ("periodic",) * 6,
    "channel": ("inlet", "outlet", "wall", "wall", "wall", "wall"),
    "mixed": ("inlet", "outlet", "periodic", "periodic", "wall", "wall"),
}


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


def _wl(q, storage, bc, nx=70, ny=22, nz=13, force=(1e-4, -5e-5, 2e-5)):
    return pi.Workload(f"obst_{q}_{storage}_{bc}", nx, ny, nz, q, storage, 0.8, 3 / 16, force, BCS[bc],
                       (0.04, 0.01, -0.02), 1, 0, 1, 4, [])


def _near_count(wl, solid, c):
    """Fluid cells with a link into an obstacle cell (numpy, periodic wrap;
    sources beyond a non-periodic face do not count)."""
    s = solid.reshape(wl.nz, wl.ny, wl.nx).astype(bool)
    per = [wl.bc[0] == "periodic", wl.bc[2] == "periodic", wl.bc[4] == "periodic"]
    near = np.zeros_like(s)
    z, y, x = np.meshgrid(np.arange(wl.nz), np.arange(wl.ny), np.arange(wl.nx), indexing="ij")
    for k in range(1, len(c)):
        sx, sy, sz = x - c[k][0], y - c[k][1], z - c[k][2]
        ok = np.ones_like(s)
        for v, n, p in ((sx, wl.nx, per[0]), (sy, wl.ny, per[1]), (sz, wl.nz, per[2])):
            if not p:
                ok &= (v >= 0) & (v < n)
        near |= ok & s[sz % wl.nz, sy % wl.ny, sx % wl.nx]
    return int((near & ~s).sum())


def _run_pair(orc, sim, gc, wl, solid_np, steps, seed=11):
    import torch

    f = sim.Field(wl, psm=False)
    gc.load_random_state(f, seed)
    solid = torch.from_numpy(solid_np).to(f.pdf.device)
    n_near = f.set_obstacle(solid)
    cfg = orc.make_config(wl, psm=0)
    fo = gc.oracle_state(orc, wl, seed)
    for t in range(steps):
        f.step(t)
        orc.step_obstacle(cfg, fo, solid_np)
    torch.cuda.synchronize()
    return f, fo, n_near


@pytest.mark.parametrize("bc", list(BCS))
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("q", [19, 27])
def test_obstacle_matches_oracle(orc, sim, gc, q, storage, bc):
    """Random obstacle cells (15%), four steps (both parities twice) on a
    70x22x13 lattice (several tiles, ragged rows); f of every cell in the
    standard layout against the oracle; the near-cell list length against a
    numpy count."""
    wl = _wl(q, storage, bc)
    _say(f"[obstacle] q={q} {storage} {bc}")
    solid = pi.random_obstacle(21 + q, wl.n_cells, 0.15)
    f, fo, n_near = _run_pair(orc, sim, gc, wl, solid, 4)
    c, _, _ = sim.lattice(q)
    assert n_near == _near_count(wl, solid, c)
    got = gc.gpu_state_oracle_order(f, orc, sim)
    err = np.abs(got - fo).max()
    _say(f"  near cells {n_near}, max |f - f_oracle| = {err:.2e}")
    assert err < 2 * TOL[storage]


@pytest.mark.parametrize("nx", [128, 40])
def test_obstacle_f16_matches_oracle(orc, sim, gc, nx):
    """FP16 storage: nx = 128 takes the paired odd-step kernel, nx = 40 the
    per-cell one."""
    wl = _wl(19, "f16", "mixed", nx=nx, ny=9, nz=7)
    _say(f"[obstacle f16] nx={nx}")
    solid = pi.random_obstacle(33, wl.n_cells, 0.1)
    f, fo, _ = _run_pair(orc, sim, gc, wl, solid, 2)
    got = gc.gpu_state_oracle_order(f, orc, sim)
    bound = 4 * 2.0**-11 * np.abs(fo - orc.lattice(19)[1][:, None]).max() + 2e-6
    err = np.abs(got - fo).max()
    _say(f"  max err {err:.2e} (bound {bound:.2e})")
    assert err < bound


def test_obstacle_cells_untouched_and_general_path_bitwise(sim, gc):
    """Obstacle cells keep their values bit for bit; the general per-cell path
    (PSM_OPT_GENERAL_PATH) gives the same bits as the fast row kernels."""
    import torch

    wl = _wl(19, "f32", "channel", nx=96, ny=20, nz=17)
    solid_np = pi.random_obstacle(5, wl.n_cells, 0.2)
    solid = torch.from_numpy(solid_np).cuda()
    outs = []
    for general in (False, True):
        f = sim.Field(wl, psm=False)
        f.set_option(1, 1 if general else 0)
        gc.load_random_state(f, 3)
        f0 = f.pdf_view().clone()
        f.set_obstacle(solid)
        for t in range(6):
            f.step(t)
        torch.cuda.synchronize()
        st = f.pdf_view().clone()
        m = solid.bool()
        assert torch.equal(st[:, m], f0[:, m])
        outs.append(st)
    assert torch.equal(outs[0], outs[1])


def test_obstacle_slab_equals_wall_faces_bitwise(sim, gc):
    """Obstacle planes y = 0 and y = ny-1 of a y-periodic lattice give the
    same bits in the fluid as wall faces on the lattice without them."""
    import torch

    nx, ny, nz = 64, 12, 10
    wa = pi.Workload("slab", nx, ny, nz, 19, "f32", 0.8, 3 / 16, (1e-4, 0, 2e-5), ("periodic",) * 6,
                     (0, 0, 0), 1, 0, 1, 4, [])
    wb = pi.Workload("walls", nx, ny - 2, nz, 19, "f32", 0.8, 3 / 16, (1e-4, 0, 2e-5),
                     ("periodic", "periodic", "wall", "wall", "periodic", "periodic"), (0, 0, 0), 1, 0, 1, 4, [])
    fa = sim.Field(wa, psm=False)
    fb = sim.Field(wb, psm=False)
    gc.load_random_state(fa, 9)
    q = 19
    fb.pdf_view().copy_(fa.pdf_view().view(q, nz, ny, nx)[:, :, 1:ny - 1, :].reshape(q, -1))
    solid = torch.zeros((nz, ny, nx), dtype=torch.uint8, device="cuda")
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    n_near = fa.set_obstacle(solid.view(-1))
    assert n_near == 2 * nx * nz
    for t in range(6):
        fa.step(t)
        fb.step(t)
    torch.cuda.synchronize()
    got = fa.pdf_view().view(q, nz, ny, nx)[:, :, 1:ny - 1, :].reshape(q, -1)
    assert torch.equal(got, fb.pdf_view())


def test_obstacle_errors_and_removal(sim, gc):
    """A PSM field refuses an obstacle; a too small buffer is reported and
    leaves no obstacle; removing the obstacle restores plain LBM bit for bit."""
    import ctypes as C

    import torch
    from paper_2502_20049_amd import _capi as capi

    wl = _wl(19, "f32", "periodic", nx=32, ny=8, nz=8)
    solid = torch.from_numpy(pi.random_obstacle(2, wl.n_cells, 0.3)).cuda()
    body = pi.Body(pi.Shape("ellipsoid", (3.0, 2.0, 2.0)), pi.Motion(x0=(16.0, 4.0, 4.0)), s=1)
    wp = pi.Workload("p", 32, 8, 8, 19, "f32", 0.8, 3 / 16, (0, 0, 0), ("periodic",) * 6, (0, 0, 0), 1, 0, 1, 2,
                     [body])
    fp = sim.Field(wp)
    buf = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    rc = capi.lib.lbm_set_obstacle(fp.handle, C.c_void_p(solid.data_ptr()), C.c_void_p(buf.data_ptr()),
                                   buf.numel(), None, None)
    assert rc == capi.PSM_EUNSUP
    f = sim.Field(wl, psm=False)
    small = 256 + wl.n_cells + 8 * 10  # room for 10 list entries
    n = C.c_int64()
    rc = capi.lib.lbm_set_obstacle(f.handle, C.c_void_p(solid.data_ptr()), C.c_void_p(buf.data_ptr()), small,
                                   C.byref(n), None)
    assert rc == capi.PSM_ESIZE and n.value > 10
    g = sim.Field(wl, psm=False)
    for fld in (f, g):
        gc.load_random_state(fld, 4)
    f.set_obstacle(solid)
    f.set_obstacle(None)
    for t in range(2):
        f.step(t)
        g.step(t)
    torch.cuda.synchronize()
    assert torch.equal(f.pdf_view(), g.pdf_view())


def test_obstacle_mass_conserved(sim, gc):
    """Periodic lattice with a body force and a random obstacle: FP64 mass of
    all slots conserved over 10 steps."""
    import torch

    wl = _wl(27, "f64", "periodic", nx=48, ny=20, nz=18)
    f = sim.Field(wl, psm=False)
    gc.load_random_state(f, 8)
    f.set_obstacle(torch.from_numpy(pi.random_obstacle(6, wl.n_cells, 0.25)).cuda())
    m0 = float(f.mass(0).item())
    for t in range(10):
        f.step(t)
    m1 = float(f.mass(10).item())
    assert abs(m1 - m0) / m0 < 1e-13


@pytest.mark.parametrize("q", [19, 27])
def test_obstacle_macroscopic_odd_parity(orc, sim, gc, q):
    """rho and u read back after an odd number of steps (the in-place layout
    is then permuted; links into obstacle cells hold bounce-back values in the
    cell's own slot) against the oracle's, every cell."""
    import torch

    wl = _wl(q, "f64", "channel", nx=30, ny=14, nz=11)
    solid = pi.random_obstacle(40 + q, wl.n_cells, 0.2)
    f, fo, _ = _run_pair(orc, sim, gc, wl, solid, 3)
    rho, u = f.macroscopic(3)
    torch.cuda.synchronize()
    ro, uo = orc.macro(orc.make_config(wl, psm=0), fo)
    er = np.abs(rho.cpu().numpy() - ro).max()
    eu = np.abs(u.cpu().numpy() - uo).max()
    _say(f"[obstacle macro] q={q} rho {er:.1e} u {eu:.1e}")
    assert er < 1e-12 and eu < 1e-12


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_obstacle_cumulant_matches_oracle(orc, sim, gc, storage):
    """The no-slip obstacle with the cumulant collision (D3Q27, no force)."""
    wl = _wl(27, storage, "channel", force=(0.0, 0.0, 0.0))
    wl.collision = "cumulant"
    _say(f"[obstacle cumulant] {storage}")
    solid = pi.random_obstacle(61, wl.n_cells, 0.15)
    f, fo, _ = _run_pair(orc, sim, gc, wl, solid, 4)
    got = gc.gpu_state_oracle_order(f, orc, sim)
    err = np.abs(got - fo).max()
    _say(f"  max |f - f_oracle| = {err:.2e}")
    assert err < 2 * TOL[storage]
