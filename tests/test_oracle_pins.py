"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
moments, textbook special cases, exact invariants, analytic steady states and
brute force.  CPU only.
"""
import itertools
import math

import numpy as np
import pytest

import psm_inputs as pi


def _cfg(orc, q=19, **kw):
    d = dict(nx=4, ny=4, nz=4, q=q, tau=0.8, magic=3 / 16, force=(0, 0, 0), bc=("periodic",) * 6,
             u_in=(0, 0, 0), sc=1, psm=1)
    d.update(kw)
    return orc.make_config(**d)


def _pose_fixed(orc, R, X, V=(0, 0, 0), W=(0, 0, 0)):
    import ctypes as C

    p = orc.Pose()
    p.R = (C.c_double * 9)(*np.asarray(R, dtype=np.float64).ravel())
    p.X = (C.c_double * 3)(*X)
    p.V = (C.c_double * 3)(*V)
    p.W = (C.c_double * 3)(*W)
    return p


def _rand_f(q, w, seed, amp=1.0):
    dev = pi.pdf_deviation(seed, q, 1, np.arange(q), 0) * amp * 10
    return w + dev


# --- lattice and equilibrium (eq. 3) ----------------------------------------
@pytest.mark.parametrize("q", [19, 27])
def test_lattice_isotropy(orc, q):
    c, w, opp = orc.lattice(q)
    assert abs(w.sum() - 1) < 1e-15
    assert np.all(c[opp] == -c)
    m2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(m2, np.eye(3) / 3, atol=1e-15)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(m4, iso, atol=1e-15)


@pytest.mark.parametrize("q", [19, 27])
def test_equilibrium_moments(orc, q):
    """sum feq = rho, sum c feq = rho u, sum cc feq = rho cs2 I + rho u u (fails with the printed '+')."""
    c, w, _ = orc.lattice(q)
    for rho, u in [(1.0, (0.05, -0.02, 0.03)), (0.97, (0.1, 0.07, -0.12)), (1.2, (0, 0, 0))]:
        u = np.array(u)
        f = orc.feq(q, rho, u)
        assert abs(f.sum() - rho) < 1e-15
        assert np.allclose(c.T @ f, rho * u, atol=1e-15)
        P = np.einsum("i,ia,ib->ab", f, c, c)
        assert np.allclose(P, rho / 3 * np.eye(3) + rho * np.outer(u, u), atol=2e-15)


# --- TRT / SRT collision -----------------------------------------------------
@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("force", [(0, 0, 0), (1e-3, -2e-3, 5e-4)])
def test_trt_conservation(orc, q, force):
    """B = 0: per-cell mass conserved, momentum gains exactly F."""
    cfg = _cfg(orc, q, force=force)
    c, w, _ = orc.lattice(q)
    for seed in range(5):
        f = _rand_f(q, w, seed)
        fo, _ = orc.collide_cell(cfg, f)
        assert abs(fo.sum() - f.sum()) < 1e-15
        assert np.allclose(c.T @ fo - c.T @ f, force, atol=1e-15)


@pytest.mark.parametrize("q", [19, 27])
def test_trt_reduces_to_srt_guo(orc, q):
    """Lambda = (tau - 1/2)^2 makes both rates 1/tau: the textbook SRT with Guo
    forcing, f* = f - (f - feq)/tau + (1 - 1/(2 tau)) w_i[3(c-u) + 9(c.u)c].F."""
    tau = 0.73
    F = np.array([2e-3, -1e-3, 3e-3])
    cfg = _cfg(orc, q, tau=tau, magic=(tau - 0.5) ** 2, force=tuple(F))
    c, w, _ = orc.lattice(q)
    for seed in range(4):
        f = _rand_f(q, w, 10 + seed)
        rho = f.sum()
        u = (c.T @ f + F / 2) / rho
        cu = c @ u
        feq = w * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u)
        S = w * (3 * (c @ F - u @ F) + 9 * cu * (c @ F))
        ref = f - (f - feq) / tau + (1 - 0.5 / tau) * S
        fo, _ = orc.collide_cell(cfg, f)
        assert np.allclose(fo, ref, atol=1e-15, rtol=0)


# --- PSM rule and solid collision (eqs. 4, 7-9) ------------------------------
@pytest.mark.parametrize("q", [19, 27])
def test_psm_b0_is_plain_lbm(orc, q):
    c, w, _ = orc.lattice(q)
    f = _rand_f(q, w, 3)
    a, _ = orc.collide_cell(_cfg(orc, q, psm=1), f, B=[0.0], us=[(0.01, 0.02, 0.0)])
    b, _ = orc.collide_cell(_cfg(orc, q, psm=0), f)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("sc,factor", [(1, 1.0), (2, None), (3, 2.0)])
def test_solid_collision_moments(orc, q, sc, factor):
    """sum Omega^S = 0; sum c Omega^S = rho (u_s - u) * {1, 1/tau, 2} for SC1/2/3 (F = 0)."""
    tau = 0.8
    cfg = _cfg(orc, q, sc=sc, tau=tau)
    c, w, _ = orc.lattice(q)
    fac = 1 / tau if factor is None else factor
    for seed in range(4):
        f = _rand_f(q, w, 20 + seed)
        rho = f.sum()
        u = c.T @ f / rho
        us = np.array([0.03, -0.01, 0.02]) * (seed + 1)
        f0, _ = orc.collide_cell(cfg, f, B=[0.0], us=[us])
        f1, dF = orc.collide_cell(cfg, f, B=[1.0], us=[us])
        fl, _ = orc.collide_cell(_cfg(orc, q, sc=sc, psm=0), f)
        om_s = f1 - f  # B = 1: f* = f + Omega^S
        assert abs(om_s.sum()) < 1e-15
        assert np.allclose(c.T @ om_s, rho * (us - u) * fac, atol=1e-15)
        # force on the body is minus the momentum given to the fluid (eq. 10, body side)
        assert np.allclose(dF[0], -rho * (us - u) * fac, atol=1e-15)
        # linear blend in B (eq. 4)
        fh, dFh = orc.collide_cell(cfg, f, B=[0.375], us=[us])
        assert np.allclose(fh, f + 0.625 * (fl - f) + 0.375 * om_s, atol=1e-15)


def test_sc1_b1_gives_solid_velocity(orc):
    """B = 1 with SC1: the post-collision momentum is exactly rho u_s (F = 0)."""
    cfg = _cfg(orc, 19)
    c, w, _ = orc.lattice(19)
    f = _rand_f(19, w, 7)
    us = np.array([0.04, -0.03, 0.01])
    fo, _ = orc.collide_cell(cfg, f, B=[1.0], us=[us])
    assert np.allclose(c.T @ fo, f.sum() * us, atol=1e-15)


def test_sc2_relaxes_nonequilibrium(orc):
    """B = 1 with SC2: f* - feq(u_s) = (1 - 1/tau)(f - feq(u_s)) (geometric relaxation)."""
    tau = 0.9
    cfg = _cfg(orc, 19, sc=2, tau=tau)
    c, w, _ = orc.lattice(19)
    f = _rand_f(19, w, 8)
    us = np.array([0.02, 0.0, -0.01])
    fe = orc.feq(19, f.sum(), us)
    fo, _ = orc.collide_cell(cfg, f, B=[1.0], us=[us])
    assert np.allclose(fo - fe, (1 - 1 / tau) * (f - fe), atol=1e-15)


@pytest.mark.parametrize("sc", [1, 2, 3])
def test_galilean_fixed_point(orc, sc):
    """A uniform equilibrium at u with u_s = u is unchanged for any B."""
    cfg = _cfg(orc, 19, sc=sc)
    u = np.array([0.03, -0.02, 0.01])
    f = orc.feq(19, 1.02, u)
    for B in (0.0, 0.3, 1.0):
        fo, dF = orc.collide_cell(cfg, f, B=[B], us=[u])
        assert np.allclose(fo, f, atol=1e-16)
        assert np.allclose(dF, 0, atol=1e-16)


def test_two_body_blend_normalised(orc):
    """Two slots with sum B > 1 are scaled to sum 1: no fluid collision remains."""
    cfg = _cfg(orc, 19)
    c, w, _ = orc.lattice(19)
    f = _rand_f(19, w, 9)
    u1, u2 = np.array([0.01, 0, 0]), np.array([0, 0.02, 0])
    fo, dF = orc.collide_cell(cfg, f, B=[0.75, 0.75], us=[u1, u2])
    a, _ = orc.collide_cell(cfg, f, B=[1.0], us=[u1])
    b, _ = orc.collide_cell(cfg, f, B=[1.0], us=[u2])
    assert np.allclose(fo, f + 0.5 * (a - f) + 0.5 * (b - f), atol=1e-15)


# --- full steps: invariants --------------------------------------------------
def _random_state(orc, q, N, seed):
    c, w, _ = orc.lattice(q)
    return w[:, None] + pi.pdf_deviation_full(seed, q, N) * 20


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("sc", [1, 2, 3])
def test_periodic_mass_and_momentum_balance(orc, q, sc):
    """Periodic box, random B and solid velocities: mass conserved to 1e-13 and
    P(t+1) - P(t) = sum_x (1 - B) F - F_body exactly (sign of eq. 10 pinned)."""
    nx, ny, nz = 6, 5, 4
    N = nx * ny * nz
    F = np.array([1e-4, -2e-4, 5e-5])
    cfg = _cfg(orc, q, nx=nx, ny=ny, nz=nz, sc=sc, force=tuple(F))
    c, w, _ = orc.lattice(q)
    f = _random_state(orc, q, N, 40 + sc)
    B = pi.random_fractions(5 + sc, N)[None, :].copy()
    pose = _pose_fixed(orc, np.eye(3), (3.0, 2.5, 2.0), V=(0.01, 0.0, -0.005), W=(0.0, 0.0, 0.004))
    m0 = orc.mass(cfg, f)
    for _ in range(10):
        P0 = (f.sum(axis=1) @ c)
        ft = orc.step(cfg, f, B, [pose])
        P1 = (f.sum(axis=1) @ c)
        expect = (1 - B[0]).sum() * F - ft[0, :3]
        assert np.allclose(P1 - P0, expect, atol=1e-13)
    assert abs(orc.mass(cfg, f) - m0) / m0 < 1e-13


def _angular_momentum(c, f, dims, O):
    """L = sum_x sum_i (x_c - O) x c_i f_i(x) about the point O (cell centres at
    index + 1/2, cell n = x + nx (y + ny z))."""
    nx, ny, nz = dims
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.stack([xx.ravel() + 0.5, yy.ravel() + 0.5, zz.ravel() + 0.5], axis=1) - np.asarray(O)
    j = f.T @ c  # momentum per cell (N, 3)
    return np.cross(r, j).sum(axis=0)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("sc", [1, 2, 3])
def test_periodic_angular_momentum_balance_pins_torque(orc, q, sc):
    """Eq. (11): in a periodic box without body force, where the bodies and all
    non-equilibrium cells stay two cells away from the faces and rest
    equilibrium fills the rest, one step changes the fluid's angular momentum
    about any point O by exactly -sum_k (T_k + (X_k - O) x F_k).  Collision
    hands each body the momentum -dF at x_c; streaming keeps (x - O) x c f
    (c x c = 0), and the uniform rest populations crossing the periodic wrap
    are only permuted.  Two bodies with different centres pin the lever arm
    x_c - X_k and the sign of the cross product."""
    nx, ny, nz = 12, 11, 10
    N = nx * ny * nz
    cfg = _cfg(orc, q, nx=nx, ny=ny, nz=nz, sc=sc)
    c, w, _ = orc.lattice(q)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inner = ((xx >= 2) & (xx < nx - 2) & (yy >= 2) & (yy < ny - 2) & (zz >= 2) & (zz < nz - 2)).ravel()
    core = ((xx >= 3) & (xx < nx - 3) & (yy >= 3) & (yy < ny - 3) & (zz >= 3) & (zz < nz - 3)).ravel()
    f = np.repeat(w[:, None], N, axis=1)
    f[:, inner] = _random_state(orc, q, N, 90 + sc)[:, inner]
    B = np.stack([pi.random_fractions(11 + sc, N) * 0.5, pi.random_fractions(21 + sc, N, stream=5) * 0.5])
    B[:, ~core] = 0.0
    poses = [_pose_fixed(orc, np.eye(3), (5.3, 4.6, 5.2), V=(0.01, -0.004, 0.002), W=(0.003, -0.002, 0.005)),
             _pose_fixed(orc, np.eye(3), (6.9, 5.8, 3.7), V=(-0.006, 0.0, 0.008), W=(-0.004, 0.006, 0.001))]
    for O in [(0.0, 0.0, 0.0), (4.25, 7.5, 3.0)]:
        g = f.copy()
        L0 = _angular_momentum(c, g, (nx, ny, nz), O)
        ft = orc.step(cfg, g, B, poses)
        L1 = _angular_momentum(c, g, (nx, ny, nz), O)
        expect = -sum(ft[k, 3:] + np.cross(np.array(poses[k].X[:]) - O, ft[k, :3]) for k in range(2))
        assert np.abs(ft[:, 3:]).max() > 1e-3  # the torques are not trivially small
        assert np.allclose(L1 - L0, expect, rtol=0, atol=1e-12)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("u_in", [(0.05, 0.0, 0.0), (0.04, 0.012, -0.007)])
def test_uniform_inflow_is_fixed_point_pins_outlet(orc, q, u_in):
    """Uniform flow at the inlet velocity (rho = 1) through an inlet (-x) /
    outlet (+x) channel, periodic in y and z, is an exact fixed point: the
    inlet's moving-wall rule returns f^eq_k = f^eq_kbar + 2 w_k c_k.u/c_s^2 (the
    odd part of eq. 3), and the zero-gradient outlet returns the cell's own
    post-collision f_k.  Bounce-back at the outlet (f*_kbar) would break it."""
    nx, ny, nz = 7, 4, 3
    N = nx * ny * nz
    cfg = _cfg(orc, q, nx=nx, ny=ny, nz=nz, u_in=u_in,
               bc=("inlet", "outlet", "periodic", "periodic", "periodic", "periodic"))
    feq = orc.feq(q, 1.0, np.array(u_in))
    f = np.repeat(feq[:, None], N, axis=1).copy()
    for _ in range(5):
        orc.step(cfg, f, None, [])
    assert np.abs(f - feq[:, None]).max() < 1e-14


def test_closed_box_walls_conserve_mass(orc):
    nx, ny, nz = 5, 6, 7
    cfg = _cfg(orc, 19, nx=nx, ny=ny, nz=nz, bc=("wall",) * 6)
    f = _random_state(orc, 19, nx * ny * nz, 77)
    m0 = orc.mass(cfg, f)
    for _ in range(12):
        orc.step(cfg, f, None, [])
    assert abs(orc.mass(cfg, f) - m0) / m0 < 1e-13


def _steady(orc, cfg, f, tol=1e-14, max_steps=200000, chunk=500):
    prev = f.copy()
    for _ in range(max_steps // chunk):
        for _ in range(chunk):
            orc.step(cfg, f, None, [])
        if np.abs(f - prev).max() < tol:
            return f
        prev = f.copy()
    raise AssertionError("no steady state")


def test_poiseuille_exact(orc):
    """Body-force channel between halfway bounce-back walls, TRT Lambda = 3/16:
    u_x(y) = F/(2 nu) y (H - y) at cell centres y = j + 1/2 (analytic parabola)."""
    ny, tau, F = 10, 0.8, 1e-5
    cfg = _cfg(orc, 19, nx=1, ny=ny, nz=1, tau=tau, force=(F, 0, 0),
               bc=("periodic", "periodic", "wall", "wall", "periodic", "periodic"))
    c, w, _ = orc.lattice(19)
    f = np.repeat(w[:, None], ny, axis=1).copy()
    _steady(orc, cfg, f)
    rho, u = orc.macro(cfg, f)
    nu = (tau - 0.5) / 3
    y = np.arange(ny) + 0.5
    ua = F / (2 * nu) * y * (ny - y)
    assert np.abs(u[:, 0] - ua).max() / ua.max() < 1e-10
    assert np.abs(u[:, 1:]).max() < 1e-15


def test_couette_exact(orc):
    """Wall at -y, moving wall (inlet rule, Ladd bounce-back) at +y: linear profile."""
    ny, U = 8, 0.02
    cfg = _cfg(orc, 19, nx=1, ny=ny, nz=1, tau=0.9, u_in=(U, 0, 0),
               bc=("periodic", "periodic", "wall", "inlet", "periodic", "periodic"))
    c, w, _ = orc.lattice(19)
    f = np.repeat(w[:, None], ny, axis=1).copy()
    _steady(orc, cfg, f)
    rho, u = orc.macro(cfg, f)
    y = np.arange(ny) + 0.5
    assert np.abs(u[:, 0] - U * y / ny).max() / U < 1e-10


# --- kinematics --------------------------------------------------------------
def test_pose_rotation(orc):
    for ax in [(0, 0, 1), (1, 0, 0), (0.6, 0.0, 0.8), (2 / 3, -1 / 3, 2 / 3)]:
        m = pi.Motion(axis=ax, theta0=0.3, omega=1e-3, x0=(1.0, 2.0, 3.0), v=(0.1, 0, 0))
        R, X, V, W = orc.pose_arrays(orc.pose_at(m, 250))
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-15)
        assert abs(np.linalg.det(R) - 1) < 1e-15
        assert np.allclose(R @ np.array(ax), ax, atol=1e-15)
        assert np.allclose(X, (26.0, 2.0, 3.0)) and np.allclose(W, 1e-3 * np.array(ax))
    R, *_ = orc.pose_arrays(orc.pose_at(pi.Motion(axis=(0, 0, 1), omega=0.5), 1))
    c, s = math.cos(0.5), math.sin(0.5)
    assert np.allclose(R, [[c, -s, 0], [s, c, 0], [0, 0, 1]], atol=1e-16)
    R0, *_ = orc.pose_arrays(orc.pose_at(pi.Motion(axis=(0.6, 0.0, 0.8), omega=0.5), 0))
    assert np.array_equal(R0, np.eye(3))


# --- geometry mapping (section III) ------------------------------------------


def test_static_sphere_bruteforce(orc):
    """32^3, sphere r=6 at (16,16,16), s=2: B = #{odd (a,b,c) in the cell:
    a^2+b^2+c^2 < 2304}/64 (integer brute force); 48-fold symmetric."""
    wl = pi.workload_sphere32()
    cfg = orc.make_config(wl)
    g = orc.OracleGeometry(wl.bodies[0].shape, 2)
    B = orc.map_body(cfg, g, _pose_fixed(orc, np.eye(3), (16.0, 16.0, 16.0))).reshape(32, 32, 32)
    ref = np.zeros((32, 32, 32))
    for z, y, x in itertools.product(range(8, 24), repeat=3):
        cnt = 0
        for kz, ky, kx in itertools.product(range(4), repeat=3):
            a, b, c_ = 8 * (x - 16) + 2 * kx + 1, 8 * (y - 16) + 2 * ky + 1, 8 * (z - 16) + 2 * kz + 1
            cnt += a * a + b * b + c_ * c_ < 2304
        ref[z, y, x] = cnt / 64
    assert np.array_equal(B, ref)
    # symmetric under the cube group about the corner (16,16,16)
    assert np.array_equal(B, B[::-1, :, :]) and np.array_equal(B, B.transpose(1, 0, 2))
    assert np.array_equal(B, B.transpose(2, 1, 0)) and np.array_equal(B, B[:, ::-1, ::-1])
    assert abs(B.sum() - 4 / 3 * math.pi * 216) / (4 / 3 * math.pi * 216) < 5e-3


def test_mapping_theta0_is_nested_average(orc):
    """theta = 0, integer centre: every sub-sample hits a lattice centre; eps =
    average of the analytic inside test at the (2^s)^3 sub-cell centres."""
    a, b, c = 5.0, 3.0, 2.0
    g = orc.OracleGeometry(pi.Shape("ellipsoid", (a, b, c)), 2)
    X = (8.0, 7.0, 6.0)
    p = _pose_fixed(orc, np.eye(3), X)
    for (x, y, z) in [(8, 7, 6), (12, 7, 6), (8, 9, 7), (3, 7, 6), (10, 8, 7)]:
        pts = [((x + (kx + 0.5) / 4) - X[0], (y + (ky + 0.5) / 4) - X[1], (z + (kz + 0.5) / 4) - X[2])
               for kx, ky, kz in itertools.product(range(4), repeat=3)]
        ref = np.mean([(px / a) ** 2 + (py / b) ** 2 + (pz / c) ** 2 < 1 for px, py, pz in pts])
        assert orc.map_cell(g, p, x, y, z) == ref


def test_mapping_quarter_turn_is_permutation(orc):
    """A rotation by pi/2 about z through an integer point permutes the field."""
    cfg = orc.make_config(nx=24, ny=24, nz=12, q=19, tau=0.8)
    g = orc.OracleGeometry(pi.Shape("ellipsoid", (8.0, 4.0, 3.0)), 2)
    X = (12.0, 12.0, 6.0)
    B0 = orc.map_body(cfg, g, _pose_fixed(orc, np.eye(3), X)).reshape(12, 24, 24)
    Rq = orc.pose_arrays(orc.pose_at(pi.Motion(axis=(0, 0, 1), omega=math.pi / 2), 1))[0]
    B1 = orc.map_body(cfg, g, _pose_fixed(orc, Rq, X)).reshape(12, 24, 24)
    # lab cell (x, y) of the rotated body sees body point R^T(x - X): (x,y) -> (y', -x')
    assert B0.sum() > 100
    assert np.array_equal(B1, np.rot90(B0, k=1, axes=(2, 1)))


@pytest.mark.parametrize("s_depth,trials,cells", [(1, 6, 5), (2, 4, 4), (3, 2, 2)])
def test_mapping_fixed_point_matches_exact_arithmetic(orc, s_depth, trials, cells):
    """Fixed-point lookup equals exact rational arithmetic on the same FP64
    rotation, except for samples within 2^-28 sub-cells of a lattice plane;
    s = 1, 2 and 3 (the depths the mapping runs at)."""
    from fractions import Fraction as Fr

    n = 2 ** s_depth
    g = orc.OracleGeometry(pi.Shape("ellipsoid", (3.0, 2.0, 1.5)), s_depth)
    rng = np.random.default_rng(5 + s_depth)
    all_cells = [(5, 5, 5), (6, 4, 5), (3, 5, 6), (7, 6, 4), (4, 4, 4)]
    mism = checked = 0
    for trial in range(trials):
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        m = pi.Motion(axis=tuple(ax), omega=float(rng.uniform(0, 6)), x0=(5.0, 5.0, 5.0))
        pose = orc.pose_at(m, 1)
        R = np.array(pose.R[:]).reshape(3, 3)
        Rf = [[Fr(float(R[i, j])) for j in range(3)] for i in range(3)]
        for (x, y, z) in all_cells[:cells]:
            pts, near = [], False
            for kx, ky, kz in itertools.product(range(n), repeat=3):
                q = [Fr(x) + Fr(2 * kx + 1, 2 * n) - 5, Fr(y) + Fr(2 * ky + 1, 2 * n) - 5,
                     Fr(z) + Fr(2 * kz + 1, 2 * n) - 5]
                p = [sum(Rf[j][a] * q[j] for j in range(3)) * n for a in range(3)]  # sub-cell units
                pts.append([math.floor(v) for v in p])
                if any(abs(v - round(v)) < Fr(1, 2 ** 28) for v in p):
                    near = True
            cnt = int(g.inside(pts).sum())
            checked += 0 < cnt < n ** 3
            if Fr(cnt, n ** 3) != Fr(orc.map_cell(g, pose, x, y, z)):
                assert near
                mism += 1
    assert mism == 0
    assert checked >= 1  # at least one cell cuts the surface


def _ellipsoid_inside_exact(m, h, abc):
    """Exact test of lattice centre (m + 1/2) h against the ellipsoid with
    semi-axes abc (rational arithmetic)."""
    from fractions import Fraction as Fr

    return sum((Fr(2 * int(mi) + 1) * h / 2 / Fr(a)) ** 2 for mi, a in zip(m, abc)) < 1


@pytest.mark.parametrize("s_depth", [1, 2, 3])
def test_mapping_block_reading_matches_exact_arithmetic(orc, s_depth):
    """The block reading (centre rotated, axis-aligned block averaged): eps
    equals the count over the (2^s)^3 lattice cells from j0 = floor(q - 2^(s-1)
    + 1/2), q the body-frame centre in sub-cell units, computed here in
    rational arithmetic from the same FP64 rotation with the analytic inside
    test, except for centres within 2^-28 sub-cells of a rounding tie."""
    from fractions import Fraction as Fr

    n = 2 ** s_depth
    abc = (3.0, 2.0, 1.5)
    g = orc.OracleGeometry(pi.Shape("ellipsoid", abc), s_depth)
    rng = np.random.default_rng(40 + s_depth)
    X = (5.25, 4.75, 5.0)
    mism = cut = 0
    for trial in range(4):
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        m = pi.Motion(axis=tuple(ax), omega=float(rng.uniform(0, 6)), x0=X)
        pose = orc.pose_at(m, 1)
        R = np.array(pose.R[:]).reshape(3, 3)
        Rf = [[Fr(float(R[i, j])) for j in range(3)] for i in range(3)]
        for (x, y, z) in [(5, 4, 5), (6, 5, 5), (3, 4, 6), (7, 6, 4), (4, 2, 5), (5, 5, 3)]:
            d = [Fr(2 * x + 1, 2) - Fr(X[0]), Fr(2 * y + 1, 2) - Fr(X[1]), Fr(2 * z + 1, 2) - Fr(X[2])]
            q = [sum(Rf[j][a] * d[j] for j in range(3)) * n for a in range(3)]
            t = [v - Fr(n, 2) + Fr(1, 2) for v in q]
            near = any(abs(v - round(v)) < Fr(1, 2 ** 28) for v in t)
            j0 = [math.floor(v) for v in t]
            cnt = sum(_ellipsoid_inside_exact((j0[0] + kx, j0[1] + ky, j0[2] + kz), Fr(1, n), abc)
                      for kx, ky, kz in itertools.product(range(n), repeat=3))
            cut += 0 < cnt < n ** 3
            if Fr(cnt, n ** 3) != Fr(orc.map_cell(g, pose, x, y, z, reading=1)):
                assert near
                mism += 1
    assert mism == 0
    assert cut >= 3  # cells that cut the surface were checked


@pytest.mark.parametrize("X", [(8.0, 7.0, 6.0), (8.3, 6.85, 6.6)])
def test_mapping_block_reading_agrees_at_theta0_and_s0(orc, X):
    """Both readings select the same geometry cells at theta = 0 (any centre,
    any s) and for s = 0 (any rotation): the dense fields are equal."""
    cfg = orc.make_config(nx=16, ny=14, nz=12, q=19, tau=0.8)
    shp = pi.Shape("ellipsoid", (5.0, 3.5, 2.5))
    for s_depth in (0, 1, 2, 3):
        g = orc.OracleGeometry(shp, s_depth)
        p0 = _pose_fixed(orc, np.eye(3), X)
        Ba, Bb = orc.map_body(cfg, g, p0, reading=1), orc.map_body(cfg, g, p0, reading=0)
        assert Bb.sum() > 50 and np.array_equal(Ba, Bb)
    g = orc.OracleGeometry(shp, 0)
    for t in (1, 3, 7):
        pr = orc.pose_at(pi.Motion(axis=(0.36, 0.48, 0.8), omega=0.37, x0=X), t)
        assert np.array_equal(orc.map_body(cfg, g, pr, reading=1), orc.map_body(cfg, g, pr, reading=0))


def test_mapping_block_reading_quarter_turn_is_permutation(orc):
    """A rotation by pi/2 about z through an integer point permutes the block
    reading's field too (the rotated lab cell is again an axis-aligned block)."""
    cfg = orc.make_config(nx=24, ny=24, nz=12, q=19, tau=0.8)
    g = orc.OracleGeometry(pi.Shape("ellipsoid", (8.0, 4.0, 3.0)), 2)
    X = (12.0, 12.0, 6.0)
    B0 = orc.map_body(cfg, g, _pose_fixed(orc, np.eye(3), X), reading=1).reshape(12, 24, 24)
    Rq = orc.pose_arrays(orc.pose_at(pi.Motion(axis=(0, 0, 1), omega=math.pi / 2), 1))[0]
    B1 = orc.map_body(cfg, g, _pose_fixed(orc, Rq, X), reading=1).reshape(12, 24, 24)
    assert B0.sum() > 100
    assert np.array_equal(B1, np.rot90(B0, k=1, axes=(2, 1)))


def _true_fractions(R, X, abc, cells, m=16):
    """Overlap of each lab cell with the rotated ellipsoid, by m^3 midpoint
    samples per cell (numpy, independent of the oracle's lookup)."""
    k = (np.arange(m) + 0.5) / m
    oz, oy, ox = np.meshgrid(k, k, k, indexing="ij")
    off = np.stack([ox.ravel(), oy.ravel(), oz.ravel()], axis=1)
    out = np.empty(len(cells))
    for i, c in enumerate(cells):
        pts = (c + off - np.asarray(X)) @ R  # rows: R^T (x - X)
        out[i] = np.mean(np.sum((pts / np.asarray(abc)) ** 2, axis=1) < 1)
    return out


@pytest.mark.parametrize("axis,angle", [((0, 0, 1), math.pi / 4), ((1, 1, 1), 0.7)])
def test_mapping_block_reading_error_under_rotation(orc, axis, angle):
    """Turned by 45 degrees (and about a body diagonal) the block reading
    samples a cube turned against the lab cell: at s = 2 and 3 its mean
    per-cell error against the true overlap is more than twice that of the
    rotated sub-samples (whose error is the sub-sampling error alone), while
    both volumes stay within the surface bound (eq. 12)."""
    abc = (6.0, 4.0, 3.0)
    X = (10.0, 10.0, 8.0)
    cfg = orc.make_config(nx=20, ny=20, nz=16, q=19, tau=0.8)
    ax = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
    pose = orc.pose_at(pi.Motion(axis=tuple(ax), omega=angle, x0=X), 1)
    R = np.array(pose.R[:]).reshape(3, 3)
    cells = np.array([(x, y, z) for z in range(16) for y in range(20) for x in range(20)])
    ref = _true_fractions(R, X, abc, cells)
    surf = (ref > 0) & (ref < 1)
    vol = 4 / 3 * math.pi * np.prod(abc)
    # Knud Thomsen's surface-area approximation (within ~1%)
    area = 4 * math.pi * ((abc[0] * abc[1]) ** 1.6 + (abc[0] * abc[2]) ** 1.6 + (abc[1] * abc[2]) ** 1.6) ** (1 / 1.6) \
        / 3 ** (1 / 1.6)
    for s_depth in (2, 3):
        g = orc.OracleGeometry(pi.Shape("ellipsoid", abc), s_depth)
        Bb = orc.map_body(cfg, g, pose, reading=0)
        Ba = orc.map_body(cfg, g, pose, reading=1)
        eb, ea = np.abs(Bb - ref)[surf], np.abs(Ba - ref)[surf]
        assert ea.mean() > 2.0 * eb.mean() and ea.max() > eb.max(), (s_depth, ea.max(), ea.mean(), eb.mean())
        assert eb.max() < 0.1
        for B in (Ba, Bb):
            assert abs(B.sum() - vol) < area * math.sqrt(3) * 2.0 ** -s_depth


def test_b_tau_weighted_form(orc):
    """Eq. (6) limits: eps 0 -> 0, eps 1 -> 1, monotone, below eps for tau < 1.5."""
    tau = 0.8
    assert orc.b_from_eps(0.0, tau, 1) == 0.0 and orc.b_from_eps(1.0, tau, 1) == 1.0
    e = np.linspace(0, 1, 65)
    b = np.array([orc.b_from_eps(x, tau, 1) for x in e])
    assert np.all(np.diff(b) > 0) and np.all(b[1:-1] < e[1:-1])
    assert orc.b_from_eps(0.25, tau, 0) == 0.25


# --- meshes -----------------------------------------------------------------
def test_mesh_volume_divergence(orc):
    m = pi.cube_mesh(1.5)
    assert abs(orc.mesh_volume(m.verts, m.tris) - 27.0) < 1e-13
    errs = []
    for n in (12, 24, 48):
        e = pi.ellipsoid_mesh(4.0, 3.0, 2.0, n_lat=n, n_lon=2 * n)
        errs.append(abs(orc.mesh_volume(e.verts, e.tris) - 4 / 3 * math.pi * 24) / (4 / 3 * math.pi * 24))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 2e-3
    assert errs[0] / errs[1] > 3.5  # second-order convergence of the polyhedral volume


def test_winding_number_cube(orc):
    """Winding number of a cube mesh equals the analytic inside test (no sample on the surface)."""
    m = pi.cube_mesh(1.3)
    h = 0.25
    mm = np.arange(-8, 8)
    inside = orc.voxelize(m.verts, m.tris, 2, (-8, -8, -8), (16, 16, 16)).reshape(16, 16, 16)
    cz, cy, cx = np.meshgrid((mm + 0.5) * h, (mm + 0.5) * h, (mm + 0.5) * h, indexing="ij")
    ref = (np.abs(cx) < 1.3) & (np.abs(cy) < 1.3) & (np.abs(cz) < 1.3)
    assert np.array_equal(inside.astype(bool), ref)


def test_winding_rotor_parity_bruteforce(orc):
    """Rotor mesh: winding-number inside test equals brute-force ray parity
    (numpy, +z rays, exact edge tests) away from the surface."""
    spec = pi.RotorSpec(n_blades=3, radius=6.0, hub_radius=1.5, hub_length=3.0, chord_root=1.8,
                        chord_tip=0.9, n_chord=6, n_span=4, n_hub=12, seed=1)
    m = pi.rotor_mesh(spec)
    V = m.verts
    T = m.tris
    assert orc.mesh_volume(V, T) > 0
    rng = np.random.default_rng(0)
    pts = rng.uniform(-6.5, 6.5, size=(300, 3))
    pts[:, 0] = rng.uniform(-2, 2, size=300)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    for p in pts:
        w = orc.winding(V, T, p)
        # ray p + t e_z, t > 0: crossing if (px,py) inside the projected triangle
        d = lambda u, v: (u[:, 0] - p[0]) * (v[:, 1] - p[1]) - (u[:, 1] - p[1]) * (v[:, 0] - p[0])
        s1, s2, s3 = d(a, b), d(b, c), d(c, a)
        hit = ((s1 > 0) & (s2 > 0) & (s3 > 0)) | ((s1 < 0) & (s2 < 0) & (s3 < 0))
        nrm = np.cross(b - a, c - a)
        with np.errstate(divide="ignore", invalid="ignore"):
            tz = (np.einsum("ij,ij->i", nrm, a - p)) / nrm[:, 2]
        crossings = int(np.sum(hit & (tz > 0)))
        assert (w > 0.5) == (crossings % 2 == 1), (p, w, crossings)
        assert abs(w - round(w)) < 1e-9


# --- volume consistency (eq. 12) ---------------------------------------------
def test_fraction_volume_rotating_cube(orc):
    """Sum of B over a rotating cube vs the cube volume (eq. 12): every
    sample is within the sub-sample surface bound, and the RMS error over time
    falls with s (the trend of table 1; its printed values are not reproducible
    because the paper's error norm is undefined)."""
    N = 10
    cfg = orc.make_config(nx=24, ny=24, nz=24, q=19, tau=0.8)
    ax = np.array([1.0, 2.0, 3.0])
    ax /= np.linalg.norm(ax)
    rms = []
    for s in (0, 1, 2, 3):
        g = orc.OracleGeometry(pi.Shape("cube", (0.5 * N,)), s)
        vals = np.array([orc.map_body(cfg, g, orc.pose_at(pi.Motion(axis=tuple(ax), omega=0.05,
                                                                     x0=(12.0, 12.0, 12.0)), t)).sum()
                         for t in range(0, 100, 5)])
        bound = 6 * N * N * (math.sqrt(3) * 2.0 ** -s)
        assert np.all(np.abs(vals - N ** 3) < bound)
        rms.append(np.sqrt(np.mean((vals - N ** 3) ** 2)) / N ** 3)
    assert rms[0] > rms[1] > rms[2] > rms[3]


@pytest.mark.parametrize("bc", [("periodic",) * 6, ("inlet", "outlet", "wall", "wall", "wall", "wall"),
                                ("wall", "wall", "periodic", "periodic", "inlet", "outlet")])
def test_sampled_update_equals_full_step(orc, bc):
    """The one-cell update (used for sampled checks on full-size grids) gives
    the same two steps as the full-domain step on every cell of a small grid."""
    wl = pi.Workload("t", 9, 7, 6, 19, "f64", 0.8, 3 / 16, (1e-4, 0, 0), bc, (0.03, 0.0, 0.01), 1, 0, 1, 2,
                     [pi.Body(pi.Shape("ellipsoid", (2.0, 1.5, 1.0)),
                              pi.Motion(axis=(0, 0, 1), omega=0.2, x0=(4.0, 3.0, 3.0)), s=1)])
    c, w, _ = orc.lattice(19)
    f0 = w[:, None] + pi.pdf_deviation_full(11, 19, wl.n_cells) * 10
    run = orc.Run(wl, f0=f0.copy()).advance(2)
    geoms = [orc.OracleGeometry(b.shape, b.s) for b in wl.bodies]

    def f_at(xyz):
        n = xyz[:, 0] + wl.nx * (xyz[:, 1] + wl.ny * xyz[:, 2])
        return f0[:, n].T

    cells = np.array([(x, y, z) for z in range(6) for y in range(7) for x in range(9)])[::5]
    got = orc.sampled_steps(wl, cells, f_at, geoms, 2)
    n = cells[:, 0] + 9 * (cells[:, 1] + 7 * cells[:, 2])
    assert np.allclose(got, run.f[:, n].T, atol=1e-15, rtol=0)


# --- static no-slip obstacle (the LBM variant of section V's node benchmark) ---
def _obstacle_steps(orc, cfg, f, solid, n):
    for _ in range(n):
        orc.step_obstacle(cfg, f, solid)


@pytest.mark.parametrize("q", [19, 27])
def test_obstacle_slab_equals_wall_faces(orc, q):
    """Obstacle rows y = 0 and y = ny-1 of a periodic box give bit for bit the
    fluid of the box without them whose -y / +y faces are halfway bounce-back
    walls (the diagonal links cross the periodic x / z wrap as well); obstacle
    cells keep their values."""
    nx, ny, nz = 4, 8, 3
    F = (1e-4, 0.0, 2e-5)
    cfg_a = _cfg(orc, q, nx=nx, ny=ny, nz=nz, force=F, psm=0)
    cfg_b = _cfg(orc, q, nx=nx, ny=ny - 2, nz=nz, force=F, psm=0,
                 bc=("periodic", "periodic", "wall", "wall", "periodic", "periodic"))
    fa = _random_state(orc, q, nx * ny * nz, 91)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    solid = solid.ravel()
    fb = fa.reshape(q, nz, ny, nx)[:, :, 1:ny - 1, :].reshape(q, -1).copy()
    f0 = fa.copy()
    _obstacle_steps(orc, cfg_a, fa, solid, 7)
    for _ in range(7):
        orc.step(cfg_b, fb, None, [])
    got = fa.reshape(q, nz, ny, nx)[:, :, 1:ny - 1, :].reshape(q, -1)
    assert np.array_equal(got, fb)
    assert np.array_equal(fa[:, solid == 1], f0[:, solid == 1])


def test_obstacle_poiseuille_exact(orc):
    """Body-force channel between obstacle rows: the halfway walls sit one cell
    in, u_x = F/(2 nu) (y - 1)(ny - 1 - y) at the fluid cell centres."""
    ny, tau, F = 12, 0.8, 1e-5
    cfg = _cfg(orc, 19, nx=1, ny=ny, nz=1, tau=tau, force=(F, 0, 0), psm=0)
    c, w, _ = orc.lattice(19)
    f = np.repeat(w[:, None], ny, axis=1).copy()
    solid = np.zeros(ny, np.uint8)
    solid[0] = solid[-1] = 1
    prev = f.copy()
    for _ in range(400):
        _obstacle_steps(orc, cfg, f, solid, 500)
        if np.abs(f - prev).max() < 1e-14:
            break
        prev = f.copy()
    else:
        raise AssertionError("no steady state")
    rho, u = orc.macro(cfg, f)
    nu = (tau - 0.5) / 3
    y = np.arange(1, ny - 1) + 0.5
    ua = F / (2 * nu) * (y - 1) * (ny - 1 - y)
    assert np.abs(u[1:-1, 0] - ua).max() / ua.max() < 1e-10


@pytest.mark.parametrize("q", [19, 27])
def test_obstacle_conserves_fluid_mass(orc, q):
    """Random obstacle cells in a periodic box with a body force: every
    post-collision value of a fluid cell lands in exactly one fluid slot, so
    the fluid mass is conserved; obstacle cells never change."""
    nx, ny, nz = 6, 5, 4
    N = nx * ny * nz
    cfg = _cfg(orc, q, nx=nx, ny=ny, nz=nz, force=(2e-4, -1e-4, 5e-5), psm=0)
    f = _random_state(orc, q, N, 93)
    solid = pi.random_obstacle(7, N, 0.3)
    assert 0 < solid.sum() < N
    f0 = f.copy()
    m0 = f[:, solid == 0].sum()
    _obstacle_steps(orc, cfg, f, solid, 10)
    assert abs(f[:, solid == 0].sum() - m0) / m0 < 1e-13
    assert np.array_equal(f[:, solid == 1], f0[:, solid == 1])


def test_obstacle_rest_is_fixed_point(orc):
    """Rest equilibrium around any obstacle stays at rest (no force)."""
    nx, ny, nz = 5, 4, 6
    cfg = _cfg(orc, 19, nx=nx, ny=ny, nz=nz, psm=0, bc=("wall", "wall", "periodic", "periodic", "wall", "wall"))
    c, w, _ = orc.lattice(19)
    N = nx * ny * nz
    f = np.repeat(w[:, None], N, axis=1).copy()
    solid = pi.random_obstacle(8, N, 0.35)
    _obstacle_steps(orc, cfg, f, solid, 5)
    assert np.abs(f - w[:, None]).max() < 1e-15


def test_obstacle_empty_mask_is_plain_step(orc):
    nx, ny, nz = 5, 4, 3
    cfg = _cfg(orc, 27, nx=nx, ny=ny, nz=nz, psm=0, force=(1e-4, 0, 0),
               bc=("inlet", "outlet", "wall", "wall", "periodic", "periodic"), u_in=(0.03, 0, 0))
    f = _random_state(orc, 27, nx * ny * nz, 95)
    g = f.copy()
    _obstacle_steps(orc, cfg, f, np.zeros(nx * ny * nz, np.uint8), 4)
    for _ in range(4):
        orc.step(cfg, g, None, [])
    assert np.array_equal(f, g)


# --- two-way coupling: rigid-body integrator (section IV's settling sphere) ---
def _rigid(orc, m=3.0, I=(2.0, 2.0, 2.0), F_ext=(0.0, 0.0, 0.0), X0=(1.0, 2.0, 3.0), average=False):
    return orc.rigid_state(dict(m=m, I=I, F_ext=F_ext, X0=X0), average=average)


def test_rigid_force_averaging_closed_form(orc):
    """With two-step averaging from rest, a constant hydrodynamic force enters
    the first step at half strength: V(t) = (F_ext t + F_h (t - 1/2)) / m."""
    F_ext = np.array([0.0, 0.0, -0.2])
    Fh = np.array([0.05, 0.0, 0.12])
    st = _rigid(orc, m=2.0, F_ext=tuple(F_ext), average=True)
    for _ in range(9):
        orc.rigid_advance(st, np.concatenate([Fh, np.zeros(3)]))
    assert np.allclose(st["V"], (F_ext * 9 + Fh * 8.5) / 2.0, rtol=0, atol=1e-15)


def test_coupled_averaging_keeps_light_sphere_stable(orc):
    """SC2 at tau = 0.575 hands the body 1/tau times its inner fluid's momentum
    change one step late: for a density ratio 1.16 the explicit update
    oscillates with growing amplitude (ratio rho_f V / (m tau) ~ 1.5 > 1);
    averaging the last two steps' force (roots of z^2 + k/2 z + k/2, |z|^2 =
    k/2 < 1) keeps it settling smoothly."""
    wl, rg = pi.workload_settling_sphere(20, 20, 30, r=3.5, storage="f64", tau=0.575, rho_s=1.16, g=7.4e-4)
    runs = {}
    for avg in (False, True):
        st = [orc.rigid_state(rg, average=avg)]
        _, tr = orc.coupled_run(wl, st, 40)
        runs[avg] = np.array([r[0]["V"][2] for r in tr])
    assert np.abs(runs[False]).max() > 1e-2  # the plain explicit update runs away
    v = runs[True]
    assert v[-1] < 0 and np.abs(v).max() < 2e-3 and np.all(np.diff(v[5:]) < 2e-5)


def test_rigid_constant_force_closed_form(orc):
    """Semi-implicit Euler from rest under a constant force: V(t) = F t / m and
    X(t) = X0 + F t (t + 1) / (2 m)."""
    F_ext = np.array([0.1, 0.0, 0.0])
    Fh = np.array([0.2, -0.2, 0.05])  # hydrodynamic part; the total is F_ext + Fh
    st = _rigid(orc, m=4.0, F_ext=tuple(F_ext))
    for _ in range(25):
        orc.rigid_advance(st, np.concatenate([Fh, np.zeros(3)]))
    t, F = 25, F_ext + Fh
    assert np.allclose(st["V"], F * t / 4.0, rtol=0, atol=1e-14)
    assert np.allclose(st["X"], np.array([1.0, 2.0, 3.0]) + F * t * (t + 1) / 8.0, rtol=0, atol=1e-12)
    assert np.array_equal(st["R"], np.eye(3)) and np.array_equal(st["W"], np.zeros(3))


def test_rigid_constant_torque_isotropic_closed_form(orc):
    """Isotropic body from rest under a constant torque T: W(t) = T t / I and
    the orientation turned by |T| t (t + 1) / (2 I) about T (rotations about
    one axis add)."""
    T = np.array([0.02, -0.01, 0.03])
    I = 5.0
    st = _rigid(orc, I=(I, I, I))
    R0 = orc.rodrigues(np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0), 0.7)
    st["R"] = R0.copy()
    for _ in range(30):
        orc.rigid_advance(st, np.concatenate([np.zeros(3), T]))
    t = 30
    a = T / np.linalg.norm(T)
    assert np.allclose(st["W"], T * t / I, rtol=0, atol=1e-15)
    ang = np.linalg.norm(T) * t * (t + 1) / (2 * I)
    assert np.allclose(st["R"], orc.rodrigues(a, ang) @ R0, rtol=0, atol=1e-12)
    assert np.allclose(st["R"] @ st["R"].T, np.eye(3), atol=1e-13)


def test_rigid_asymmetric_gyroscopic_term(orc):
    """Asymmetric body spinning about a principal axis (no torque): the
    gyroscopic term vanishes and W stays put; spinning about a tilted axis it
    does not, and the step changes W by -dt I_lab^-1 (W x I_lab W) exactly."""
    st = _rigid(orc, I=(1.0, 2.0, 3.0))
    st["W"] = np.array([0.0, 0.05, 0.0])
    orc.rigid_advance(st, np.zeros(6))
    assert np.allclose(st["W"], [0.0, 0.05, 0.0], atol=1e-17)
    st = _rigid(orc, I=(1.0, 2.0, 3.0))
    W0 = np.array([0.03, 0.04, 0.0])
    st["W"] = W0.copy()
    orc.rigid_advance(st, np.zeros(6))
    I = np.diag([1.0, 2.0, 3.0])
    expect = W0 - np.linalg.inv(I) @ np.cross(W0, I @ W0)
    assert np.allclose(st["W"], expect, atol=1e-16)
    assert abs(np.cross(W0, I @ W0)[2]) > 1e-4  # the term is really exercised


def test_coupled_momentum_balance(orc):
    """Freely moving sphere in a periodic box (no fluid force): every step the
    fluid's momentum change plus the body's, m (V(t+1) - V(t)), equals the
    external force on the body exactly (the force of eq. (10) leaves the
    fluid and enters the body)."""
    wl, rg = pi.workload_settling_sphere(16, 16, 20, r=3.0, storage="f64", tau=0.8, rho_s=1.4, g=5e-4, z0=10.0)
    wl.bc = ("periodic",) * 6
    st = [orc.rigid_state(rg, average=False)]  # the balance holds step by step without averaging
    st[0]["V"] = np.array([0.002, -0.001, 0.0])
    st[0]["W"] = np.array([0.0, 0.003, 0.001])
    c, w, _ = orc.lattice(19)
    f = w[:, None] + pi.pdf_deviation_full(12, 19, wl.n_cells) * 4
    P = lambda g: g.sum(axis=1) @ c
    Fe = np.array(rg["F_ext"])
    for _ in range(6):
        p0, v0 = P(f), st[0]["V"].copy()
        f, _ = orc.coupled_run(wl, st, 1, f0=f)
        dP = P(f) - p0 + rg["m"] * (st[0]["V"] - v0)
        assert np.allclose(dP, Fe, rtol=0, atol=1e-12)


# --- cumulant collision (D3Q27; section II.B lists it, section V runs with it) ---
def _cum_cfg(orc, tau=0.7, **kw):
    return _cfg(orc, 27, tau=tau, psm=0, collision="cumulant", **kw)


def _cum_collide(orc, cfg, f):
    fo, _ = orc.collide_cell(cfg, f)
    return fo


def test_cumulant_rate_one_gives_product_equilibrium(orc):
    """With every rate one the post-collision state has all cumulants of
    order >= 3 zero and the second-order ones at c_s^2 delta: it is the
    product of the three 1-D distributions on {-1, 0, 1} with mean u_a and
    variance 1/3, rho prod_a phi(c_a; u_a), phi(+-1) = (1/3 + u^2 +- u)/2,
    phi(0) = 2/3 - u^2."""
    cfg = _cum_cfg(orc, tau=1.0)
    c, w, _ = orc.lattice(27)
    for seed in range(4):
        f = _rand_f(27, w, 60 + seed, amp=3.0)
        rho = f.sum()
        u = (f @ c) / rho
        def phi(k, v):
            return {-1: (1 / 3 + v * v - v) / 2, 0: 2 / 3 - v * v, 1: (1 / 3 + v * v + v) / 2}[k]
        expect = np.array([rho * phi(cc[0], u[0]) * phi(cc[1], u[1]) * phi(cc[2], u[2]) for cc in c])
        got = _cum_collide(orc, cfg, f)
        assert np.abs(got - expect).max() < 1e-15


def test_cumulant_conserves_mass_and_momentum(orc):
    cfg = _cum_cfg(orc, tau=0.63)
    c, w, _ = orc.lattice(27)
    for seed in range(4):
        f = _rand_f(27, w, 70 + seed, amp=3.0)
        g = _cum_collide(orc, cfg, f)
        assert abs(g.sum() - f.sum()) < 1e-15
        assert np.abs(g @ c - f @ c).max() < 1e-15
        assert np.abs(g - f).max() > 1e-4  # it does relax


@pytest.mark.parametrize("perm,sign", [((1, 0, 2), (1, 1, 1)), ((2, 0, 1), (1, 1, 1)), ((0, 1, 2), (-1, 1, 1)),
                                       ((0, 2, 1), (1, -1, -1))])
def test_cumulant_commutes_with_lattice_symmetries(orc, perm, sign):
    """Collision commutes with the cube's symmetries (axis permutations and
    reflections) of the D3Q27 velocity set."""
    cfg = _cum_cfg(orc, tau=0.71)
    c, w, _ = orc.lattice(27)
    lut = {tuple(v): k for k, v in enumerate(c)}
    img = np.array([lut[tuple(np.array(sign) * v[list(perm)])] for v in c])  # velocity k -> its image
    f = _rand_f(27, w, 81, amp=3.0)
    g = np.empty_like(f)
    g[img] = f
    a = _cum_collide(orc, cfg, f)
    b = _cum_collide(orc, cfg, g)
    assert np.abs(b[img] - a).max() < 1e-15


def test_cumulant_shear_wave_viscosity(orc):
    """A decaying shear wave u_x(y) = U sin(k y) (periodic, D3Q27): the
    amplitude decays at the rate nu k^2 with nu = c_s^2 (tau - 1/2) (the shear
    rate 1/tau sets the viscosity); 1% on the rate at k = 2 pi / 32."""
    L, tau, U = 32, 0.8, 1e-3
    cfg = _cum_cfg(orc, tau=tau, nx=1, ny=L, nz=1)
    c, w, _ = orc.lattice(27)
    y = np.arange(L) + 0.0
    ux = U * np.sin(2 * np.pi * y / L)
    f = np.stack([orc.feq(27, 1.0, (ux[n], 0.0, 0.0)) for n in range(L)], axis=1)
    amps = {}
    for t in range(1, 301):
        orc.step(cfg, f, None, [])
        if t in (100, 300):
            _, u = orc.macro(cfg, f)
            amps[t] = 2 / L * np.sum(u[:, 0] * np.sin(2 * np.pi * y / L))
    rate = np.log(amps[100] / amps[300]) / 200
    nu = (tau - 0.5) / 3
    k = 2 * np.pi / L
    assert abs(rate / (nu * k * k) - 1) < 0.01


def test_cumulant_post_collision_central_moments(orc):
    """Second- and third-order central moments of the collision's output, from
    their definition C_abc = sum_i f_i (c_x - u_x)^a (c_y - u_y)^b (c_z - u_z)^c
    (u conserved): the trace relaxes to rho (3 c_s^2 rho, bulk rate one), the
    deviators C_xx - C_yy, C_xx - C_zz and the off-diagonal C_xy, C_xz, C_yz keep
    (1 - 1/tau) of their value, and the third-order ones with exponents <= 2 per
    axis (third-order cumulants, rate one) vanish.  At tau != 1, so a wrong
    deviator or bulk rate shows."""
    tau = 0.66
    om = 1 / tau
    cfg = _cum_cfg(orc, tau=tau)
    c, w, _ = orc.lattice(27)

    def central(f, u, e):
        d = c - u
        return float(np.sum(f * d[:, 0] ** e[0] * d[:, 1] ** e[1] * d[:, 2] ** e[2]))

    for seed in range(5):
        f = _rand_f(27, w, 120 + seed, amp=3.0)
        g = _cum_collide(orc, cfg, f)
        rho = f.sum()
        u = (f @ c) / rho
        assert np.abs((g @ c) / g.sum() - u).max() < 1e-15
        Cf = {e: central(f, u, e) for e in itertools.product(range(3), repeat=3) if sum(e) == 2}
        Cg = {e: central(g, u, e) for e in Cf}
        xx, yy, zz = (2, 0, 0), (0, 2, 0), (0, 0, 2)
        assert abs(Cg[xx] + Cg[yy] + Cg[zz] - rho) < 1e-14
        assert abs(Cf[xx] + Cf[yy] + Cf[zz] - rho) > 1e-3  # the input is off the trace equilibrium
        for a, b in [(xx, yy), (xx, zz)]:
            assert abs((Cg[a] - Cg[b]) - (1 - om) * (Cf[a] - Cf[b])) < 1e-14
            assert abs(Cf[a] - Cf[b]) > 1e-3
        for e in [(1, 1, 0), (1, 0, 1), (0, 1, 1)]:
            assert abs(Cg[e] - (1 - om) * Cf[e]) < 1e-14
            assert abs(Cf[e]) > 1e-4
        for e in itertools.product(range(3), repeat=3):
            if sum(e) == 3:
                assert abs(central(g, u, e)) < 1e-14
                assert abs(central(f, u, e)) > 1e-6 or e == (1, 1, 1)


def test_cumulant_diagonal_shear_wave_viscosity(orc):
    """A shear wave along the face diagonal, u = U sin(k.x) (1, -1, 0)/sqrt 2
    with k = 2 pi (1, 1, 0)/L (periodic, D3Q27): its strain is purely diagonal
    in the lattice frame (S_xx = -S_yy, S_xy = 0), so the decay rate nu |k|^2,
    nu = c_s^2 (tau - 1/2), is set by the deviator rate, which the axis-aligned
    wave never sees; 1% on the rate."""
    L, tau, U = 24, 0.8, 1e-3
    cfg = _cum_cfg(orc, tau=tau, nx=L, ny=L, nz=1)
    yy, xx = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    ph = 2 * np.pi * (xx + yy).ravel() / L
    amp = U * np.sin(ph) / np.sqrt(2)
    f = np.stack([orc.feq(27, 1.0, (a, -a, 0.0)) for a in amp], axis=1)
    amps = {}
    for t in range(1, 121):
        orc.step(cfg, f, None, [])
        if t in (40, 120):
            _, u = orc.macro(cfg, f)
            amps[t] = 2 / (L * L) * np.sum((u[:, 0] - u[:, 1]) / np.sqrt(2) * np.sin(ph))
    rate = np.log(amps[40] / amps[120]) / 80
    nu = (tau - 0.5) / 3
    k2 = 2 * (2 * np.pi / L) ** 2
    assert abs(rate / (nu * k2) - 1) < 0.01


def test_cumulant_refuses_force_and_d3q19(orc):
    cfg = _cfg(orc, 19, psm=0, collision="cumulant")
    c, w, _ = orc.lattice(19)
    with pytest.raises(RuntimeError):
        orc.collide_cell(cfg, w.copy())
    cfg = _cum_cfg(orc, force=(1e-5, 0, 0))
    c, w, _ = orc.lattice(27)
    with pytest.raises(RuntimeError):
        orc.collide_cell(cfg, w.copy())


# --- the roofline model of the measurement (section V's worked figures) ------
def test_roofline_bytes_model_matches_section_v():
    """bench.py's algorithmic bytes per plain-LBM cell update, 2 Q sizeof, give
    the paper's CPU roofline exactly (247,000 MB/s / 304 B = 812.5 MLUPS) and
    its printed fractions (> 72% on the CPU, > 93% on the A100 node).  The
    printed A100 roofline, 18,092 MLUPS, is 0.66% above 4 x 1366 GB/s / 304 B
    = 17,974 (the text's figures disagree slightly); both readings give the
    printed > 93%."""
    import json
    import os

    import bench

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "roofline_section_v.json")))
    cpu, gpu = g["cpu_lumi_c"], g["gpu_a100_node"]
    b = bench.bytes_per_cell(cpu["stencil_q"], "f64", psm=False)
    assert b == 2 * 19 * 8 == 304
    assert cpu["stream_bandwidth_MBps"] * 1e6 / b / 1e6 == cpu["roofline_mlups_printed"]
    for v in cpu["lbm_mlups_printed"].values():
        assert v / cpu["roofline_mlups_printed"] > cpu["fraction_of_roofline_printed_at_least"]
    roof = gpu["gpus"] * gpu["stream_bandwidth_GBps_per_gpu"] * 1e9 / b / 1e6
    assert abs(roof / gpu["roofline_mlups_printed"] - 1) < 0.007
    for r in (roof, gpu["roofline_mlups_printed"]):
        assert gpu["lbm_mlups_printed_scenario_B"] / r > gpu["fraction_of_roofline_printed_at_least"]
