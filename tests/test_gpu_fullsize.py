"""Full-size parity on sampled outputs, in the launch configuration bench.py
times (same Field setup): two steps (even + odd) from a seeded random state,
then f at sampled cells against the oracle's one-cell updates over each cell's
two-step dependence cone; solid fractions at sampled surface cells bit for bit.

Samples cover corners, edges and faces of the domain (every face rule),
random interior cells and cells next to the bodies.  PDF samples next to mesh
bodies are left to the mapping checks (the oracle's on-demand winding number
over ~10^5 triangles per point is too slow for a whole dependence cone).
"""
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

    assert torch.cuda.is_available()
    from paper_2502_20049_amd import sim as s

    return s


def _perm(orc, sim, q):
    c, _, _ = sim.lattice(q)
    oc, _, _ = orc.lattice(q)
    lut = {tuple(v): k for k, v in enumerate(c)}
    return np.array([lut[tuple(v)] for v in oc])


def _edge_cells(wl, rng, n_rand=12):
    nx, ny, nz = wl.nx, wl.ny, wl.nz
    pts = set()
    for x in (0, 1, nx // 2, nx - 2, nx - 1):
        for y in (0, 1, ny // 2, ny - 1):
            for z in (0, nz // 3, nz - 1):
                pts.add((x, y, z))
    for _ in range(n_rand):
        pts.add((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    return sorted(pts)


def _far_from_bodies(wl, cells, margin):
    out = []
    for c in cells:
        ok = True
        for b in wl.bodies:
            r = max(np.linalg.norm(b.shape.mesh.verts, axis=1).max() if b.shape.kind == "mesh" else max(b.shape.params),
                    0.0)
            if np.linalg.norm(np.array(c) + 0.5 - np.array(b.motion.x0)) < r + margin:
                ok = False
        if ok:
            out.append(c)
    return out


def _run(orc, sim, wl, seed, cells, tol_fn, lazy=False):
    import torch

    f = sim.Field(wl)
    c, _, _ = sim.lattice(wl.q)
    for k in range(wl.q):  # per direction, to bound temporary memory
        f.pdf_view()[k].copy_(pi.random_state_torch(seed, c[k:k + 1], wl.n_cells, f.pdf.device, f.dtype)[0])
    torch.cuda.synchronize()
    f.step(0)
    f.step(1)
    torch.cuda.synchronize()
    oc, ow, _ = orc.lattice(wl.q)
    idx = _perm(orc, sim, wl.q)
    cells = np.array(cells, dtype=np.int64)
    n = cells[:, 0] + wl.nx * (cells[:, 1] + wl.ny * cells[:, 2])
    nt = torch.tensor(n, device=f.pdf.device)
    g = f.pdf_view()[:, nt].double().cpu().numpy()[idx].T + ow[None, :]
    geoms = [orc.OracleGeometry(b.shape, b.s, lazy=lazy) for b in wl.bodies]

    def f_at(xyz):
        m = xyz[:, 0] + wl.nx * (xyz[:, 1] + wl.ny * xyz[:, 2])
        return ow[None, :] + pi.random_state(seed, oc, wl.n_cells, m)

    ref = orc.sampled_steps(wl, cells, f_at, geoms, 2)
    err = np.abs(g - ref)
    bound = tol_fn(ref - ow[None, :])
    _say(f"  {wl.name}: {len(cells)} cells, max err {err.max():.2e}, max err/bound {(err / bound).max():.2f}")
    assert np.all(err <= bound)
    return f, geoms


def _map_samples(orc, f, wl, geoms, cells, t):
    import torch

    B, meta = f.b_view()
    cells = np.array(cells, dtype=np.int64)
    n = cells[:, 0] + wl.nx * (cells[:, 1] + wl.ny * cells[:, 2])
    nt = torch.tensor(n, device=B.device)
    Bg = B[0, nt].double().cpu().numpy()
    ids = meta[nt].cpu().numpy() & 15
    for j, cidx in enumerate(cells):
        vals = [orc.b_from_eps(orc.map_cell(g, orc.pose_at(b.motion, t), *map(int, cidx)), wl.tau, wl.b_form)
                for g, b in zip(geoms, wl.bodies)]
        nz = [(bi, v) for bi, v in enumerate(vals) if v != 0]
        if not nz:
            assert Bg[j] == 0.0
        else:
            assert len(nz) == 1 and ids[j] == nz[0][0] and Bg[j] == nz[0][1], (cidx, Bg[j], vals)
    return Bg


def test_ellipsoid_channel_256_full_size(orc, sim):
    _say("[full-size] 256^3 channel, rotating ellipsoid s=3, FP32")
    wl = pi.workload_ellipsoid_channel(256, "f32", steps=2, s=3)
    rng = np.random.default_rng(1)
    cells = _edge_cells(wl, rng)
    # cells on and near the ellipsoid surface (x axis tip, y tip, z tip)
    cells += [(128 + 40, 128, 128), (128 - 41, 127, 128), (128, 128 + 20, 129), (127, 128, 128 - 10),
              (150, 140, 131), (100, 120, 124)]
    _run(orc, sim, wl, 3, cells, lambda d: np.full_like(d, 2e-6))


def test_cror_768_fp16_full_size(orc, sim):
    _say("[full-size] 768x384x384 D3Q27 counter-rotating rotors, FP16 storage")
    wl = pi.workload_cror(storage="f16")
    rng = np.random.default_rng(2)
    cells = _far_from_bodies(wl, _edge_cells(wl, rng), 4.0)
    f, geoms = _run(orc, sim, wl, 4, cells,
                    lambda d: np.full_like(d, 4 * 2.0 ** -11 * np.abs(d).max() + 2e-6), lazy=True)
    # solid fractions at sampled cells on the blades (B after the odd step's mapping, t = 1)
    bcells = []
    for b in wl.bodies:
        X = np.array(b.motion.x0)
        for r, ang in [(60.0, 0.3), (90.0, 1.1), (110.0, 2.5), (45.0, 4.0)]:
            bcells.append((int(X[0]), int(X[1] + r * np.cos(ang)), int(X[2] + r * np.sin(ang))))
    Bg = _map_samples(orc, f, wl, geoms, bcells, 1)
    _say(f"  sampled B: {Bg}")


def test_capacity_1024_full_size(orc, sim):
    import torch

    _say("[full-size] 1024^3 capacity run, two 6-blade rotors, FP32 in place")
    free, total = torch.cuda.mem_get_info()
    if free < 100 * 2**30:
        pytest.skip(f"needs ~90 GiB of device memory, {free / 2**30:.0f} GiB free")
    wl = pi.workload_capacity()
    rng = np.random.default_rng(3)
    cells = _far_from_bodies(wl, _edge_cells(wl, rng, 8), 4.0)
    f, geoms = _run(orc, sim, wl, 5, cells, lambda d: np.full_like(d, 2e-6), lazy=True)
    bcells = []
    for b in wl.bodies:
        X = np.array(b.motion.x0)
        for r, ang in [(150.0, 0.2), (250.0, 1.4)]:
            bcells.append((int(X[0]), int(X[1] + r * np.cos(ang)), int(X[2] + r * np.sin(ang))))
    _map_samples(orc, f, wl, geoms, bcells, 1)
    mass = f.mass(2).item()
    assert np.isfinite(mass)


def test_direction_arrays_over_4gib_sc2(orc, sim):
    """A 1056 x 1024 x 1024 channel in FP32 (4.4 GB per direction array, so
    byte offsets past 2^32 inside each array) with SC2 and a rotating
    ellipsoid at the top of the lattice, where the offsets are largest: two
    steps against the oracle's one-cell updates on sampled cells, including
    the body's surface cells."""
    import torch

    free, total = torch.cuda.mem_get_info()
    if free < 100 * 2**30:
        pytest.skip(f"needs ~92 GiB of device memory, {free / 2**30:.0f} GiB free")
    _say("[full-size] 1056x1024x1024 channel, SC2, FP32 (direction arrays over 4 GiB)")
    ell = pi.Body(pi.Shape("ellipsoid", (12.0, 8.0, 6.0)),
                  pi.Motion(axis=(0.0, 0.6, 0.8), theta0=0.4, omega=0.05, x0=(528.0, 512.0, 1000.0)), s=1)
    wl = pi.Workload("channel_1056x1024x1024_sc2", 1056, 1024, 1024, 19, "f32", 0.8, 3 / 16, (0, 0, 0),
                     ("inlet", "outlet", "wall", "wall", "wall", "wall"), (0.05, 0, 0), 2, 0, 1, 2, [ell])
    assert 4 * wl.n_cells > 2**32
    rng = np.random.default_rng(9)
    cells = _edge_cells(wl, rng, 8)
    cells += [(528 + 12, 512, 1000), (528 - 12, 511, 1000), (528, 512 + 7, 1001), (527, 512, 1000 + 6),
              (520, 505, 997), (533, 516, 1003), (528, 512, 1000)]
    _run(orc, sim, wl, 11, cells, lambda d: np.full_like(d, 2e-6))


def test_cror_768_cumulant_full_size(orc, sim):
    """The rotor pair with the cumulant collision (FP16 storage, the odd steps
    on the one-cell-per-lane kernel): sampled cells against the oracle's
    one-cell updates."""
    _say("[full-size] 768x384x384 D3Q27 rotor pair, cumulant, FP16 storage")
    wl = pi.workload_cror(storage="f16")
    wl.collision = "cumulant"
    rng = np.random.default_rng(6)
    cells = _far_from_bodies(wl, _edge_cells(wl, rng), 4.0)
    _run(orc, sim, wl, 7, cells, lambda d: np.full_like(d, 4 * 2.0 ** -11 * np.abs(d).max() + 2e-6), lazy=True)


def test_rotor_box_256_obstacle_full_size(sim):
    """LBM with the voxelised 8-blade rotor (r = 120) as a static no-slip
    obstacle on the 256^3 periodic box, two steps from a seeded state:
    obstacle cells keep their values bit for bit; cells whose two-step
    dependence cone holds no obstacle cell or neighbour match plain LBM bit for
    bit (same kernel path); FP64 mass of all slots conserved up to the FP32
    rounding of the stored deviations."""
    import dataclasses

    import torch
    import torch.nn.functional as F

    _say("[full-size] 256^3 rotor box, LBM + no-slip obstacle, FP32")
    wl = dataclasses.replace(pi.workload_rotor_box(steps=2), bc=("periodic",) * 6, u_in=(0.0, 0.0, 0.0))
    solid = sim.voxelize_obstacle(wl, 0)
    c, _, _ = sim.lattice(19)
    runs = []
    for with_obst in (True, False):
        f = sim.Field(wl, psm=False)
        for k in range(19):
            f.pdf_view()[k].copy_(pi.random_state_torch(8, c[k:k + 1], wl.n_cells, f.pdf.device, f.dtype)[0])
        if with_obst:
            n_near = f.set_obstacle(solid)
            f0 = f.pdf_view()[:, solid.bool()].clone()
            m0 = float(f.mass(0).item())
        f.step(0)
        f.step(1)
        torch.cuda.synchronize()
        if with_obst:
            assert torch.equal(f.pdf_view()[:, solid.bool()], f0)
            m1 = float(f.mass(2).item())
            assert abs(m1 - m0) / abs(m0) < 1e-7  # FP32 rounding of ~3e8 stored deviations
        runs.append(f.pdf_view().clone())
        del f
        torch.cuda.empty_cache()
    # cells at distance > 3 from every obstacle cell (periodic): a 7^3 max filter of the mask
    s3 = solid.view(1, 1, wl.nz, wl.ny, wl.nx).float()
    s3 = torch.cat([s3[..., -3:, :, :], s3, s3[..., :3, :, :]], dim=2)
    s3 = torch.cat([s3[..., :, -3:, :], s3, s3[..., :, :3, :]], dim=3)
    s3 = torch.cat([s3[..., :, :, -3:], s3, s3[..., :, :, :3]], dim=4)
    near = F.max_pool3d(s3, 7, stride=1).view(-1) > 0
    far = ~near
    _say(f"  near cells {n_near}, far cells {int(far.sum())}")
    assert int(far.sum()) > wl.n_cells // 2
    assert torch.equal(runs[0][:, far], runs[1][:, far])
