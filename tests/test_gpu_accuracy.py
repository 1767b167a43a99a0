"""Accuracy of the reduced-precision storage forms against the FP64 oracle at
the benchmark configurations' own sizes, and of the adjoint at full size.

Metrics: velocity rel. L2 ||u - u_ref|| / ||u_ref|| over all cells at the last
step (also max |u - u_ref| / max |u_ref|); torque: the series max
|T(t) - T_ref(t)| / max |T_ref| and the window mean.  Targets for FP32
storage (FP32 arithmetic): 1e-5 in velocity and 1e-4 in torque.  FP16 storage
rounds every stored deviation to 11 bits each step: its error is reported and
held to the bound the reduced tests established.
"""
import dataclasses
import json
import os
import sys

import numpy as np
import pytest

import psm_inputs as pi

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2502_20049_amd import sim as s

    return s


def _gpu_run(sim, wl, storage, steps, body=0, comp=5):
    """(u (N, 3) at `steps`, torque component `comp` series of body `body`)."""
    import torch

    f = sim.Field(wl, storage=storage)
    tz = []
    for t in range(steps):
        f.step(t)
        tz.append(f.force_torque()[body, comp].item())
    _, u = f.macroscopic(steps)
    torch.cuda.synchronize()
    u = u.cpu().numpy()
    del f
    torch.cuda.empty_cache()
    return u, np.array(tz)


def _errors(u, uo, tz, tzo, window):
    relu = float(np.linalg.norm(u - uo) / np.linalg.norm(uo))
    maxu = float(np.abs(u - uo).max() / np.abs(uo).max())
    relT = float(np.abs(tz - tzo).max() / np.abs(tzo).max())
    relJ = float(abs(tz[-window:].mean() - tzo[-window:].mean()) / abs(tzo[-window:].mean()))
    return relu, maxu, relT, relJ


@pytest.fixture(scope="module")
def channel_256_oracle(orc):
    """The rotating-ellipsoid channel at full size (256^3, semi-axes 40, 20, 10,
    1e-3 rad/step about z, s = 3, inlet 0.05, outlet, walls), 200 steps from
    rest in the FP64 oracle: u at the last step and the z-torque series."""
    wl = pi.workload_ellipsoid_channel(256, "f32", steps=200, s=3)
    _say("[channel 256^3] oracle, 200 steps (FP64, host cores) ...")
    run = orc.Run(wl).advance(wl.steps)
    _, uo = run.macro()
    tzo = np.array(run.ft)[:, 0, 5]
    del run
    return wl, uo, tzo


@pytest.mark.timeout(900)
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_channel_256_accuracy_vs_fp64_oracle(sim, channel_256_oracle, storage):
    """The benchmark workload itself (256^3, 200 steps): FP32 storage within
    1e-5 (u) and 1e-4 (torque) of the FP64 oracle; FP16 storage reported and
    held to 5e-4 / 1e-3."""
    wl, uo, tzo = channel_256_oracle
    u, tz = _gpu_run(sim, wl, storage, wl.steps)
    relu, maxu, relT, relJ = _errors(u, uo, tz, tzo, 50)
    _say(f"[channel 256^3] {storage}: u rel L2 {relu:.2e} (max {maxu:.2e}); torque series rel {relT:.2e}, "
         f"last-50 mean rel {relJ:.2e}")
    if storage == "f32":
        assert relu < 1e-5 and relT < 1e-4 and relJ < 1e-4
    else:
        assert relu < 5e-4 and relT < 1e-3


@pytest.fixture(scope="module")
def rotor_pair_oracle(orc):
    """A reduced copy of the counter-rotating rotor pair (D3Q27, 96 x 48 x 48,
    two 8-blade rotors of radius 15, 832 triangles each, s = 1, tip speed 0.24
    as in the full scene (+-0.016 rad/step), inflow 0.05, tau 0.6), 300 steps
    in the FP64 oracle (meshes voxelised by the winding number)."""
    wl = pi.workload_cror(nx=96, ny=48, nz=48, radius=15.0, s=1, n_chord=4, n_span=3, steps=300)
    for b in wl.bodies:
        b.motion.omega = 8.0 * b.motion.omega
    _say("[rotor pair q27] oracle, 300 steps ...")
    run = orc.Run(wl)
    run.map(0)
    B0 = run.B.copy()
    run.advance(wl.steps)
    _, uo = run.macro()
    ft = np.array(run.ft)
    return wl, B0, uo, ft


@pytest.mark.timeout(600)
def test_rotor_pair_q27_storage_accuracy(sim, rotor_pair_oracle):
    """D3Q27 rotor pair: FP32 and FP16 storage against the FP64 oracle (the
    rotor scene's error is reported; FP32 held to 1e-5 / 1e-4, FP16 to the
    storage bound 2e-3 / 5e-3).  B of both rotors bit-exact at t = 0."""
    import torch

    import gpu_common as gc

    wl, B0, uo, ft = rotor_pair_oracle
    f = sim.Field(wl)
    f.map(0)
    torch.cuda.synchronize()
    Bg = gc.gpu_B_per_body(f, 2)
    assert np.array_equal(Bg, B0), (Bg != B0).sum()
    del f
    res = {}
    for storage in ("f32", "f16"):
        u, tx0 = _gpu_run(sim, wl, storage, wl.steps, body=0, comp=3)
        relu, maxu, relT, relJ = _errors(u, uo, tx0, ft[:, 0, 3], 100)
        res[storage] = (relu, relT)
        _say(f"[rotor pair q27] {storage}: u rel L2 {relu:.2e} (max {maxu:.2e}); rotor-1 axial torque series rel "
             f"{relT:.2e}, last-100 mean rel {relJ:.2e}")
    assert res["f32"][0] < 1e-5 and res["f32"][1] < 1e-4
    assert res["f16"][0] < 2e-3 and res["f16"][1] < 5e-3


def _golden_adjoint():
    p = os.path.join(GOLDEN, "adjoint_rotor_128.json")
    with open(p) as fh:
        return json.load(fh)


def _v_field(rec, n):
    """The direction of the dJ/dB check, rebuilt from its recipe."""
    lo, hi = rec["v_box_lo"], rec["v_box_hi"]
    rng = np.random.default_rng(rec["v_seed"])
    shape = tuple(h - l + 1 for l, h in zip(lo, hi))[::-1]
    vals = (rec["v_scale"] * rng.standard_normal(shape)).astype(np.float32).astype(np.float64)
    v = np.zeros((n, n, n))
    v[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = vals
    return v.reshape(-1)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_adjoint_rotor_128_full_size(sim, storage):
    """The adjoint configuration at full size (128^3, 4-blade rotor of ~41k
    triangles, 800 steps, torque averaged over the last 200): J, dJ/dOmega and
    dJ/dB along a seeded direction from the hand-written adjoint (the whole
    trajectory kept, or sqrt(T) checkpoints, as memory allows), against the FP64 oracle's J and its central differences
    (frozen B; tests/golden/make_adjoint_rotor_128.py).  The GPU mapping's sums
    of B equal the oracle's exactly."""
    import torch

    import gpu_common as gc
    from paper_2502_20049_amd import adjoint

    rec = _golden_adjoint()
    wl = pi.workload_adjoint_rotor(steps=rec["steps"], storage=storage)
    f = sim.Field(wl)
    for t, s_ref in rec["sum_B"].items():
        f.map(int(t))
        torch.cuda.synchronize()
        sB = float(gc.gpu_B_per_body(f, 1).sum())
        assert sB == s_ref, (t, sB, s_ref)
    del f
    T, win = rec["steps"], rec["window"]
    w = np.zeros(T)
    w[-win:] = 1.0 / win
    # FP32: the whole trajectory (about 136 GB) where the device holds it,
    # else sqrt(T) checkpoints; FP64 (twice that): checkpoints
    obj = adjoint.TorqueAdjoint(wl, T, w)
    _say(f"[adjoint rotor 128^3] {storage}: store_all={obj.store_all}")
    J = obj.forward()
    gB, gW, _ = obj.backward()
    torch.cuda.synchronize()
    v = _v_field(rec, wl.nx)
    gBv = float(np.dot(gB.double().cpu().numpy(), v))
    eJ = abs(J - rec["J"]) / abs(rec["J"])
    eW = abs(gW - rec["dJ_dOmega_fd"]) / abs(rec["dJ_dOmega_fd"])
    eB = abs(gBv - rec["dJ_dB_dot_v_fd"]) / abs(rec["dJ_dB_dot_v_fd"])
    _say(f"[adjoint rotor 128^3] {storage}: J {J:.9e} vs {rec['J']:.9e} ({eJ:.1e}); dJ/dOmega {gW:.6e} vs FD "
         f"{rec['dJ_dOmega_fd']:.6e} ({eW:.1e}); dJ/dB.v {gBv:.6e} vs FD {rec['dJ_dB_dot_v_fd']:.6e} ({eB:.1e})")
    del obj, gB
    torch.cuda.empty_cache()
    if storage == "f64":
        assert eJ < 1e-10 and eW < 1e-5 and eB < 1e-5
    else:
        assert eJ < 1e-4 and eW < 1e-3 and eB < 1e-3
