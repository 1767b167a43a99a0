"""GPU adjoint (psm_adjoint_step + sqrt(T) driver + autograd.Function) against
the oracle's complex-step adjoint.

Tolerances: FP64 storage/arithmetic runs the same operations in another
order, so gradients agree to ~1e-10 relative; FP32 arithmetic on the forward
and adjoint (deviations ~1e-2, sums over Q and over the window) gives ~1e-4
relative on dJ/dOmega and on the dJ/dB field (max-norm).
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
def adjmod():
    import torch

    assert torch.cuda.is_available()
    from paper_2502_20049_amd import adjoint, sim

    return adjoint, sim


def _small(orc, storage, bc, sc=1):
    body = pi.Body(pi.Shape("ellipsoid", (3.0, 2.0, 1.5)),
                   pi.Motion(axis=(0.0, 0.6, 0.8), theta0=0.2, omega=0.05, x0=(5.0, 4.0, 3.0)), s=1)
    wl = pi.Workload("adj", 10, 8, 7, 19, storage, 0.8, 3 / 16, (1e-4, -5e-5, 0.0), bc, (0.03, 0.01, 0.0), sc, 0,
                     1, 6, [body])
    oc, ow, _ = orc.lattice(19)
    dev = pi.pdf_deviation_full(21, 19, wl.n_cells) * 4  # oracle direction order
    rng = np.random.default_rng(4)
    dB = (0.02 * rng.standard_normal(wl.n_cells)).astype(np.float32).astype(np.float64)
    weights = np.array([0.0, 0.5, 1.0, 1.0, 1.0, 1.0])
    return wl, ow[:, None] + dev, dev, dB, weights


def _perm(orc, sim, q):
    c, _, _ = sim.lattice(q)
    oc, _, _ = orc.lattice(q)
    lut = {tuple(v): k for k, v in enumerate(c)}
    return np.array([lut[tuple(v)] for v in oc])  # oracle j -> library k


BCS = {"periodic": ("periodic",) * 6, "channel": ("inlet", "outlet", "wall", "wall", "periodic", "periodic"),
       "box": ("wall", "wall", "inlet", "outlet", "wall", "wall")}


@pytest.mark.parametrize("store_all", [False, True], ids=["sqrtT", "whole"])
@pytest.mark.parametrize("bc", list(BCS))
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_adjoint_matches_oracle(orc, adjmod, bc, storage, store_all):
    """Both trajectory modes (sqrt(T) checkpoints with recompute, and the
    whole trajectory kept by the forward) against the oracle's adjoint."""
    import torch

    adjoint, sim = adjmod
    _say(f"[adjoint] {storage} {bc} store_all={store_all}")
    wl, f0, dev, dB, wts = _small(orc, storage, BCS[bc])
    om = wl.bodies[0].motion.omega
    Jo, gBo, gWo, gFo = orc.torque_adjoint(wl, f0, 6, wts, dB=dB, omega_us=om)
    idx = _perm(orc, sim, 19)
    dev_lib = np.empty_like(dev)
    dev_lib[idx] = dev
    adj = adjoint.TorqueAdjoint(wl, 6, wts, storage=storage, segment=2, store_all=store_all)
    assert adj.store_all == store_all
    J = adj.forward(dB=torch.tensor(dB, dtype=torch.float32), omega=om,
                    f0=torch.tensor(dev_lib, device="cuda"))
    gB, gW, gF = adj.backward()
    torch.cuda.synchronize()
    gB = gB.double().cpu().numpy()
    gF = gF.double().cpu().numpy()[idx]
    eJ = abs(J - Jo) / abs(Jo)
    eB = np.abs(gB - gBo).max() / np.abs(gBo).max()
    eW = abs(gW - gWo) / abs(gWo)
    eF = np.abs(gF - gFo).max() / np.abs(gFo).max()
    _say(f"  J {J:.6e} vs {Jo:.6e} rel {eJ:.1e}; dJ/dB {eB:.1e}; dJ/dOmega {gW:.6e} vs {gWo:.6e} rel {eW:.1e}; "
         f"dJ/df0 {eF:.1e}")
    tol = 1e-10 if storage == "f64" else 2e-4
    assert eJ < (1e-12 if storage == "f64" else 1e-4)
    assert eB < tol and eW < tol and eF < tol


def test_checkpoint_segment_does_not_change_gradients(orc, adjmod):
    """Segments of 2, 4 and 6 steps and the whole-trajectory mode give the
    same J and gradients bit for bit (the same states and B(t) reach the
    adjoint steps); the size rule picks the whole trajectory only within
    the budget."""
    import torch

    adjoint, sim = adjmod
    wl, f0, dev, dB, wts = _small(orc, "f32", BCS["channel"])
    res = []
    for L, whole in ((2, False), (4, False), (6, False), (2, True)):
        adj = adjoint.TorqueAdjoint(wl, 6, wts, segment=L, store_all=whole)
        adj.forward(dB=torch.tensor(dB, dtype=torch.float32), omega=0.05)
        gB, gW, gF = adj.backward()
        torch.cuda.synchronize()
        res.append((gB.cpu(), gW, gF.cpu()))
    for r in res[1:]:
        assert torch.equal(r[0], res[0][0]) and r[1] == res[0][1] and torch.equal(r[2], res[0][2])
    assert adjoint.TorqueAdjoint(wl, 6, wts, memory_budget=0).store_all is False
    big = adjoint.TorqueAdjoint(wl, 6, wts, memory_budget=1 << 40)
    assert big.store_all is True and big.trajectory_bytes > 0


def test_autograd_rotor_gradient(orc, adjmod):
    """Reduced copy of the rotor objective (32^3, 4-blade rotor r=10, inflow
    0.04, 60 steps, torque averaged over the last 20): torch.autograd through
    PSMTorque (FP32) against the oracle's FP64 adjoint."""
    import torch

    adjoint, sim = adjmod
    _say("[autograd rotor 32^3]")
    wl = pi.workload_adjoint_rotor(n=32, steps=60, radius=10.0, s=2, n_chord=8, n_span=8)
    T = 60
    wts = np.zeros(T)
    wts[-20:] = 1.0 / 20
    om0 = wl.bodies[0].motion.omega
    obj = adjoint.TorqueAdjoint(wl, T, wts)
    dB = torch.zeros(wl.n_cells, dtype=torch.float32, requires_grad=True)
    om = torch.tensor(om0, dtype=torch.float64, requires_grad=True)
    J = adjoint.PSMTorque.apply(dB, om, obj)
    J.backward()
    _, ow, _ = orc.lattice(19)
    f0 = np.repeat(ow[:, None], wl.n_cells, axis=1)
    Jo, gBo, gWo, _ = orc.torque_adjoint(wl, f0, T, wts, dB=None, omega_us=om0)
    eJ = abs(J.item() - Jo) / abs(Jo)
    eW = abs(om.grad.item() - gWo) / abs(gWo)
    gB = dB.grad.double().numpy()
    eB = np.linalg.norm(gB - gBo) / np.linalg.norm(gBo)
    _say(f"  J {J.item():.6e} vs {Jo:.6e} ({eJ:.1e}); dJ/dOmega {om.grad.item():.6e} vs {gWo:.6e} ({eW:.1e}); "
         f"dJ/dB rel L2 {eB:.1e}")
    assert eJ < 1e-4 and eW < 1e-3 and eB < 1e-3
