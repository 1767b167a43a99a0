"""Pins of the oracle's discrete adjoint (complex-step Jacobians + scattered
transposed streaming) against central finite differences of the oracle
forward, under the frozen-B convention (the mapping follows the prescribed
motion; the rotation rate enters the solid velocity only).  CPU only."""
import numpy as np
import pytest

import psm_inputs as pi


def _setup(orc, sc, bc):
    body = pi.Body(pi.Shape("ellipsoid", (3.0, 2.0, 1.5)),
                   pi.Motion(axis=(0.0, 0.6, 0.8), theta0=0.2, omega=0.05, x0=(5.0, 4.0, 3.0)), s=1)
    wl = pi.Workload("adj", 10, 8, 7, 19, "f64", 0.8, 3 / 16, (1e-4, -5e-5, 0.0), bc, (0.03, 0.01, 0.0), sc, 0, 1,
                     6, [body])
    c, w, _ = orc.lattice(19)
    f0 = w[:, None] + pi.pdf_deviation_full(21, 19, wl.n_cells) * 4
    rng = np.random.default_rng(4)
    dB = 0.02 * rng.standard_normal(wl.n_cells)
    weights = np.array([0.0, 0.5, 1.0, 1.0, 1.0, 1.0])
    return wl, f0, dB, weights, rng


BCS = [("periodic",) * 6, ("inlet", "outlet", "wall", "wall", "periodic", "periodic"),
       ("wall", "wall", "inlet", "outlet", "wall", "wall")]


@pytest.mark.parametrize("sc", [1, 2, 3])
@pytest.mark.parametrize("bc", BCS)
def test_adjoint_matches_finite_differences(orc, sc, bc):
    wl, f0, dB, wts, rng = _setup(orc, sc, bc)
    om = wl.bodies[0].motion.omega
    J, gB, gW, gf0 = orc.torque_adjoint(wl, f0, 6, wts, dB=dB, omega_us=om)
    assert abs(J) > 1e-9

    def Jof(dBv=dB, omv=om, f0v=f0):
        return orc.torque_forward(wl, f0v, 6, wts, dB=dBv, omega_us=omv)[0]

    eps = 1e-5
    fdW = (Jof(omv=om + eps) - Jof(omv=om - eps)) / (2 * eps)
    assert abs(fdW - gW) <= 1e-7 * max(abs(fdW), 1e-12) + 1e-13, (fdW, gW)
    v = rng.standard_normal(wl.n_cells)
    fdB = (Jof(dBv=dB + 1e-6 * v) - Jof(dBv=dB - 1e-6 * v)) / 2e-6
    assert abs(fdB - v @ gB) <= 1e-7 * abs(fdB) + 1e-13, (fdB, v @ gB)
    V = rng.standard_normal(f0.shape)
    fdF = (Jof(f0v=f0 + 1e-6 * V) - Jof(f0v=f0 - 1e-6 * V)) / 2e-6
    assert abs(fdF - np.sum(V * gf0)) <= 1e-7 * abs(fdF) + 1e-13, (fdF, np.sum(V * gf0))
