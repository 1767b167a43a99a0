"""Writes adjoint_rotor_128.json: FP64 oracle values of the torque objective
on the 128^3 single-rotor workload (4 blades, radius 40, ~41k triangles, s = 2,
inflow 0.04, periodic y/z, tau 0.8, 800 steps from rest, J = mean axial torque
over the last 200 steps), for the GPU adjoint at full size.

Frozen-B convention: B(t) follows the prescribed motion (Omega = 1e-3) in every
run; the rate enters only the solid velocity.  Recorded:
  J                 at Omega = 1e-3
  dJ/dOmega         central difference, step dW (two runs)
  dJ/dB . v         central difference along v (B_eff = B_map + eps v), where
                    v = 0.1 * standard normal (numpy default_rng(seed)) rounded
                    to float32, on the cells of the box lo..hi (x fastest),
                    zero elsewhere (two runs)
  sum B(t)          of the oracle's mapping at a few steps (B = k/64 exactly,
                    so the sums are exact and must match the GPU mapping)

Calls only the oracle (and the seeded input module).  About 40 minutes on 8
cores: the winding-number voxelisation of the mesh dominates.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as orc  # noqa: E402
import psm_inputs as pi  # noqa: E402

STEPS, WINDOW = 800, 200
DW = 1e-6
EPS = 1e-3
SEED = 128
BOX = ((48, 16, 16), (80, 112, 112))  # lo, hi inclusive: the rotor's swept region


def direction_v(n):
    lo, hi = BOX
    rng = np.random.default_rng(SEED)
    shape = tuple(h - l + 1 for l, h in zip(lo, hi))[::-1]  # (z, y, x)
    vals = (0.1 * rng.standard_normal(shape)).astype(np.float32).astype(np.float64)
    v = np.zeros((n, n, n))
    v[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = vals
    return v.reshape(-1)


def main():
    t0 = time.time()
    orc.build(force=False)
    wl = pi.workload_adjoint_rotor(steps=STEPS)
    om = wl.bodies[0].motion.omega
    w = np.zeros(STEPS)
    w[-WINDOW:] = 1.0 / WINDOW
    geom = orc.OracleGeometry(wl.bodies[0].shape, wl.bodies[0].s)
    print(f"voxelised in {time.time() - t0:.0f} s", flush=True)
    _, ow, _ = orc.lattice(19)
    f0 = np.repeat(ow[:, None], wl.n_cells, axis=1)
    sums = {}
    J0, *_ = orc.torque_forward(wl, f0, STEPS, w, omega_us=om, geom=geom, sums=sums)
    print(f"J = {J0!r} ({time.time() - t0:.0f} s)", flush=True)
    Jp, *_ = orc.torque_forward(wl, f0, STEPS, w, omega_us=om + DW, geom=geom)
    Jm, *_ = orc.torque_forward(wl, f0, STEPS, w, omega_us=om - DW, geom=geom)
    dJdW = (Jp - Jm) / (2 * DW)
    print(f"dJ/dOmega = {dJdW!r} ({time.time() - t0:.0f} s)", flush=True)
    v = direction_v(wl.nx)
    Jbp, *_ = orc.torque_forward(wl, f0, STEPS, w, dB=EPS * v, omega_us=om, geom=geom)
    Jbm, *_ = orc.torque_forward(wl, f0, STEPS, w, dB=-EPS * v, omega_us=om, geom=geom)
    dJdBv = (Jbp - Jbm) / (2 * EPS)
    print(f"dJ/dB.v = {dJdBv!r} ({time.time() - t0:.0f} s)", flush=True)
    rec = {
        "workload": wl.name, "steps": STEPS, "window": WINDOW, "omega": om,
        "J": J0, "dJ_dOmega_fd": dJdW, "fd_step_omega": DW, "J_plus": Jp, "J_minus": Jm,
        "dJ_dB_dot_v_fd": dJdBv, "fd_step_B": EPS, "v_seed": SEED, "v_box_lo": BOX[0], "v_box_hi": BOX[1],
        "v_scale": 0.1, "sum_B": {str(t): sums[t] for t in (0, 1, 400, 799)},
        "oracle": "FP64, two-buffer pull streaming, winding-number voxelisation, frozen B",
    }
    with open(os.path.join(HERE, "adjoint_rotor_128.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
