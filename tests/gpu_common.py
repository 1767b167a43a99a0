"""Helpers shared by the GPU tests (test side only): set up fields through the
C ABI, load seeded states, read results back in the oracle's direction order."""
import numpy as np
import torch

import psm_inputs as pi


def lib_sim():
    from paper_2502_20049_amd import sim

    return sim


def perm_to_oracle(orc, sim, q):
    """idx[j] = library direction with the oracle's velocity j."""
    c, _, _ = sim.lattice(q)
    oc, _, _ = orc.lattice(q)
    lut = {tuple(v): k for k, v in enumerate(c)}
    return np.array([lut[tuple(v)] for v in oc])


def load_random_state(field, seed, amp=8.0):
    sim = lib_sim()
    c, _, _ = sim.lattice(field.q)
    st = pi.random_state_torch(seed, c, field.N, field.pdf.device, field.dtype, amp)
    field.load_pdf_std(st)
    torch.cuda.synchronize()


def oracle_state(orc, wl, seed, amp=8.0):
    oc, ow, _ = orc.lattice(wl.q)
    dev = pi.random_state(seed, oc, wl.n_cells, np.arange(wl.n_cells), amp)
    return (ow[None, :] + dev).T.copy()


def gpu_state_oracle_order(field, orc, sim):
    """f (q, N) in float64 in the oracle's direction order (standard layout:
    call after an even number of steps)."""
    idx = perm_to_oracle(orc, sim, field.q)
    _, ow, _ = orc.lattice(field.q)
    d = field.pdf_std().double().cpu().numpy()
    return ow[:, None] + d[idx]


def gpu_B_per_body(field, nb):
    """Dense (nb, N) solid fractions from the slot fields and body ids."""
    B, meta = field.b_view()
    B = B.double().cpu().numpy()
    meta = meta.cpu().numpy().astype(np.int64)
    out = np.zeros((nb, field.N))
    idx0 = meta & 15
    for b in range(nb):
        m0 = (idx0 == b) & (B[0] > 0)
        out[b, m0] = B[0, m0]
    if B.shape[0] == 2:
        id1 = (meta >> 4) - 1
        for b in range(nb):
            m1 = (id1 == b) & (B[1] > 0)
            out[b, m1] += B[1, m1]
    return out
