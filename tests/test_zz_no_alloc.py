"""pdf_field_create_noalloc (the library's static work area) against
pdf_field_create (a caller work buffer), through the C ABI.

Both handles run the same kernels, so every output must match bit for bit:
PDFs, solid fractions and body ids, per-step force/torque, FP64 mass and the
error flags.  Two creations in a row, the second on a smaller lattice, so the
second one starts from what the first left in the static array.  Also: an
earlier field on the static area is refused once a newer one has claimed it,
and psm_field_reset claims it back.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import psm_inputs as pi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sim():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2502_20049_amd import sim as s

    return s


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bodies(scale):
    return [pi.Body(pi.Shape("ellipsoid", (9.0 * scale, 5.0 * scale, 4.0 * scale)),
                    pi.Motion(axis=(0.0, 0.6, 0.8), theta0=0.3, omega=0.05, x0=(31.0 * scale, 11.0 * scale, 9.0 * scale)),
                    s=3),
            pi.Body(pi.Shape("ellipsoid", (4.0 * scale, 4.0 * scale, 3.0 * scale)),
                    pi.Motion(axis=(0, 0, 1), omega=-0.1, x0=(52.0 * scale, 12.0 * scale, 8.0 * scale),
                              v=(0.2, 0.0, 0.0)), s=2)]


CASES = [
    # (name, nx, ny, nz, q, storage, slots, max_bodies, scale, steps)
    ("large_q19_f32", 96, 40, 24, 19, "f32", 2, 8, 1.0, 6),
    ("small_q27_f16", 48, 20, 16, 27, "f16", 1, 2, 0.5, 4),
]


def _workload(name, nx, ny, nz, q, storage, slots, scale):
    return pi.Workload(name, nx, ny, nz, q, storage, 0.8, 3 / 16, (0, 0, 0),
                       ("inlet", "outlet", "wall", "wall", "wall", "wall"), (0.04, 0.01, -0.02), 1, 0, slots, 2,
                       _bodies(scale))


def _run(sim, wl, max_bodies, steps, noalloc, seed):
    import torch

    from paper_2502_20049_amd import _capi as capi

    f = sim.Field(wl, max_bodies=max_bodies, noalloc=noalloc)
    c, _, _ = sim.lattice(wl.q)
    f.pdf_view().copy_(pi.random_state_torch(seed, c, f.N, f.pdf.device, f.dtype, 8.0))
    fts, masses = [], []
    ft = torch.zeros((len(wl.bodies), 6), dtype=torch.float64, device=f.pdf.device)
    for t in range(steps):
        f.step(t, ft=ft)
        fts.append(ft.clone())
        masses.append(f.mass(t + 1))
    torch.cuda.synchronize()
    B, meta = f.b_view()
    out = {"pdf": f.pdf_view().clone().cpu().numpy(), "B": B.clone().cpu().numpy(), "meta": meta.clone().cpu().numpy(),
           "ft": torch.stack(fts).cpu().numpy(), "mass": torch.cat(masses).cpu().numpy(),
           "flags": f.error_flags().cpu().numpy()}
    assert f.work is None if noalloc else f.work is not None
    return f, out, capi


def test_noalloc_field_matches_caller_work_buffer(sim):
    import torch

    torch.cuda.set_device(0)
    prev = None
    for k, (name, nx, ny, nz, q, storage, slots, mb, scale, steps) in enumerate(CASES):
        _say(f"no-alloc case {name}: {nx}x{ny}x{nz} D3Q{q} {storage}, slots {slots}, max_bodies {mb}, {steps} steps")
        wl = _workload(name, nx, ny, nz, q, storage, slots, scale)
        f_ref, ref, capi = _run(sim, wl, mb, steps, noalloc=False, seed=11 + k)
        f_st, got, _ = _run(sim, wl, mb, steps, noalloc=True, seed=11 + k)
        assert np.abs(ref["ft"]).max() > 0 and np.count_nonzero(ref["B"]) > 0
        for key in ("pdf", "B", "meta", "ft", "mass", "flags"):
            a, b = ref[key], got[key]
            assert a.shape == b.shape, key
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"{name}: {key} differs"
        _say(f"  {name}: bitwise equal ({ref['pdf'].size} PDF values, ft max {np.abs(ref['ft']).max():.3e})")
        if prev is not None:
            # the earlier static-area field lost the array to this one
            out = torch.zeros(4, dtype=torch.int32, device="cuda")
            rc = capi.lib.psm_error_flags(prev.handle, C.c_void_p(out.data_ptr()), sim._stream())
            assert rc == capi.PSM_EINVAL and "claimed" in capi.last_error()
            prev.reset()  # claims it back
            prev.error_flags()
            f_st.reset()
        prev = f_st
        del f_ref
    torch.cuda.synchronize()
