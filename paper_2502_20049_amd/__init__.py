"""PSM lattice Boltzmann hot path for MI355X (gfx950).

The compute path is ``libpsm.so`` (hand-written HIP kernels behind a C ABI,
``include/psm.h``).  ``_capi`` binds its entry points under the same names;
``sim`` drives them with torch-owned device memory and streams.  Importing
``_capi`` fails loudly if the library has not been built.
"""
__all__ = ["build"]


def build(verbose: bool = False) -> str:
    from .build import build as _b

    return _b(verbose=verbose)
