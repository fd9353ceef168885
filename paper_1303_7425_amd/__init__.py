"""MI355X-native sparse multivariate polynomial multiplication.

The product h = f * g of two polynomials in distributed format (sorted term
arrays with packed 64-bit exponent keys) runs in hand-written HIP kernels for
gfx950 behind a C ABI (`include/polymul.h`).  `polymul` is the thin ctypes
binding; `workloads` builds seeded synthetic operands.  Submodules are
imported lazily so that the input generators can be used without a GPU.
"""
__all__ = ["polymul", "workloads"]
