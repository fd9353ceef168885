"""Seeded synthetic inputs for the sparse polynomial product.

This module builds operands only.  It holds none of the product's arithmetic:
every polynomial here is produced either by the multinomial theorem applied to
a base polynomial whose non-constant terms are powers of pairwise distinct
variables (so every multinomial index vector maps to its own monomial and no
two terms ever merge), or by drawing random distinct exponent vectors.  Both
the CPU oracle and the GPU path consume these arrays; neither is imported here.

Representation (distributed format, Section 2 of the paper): a polynomial is a
list of terms sorted by a monomial order.  Exponents are packed into one
unsigned 64-bit key (the paper packs exponents into a 64-bit word in its
benchmark section); variable 0 occupies the most significant field, so the
unsigned order of keys is the lexicographic order with x_0 > x_1 > ...

Workloads:
  * dense power   (1 + x_1 + ... + x_v)^n        -- Example 1 family
  * sparse power  (1 + x + y + 2z^2 + 3t^3 + 5u^5)^n and its mirror
                  (1 + u + t + 2z^2 + 3y^3 + 5x^5)^n -- Example 2 family
  * Example 3 operands (1+u^2+v+w^2+x-y^2)^n and (1+u+v^2+w+x^2+y^3)^n + 1
  * random sparse 6-variable operands for the batched workload
  * a Poisson request stream for the serving workload
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

P61 = (1 << 61) - 1
Q64 = (1 << 64) - 59

RING_MODP = "modp"
RING_F64 = "f64"
RING_I64 = "i64"
RING_MODQ = "modq"      # integers mod the prime 2^64 - 59
RING_Z192 = "z192"      # integers as three-word two's-complement values (least significant word first)
RINGS = (RING_MODP, RING_F64, RING_I64, RING_MODQ, RING_Z192)


@dataclass
class Layout:
    """Packing of an exponent vector into a u64 key: nvars fields of `bits`
    bits each, variable 0 in the most significant field."""
    nvars: int
    bits: int
    ring: str

    def shift(self, v: int) -> int:
        return (self.nvars - 1 - v) * self.bits


@dataclass
class Poly:
    """Sorted term list: keys strictly ascending (u64), coefs aligned.

    coefs dtype: uint64 residues in [0, p) for modp, int64 for i64, float64
    for f64.  `exact` optionally keeps the exact integer coefficients (Python
    ints) when the polynomial came from a closed-form generator."""
    layout: Layout
    keys: np.ndarray
    coefs: np.ndarray
    exact: list | None = field(default=None, repr=False)

    def __len__(self) -> int:
        return int(self.keys.shape[0])


def pack(exps: np.ndarray, nvars: int, bits: int) -> np.ndarray:
    """Pack an (n, nvars) array of exponents into u64 keys."""
    exps = np.asarray(exps, dtype=np.uint64).reshape(-1, nvars)
    if exps.size and int(exps.max()) >= (1 << bits):
        raise ValueError("exponent does not fit its field")
    keys = np.zeros(exps.shape[0], dtype=np.uint64)
    for v in range(nvars):
        keys |= exps[:, v] << np.uint64((nvars - 1 - v) * bits)
    return keys


def unpack(keys: np.ndarray, nvars: int, bits: int) -> np.ndarray:
    keys = np.asarray(keys, dtype=np.uint64)
    mask = np.uint64((1 << bits) - 1)
    out = np.empty((keys.shape[0], nvars), dtype=np.int64)
    for v in range(nvars):
        out[:, v] = ((keys >> np.uint64((nvars - 1 - v) * bits)) & mask).astype(np.int64)
    return out


def to_ring(values, ring: str) -> np.ndarray:
    """Map exact integers into the coefficient ring's storage type.
    Negative integers map to p - |v| under mod p (residues in [0, p))."""
    if ring == RING_MODP:
        return np.array([int(v) % P61 for v in values], dtype=np.uint64)
    if ring == RING_I64:
        for v in values:
            if not (-(1 << 63) <= int(v) < (1 << 63)):
                raise OverflowError("coefficient does not fit int64")
        return np.array([int(v) for v in values], dtype=np.int64)
    if ring == RING_F64:
        return np.array([float(v) for v in values], dtype=np.float64)
    if ring == RING_MODQ:
        return np.array([int(v) % Q64 for v in values], dtype=np.uint64)
    if ring == RING_Z192:
        return z192_words(values)
    raise ValueError(ring)


def z192_words(values) -> np.ndarray:
    """Exact integers in [-2^191, 2^191) -> (n, 3) uint64 words of their
    two's-complement form, least significant first."""
    out = np.zeros((len(values), 3), dtype=np.uint64)
    m = (1 << 64) - 1
    for i, v in enumerate(values):
        v = int(v)
        if not (-(1 << 191) <= v < (1 << 191)):
            raise OverflowError("coefficient does not fit 192 bits")
        u = v % (1 << 192)
        out[i] = (u & m, (u >> 64) & m, u >> 128)
    return out


def z192_ints(words: np.ndarray) -> list:
    """(n, 3) uint64 two's-complement words -> exact Python integers."""
    out = []
    for w0, w1, w2 in np.asarray(words, dtype=np.uint64).reshape(-1, 3).tolist():
        u = int(w0) | (int(w1) << 64) | (int(w2) << 128)
        out.append(u - (1 << 192) if u >> 191 else u)
    return out


def _compositions(n: int, m: int):
    """All (k_0..k_{m-1}) with k_i >= 0 and sum n, as an int array."""
    if m == 1:
        return np.array([[n]], dtype=np.int64)
    rows = []
    for k0 in range(n + 1):
        sub = _compositions(n - k0, m - 1)
        rows.append(np.concatenate([np.full((sub.shape[0], 1), k0, dtype=np.int64), sub], axis=1))
    return np.concatenate(rows, axis=0)


def multinomial_power(base, n: int, nvars: int):
    """Terms of (sum_i c_i * x_{v_i}^{p_i})^n by the multinomial theorem.

    `base` lists (coef, var, power); the constant term is (c, None, 0).  The
    non-constant monomials must be powers of pairwise distinct variables, so
    each index vector k yields a distinct exponent sum_i k_i * p_i * e_{v_i}.
    Returns (exponents (N, nvars) int64, exact coefficients list of int)."""
    vars_used = [v for (_, v, _) in base if v is not None]
    if len(set(vars_used)) != len(vars_used):
        raise ValueError("base monomials must use distinct variables")
    m = len(base)
    ks = _compositions(n, m)
    exps = np.zeros((ks.shape[0], nvars), dtype=np.int64)
    for i, (_, v, p) in enumerate(base):
        if v is not None:
            exps[:, v] += ks[:, i] * p
    fact = [math.factorial(i) for i in range(n + 1)]
    pw = [[c ** k for k in range(n + 1)] for (c, _, _) in base]
    coefs = []
    nf = fact[n]
    for row in ks.tolist():
        c = nf
        for i, k in enumerate(row):
            c //= fact[k]
        for i, k in enumerate(row):
            c *= pw[i][k]
        coefs.append(c)
    return exps, coefs


def _assemble(exps, coefs, layout: Layout) -> Poly:
    keys = pack(exps, layout.nvars, layout.bits)
    order = np.argsort(keys, kind="stable")
    keys = keys[order]
    exact = [coefs[i] for i in order.tolist()]
    if keys.size > 1 and not np.all(keys[1:] > keys[:-1]):
        raise AssertionError("generator produced duplicate monomials")
    return Poly(layout, keys, to_ring(exact, layout.ring), exact)


def add_constant(p: Poly, c: int) -> Poly:
    """p + c; the constant term is the smallest key (0) when present."""
    if p.exact is None:
        raise ValueError("needs exact coefficients")
    exact = list(p.exact)
    keys = p.keys.copy()
    if keys.size and int(keys[0]) == 0:
        exact[0] += c
    else:
        keys = np.concatenate([np.zeros(1, dtype=np.uint64), keys])
        exact = [c] + exact
    if exact[0] == 0:
        keys, exact = keys[1:], exact[1:]
    return Poly(p.layout, keys, to_ring(exact, p.layout.ring), exact)


def dense_power(n: int, nvars: int = 4, bits: int = 16, ring: str = RING_MODP) -> Poly:
    """(1 + x_0 + ... + x_{nvars-1})^n; C(n+nvars, nvars) terms."""
    base = [(1, None, 0)] + [(1, v, 1) for v in range(nvars)]
    exps, coefs = multinomial_power(base, n, nvars)
    return _assemble(exps, coefs, Layout(nvars, bits, ring))


# variable indices for the 5-variable sparse family: x, y, z, t, u
X, Y, Z, T, U = range(5)
SPARSE_F_BASE = [(1, None, 0), (1, X, 1), (1, Y, 1), (2, Z, 2), (3, T, 3), (5, U, 5)]
SPARSE_G_BASE = [(1, None, 0), (1, U, 1), (1, T, 1), (2, Z, 2), (3, Y, 3), (5, X, 5)]


def sparse_power(n: int, which: str = "f", bits: int = 12, ring: str = RING_MODP) -> Poly:
    """(1+x+y+2z^2+3t^3+5u^5)^n (which='f') or (1+u+t+2z^2+3y^3+5x^5)^n
    (which='g'); C(n+5, 5) terms each."""
    base = SPARSE_F_BASE if which == "f" else SPARSE_G_BASE
    exps, coefs = multinomial_power(base, n, 5)
    return _assemble(exps, coefs, Layout(5, bits, ring))


# Example 3 variables u, v, w, x, y
EX3_F_BASE = [(1, None, 0), (1, 0, 2), (1, 1, 1), (1, 2, 2), (1, 3, 1), (-1, 4, 2)]
EX3_G_BASE = [(1, None, 0), (1, 0, 1), (1, 1, 2), (1, 2, 1), (1, 3, 2), (1, 4, 3)]


def example3(n: int, bits: int = 12, ring: str = RING_MODP):
    """(1+u^2+v+w^2+x-y^2)^n and (1+u+v^2+w+x^2+y^3)^n + 1."""
    ef, cf = multinomial_power(EX3_F_BASE, n, 5)
    eg, cg = multinomial_power(EX3_G_BASE, n, 5)
    lay = Layout(5, bits, ring)
    return _assemble(ef, cf, lay), add_constant(_assemble(eg, cg, lay), 1)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_pm1(rng: np.random.Generator, n: int) -> np.ndarray:
    """FP64 coefficients uniform in [-1, 1]; an exact 0.0 is redrawn."""
    out = rng.uniform(-1.0, 1.0, size=n)
    bad = out == 0.0
    while bad.any():
        out[bad] = rng.uniform(-1.0, 1.0, size=int(bad.sum()))
        bad = out == 0.0
    return out


def residues(rng: np.random.Generator, n: int) -> np.ndarray:
    """Coefficients mod p drawn uniformly from [1, p)."""
    return rng.integers(1, P61, size=n, dtype=np.uint64)


def big_signed(rng: np.random.Generator, n: int, bits: int) -> list:
    """Exact integers uniform in (-2^bits, 2^bits), zero redrawn."""
    out = []
    while len(out) < n:
        w = rng.integers(0, 1 << 62, size=(n - len(out), (bits + 61) // 62 + 1), dtype=np.int64).tolist()
        for row in w:
            v = 0
            for x in row[1:]:
                v = (v << 62) | int(x)
            v &= (1 << bits) - 1
            if v:
                out.append(-v if row[0] & 1 else v)
    return out


def with_random_coefs(p: Poly, rng: np.random.Generator, ring: str, bits: int = 80) -> Poly:
    """Fresh random coefficients; for z192 exact integers of up to `bits` bits."""
    lay = Layout(p.layout.nvars, p.layout.bits, ring)
    n = len(p)
    if ring == RING_F64:
        c = uniform_pm1(rng, n)
    elif ring == RING_MODP:
        c = residues(rng, n)
    elif ring == RING_MODQ:
        c = rng.integers(1, Q64, size=n, dtype=np.uint64)
    elif ring == RING_Z192:
        ex = big_signed(rng, n, bits)
        return Poly(lay, p.keys.copy(), z192_words(ex), ex)
    else:
        c = rng.integers(-(1 << 20), (1 << 20) + 1, size=n, dtype=np.int64)
    return Poly(lay, p.keys.copy(), c)


def random_sparse(rng: np.random.Generator, n: int, nvars: int = 6, bits: int = 10,
                  max_exp: int = 15, ring: str = RING_MODP) -> Poly:
    """n distinct exponent vectors with entries uniform in 0..max_exp: draw,
    dedupe, top up until n distinct, then sort."""
    if n > (max_exp + 1) ** nvars:
        raise ValueError("more terms than monomials")
    keys = np.zeros(0, dtype=np.uint64)
    while keys.size < n:
        need = n - keys.size
        e = rng.integers(0, max_exp + 1, size=(need + 8, nvars), dtype=np.int64)
        keys = np.unique(np.concatenate([keys, pack(e, nvars, bits)]))
    if keys.size > n:
        keys = np.sort(rng.choice(keys, size=n, replace=False))
    lay = Layout(nvars, bits, ring)
    if ring == RING_F64:
        c = uniform_pm1(rng, n)
    elif ring == RING_MODP:
        c = residues(rng, n)
    elif ring == RING_MODQ:
        c = rng.integers(1, Q64, size=n, dtype=np.uint64)
    elif ring == RING_Z192:
        ex = big_signed(rng, n, 80)
        return Poly(lay, keys, z192_words(ex), ex)
    else:
        c = rng.integers(-(1 << 20), (1 << 20) + 1, size=n, dtype=np.int64)
    return Poly(lay, keys, c)


# ----------------------------------------------------------------------------
# The five workload configurations
# ----------------------------------------------------------------------------

def config1():
    """Dense 4-var, n=10, int64, 16 bits/var: f=(1+x+y+z+t)^10, g=f+1."""
    f = dense_power(10, 4, 16, RING_I64)
    return f, add_constant(f, 1)


def config2(n: int = 20):
    """Dense 4-var, n=20, mod p, 16 bits/var: f=(1+x+y+z+t)^20, g=f+1."""
    f = dense_power(n, 4, 16, RING_MODP)
    return f, add_constant(f, 1)


def config3(ring: str = RING_MODP, n: int = 12, seed: int = 3):
    """Sparse 5-var, n=12, 12 bits/var.  mod p keeps the generator's exact
    coefficients; the FP64 variant replaces them by seeded uniform[-1,1]."""
    f = sparse_power(n, "f", 12, RING_MODP)
    g = sparse_power(n, "g", 12, RING_MODP)
    if ring == RING_MODP:
        return f, g
    rng = rng_for(seed)
    return with_random_coefs(f, rng, ring), with_random_coefs(g, rng, ring)


def config4_sizes(count: int = 4096, seed: int = 4, lo: int = 50, hi: int = 20000):
    """Term counts exp(U(ln lo, ln hi)) for the f and g of each pair."""
    rng = rng_for(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=(count, 2))
    return np.floor(np.exp(u)).astype(np.int64), rng


def config4(ring: str = RING_MODP, count: int = 4096, seed: int = 4, lo: int = 50, hi: int = 20000,
            scale: float = 1.0):
    """Batched: `count` pairs of random sparse 6-var operands, 10 bits/var,
    exponents uniform 0..15.  `scale` shrinks every size (tests use it)."""
    sizes, rng = config4_sizes(count, seed, lo, hi)
    sizes = np.maximum(1, np.floor(sizes * scale)).astype(np.int64)
    pairs = []
    for na, nb in sizes.tolist():
        f = random_sparse(rng, na, 6, 10, 15, ring)
        g = random_sparse(rng, nb, 6, 10, 15, ring)
        pairs.append((f, g))
    return pairs


@dataclass
class Request:
    arrival_s: float
    kind: str          # "small" or "large"
    f: Poly
    g: Poly


def config5_stream(n_requests: int, rate_per_s: float, seed: int = 5, large_frac: float = 0.02,
                   large_n: int = 30, small_range=(6, 12)):
    """Poisson arrivals.  98% small requests: the sparse 5-var pair at power
    k ~ U{small_range} with re-randomised residues; 2% large dense requests
    (1+x+y+z+t)^large_n times itself plus one.  All mod p."""
    rng = rng_for(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps)
    cache = {}
    big_f = dense_power(large_n, 4, 16, RING_MODP)
    big = (big_f, add_constant(big_f, 1))
    out = []
    for i in range(n_requests):
        if rng.uniform() < large_frac:
            out.append(Request(float(t[i]), "large", big[0], big[1]))
            continue
        k = int(rng.integers(small_range[0], small_range[1] + 1))
        if k not in cache:
            cache[k] = (sparse_power(k, "f", 12, RING_MODP), sparse_power(k, "g", 12, RING_MODP))
        f0, g0 = cache[k]
        out.append(Request(float(t[i]), "small",
                           with_random_coefs(f0, rng, RING_MODP), with_random_coefs(g0, rng, RING_MODP)))
    return out
