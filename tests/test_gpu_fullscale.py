"""Full-size products on the GPU checked against closed forms and the oracle.

  * (1+x+y+z+t)^30 * ((1+x+y+z+t)^30 + 1) mod p, the large request of the
    serving mix: all C(64,4) = 635,376 terms against M(60; e) + M(30; e),
    plus evaluation at 16 random points.
  * Example 1 of the paper's benchmark section at n = 40 mod p:
    (1+x+y+z+t)^40 * ((1+x+y+z+t)^40 + 1), 1.84e10 term products; the paper
    reports 1,929,501 result terms, each equal to M(80; e) + M(40; e).
  * Examples 2 and 3 of the paper mod p (2.03e10 and 5.63e10 term
    products, degree boxes of 2.35e10 and 7.36e9 cells): the paper's
    312,855,140 and 144,049,555 result terms, keys ascending, and 202 terms
    each against the definition of the product.
  * The largest pairs of the batched workload recipe (6 variables, 10 bits,
    exponents 0..15, log-uniform sizes in [50, 20000], seed 4), term by term
    against the oracle.

M(n; e) is the multinomial coefficient n! / (e_1! ... e_4! (n - |e|)!), the
coefficient of x^e in (1+x+y+z+t)^n; it is reduced mod p through inverse
factorials (p is a prime larger than n).
"""
import math
import random
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from paper_1303_7425_amd import workloads as W

P = W.P61
MASK31 = (1 << 31) - 1


def mulmod_np(a, b):
    """Elementwise a*b mod 2^61-1 on uint64 arrays of residues (31-bit limbs)."""
    a = a.astype(np.uint64)
    b = b.astype(np.uint64)
    a1, a0 = a >> np.uint64(31), a & np.uint64(MASK31)
    b1, b0 = b >> np.uint64(31), b & np.uint64(MASK31)
    hi = a1 * b1                       # < 2^60, weight 2^62 = 2 (mod p)
    mid = a1 * b0 + a0 * b1            # < 2^62, weight 2^31
    lo = a0 * b0                       # < 2^62
    m_hi, m_lo = mid >> np.uint64(30), mid & np.uint64((1 << 30) - 1)   # mid*2^31 = m_hi*2^61 + m_lo*2^31
    x = np.uint64(2) * hi + m_hi + (m_lo << np.uint64(31))              # < 2^62
    x = (x & np.uint64(P)) + (x >> np.uint64(61))
    x = (x & np.uint64(P)) + (x >> np.uint64(61))
    lo = (lo & np.uint64(P)) + (lo >> np.uint64(61))
    x = x + lo                         # < 2^62 + 2
    x = (x & np.uint64(P)) + (x >> np.uint64(61))
    return np.where(x >= np.uint64(P), x - np.uint64(P), x)


def summod_np(v):
    v = v.astype(np.uint64)
    s = int((v & np.uint64(0xFFFFFFFF)).sum()) + (int((v >> np.uint64(32)).sum()) << 32)
    return s % P


def test_mulmod_np_helper():
    rr = random.Random(7)
    a = [rr.randrange(P) for _ in range(2000)] + [0, 1, P - 1, P - 1]
    b = [rr.randrange(P) for _ in range(2000)] + [P - 1, P - 1, P - 1, 1]
    got = mulmod_np(np.array(a, np.uint64), np.array(b, np.uint64)).tolist()
    assert got == [x * y % P for x, y in zip(a, b)]
    assert summod_np(np.array(a, np.uint64)) == sum(a) % P


def fact_tables(n):
    f = [1] * (n + 1)
    for i in range(1, n + 1):
        f[i] = f[i - 1] * i % P
    inv = [pow(x, P - 2, P) for x in f]
    return np.array(f, np.uint64), np.array(inv, np.uint64)


def multinomial_modp(n, ex, fact, inv):
    """M(n; e) mod p for every row e of ex (|e| <= n assumed where used)."""
    s = ex.sum(axis=1)
    ok = s <= n
    r = np.full(ex.shape[0], int(fact[n]), np.uint64)
    for v in range(ex.shape[1]):
        r = mulmod_np(r, inv[ex[:, v]])
    r = mulmod_np(r, inv[np.where(ok, n - s, 0)])
    return np.where(ok, r, np.uint64(0))


def check_dense_family(n, hk, hc):
    """h = f (f + 1) with f = (1+x+y+z+t)^n: every term M(2n; e) + M(n; e)."""
    ex = W.unpack(hk, 4, 16).astype(np.int64)
    fact, inv = fact_tables(2 * n)
    want = multinomial_modp(2 * n, ex, fact, inv) + multinomial_modp(n, ex, fact, inv)
    want = np.where(want >= np.uint64(P), want - np.uint64(P), want)
    assert np.array_equal(hc.view(np.uint64), want)
    return ex


def gpu_mul(f, g):
    from paper_1303_7425_amd import polymul as pm
    lay = (f.layout.nvars, f.layout.bits, f.layout.ring)
    t = time.perf_counter()
    h = pm.mul(lay, pm.to_device(f), pm.to_device(g))
    hk, hc = h.numpy()
    dt = time.perf_counter() - t
    assert pm.last_call_status() == 0
    return hk, hc, dt


def test_serve_large_request_n30_closed_form_and_evaluation():
    n = 30
    f = W.dense_power(n, 4, 16, "modp")
    g = W.add_constant(f, 1)
    assert len(f) == math.comb(34, 4) == 46376
    print(f"[fullscale] (1+x+y+z+t)^{n} x (same+1) mod p, {len(f) * len(g):.3e} pairs", flush=True)
    hk, hc, dt = gpu_mul(f, g)
    assert hk.size == math.comb(64, 4) == 635376
    assert np.all(hk[1:] > hk[:-1])
    ex = check_dense_family(n, hk, hc)
    # h(a) = f(a) (f(a) + 1) at 16 random points mod p
    rr = random.Random(2)
    for _ in range(16):
        a = [rr.randrange(P) for _ in range(4)]
        v = hc.view(np.uint64)
        for k in range(4):
            pw = np.array([pow(a[k], e, P) for e in range(2 * n + 1)], np.uint64)
            v = mulmod_np(v, pw[ex[:, k]])
        fa = pow((1 + sum(a)) % P, n, P)
        assert summod_np(v) == fa * (fa + 1) % P


def test_example1_n40_term_count_and_closed_form():
    # the paper's Example 1: 1,929,501 result terms
    n = 40
    f = W.dense_power(n, 4, 16, "modp")
    g = W.add_constant(f, 1)
    assert len(f) == math.comb(44, 4) == 135751
    print(f"[fullscale] Example 1 n={n} mod p, {len(f) * len(g):.3e} pairs", flush=True)
    hk, hc, dt = gpu_mul(f, g)
    print(f"[fullscale] Example 1: {hk.size} terms in {dt:.3f} s (including upload and read-back)", flush=True)
    assert hk.size == 1929501 == math.comb(84, 4)
    assert np.all(hk[1:] > hk[:-1])
    check_dense_family(n, hk, hc)


def coefficient_by_definition(f, g, key):
    """Coefficient of monomial `key` in f*g from Section 2's definition: the
    sum of a_i b_j over the pairs with alpha_i + beta_j = key (each alpha_i
    with alpha_i <= key fieldwise names its partner beta_j = key - alpha_i,
    looked up in g's sorted keys), mod p."""
    nv, bits = f.layout.nvars, f.layout.bits
    e = W.unpack(np.array([key], np.uint64), nv, bits)[0].astype(np.int64)
    fa = W.unpack(f.keys, nv, bits).astype(np.int64)
    ok = np.all(fa <= e, axis=1)
    want = W.pack((e - fa[ok]).astype(np.uint64), nv, bits)
    pos = np.searchsorted(g.keys, want)
    pos_c = np.minimum(pos, len(g.keys) - 1)
    hit = g.keys[pos_c] == want
    a = f.coefs[ok][hit]
    b = g.coefs[pos_c[hit]]
    return summod_np(mulmod_np(a, b)) if a.size else 0


def test_example3_n28_term_count_and_sampled_terms():
    # the paper's Example 3: (1+u^2+v+w^2+x-y^2)^28 * ((1+u+v^2+w+x^2+y^3)^28 + 1),
    # 237,336 terms each, 5.63e10 term products into a 7.36e9-cell degree box
    # (64-bit compressed keys); the paper reports 144,049,555 result terms
    from paper_1303_7425_amd import polymul as pm
    f, g = W.example3(28, 12, "modp")
    assert len(f) == len(g) == math.comb(33, 5) == 237336
    lay = (5, 12, "modp")
    print(f"[fullscale] Example 3 n=28 mod p, {len(f) * len(g):.3e} pairs", flush=True)
    import torch
    torch.cuda.empty_cache()
    t = time.perf_counter()
    h = pm.mul(lay, pm.to_device(f), pm.to_device(g), out=pm.alloc_out(150_000_000, "modp"))
    assert pm.last_call_status() == 0
    hk, hc = h.numpy()
    del h
    torch.cuda.empty_cache()
    print(f"[fullscale] Example 3: {hk.size} terms in {time.perf_counter() - t:.3f} s "
          f"(including upload and read-back)", flush=True)
    assert hk.size == 144049555
    assert np.all(hk[1:] > hk[:-1])
    assert np.all(hc != 0) and np.all(hc < np.uint64(P))
    rr = np.random.default_rng(28)
    for k in [0, hk.size - 1] + rr.integers(0, hk.size, 200).tolist():
        assert int(hc[k]) == coefficient_by_definition(f, g, hk[k]), k


def test_example2_n25_term_count_and_sampled_terms():
    # the paper's Example 2: (1+x+y+2z^2+3t^3+5u^5)^25 * (1+u+t+2z^2+3y^3+5x^5)^25,
    # 142,506 terms each, 2.03e10 term products (beyond the sparse paths' 2^32 - 1)
    # into a 2.35e10-cell degree box (188 GB of cells); the paper reports
    # 312,855,140 result terms
    import torch
    from paper_1303_7425_amd import polymul as pm
    torch.cuda.empty_cache()  # earlier tests' cached workspaces
    f, g = W.config3("modp", n=25)
    assert len(f) == len(g) == math.comb(30, 5) == 142506
    lay = (5, 12, "modp")
    print(f"[fullscale] Example 2 n=25 mod p, {len(f) * len(g):.3e} pairs", flush=True)
    t = time.perf_counter()
    h = pm.mul(lay, pm.to_device(f), pm.to_device(g), out=pm.alloc_out(320_000_000, "modp"))
    assert pm.last_call_status() == 0
    hk, hc = h.numpy()
    del h
    torch.cuda.empty_cache()
    print(f"[fullscale] Example 2: {hk.size} terms in {time.perf_counter() - t:.3f} s "
          f"(including upload and read-back)", flush=True)
    assert hk.size == 312855140
    assert np.all(hk[1:] > hk[:-1])
    assert np.all(hc != 0) and np.all(hc < np.uint64(P))
    rr = np.random.default_rng(25)
    for k in [0, hk.size - 1] + rr.integers(0, hk.size, 200).tolist():
        assert int(hc[k]) == coefficient_by_definition(f, g, hk[k]), k


def _config4_largest(k):
    sizes, _ = W.config4_sizes()
    order = np.argsort(sizes[:, 0] * sizes[:, 1])[::-1]
    return [tuple(int(x) for x in sizes[q]) for q in order[:k]]


@pytest.mark.parametrize("rank,ring", [(0, "modp"), (1, "modp"), (0, "f64")])
def test_config4_largest_pairs_vs_oracle(rank, ring):
    from test_gpu_parity import assert_same
    na, nb = _config4_largest(2)[rank]
    rng = W.rng_for(4000 + rank)
    f = W.random_sparse(rng, na, 6, 10, 15, ring)
    g = W.random_sparse(rng, nb, 6, 10, 15, ring)
    print(f"[fullscale] config-4 pair of rank {rank} by size: {na} x {nb} = {na * nb:.3e} pairs, {ring}", flush=True)
    hk, hc, _ = gpu_mul(f, g)
    want = oracle.mul(f, g)
    assert_same((hk, hc), want, ring, f"cfg4 rank {rank}")
