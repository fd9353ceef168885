"""Pins for the CPU oracle: checks against facts fixed by the paper and by
mathematics, never against the oracle's own formula.

  P1 closed form      f*(f+1) = f^2 + f for f = (1+x+y+z+t)^n, so every output
                      coefficient is a sum of two multinomial coefficients and
                      the term count is C(2n+4, 4) (the paper's Example 1 output,
                      1929501 terms, is this count at n = 40).
  P2 evaluation       h(a) = f(a) g(a) mod p at random points, with f(a), g(a)
                      computed from the generating expression by modular powers.
  P3 brute force      dense convolution over exponent vectors in Python ints.
  P4 special cases    cancellation, identities, commutativity, associativity.
  P5 FP64 integers    integer-valued doubles give the int64 result bit for bit.
  P6 FP64 rounding    the double result lies within the recursive-summation
                      error bound of the exact rational sum.
"""
import json
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1303_7425_amd import workloads as W

P = W.P61
HERE = os.path.dirname(os.path.abspath(__file__))


def multinom(n, e):
    s = sum(e)
    if s > n or min(e) < 0:
        return 0
    r = math.factorial(n) // math.factorial(n - s)
    for x in e:
        r //= math.factorial(x)
    return r


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("n,ring", [(2, "i64"), (5, "i64"), (10, "i64"), (6, "modp"), (10, "modp")])
def test_p1_dense_closed_form(n, ring):
    f = W.dense_power(n, 4, 16, ring)
    g = W.add_constant(f, 1)
    hk, hc, _ = oracle.mul(f, g)
    assert len(hk) == math.comb(2 * n + 4, 4)
    exps = W.unpack(hk, 4, 16)
    for e, c in zip(exps.tolist(), hc.tolist()):
        want = multinom(2 * n, e) + multinom(n, e)
        if ring == "modp":
            want %= P
        assert int(c) == want, (e, c, want)


def test_p1_dense_closed_form_3var():
    n = 7
    f = W.dense_power(n, 3, 8, "i64")
    g = W.add_constant(f, 1)
    hk, hc, _ = oracle.mul(f, g)
    assert len(hk) == math.comb(2 * n + 3, 3)
    for e, c in zip(W.unpack(hk, 3, 8).tolist(), hc.tolist()):
        assert int(c) == multinom(2 * n, e) + multinom(n, e)


def test_p1_paper_example1_count_is_closed_form():
    gold = json.load(open(os.path.join(HERE, "golden", "paper_counts.json")))
    # Example 1: (1+x+y+z+t)^40 has C(44,4) terms; f1*(f1+1) has C(84,4).
    assert math.comb(40 + 4, 4) == gold["example1"]["input_terms"]
    assert math.comb(80 + 4, 4) == gold["example1"]["output_terms"]


# ---------------------------------------------------------------- P2
def eval_terms(keys, coefs, nvars, bits, point):
    """sum c * prod a_v^{e_v} mod p, with Python ints."""
    exps = W.unpack(keys, nvars, bits)
    maxe = exps.max(axis=0) if exps.size else np.zeros(nvars, dtype=np.int64)
    pw = []
    for v in range(nvars):
        t = [1]
        for _ in range(int(maxe[v])):
            t.append(t[-1] * point[v] % P)
        pw.append(t)
    s = 0
    for e, c in zip(exps.tolist(), coefs.tolist()):
        m = int(c) % P
        for v in range(nvars):
            m = m * pw[v][e[v]] % P
        s = (s + m) % P
    return s


def base_value(base, point):
    s = 0
    for c, v, p in base:
        s += c * (1 if v is None else pow(point[v], p, P))
    return s % P


@pytest.mark.parametrize("n", [4, 7])
def test_p2_sparse_family_evaluation(n):
    f = W.sparse_power(n, "f", 12, "modp")
    g = W.sparse_power(n, "g", 12, "modp")
    hk, hc, _ = oracle.mul(f, g)
    rng = random.Random(2)
    for _ in range(6):
        a = [rng.randrange(P) for _ in range(5)]
        fa = pow(base_value(W.SPARSE_F_BASE, a), n, P)
        ga = pow(base_value(W.SPARSE_G_BASE, a), n, P)
        assert eval_terms(hk, hc, 5, 12, a) == fa * ga % P


def test_p2_dense_evaluation():
    n = 8
    f = W.dense_power(n, 4, 16, "modp")
    g = W.add_constant(f, 1)
    hk, hc, _ = oracle.mul(f, g)
    rng = random.Random(2)
    for _ in range(16):
        a = [rng.randrange(P) for _ in range(4)]
        fa = pow((1 + sum(a)) % P, n, P)
        assert eval_terms(hk, hc, 4, 16, a) == fa * ((fa + 1) % P) % P


def test_p2_example3_small_power_evaluation():
    # Example 3 family (negative coefficient -y^2 maps to p - 1), small power.
    n = 4
    f, g = W.example3(n, 12, "modp")
    hk, hc, _ = oracle.mul(f, g)
    rng = random.Random(2)
    for _ in range(6):
        a = [rng.randrange(P) for _ in range(5)]
        fa = pow(base_value(W.EX3_F_BASE, a), n, P)
        ga = (pow(base_value(W.EX3_G_BASE, a), n, P) + 1) % P
        assert eval_terms(hk, hc, 5, 12, a) == fa * ga % P


def test_p2_random_sparse_6var_evaluation():
    rng = W.rng_for(11)
    f = W.random_sparse(rng, 300, 6, 10, 15, "modp")
    g = W.random_sparse(rng, 200, 6, 10, 15, "modp")
    hk, hc, _ = oracle.mul(f, g)
    r = random.Random(5)
    for _ in range(4):
        a = [r.randrange(P) for _ in range(6)]
        assert eval_terms(hk, hc, 6, 10, a) == \
            eval_terms(f.keys, f.coefs, 6, 10, a) * eval_terms(g.keys, g.coefs, 6, 10, a) % P


# ---------------------------------------------------------------- P3
def brute(fe, fc, ge, gc, nvars):
    """Dense convolution over exponent vectors (no packed keys, no hashing):
    H[e] = sum over f-box cells a of F[a] * G[e - a]."""
    F = {tuple(e): c for e, c in zip(fe, fc)}
    G = {tuple(e): c for e, c in zip(ge, gc)}
    if not F or not G:
        return {}
    fmax = [max(e[v] for e in F) for v in range(nvars)]
    gmax = [max(e[v] for e in G) for v in range(nvars)]
    import itertools
    H = {}
    for e in itertools.product(*[range(fmax[v] + gmax[v] + 1) for v in range(nvars)]):
        s = 0
        for a in itertools.product(*[range(min(e[v], fmax[v]) + 1) for v in range(nvars)]):
            fa = F.get(a)
            if fa is None:
                continue
            b = tuple(e[v] - a[v] for v in range(nvars))
            gb = G.get(b)
            if gb is not None:
                s += fa * gb
        if s != 0:
            H[e] = s
    return H


def rand_poly(rng, nvars, maxdeg, nterms, lo=-9, hi=9):
    import itertools
    cells = list(itertools.product(*[range(maxdeg + 1)] * nvars))
    rng.shuffle(cells)
    out = []
    for e in cells[:nterms]:
        c = 0
        while c == 0:
            c = rng.randint(lo, hi)
        out.append((e, c))
    return out


def to_poly(terms, nvars, bits, ring):
    lay = W.Layout(nvars, bits, ring)
    if not terms:
        return W.Poly(lay, np.zeros(0, dtype=np.uint64), np.zeros(0, dtype=oracle.COEF_DTYPE[ring]))
    exps = np.array([t[0] for t in terms], dtype=np.int64).reshape(-1, nvars)
    keys = W.pack(exps, nvars, bits)
    order = np.argsort(keys)
    cs = [terms[i][1] for i in order.tolist()]
    return W.Poly(lay, keys[order], W.to_ring(cs, ring), cs)


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("ring", ["i64", "modp", "f64"])
def test_p3_brute_force_random(seed, ring):
    rng = random.Random(1000 + seed)
    nvars = rng.randint(1, 3)
    maxdeg = rng.randint(0, 5)
    ncell = (maxdeg + 1) ** nvars
    ft = rand_poly(rng, nvars, maxdeg, rng.randint(1, ncell))
    gt = rand_poly(rng, nvars, maxdeg, rng.randint(1, ncell))
    want = brute([t[0] for t in ft], [t[1] for t in ft], [t[0] for t in gt], [t[1] for t in gt], nvars)
    if ring == "modp":
        want = {e: c % P for e, c in want.items() if c % P}
    bits = 5
    f, g = to_poly(ft, nvars, bits, ring), to_poly(gt, nvars, bits, ring)
    hk, hc, _ = oracle.mul(f, g)
    got = {tuple(e): (int(c) if ring != "f64" else c) for e, c in zip(W.unpack(hk, nvars, bits).tolist(), hc.tolist())}
    assert got == want
    assert np.all(hk[1:] > hk[:-1])


@pytest.mark.parametrize("ring", ["i64", "modp", "f64"])
def test_p3_edge_cases(ring):
    x = ((1, 0), 3)
    y = ((0, 1), -2)
    one = ((0, 0), 1)
    cases = [
        ([], [x, y]),                    # empty f
        ([x, y], []),                    # empty g
        ([x], [y]),                      # one term each
        ([one], [x, y]),                 # constant
        ([((2, 3), 5)], [x, y, one]),    # pure monomial shifts keys
        ([x, y, one], [x, y, one]),
    ]
    for ft, gt in cases:
        want = brute([t[0] for t in ft], [t[1] for t in ft], [t[0] for t in gt], [t[1] for t in gt], 2)
        if ring == "modp":
            want = {e: c % P for e, c in want.items() if c % P}
        hk, hc, _ = oracle.mul(to_poly(ft, 2, 6, ring), to_poly(gt, 2, 6, ring))
        got = {tuple(e): (int(c) if ring != "f64" else c) for e, c in zip(W.unpack(hk, 2, 6).tolist(), hc.tolist())}
        assert got == want


# ---------------------------------------------------------------- P4
def poly_from(terms, nvars=2, bits=8, ring="i64"):
    return to_poly(terms, nvars, bits, ring)


@pytest.mark.parametrize("ring", ["i64", "modp", "f64"])
def test_p4_difference_of_squares_drops_cross_term(ring):
    f = poly_from([((1, 0), 1), ((0, 1), 1)], ring=ring)          # x + y
    g = poly_from([((1, 0), 1), ((0, 1), -1)], ring=ring)         # x - y
    hk, hc, _ = oracle.mul(f, g)
    got = dict(zip(map(tuple, W.unpack(hk, 2, 8).tolist()), hc.tolist()))
    neg1 = P - 1 if ring == "modp" else -1
    assert got == {(2, 0): 1, (0, 2): neg1}


def test_p4_modp_wraparound():
    f = poly_from([((0, 0), 1), ((1, 0), 1)], ring="modp")        # x + 1
    g = poly_from([((0, 0), P - 1), ((1, 0), 1)], ring="modp")    # x + p - 1
    hk, hc, _ = oracle.mul(f, g)
    got = dict(zip(map(tuple, W.unpack(hk, 2, 8).tolist()), [int(c) for c in hc]))
    assert got == {(0, 0): P - 1, (2, 0): 1}                      # x^2 + (p - 1)
    # (p-1)^2 = 1 mod p on a single pair
    f = poly_from([((1, 0), P - 1)], ring="modp")
    g = poly_from([((0, 1), P - 1)], ring="modp")
    hk, hc, _ = oracle.mul(f, g)
    assert hc.tolist() == [1]


def add_modp(a, b):
    """Sum of two sorted term lists mod p (test helper)."""
    d = {}
    for k, c in zip(a[0].tolist(), a[1].tolist()):
        d[k] = (d.get(k, 0) + int(c)) % P
    for k, c in zip(b[0].tolist(), b[1].tolist()):
        d[k] = (d.get(k, 0) + int(c)) % P
    ks = sorted(k for k, v in d.items() if v)
    return np.array(ks, dtype=np.uint64), np.array([d[k] for k in ks], dtype=np.uint64)


def test_p4_identities_modp():
    rng = W.rng_for(7)
    f = W.random_sparse(rng, 40, 3, 8, 7, "modp")
    g = W.random_sparse(rng, 35, 3, 8, 7, "modp")
    k = W.random_sparse(rng, 30, 3, 8, 7, "modp")
    one = W.Poly(f.layout, np.zeros(1, dtype=np.uint64), np.ones(1, dtype=np.uint64))
    # f * 1 = f
    hk, hc, _ = oracle.mul(f, one)
    assert np.array_equal(hk, f.keys) and np.array_equal(hc, f.coefs)
    # commutativity, bit-exact
    a = oracle.mul(f, g)
    b = oracle.mul(g, f)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # associativity (f g) k = f (g k)
    fg = W.Poly(f.layout, a[0], a[1])
    gk = oracle.mul(g, k)
    lhs = oracle.mul(fg, k)
    rhs = oracle.mul(f, W.Poly(f.layout, gk[0], gk[1]))
    assert np.array_equal(lhs[0], rhs[0]) and np.array_equal(lhs[1], rhs[1])
    # distributivity f (g + k) = f g + f k
    s = add_modp((g.keys, g.coefs), (k.keys, k.coefs))
    lhs = oracle.mul(f, W.Poly(f.layout, s[0], s[1]))
    fk = oracle.mul(f, k)
    rhs = add_modp((a[0], a[1]), (fk[0], fk[1]))
    assert np.array_equal(lhs[0], rhs[0]) and np.array_equal(lhs[1], rhs[1])


# ---------------------------------------------------------------- P5
def test_p5_integer_valued_f64_equals_i64():
    rng = W.rng_for(9)
    fi = W.random_sparse(rng, 500, 6, 10, 15, "i64")
    gi = W.random_sparse(rng, 400, 6, 10, 15, "i64")
    # coefficients in [-2^20, 2^20]: every partial sum stays below 2^53
    a = oracle.mul(fi, gi)
    ff = W.Poly(W.Layout(6, 10, "f64"), fi.keys, fi.coefs.astype(np.float64))
    gf = W.Poly(W.Layout(6, 10, "f64"), gi.keys, gi.coefs.astype(np.float64))
    b = oracle.mul(ff, gf)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1].astype(np.float64), b[1])


def test_p5_dense_integer_f64():
    f = W.dense_power(6, 4, 16, "f64")
    g = W.add_constant(f, 1)
    fi = W.dense_power(6, 4, 16, "i64")
    gi = W.add_constant(fi, 1)
    a, b = oracle.mul(fi, gi), oracle.mul(f, g)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1].astype(np.float64), b[1])


# ---------------------------------------------------------------- P6
def test_p6_f64_within_recursive_sum_bound():
    rng = W.rng_for(3)
    f = W.random_sparse(rng, 120, 3, 8, 6, "f64")
    g = W.random_sparse(rng, 110, 3, 8, 6, "f64")
    hk, hc, ha = oracle.mul(f, g)
    exact, mult = {}, {}
    for i, (ka, ca) in enumerate(zip(f.keys.tolist(), f.coefs.tolist())):
        for kb, cb in zip(g.keys.tolist(), g.coefs.tolist()):
            k = ka + kb
            exact[k] = exact.get(k, Fraction(0)) + Fraction(ca) * Fraction(cb)
            mult[k] = mult.get(k, 0) + 1
    u = 2.0 ** -53
    got = dict(zip(hk.tolist(), hc.tolist()))
    absum = dict(zip(hk.tolist(), ha.tolist()))
    for k, e in exact.items():
        v = got.get(k, 0.0)
        if k in absum:
            A = absum[k]
            # (m+1) u A bounds the error of m rounded products summed recursively
            assert abs(Fraction(v) - e) <= Fraction((mult[k] + 1) * u) * Fraction(A) * (1 + 1e-9), k
        else:
            assert e == 0 or abs(float(e)) < 1e-300
    # A(k) is at least |h(k)| and equals it for single-contribution monomials
    for k, v in got.items():
        assert absum[k] >= abs(v)
        if mult[k] == 1:
            assert absum[k] == abs(v)


# ---------------------------------------------------------------- validation
def test_validation_codes():
    lay = (2, 8, "i64")
    k = np.array([1, 2], dtype=np.uint64)
    c = np.array([1, 1], dtype=np.int64)
    assert oracle.validate(*lay, k, c, k, c) == oracle.OK
    assert oracle.validate(*lay, k[::-1], c, k, c) == oracle.EUNSORTED
    assert oracle.validate(*lay, np.array([1, 1], dtype=np.uint64), c, k, c) == oracle.EUNSORTED
    big = np.array([200], dtype=np.uint64)       # field value 200 in the low field
    assert oracle.validate(*lay, big, c[:1], big, c[:1]) == oracle.EOVERFLOW
    assert oracle.validate(*lay, np.array([1 << 20], dtype=np.uint64), c[:1], k, c) == oracle.EINVAL
    assert oracle.validate(9, 8, "i64", k, c, k, c) == oracle.EINVAL
    r = np.array([P, 1], dtype=np.uint64)
    assert oracle.validate(2, 8, "modp", k, r, k, r) == oracle.ERANGE
    nan = np.array([np.nan, 1.0])
    assert oracle.validate(2, 8, "f64", k, nan, k, nan) == oracle.ERANGE


def test_int64_overflow_reported():
    f = poly_from([((1, 0), 1 << 62)], ring="i64")
    g = poly_from([((0, 1), 4)], ring="i64")
    with pytest.raises(oracle.OracleError) as e:
        oracle.mul(f, g)
    assert e.value.code == oracle.EINT64
