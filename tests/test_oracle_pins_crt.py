"""Pins for the oracle's two extra integer rings, used by the exact-integer
(several residues, Chinese remaindering) product:

  ring modq   integers mod the prime q = 2^64 - 59
  ring z192   integers as 192-bit two's-complement words, arithmetic mod 2^192
              (exact whenever the result lies in [-2^191, 2^191))

Each pin checks the oracle against a fact that does not come from the oracle:
the multinomial theorem (closed forms), evaluation at points, and a brute-force
dictionary convolution in Python integers.
"""
import math
import random

import numpy as np
import pytest

import oracle
from paper_1303_7425_amd import workloads as W

Q = W.Q64


def test_q_is_prime_and_below_2_64():
    # deterministic Miller-Rabin bases for 64-bit integers
    assert Q == 2 ** 64 - 59
    d, s = Q - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, Q)
        if x in (1, Q - 1):
            continue
        for _ in range(s - 1):
            x = x * x % Q
            if x == Q - 1:
                break
        else:
            pytest.fail("composite")


def multinom(n, e):
    s = sum(e)
    if s > n:
        return 0
    r = math.factorial(n) // math.factorial(n - s)
    for x in e:
        r //= math.factorial(x)
    return r


@pytest.mark.parametrize("n", [4, 9])
def test_q1_dense_closed_form_modq(n):
    f = W.dense_power(n, 4, 16, "modq")
    g = W.add_constant(f, 1)
    hk, hc, _ = oracle.mul(f, g)
    assert hk.size == math.comb(2 * n + 4, 4)
    for e, c in zip(W.unpack(hk, 4, 16).tolist(), hc.tolist()):
        assert c == (multinom(2 * n, e) + multinom(n, e)) % Q


def test_q2_sparse_family_evaluation_modq():
    n = 4
    f = W.with_random_coefs(W.sparse_power(n, "f"), W.rng_for(5), "modq")
    g = W.with_random_coefs(W.sparse_power(n, "g"), W.rng_for(6), "modq")
    hk, hc, _ = oracle.mul(f, g)
    rr = random.Random(11)

    def ev(keys, coefs, a):
        s = 0
        for e, c in zip(W.unpack(keys, 5, 12).tolist(), [int(x) for x in coefs]):
            t = c
            for v in range(5):
                t = t * pow(a[v], e[v], Q) % Q
            s = (s + t) % Q
        return s
    for _ in range(4):
        a = [rr.randrange(Q) for _ in range(5)]
        assert ev(hk, hc, a) == ev(f.keys, f.coefs, a) * ev(g.keys, g.coefs, a) % Q


def brute_dict(fk, fvals, gk, gvals, reduce):
    acc = {}
    for a, x in zip(fk.tolist(), fvals):
        for b, y in zip(gk.tolist(), gvals):
            acc[a + b] = acc.get(a + b, 0) + x * y
    out = sorted((k, reduce(v)) for k, v in acc.items())
    return [(k, v) for k, v in out if v != 0]


@pytest.mark.parametrize("seed", range(4))
def test_q3_brute_force_modq(seed):
    rng = W.rng_for(100 + seed)
    f = W.random_sparse(rng, 40 + 7 * seed, 3, 10, 6, "modq")
    g = W.random_sparse(rng, 25, 3, 10, 6, "modq")
    hk, hc, _ = oracle.mul(f, g)
    want = brute_dict(f.keys, [int(c) for c in f.coefs], g.keys, [int(c) for c in g.coefs], lambda v: v % Q)
    assert [(int(k), int(c)) for k, c in zip(hk, hc)] == want


def test_q4_range_check():
    f = W.dense_power(2, 2, 8, "modq")
    bad = f.coefs.copy()
    bad[0] = np.uint64(Q)
    with pytest.raises(oracle.OracleError):
        oracle.mul_arrays(2, 8, "modq", f.keys, bad, f.keys, f.coefs)


def test_z1_weighted_closed_form_beyond_2_61():
    # f = (3 - 5x + 7y - 11z)^10, so f*f = (3 - 5x + 7y - 11z)^20 with
    # coefficient (20)! / (a! b! c! d!) 3^d (-5)^a 7^b (-11)^c at x^a y^b z^c
    base = [(3, None, 0), (-5, 0, 1), (7, 1, 1), (-11, 2, 1)]
    ex, co = W.multinomial_power(base, 10, 3)
    lay = W.Layout(3, 16, "z192")
    f = W._assemble(ex, co, lay)
    hk, hc, _ = oracle.mul(f, f)
    assert hk.size == math.comb(23, 3)
    got = W.z192_ints(hc)
    assert max(abs(v) for v in got) > 2 ** 61
    for (a, b, c), v in zip(W.unpack(hk, 3, 16).tolist(), got):
        d = 20 - a - b - c
        want = math.factorial(20) // (math.factorial(a) * math.factorial(b) * math.factorial(c) * math.factorial(d))
        want *= 3 ** d * (-5) ** a * 7 ** b * (-11) ** c
        assert v == want


def test_z2_evaluation_exact_at_integer_points():
    rng = W.rng_for(7)
    f = W.random_sparse(rng, 120, 4, 10, 7, "z192")       # 80-bit coefficients
    g = W.random_sparse(rng, 90, 4, 10, 7, "z192")
    hk, hc, _ = oracle.mul(f, g)
    got = W.z192_ints(hc)
    assert max(abs(v) for v in got) > 2 ** 150

    def ev(keys, vals, a):
        return sum(c * math.prod(a[v] ** e[v] for v in range(4)) for e, c in zip(W.unpack(keys, 4, 10).tolist(), vals))
    for a in ([1, 1, 1, 1], [2, -3, 5, 1], [-1, 4, 0, 2]):
        assert ev(hk, got, a) == ev(f.keys, f.exact, a) * ev(g.keys, g.exact, a)


@pytest.mark.parametrize("seed", range(4))
def test_z3_brute_force_and_wraparound(seed):
    rng = W.rng_for(200 + seed)
    f = W.random_sparse(rng, 30, 3, 10, 5, "i64")
    g = W.random_sparse(rng, 20, 3, 10, 5, "i64")
    bits = 60 + 30 * seed         # seed 3: 150-bit operands, products wrap mod 2^192
    fv, gv = W.big_signed(rng, len(f), bits), W.big_signed(rng, len(g), bits)
    hk, hc, _ = oracle.mul_arrays(3, 10, "z192", f.keys, W.z192_words(fv), g.keys, W.z192_words(gv))

    def wrap(v):
        u = v % (1 << 192)
        return u - (1 << 192) if u >> 191 else u
    want = brute_dict(f.keys, fv, g.keys, gv, wrap)
    assert [(int(k), v) for k, v in zip(hk, W.z192_ints(hc))] == want


def test_z4_cancellation_drops_terms():
    # (a + b x)(a - b x) = a^2 - b^2 x^2 with 93-bit a, b: the x term cancels
    a, b = 3 ** 59, 5 ** 40
    lay = W.Layout(1, 16, "z192")
    f = W.Poly(lay, np.array([0, 1], np.uint64), W.z192_words([a, b]), [a, b])
    g = W.Poly(lay, np.array([0, 1], np.uint64), W.z192_words([a, -b]), [a, -b])
    hk, hc, _ = oracle.mul(f, g)
    assert hk.tolist() == [0, 2]
    assert W.z192_ints(hc) == [a * a, -b * b]
