"""Integer coefficients beyond 61 bits on the GPU.

  * ring modq (the prime 2^64 - 59) on every sparse and dense path, bit-exact
    against the oracle;
  * ring z192 (exact integers, three words): the product of the residues mod
    2^64, 2^61 - 1 and 2^64 - 59 recombined by the Chinese remainder theorem,
    checked against the oracle's 192-bit product, against closed forms whose
    coefficients exceed 2^61 (the dense family at n = 20 and the paper's
    Example 1 at n = 40), and for the refusal of products whose coefficient
    bound passes 2^187.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from paper_1303_7425_amd import workloads as W


def _pm():
    from paper_1303_7425_amd import polymul
    return polymul


@pytest.fixture(autouse=True)
def default_tuning():
    pm = _pm()
    pm.set_tuning(-1, -1, True)
    yield
    pm.set_tuning(-1, -1, True)


def gpu(f, g):
    pm = _pm()
    lay = (f.layout.nvars, f.layout.bits, f.layout.ring)
    h = pm.mul(lay, pm.to_device(f), pm.to_device(g))
    assert pm.last_call_status() == 0
    return h.numpy()


def same_as_oracle(f, g, tag):
    print(f"[crt] {tag} ring={f.layout.ring} na={len(f)} nb={len(g)}", flush=True)
    hk, hc = gpu(f, g)
    wk, wc, _ = oracle.mul(f, g)
    assert np.array_equal(hk, wk), tag
    assert np.array_equal(np.asarray(hc).view(np.uint64), np.asarray(wc).view(np.uint64)), tag
    return hk, hc


# ------------------------------------------------------------------ mod q
@pytest.mark.parametrize("mode", ["auto", "pairs", "combine", "intervals", "workitems", "nodense"])
def test_modq_paths_match_oracle(mode):
    pm = _pm()
    combine = {"auto": -1, "pairs": 0, "combine": 1, "intervals": 2, "workitems": 3, "nodense": -1}[mode]
    pm.set_tuning(-1, combine, mode != "nodense")
    rng = W.rng_for(61)
    f, g = W.config3("modq", n=6)
    f, g = W.with_random_coefs(f, rng, "modq"), W.with_random_coefs(g, rng, "modq")
    same_as_oracle(f, g, f"sparse n=6 {mode}")
    d = W.dense_power(7, 4, 16, "modq")
    same_as_oracle(d, W.add_constant(d, 1), f"dense n=7 {mode}")
    same_as_oracle(W.random_sparse(rng, 1000, 6, 10, 15, "modq"), W.random_sparse(rng, 333, 6, 10, 15, "modq"),
                   f"random 6-var {mode}")


def test_modq_near_modulus_coefficients():
    # residues just below q: every product and sum wraps past 2^64 repeatedly
    rng = W.rng_for(62)
    f = W.random_sparse(rng, 700, 4, 10, 7, "modq")
    g = W.random_sparse(rng, 900, 4, 10, 7, "modq")
    f.coefs[:] = W.Q64 - 1 - (f.coefs % np.uint64(1000))
    g.coefs[:] = W.Q64 - 1 - (g.coefs % np.uint64(1000))
    same_as_oracle(f, g, "near q")


# ------------------------------------------------------------------ z192
def test_z192_random_80bit_matches_oracle():
    rng = W.rng_for(63)
    for na, nb in [(1, 1), (1, 300), (257, 129), (1500, 900)]:
        same_as_oracle(W.random_sparse(rng, na, 6, 10, 15, "z192"), W.random_sparse(rng, nb, 6, 10, 15, "z192"),
                       f"z192 random {na}x{nb}")


def test_z192_sparse_family_random_coefficients():
    rng = W.rng_for(64)
    f, g = W.config3("modp", n=8)
    same_as_oracle(W.with_random_coefs(f, rng, "z192", bits=85), W.with_random_coefs(g, rng, "z192", bits=85),
                   "z192 sparse family n=8")


def test_z192_weighted_closed_form():
    # f = (3 - 5x + 7y - 11z)^10: f*f has coefficients up to about 2^94
    base = [(3, None, 0), (-5, 0, 1), (7, 1, 1), (-11, 2, 1)]
    ex, co = W.multinomial_power(base, 10, 3)
    f = W._assemble(ex, co, W.Layout(3, 16, "z192"))
    hk, hc = gpu(f, f)
    assert hk.size == math.comb(23, 3)
    got = W.z192_ints(hc)
    fact = [math.factorial(i) for i in range(21)]
    for (a, b, c), v in zip(W.unpack(hk, 3, 16).tolist(), got):
        d = 20 - a - b - c
        assert v == fact[20] // (fact[a] * fact[b] * fact[c] * fact[d]) * 3 ** d * (-5) ** a * 7 ** b * (-11) ** c


def check_dense_exact(n, hk, hc):
    ex = W.unpack(hk, 4, 16).tolist()
    got = W.z192_ints(hc)
    fact = [math.factorial(i) for i in range(2 * n + 1)]
    for e, v in zip(ex, got):
        s = sum(e)
        den = fact[e[0]] * fact[e[1]] * fact[e[2]] * fact[e[3]]
        want = fact[2 * n] // (den * fact[2 * n - s])
        if s <= n:
            want += fact[n] // (den * fact[n - s])
        assert v == want
    return max(got)


def test_z192_dense_n20_closed_form_beyond_2_61():
    n = 20
    f = W.dense_power(n, 4, 16, "z192")
    hk, hc = gpu(f, W.add_constant(f, 1))
    assert hk.size == math.comb(2 * n + 4, 4)
    assert check_dense_exact(n, hk, hc) > 2 ** 80


def test_z192_example1_n40_exact():
    # the paper's Example 1 with exact integers: 1,929,501 terms, coefficients near 2^172
    n = 40
    f = W.dense_power(n, 4, 16, "z192")
    print(f"[crt] Example 1 exact, {len(f)} x {len(f) + 1} terms", flush=True)
    hk, hc = gpu(f, W.add_constant(f, 1))
    assert hk.size == 1929501
    assert check_dense_exact(n, hk, hc) > 2 ** 170


def test_z192_cancellation_and_empty():
    pm = _pm()
    a, b = 3 ** 57, 5 ** 38              # 91 + 91 + bits(2) = 184 bits: within the bound
    lay = W.Layout(1, 16, "z192")
    f = W.Poly(lay, np.array([0, 1], np.uint64), W.z192_words([a, b]), [a, b])
    g = W.Poly(lay, np.array([0, 1], np.uint64), W.z192_words([a, -b]), [a, -b])
    hk, hc = gpu(f, g)
    assert hk.tolist() == [0, 2] and W.z192_ints(hc) == [a * a, -b * b]
    e = W.Poly(lay, np.zeros(0, np.uint64), np.zeros((0, 3), np.uint64), [])
    h = pm.mul((1, 16, "z192"), pm.to_device(f), pm.to_device(e), out=pm.alloc_out(4, "z192"))
    assert h.n == 0


def test_z192_refuses_beyond_bound():
    pm = _pm()
    lay = W.Layout(2, 8, "z192")
    big = [2 ** 95 - 1, -(2 ** 94)]
    f = W.Poly(lay, np.array([0, 1], np.uint64), W.z192_words(big), big)
    with pytest.raises(pm.PolymulError) as ei:
        pm.mul((2, 8, "z192"), pm.to_device(f), pm.to_device(f))
    assert ei.value.code == pm.PM_EOVERFLOW
    # just inside: 92 + 92 + bits(2) = 186 bits
    ok = [2 ** 92 - 1, -(2 ** 91)]
    f = W.Poly(lay, np.array([0, 1], np.uint64), W.z192_words(ok), ok)
    hk, hc = gpu(f, f)
    assert W.z192_ints(hc) == [ok[0] ** 2, 2 * ok[0] * ok[1], ok[1] ** 2]


def test_z192_rejected_by_batch_entry_points():
    pm = _pm()
    rng = W.rng_for(65)
    f = W.random_sparse(rng, 10, 3, 10, 5, "z192")
    with pytest.raises(pm.PolymulError) as ei:
        pm.mul_batch((3, 10, "z192"), [pm.to_device(f)], [pm.to_device(f)])
    assert ei.value.code == pm.PM_EINVAL
