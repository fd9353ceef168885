"""GPU path vs the CPU oracle on the same seeded inputs, through the C ABI.

Bar: mod p and int64 bit-exact (keys, coefficients, term count).  FP64: keys
identical and |h_gpu - h_oracle| <= 1e-13 * A(k) with A(k) = sum |fl(a_i b_j)|
over the union of keys; in addition the GPU sums each monomial's products in
the oracle's row-major order, so the coefficients are compared bit for bit.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from paper_1303_7425_amd import workloads as W

P = W.P61


def _pm():
    from paper_1303_7425_amd import polymul
    return polymul


def gpu_mul(f, g, ws=None):
    pm = _pm()
    lay = (f.layout.nvars, f.layout.bits, f.layout.ring)
    h = pm.mul(lay, pm.to_device(f), pm.to_device(g), workspace=ws)
    assert pm.last_call_status() == 0
    return h.numpy()


def assert_same(got, want, ring, tag=""):
    gk, gc = got
    wk, wc, wa = want
    if ring != "f64":
        assert gk.shape == wk.shape, (tag, gk.shape, wk.shape)
        assert np.array_equal(gk, wk), tag
        assert np.array_equal(gc.view(np.uint64), wc.view(np.uint64)), tag
        return
    # FP64: union of keys, missing = 0
    keys = np.union1d(gk, wk)
    gv = np.zeros(keys.size)
    wv = np.zeros(keys.size)
    av = np.zeros(keys.size)
    gv[np.searchsorted(keys, gk)] = gc
    wv[np.searchsorted(keys, wk)] = wc
    av[np.searchsorted(keys, wk)] = wa
    # a key emitted by the GPU must have contributing products: the oracle
    # keeps all keys with a non-zero sum, and a zero sum on one side only is
    # within tolerance when A(k) is large enough
    err = np.abs(gv - wv)
    assert np.all(err <= 1e-13 * av), (tag, float(err.max()))
    # stronger: row-major summation order on both sides -> identical bits
    assert np.array_equal(gk, wk), tag
    assert np.array_equal(gc.view(np.uint64), wc.view(np.uint64)), tag


def check(f, g, tag=""):
    print(f"[parity] {tag} ring={f.layout.ring} na={len(f)} nb={len(g)}", flush=True)
    want = oracle.mul(f, g)
    got = gpu_mul(f, g)
    assert_same(got, want, f.layout.ring, tag)


@pytest.fixture(autouse=True)
def default_tuning():
    pm = _pm()
    pm.set_tuning(-1, -1, True)
    yield
    pm.set_tuning(-1, -1, True)


# ------------------------------------------------------------- small configs
def test_config1_dense_int64():
    f, g = W.config1()
    check(f, g, "cfg1")


@pytest.mark.parametrize("n", [3, 8])
def test_dense_modp_small(n):
    check(*W.config2(n), f"dense n={n}")


@pytest.mark.parametrize("n", [2, 6])
@pytest.mark.parametrize("ring", ["modp", "f64"])
def test_sparse_family_small(n, ring):
    f = W.sparse_power(n, "f", 12, "modp")
    g = W.sparse_power(n, "g", 12, "modp")
    if ring == "f64":
        rng = W.rng_for(3)
        f, g = W.with_random_coefs(f, rng, "f64"), W.with_random_coefs(g, rng, "f64")
    check(f, g, f"sparse n={n}")


@pytest.mark.parametrize("ring", ["modp", "f64", "i64"])
@pytest.mark.parametrize("na,nb", [(1, 1), (1, 500), (33, 70), (257, 129), (1000, 3000)])
def test_random_6var_ragged(ring, na, nb):
    rng = W.rng_for(100 + na + nb)
    f = W.random_sparse(rng, na, 6, 10, 15, ring)
    g = W.random_sparse(rng, nb, 6, 10, 15, ring)
    check(f, g, f"rand {na}x{nb}")


@pytest.mark.parametrize("digits", [0, 1])
@pytest.mark.parametrize("ring", ["modp", "f64"])
def test_radix_digit_schedules_same_result(ring, digits):
    """Both digit schedules (8-bit digits, or balanced widths 8, 8, 7, 7 over
    the 30 significant bits of this product's keys) give the oracle's result."""
    pm = _pm()
    f, g = W.config3(ring, n=8)
    pm.set_radix(digits)
    try:
        check(f, g, f"digits={digits}")
    finally:
        pm.set_radix(-1)


@pytest.mark.parametrize("digits", [0, 1])
@pytest.mark.parametrize("ring", ["modp", "f64"])
def test_generated_pass_counts_with_narrow_digits(ring, digits):
    """Long rows of g (1089 terms) in a small degree box (11 key bits, two
    radix passes of 6 and 5 bits when balanced): the first pass counts whole
    rows from g's rotated digit histogram and partial rows item by item."""
    pm = _pm()
    rng = W.rng_for(57)
    lay = W.Layout(2, 8, ring)
    ge = np.array([(a, b) for a in range(33) for b in range(33)], dtype=np.int64)
    fe = np.unique(rng.integers(0, 12, size=(40, 2)), axis=0)[:20]
    coef = {"modp": lambda n: W.residues(rng, n), "f64": lambda n: W.uniform_pm1(rng, n)}[ring]
    g = W.Poly(lay, W.pack(ge, 2, 8), coef(len(ge)))
    f = W.Poly(lay, W.pack(fe, 2, 8), coef(len(fe)))
    pm.set_tuning(-1, -1, False)  # keep it off the degree-box path
    pm.set_radix(digits)
    try:
        check(f, g, f"narrow digits={digits}")
    finally:
        pm.set_radix(-1)


@pytest.mark.parametrize("ring", ["modp", "f64"])
def test_operand_keys_beyond_radix_lds_copy(ring):
    """14,000 operand terms (56 KB of compressed keys): the digit counts copy
    them to LDS, the radix passes regenerate keys through the vector cache."""
    rng = W.rng_for(91)
    f = W.random_sparse(rng, 13000, 6, 10, 15, ring)
    g = W.random_sparse(rng, 1000, 6, 10, 15, ring)
    check(f, g, f"keys beyond radix LDS ({ring})")


@pytest.mark.parametrize("mode", ["auto", "pairs", "combine", "intervals", "nodense", "nodense_combine",
                                  "nodense_intervals", "tile1", "tile2"])
def test_tuning_modes_same_result(mode):
    pm = _pm()
    if mode == "pairs":
        pm.set_tuning(-1, 0, True)
    elif mode == "combine":
        pm.set_tuning(-1, 1, True)
    elif mode == "nodense":
        pm.set_tuning(-1, 0, False)
    elif mode == "nodense_combine":
        pm.set_tuning(-1, 1, False)
    elif mode == "intervals":
        pm.set_tuning(-1, 2, True)
    elif mode == "nodense_intervals":
        pm.set_tuning(-1, 2, False)
    elif mode == "tile1":
        pm.set_tuning(1, -1, True)
    elif mode == "tile2":
        pm.set_tuning(2, -1, True)
    for n in (5, 9):
        check(*W.config2(n), f"dense n={n} {mode}")
    check(W.sparse_power(5, "f", 12, "modp"), W.sparse_power(5, "g", 12, "modp"), f"sparse {mode}")
    rng = W.rng_for(8)
    check(W.random_sparse(rng, 700, 6, 10, 15, "i64"), W.random_sparse(rng, 900, 6, 10, 15, "i64"), f"i64 {mode}")


# ------------------------------------------------------------- edge cases
def _poly(terms, nvars, bits, ring):
    lay = W.Layout(nvars, bits, ring)
    if not terms:
        dt = {"f64": np.float64, "i64": np.int64, "modp": np.uint64}[ring]
        return W.Poly(lay, np.zeros(0, dtype=np.uint64), np.zeros(0, dtype=dt))
    exps = np.array([t[0] for t in terms], dtype=np.int64).reshape(-1, nvars)
    keys = W.pack(exps, nvars, bits)
    o = np.argsort(keys)
    return W.Poly(lay, keys[o], W.to_ring([terms[i][1] for i in o.tolist()], ring))


@pytest.mark.parametrize("ring", ["modp", "f64", "i64"])
def test_edge_cases(ring):
    x = ((1, 0), 3)
    y = ((0, 1), -2)
    one = ((0, 0), 1)
    cases = [([], [x, y]), ([x, y], []), ([], []), ([x], [y]), ([one], [x, y]), ([((2, 3), 5)], [x, y, one]),
             ([((1, 0), 1), ((0, 1), 1)], [((1, 0), 1), ((0, 1), -1)])]
    for i, (ft, gt) in enumerate(cases):
        check(_poly(ft, 2, 8, ring), _poly(gt, 2, 8, ring), f"edge{i}")


def test_total_cancellation_gives_empty():
    # (x + y) * (x - y) with the square terms removed from f: x*(x-y) + y*(x-y) ... use
    # f = x - y and g = 0 coefficient list: every product cancels pairwise
    f = _poly([((1, 0), 1), ((0, 1), 1)], 2, 8, "modp")
    g = _poly([((1, 1), 1)], 2, 8, "modp")
    g.coefs[:] = 0
    hk, hc = gpu_mul(f, g)
    assert hk.size == 0


def _cancelling_pair(ring, n=1500, seed=31):
    """f = p + q and g = p - q with p in x0..x2 and q in x3..x5 (disjoint
    supports, no constant term): f*g = p^2 - q^2, and each of the n*n cross
    monomials x^(a_i + b_j) gets exactly p_i*q_j - q_j*p_i = 0, which is an
    exact zero in every ring (FP64 included: both products round the same)."""
    rng = W.rng_for(seed)
    lay = W.Layout(6, 10, ring)

    def embed(part, lo):
        e = W.unpack(part.keys, 3, 10)
        e[:, 0] += 1
        full = np.zeros((len(part), 6), dtype=np.int64)
        full[:, lo:lo + 3] = e
        return W.pack(full, 6, 10)

    p = W.random_sparse(rng, n, 3, 10, 15, ring)
    q = W.random_sparse(rng, n, 3, 10, 15, ring)
    keys = np.concatenate([embed(p, 0), embed(q, 3)])
    o = np.argsort(keys)
    if ring == "modp":
        neg_q = (P - q.coefs) % P
    else:
        neg_q = -q.coefs
    f = W.Poly(lay, keys[o], np.concatenate([p.coefs, q.coefs])[o])
    g = W.Poly(lay, keys[o], np.concatenate([p.coefs, neg_q])[o])
    return f, g


@pytest.mark.parametrize("ring", ["modp", "i64", "f64"])
@pytest.mark.parametrize("mode", ["pairs", "combine", "intervals", "auto"])
def test_cross_terms_cancel_on_sorted_path(ring, mode):
    # about 2.25e6 result slots cancel, spread over every sort partition
    pm = _pm()
    pm.set_tuning(-1, {"pairs": 0, "combine": 1, "intervals": 2, "auto": -1}[mode], mode == "auto")
    f, g = _cancelling_pair(ring)
    want = oracle.mul(f, g)
    assert len(want[0]) < len(f) * len(f) // 2
    print(f"[parity] cancel {ring} {mode} na={len(f)} terms={len(want[0])}", flush=True)
    assert_same(gpu_mul(f, g), want, ring, f"cancel {ring} {mode}")


def test_cancellation_with_capacity_below_slots():
    # capacity = the final term count, which is below the number of distinct
    # monomials the sorted path sees before cancelled terms are dropped
    pm = _pm()
    pm.set_tuning(-1, 0, False)
    f, g = _cancelling_pair("modp", n=600, seed=32)
    wk, wc, _ = oracle.mul(f, g)
    cnt = len(wk)
    lay = (6, 10, "modp")
    F, G = pm.to_device(f), pm.to_device(g)
    out = pm.alloc_out(cnt, "modp")
    h = pm.mul(lay, F, G, out=out)
    assert h.n >= cnt
    k = out[0].cpu().numpy().view(np.uint64)[:cnt]
    c = out[1].cpu().numpy().view(np.uint64)[:cnt]
    if h.n == cnt:
        assert np.array_equal(k, wk) and np.array_equal(c, wc)
    else:
        # truncated: a prefix of the result, then zero coefficients
        m = int(np.argmax(c == 0)) if np.any(c == 0) else cnt
        assert np.all(c[m:] == 0)
        assert np.array_equal(k[:m], wk[:m]) and np.array_equal(c[:m], wc[:m])
    # a capacity of the reported size always suffices
    out2 = pm.alloc_out(max(h.n, cnt), "modp")
    h2 = pm.mul(lay, F, G, out=out2)
    assert h2.n == cnt
    got = h2.numpy()
    assert np.array_equal(got[0], wk) and np.array_equal(got[1], wc)


def test_sort_blocks_with_range_scan():
    # one product of 68.9e6 term pairs on the sort path: more than 16 x 64 sort
    # blocks, so the radix passes take their block positions from the range
    # scan (the large sparse workload stays below that and sums its ranges)
    pm = _pm()
    pm.set_tuning(-1, 0, False)
    rng = W.rng_for(78)
    f = W.random_sparse(rng, 8300, 6, 10, 6, "modp")
    g = W.random_sparse(rng, 8300, 6, 10, 6, "modp")
    check(f, g, "range scan")
    assert pm.last_call_info()["staged"] == len(f) * len(g)


def test_single_variable_full_width():
    # one variable, 64-bit field: the degree box is not compressible
    rng = np.random.default_rng(5)
    a = np.sort(rng.choice(1 << 40, size=300, replace=False)).astype(np.uint64)
    b = np.sort(rng.choice(1 << 40, size=200, replace=False)).astype(np.uint64)
    lay = W.Layout(1, 64, "modp")
    f = W.Poly(lay, a, W.residues(W.rng_for(1), 300))
    g = W.Poly(lay, b, W.residues(W.rng_for(2), 200))
    check(f, g, "1var64")


def test_many_vars_one_bit():
    rng = W.rng_for(6)
    # 32 variables of 2 bits: exponents 0..1, so sums fit
    f = W.random_sparse(rng, 400, 32, 2, 1, "modp")
    g = W.random_sparse(rng, 300, 32, 2, 1, "modp")
    check(f, g, "32var")


def test_validation_errors_match_oracle():
    pm = _pm()
    lay = (2, 8, "i64")
    k = np.array([1, 2], dtype=np.uint64)
    c = np.array([1, 1], dtype=np.int64)
    bad = [
        (k[::-1].copy(), c, k, c, pm.PM_EUNSORTED),
        (np.array([200], dtype=np.uint64), c[:1], np.array([200], dtype=np.uint64), c[:1], pm.PM_EOVERFLOW),
        (np.array([1 << 20], dtype=np.uint64), c[:1], k, c, pm.PM_EINVAL),
    ]
    for fk, fc, gk, gc, code in bad:
        f = W.Poly(W.Layout(2, 8, "i64"), fk, fc)
        g = W.Poly(W.Layout(2, 8, "i64"), gk, gc)
        assert oracle.validate(2, 8, "i64", fk, fc, gk, gc) == code
        with pytest.raises(pm.PolymulError) as e:
            pm.mul(lay, pm.to_device(f), pm.to_device(g))
        assert e.value.code == code
    r = np.array([P, 1], dtype=np.uint64)
    f = W.Poly(W.Layout(2, 8, "modp"), k, r)
    with pytest.raises(pm.PolymulError) as e:
        pm.mul((2, 8, "modp"), pm.to_device(f), pm.to_device(f))
    assert e.value.code == pm.PM_ERANGE


def test_misaligned_workspace_rejected():
    """The workspace must be 256-byte aligned (kernels issue 16-byte loads
    from its regions); an offset pointer is refused before anything runs."""
    pm = _pm()
    import ctypes
    import torch
    f, g = W.config3("modp", n=3)
    lay = pm.make_layout(5, 12, "modp")
    df, dg = pm.to_device(f), pm.to_device(g)
    cap, wb = pm.bound(lay, df, dg)
    hk, hc, hn = pm.alloc_out(cap, "modp")
    h = pm.pm_poly(cap, hn.data_ptr(), hk.data_ptr(), hc.data_ptr())
    ws = torch.empty(wb + 512, dtype=torch.uint8, device="cuda")
    for off, code in ((16, pm.PM_EINVAL), (256, pm.PM_OK)):
        rc = pm.lib().pm_mul(ctypes.byref(lay), ctypes.byref(pm._cpoly(df)), ctypes.byref(pm._cpoly(dg)),
                             ctypes.byref(h), ctypes.c_void_p(ws.data_ptr() + off), wb, None)
        assert rc == code, (off, rc)
    torch.cuda.synchronize()
    want = oracle.mul(f, g)
    assert int(hn.item()) == len(want[0])
    assert np.array_equal(hk[:len(want[0])].cpu().numpy().view(np.uint64), want[0])


def test_truncation_reports_full_count():
    pm = _pm()
    import torch
    f, g = W.config2(4)
    want = oracle.mul(f, g)
    out = pm.alloc_out(10, "modp")
    h = pm.mul((4, 16, "modp"), pm.to_device(f), pm.to_device(g), out=out)
    assert h.n == len(want[0])
    assert np.array_equal(out[0][:10].cpu().numpy().view(np.uint64), want[0][:10])


# ------------------------------------------------------------- full sizes
def test_config1_closed_form_full():
    f, g = W.config1()
    hk, hc = gpu_mul(f, g)
    assert hk.size == math.comb(24, 4)
    fact = [math.factorial(i) for i in range(21)]

    def M(n, e):
        s = sum(e)
        if s > n:
            return 0
        r = fact[n] // fact[n - s]
        for x in e:
            r //= fact[x]
        return r
    for e, c in zip(W.unpack(hk, 4, 16).tolist()[::97], hc.tolist()[::97]):
        assert c == M(20, e) + M(10, e)


def test_config2_full_closed_form_and_evaluation():
    f, g = W.config2(20)
    hk, hc = gpu_mul(f, g)
    assert hk.size == math.comb(44, 4) == 135751
    # closed form on every term: M(40; e) + M(20; e) mod p
    fact = [math.factorial(i) for i in range(41)]
    ex = W.unpack(hk, 4, 16)
    for e, c in zip(ex.tolist(), hc.tolist()):
        s = sum(e)
        m40 = fact[40] // (fact[e[0]] * fact[e[1]] * fact[e[2]] * fact[e[3]] * fact[40 - s])
        m20 = 0
        if s <= 20:
            m20 = fact[20] // (fact[e[0]] * fact[e[1]] * fact[e[2]] * fact[e[3]] * fact[20 - s])
        assert c == (m40 + m20) % P
    # evaluation at 16 random points mod p
    import random
    rr = random.Random(2)
    for _ in range(16):
        a = [rr.randrange(P) for _ in range(4)]
        pw = [[pow(a[v], k, P) for k in range(41)] for v in range(4)]
        s = 0
        for e, c in zip(ex.tolist(), hc.tolist()):
            s = (s + c * pw[0][e[0]] % P * pw[1][e[1]] % P * pw[2][e[2]] % P * pw[3][e[3]]) % P
        fa = pow((1 + sum(a)) % P, 20, P)
        assert s == fa * (fa + 1) % P


@pytest.mark.parametrize("ring", ["modp", "f64"])
def test_config3_full(ring):
    f, g = W.config3(ring)
    check(f, g, f"cfg3 {ring}")


@pytest.mark.parametrize("ring", ["modp", "f64"])
def test_config3_full_pair_sort_path(ring):
    pm = _pm()
    pm.set_tuning(-1, 0, True)
    f, g = W.config3(ring)
    check(f, g, f"cfg3 pair sort {ring}")


def test_dense_family_through_intervals():
    # high multiplicity (up to thousands of pairs per monomial) on the interval
    # path: exercises bucket refinement and the single-monomial accumulation
    pm = _pm()
    pm.set_tuning(-1, 2, False)
    for ring in ("modp", "i64"):
        f = W.dense_power(14, 4, 16, ring)
        check(f, W.add_constant(f, 1), f"dense n=14 intervals {ring}")
    f = W.dense_power(14, 4, 16, "f64")
    check(f, W.add_constant(f, 1), "dense n=14 intervals f64")


def test_config3_modp_lds_combine():
    pm = _pm()
    pm.set_tuning(-1, 1, True)
    f, g = W.config3("modp")
    check(f, g, "cfg3 combine")
