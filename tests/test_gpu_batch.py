"""Batched products (one work queue for many uneven products) and the
HIP-graph-prepared batch, against the oracle and against single products."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from paper_1303_7425_amd import workloads as W


def _pm():
    from paper_1303_7425_amd import polymul
    return polymul


def mixed_pairs(ring, count=24, seed=41):
    """Uneven random 6-variable products (log-uniform sizes, some tiny and
    some empty) plus two structured ones."""
    rng = W.rng_for(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(1), np.log(3000), size=(count, 2)))).astype(int)
    pairs = []
    for na, nb in sizes.tolist():
        pairs.append((W.random_sparse(rng, na, 6, 10, 15, ring), W.random_sparse(rng, nb, 6, 10, 15, ring)))
    pairs[3] = (pairs[3][0], W.Poly(pairs[3][1].layout, np.zeros(0, np.uint64), pairs[3][1].coefs[:0]))
    return pairs


def check_results(pairs, results, ring):
    for q, ((f, g), (hk, hc)) in enumerate(zip(pairs, results)):
        wk, wc, _ = oracle.mul(f, g)
        assert np.array_equal(hk, wk), q
        assert np.array_equal(np.asarray(hc).view(np.uint64), wc.view(np.uint64)), q


@pytest.mark.parametrize("ring", ["modp", "f64", "i64"])
def test_batch_matches_oracle(ring):
    pm = _pm()
    pairs = mixed_pairs(ring)
    print(f"[batch] ring={ring} products={len(pairs)}", flush=True)
    fs = [pm.to_device(f) for f, _ in pairs]
    gs = [pm.to_device(g) for _, g in pairs]
    res = pm.mul_batch((6, 10, ring), fs, gs)
    assert pm.last_call_status() == 0
    check_results(pairs, res, ring)


@pytest.mark.parametrize("ring", ["modp", "f64"])
def test_batch_with_large_operand_keys(ring):
    """More than 1 MB of compressed operand keys in one launch: the pair-index
    sort carries its keys through the passes instead of regenerating them."""
    pm = _pm()
    rng = W.rng_for(77)
    pairs = [(W.random_sparse(rng, 60000, 6, 10, 15, ring), W.random_sparse(rng, 3, 6, 10, 15, ring))
             for _ in range(5)]
    pairs.append((W.random_sparse(rng, 700, 6, 10, 15, ring), W.random_sparse(rng, 900, 6, 10, 15, ring)))
    print(f"[batch] large operand keys ring={ring}", flush=True)
    res = pm.mul_batch((6, 10, ring), [pm.to_device(f) for f, _ in pairs], [pm.to_device(g) for _, g in pairs])
    assert pm.last_call_status() == 0
    check_results(pairs, res, ring)


@pytest.mark.parametrize("ring", ["modp", "f64"])
def test_batch_many_small_operand_keys(ring):
    """Forty products whose compressed operand keys each fit the LDS copies
    but total over 1 MB: the passes carry keys with the pair indices."""
    pm = _pm()
    rng = W.rng_for(78)
    pairs = [(W.random_sparse(rng, 8000, 6, 10, 15, ring), W.random_sparse(rng, 4, 6, 10, 15, ring))
             for _ in range(40)]
    print(f"[batch] many products, keys in LDS, ring={ring}", flush=True)
    res = pm.mul_batch((6, 10, ring), [pm.to_device(f) for f, _ in pairs], [pm.to_device(g) for _, g in pairs])
    assert pm.last_call_status() == 0
    assert pm.last_call_info()["payload_bytes"] == 4
    check_results(pairs, res, ring)


def test_batch_with_dense_and_sparse_members():
    pm = _pm()
    # (1+x+y+z+t+u)^10 times itself plus one takes the degree-box path; the
    # sparse family pair takes the sort path; both in one batch, 5 vars x 12 bits
    df = W.dense_power(10, 5, 12, "modp")
    d5 = (df, W.add_constant(df, 1))
    sp = (W.sparse_power(5, "f", 12, "modp"), W.sparse_power(5, "g", 12, "modp"))
    pairs = [d5, sp, d5, sp]
    res = pm.mul_batch((5, 12, "modp"), [pm.to_device(f) for f, _ in pairs], [pm.to_device(g) for _, g in pairs])
    check_results(pairs, res, "modp")


def test_f64_batch_bit_identical_to_single():
    pm = _pm()
    pairs = mixed_pairs("f64", count=12, seed=7)
    fs = [pm.to_device(f) for f, _ in pairs]
    gs = [pm.to_device(g) for _, g in pairs]
    res = pm.mul_batch((6, 10, "f64"), fs, gs)
    for q in range(len(pairs)):
        hk, hc = pm.mul((6, 10, "f64"), fs[q], gs[q]).numpy()
        assert np.array_equal(hk, res[q][0]) and np.array_equal(hc.view(np.uint64), res[q][1].view(np.uint64))


@pytest.mark.parametrize("ring", ["modp", "f64"])
def test_graph_replays_match_eager(ring):
    import torch
    pm = _pm()
    pairs = mixed_pairs(ring, count=16, seed=3)
    fs = [pm.to_device(f) for f, _ in pairs]
    gs = [pm.to_device(g) for _, g in pairs]
    eager = pm.mul_batch((6, 10, ring), fs, gs)
    call = pm.BatchCall((6, 10, ring), fs, gs)
    call.prepare_graph()
    for rep in range(4):
        call.out_k.fill_(0)
        call.out_c.fill_(0)
        call.out_n.fill_(-1)
        call.launch_graph()
        torch.cuda.synchronize()
        got = call.results()
        assert pm.last_call_status() == 0
        for q in range(len(pairs)):
            assert np.array_equal(got[q][0], eager[q][0]), (rep, q)
            assert np.array_equal(np.asarray(got[q][1]).view(np.uint64), np.asarray(eager[q][1]).view(np.uint64))
        # eager work between replays
        pm.mul((6, 10, ring), fs[0], gs[0])
    check_results(pairs, got, ring)


def test_autotune_keeps_results():
    pm = _pm()
    pm.autotune_reset()
    f, g = W.config3("modp", n=7)
    want = oracle.mul(f, g)
    fd, gd = pm.to_device(f), pm.to_device(g)
    choice = pm.autotune((5, 12, "modp"), fd, gd)
    assert choice[1] in (0, 1, 2, 3) and choice[2] in (-1, 0, 1)
    hk, hc = pm.mul((5, 12, "modp"), fd, gd).numpy()
    assert np.array_equal(hk, want[0]) and np.array_equal(hc, want[1])
    f2, g2 = W.config2(9)
    pm.autotune((4, 16, "modp"), pm.to_device(f2), pm.to_device(g2))
    hk, hc = pm.mul((4, 16, "modp"), pm.to_device(f2), pm.to_device(g2)).numpy()
    want = oracle.mul(f2, g2)
    assert np.array_equal(hk, want[0]) and np.array_equal(hc, want[1])
    pm.autotune_reset()


def test_config4_subsample_full_parity():
    """Batched workload recipe (6 vars, 10 bits, exponents 0..15, log-uniform
    sizes in [50, 20000]) on a seeded subsample of pairs spanning sizes,
    mod p and FP64, term by term against the oracle."""
    pm = _pm()
    sizes, _ = W.config4_sizes()
    order = np.argsort(sizes[:, 0] * sizes[:, 1])
    pick = order[np.linspace(0, len(order) * 0.6, 12).astype(int)]   # up to mid-size pairs
    for ring in ("modp", "f64"):
        rng = W.rng_for(4)
        pairs = []
        for q in pick.tolist():
            na, nb = sizes[q]
            pairs.append((W.random_sparse(rng, int(na), 6, 10, 15, ring), W.random_sparse(rng, int(nb), 6, 10, 15, ring)))
        print(f"[cfg4 subsample] ring={ring} pairs={[(len(f), len(g)) for f, g in pairs]}", flush=True)
        res = pm.mul_batch((6, 10, ring), [pm.to_device(f) for f, _ in pairs], [pm.to_device(g) for _, g in pairs])
        check_results(pairs, res, ring)
