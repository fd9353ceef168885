"""The output-key work-item path (pm_set_tuning(-1, 3, ...)) against the
oracle in every ring: exact fine-bin counts, the greedy cut into work items
of at most 8192 pairs (and, for the exact rings, at most 2^18 keys), the
scatter, and the per-work-item LDS sum (direct cells, presence-bitmap ranks,
or for FP64 the stable LDS sort by row then key, which keeps row-major sums),
including fine bins holding more than one work item's pairs (processed in
rounds) and ragged, empty and single-term operands."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1303_7425_amd import workloads as W
from test_gpu_parity import check


def _pm():
    from paper_1303_7425_amd import polymul
    return polymul


@pytest.fixture(autouse=True)
def work_items():
    pm = _pm()
    pm.set_tuning(-1, 3, True)
    yield
    pm.set_tuning(-1, -1, True)


def fat_bins(ring, n=60, seed=1):
    """f: all (0, t, u) with t + u <= n; g: the same plus (1000, t, u).  Many
    pairs share a monomial, so single fine bins hold more than 8192 pairs."""
    rng = W.rng_for(seed)
    tri = [(0, t, u) for t in range(n + 1) for u in range(n + 1 - t)]
    lay = W.Layout(3, 12, ring)

    def mk(exps):
        keys = W.pack(np.array(exps), 3, 12)
        o = np.argsort(keys)
        if ring == "modp":
            c = W.residues(rng, len(exps))
        elif ring == "f64":
            c = W.uniform_pm1(rng, len(exps))
        else:
            c = rng.integers(-5, 6, len(exps)).astype(np.int64)
        return W.Poly(lay, keys[o], c[o])
    return mk(tri), mk(tri + [(1000, t, u) for (_, t, u) in tri])


@pytest.mark.parametrize("ring", ["modp", "f64", "i64"])
def test_workitems_random_ragged(ring):
    rng = W.rng_for(11)
    for na, nb in ((1, 1), (1, 500), (33, 70), (257, 129), (1000, 3000)):
        check(W.random_sparse(rng, na, 6, 10, 15, ring), W.random_sparse(rng, nb, 6, 10, 15, ring),
              f"work items {na}x{nb}")


@pytest.mark.parametrize("ring", ["modp", "f64", "i64"])
def test_workitems_fat_bins(ring):
    check(*fat_bins(ring), "work items, fat bins")


@pytest.mark.parametrize("ring", ["modp", "f64"])
def test_workitems_sparse_family(ring):
    check(*W.config3(ring, n=8), "work items, sparse family n=8")


def test_workitems_dense_family_without_box():
    pm = _pm()
    pm.set_tuning(-1, 3, False)
    check(*W.config2(9), "work items, dense n=9 mod p")
    f, g = W.config2(9)
    check(W.with_random_coefs(f, W.rng_for(3), "f64"), W.with_random_coefs(g, W.rng_for(4), "f64"),
          "work items, dense n=9 f64")


def test_workitems_cancellation_and_empty():
    pm = _pm()
    lay = W.Layout(2, 8, "modp")
    # (x + y)(x - y) = x^2 - y^2 with the cross terms cancelling in one work item
    f = W.Poly(lay, W.pack(np.array([[0, 1], [1, 0]]), 2, 8), np.array([1, 1], np.uint64))
    g = W.Poly(lay, W.pack(np.array([[0, 1], [1, 0]]), 2, 8), np.array([W.P61 - 1, 1], np.uint64))
    check(f, g, "work items, cancellation")
    e = W.Poly(lay, np.zeros(0, np.uint64), np.zeros(0, np.uint64))
    check(f, e, "work items, empty operand")
