"""pm_mul_noalloc (static device scratch, no allocation) against pm_mul on
the same operands: identical results on consecutive calls, the second one
smaller than the first, and products beyond the scratch rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1303_7425_amd import workloads as W


def _pm():
    from paper_1303_7425_amd import polymul
    return polymul


def _both(f, g):
    pm = _pm()
    lay = (f.layout.nvars, f.layout.bits, f.layout.ring)
    fd, gd = pm.to_device(f), pm.to_device(g)
    ref = pm.mul(lay, fd, gd)
    cap, ws = pm.bound(lay, fd, gd)
    assert ws <= pm.NOALLOC_SCRATCH_BYTES
    out = pm.alloc_out(cap, f.layout.ring)
    out[0].fill_(-1)
    out[1].fill_(-1)
    got = pm.mul_noalloc(lay, fd, gd, out)
    assert pm.last_call_status() == 0
    rk, rc = ref.numpy()
    gk, gc = got.numpy()
    assert got.n == ref.n
    assert np.array_equal(gk, rk)
    assert np.array_equal(np.asarray(gc).view(np.uint64), np.asarray(rc).view(np.uint64))
    return got.n


@pytest.mark.parametrize("ring", ["modp", "f64", "i64"])
def test_noalloc_matches_pm_mul_twice_shrinking(ring):
    rng = W.rng_for(71)
    # first: the 5-variable sparse family at n = 8 (1287 x 1287 terms)
    f1, g1 = W.config3(ring if ring != "i64" else "modp", n=8)
    if ring == "i64":
        f1, g1 = W.with_random_coefs(f1, rng, "i64"), W.with_random_coefs(g1, rng, "i64")
    n1 = _both(f1, g1)
    # second, smaller: random 6-variable operands with a ragged tail
    f2 = W.random_sparse(rng, 333, 6, 10, 15, ring)
    g2 = W.random_sparse(rng, 71, 6, 10, 15, ring)
    n2 = _both(f2, g2)
    assert 0 < n2 < n1


def test_noalloc_dense_then_sparse():
    # the degree-box path, then a product on the sparse path, then a dense one again
    f = W.dense_power(8, 4, 16, "modp")
    _both(f, W.add_constant(f, 1))
    rng = W.rng_for(72)
    _both(W.random_sparse(rng, 900, 6, 10, 15, "modp"), W.random_sparse(rng, 500, 6, 10, 15, "modp"))
    f = W.dense_power(5, 4, 16, "modp")
    _both(f, W.add_constant(f, 1))


def test_noalloc_rejects_beyond_scratch_then_recovers():
    pm = _pm()
    f, g = W.config3("modp")                      # about 480 MiB of workspace
    lay = (5, 12, "modp")
    fd, gd = pm.to_device(f), pm.to_device(g)
    cap, ws = pm.bound(lay, fd, gd)
    assert ws > pm.NOALLOC_SCRATCH_BYTES
    out = pm.alloc_out(16, "modp")
    with pytest.raises(pm.PolymulError) as ei:
        pm.mul_noalloc(lay, fd, gd, out)
    assert ei.value.code == pm.PM_ENOMEM
    # a product that fits still runs correctly afterwards
    f2, g2 = W.config3("modp", n=5)
    _both(f2, g2)
