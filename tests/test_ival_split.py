"""The output-key interval split of the interval path, on the host (no GPU).

Section 5 samples the pp-matrix on a grid of (l+1)^2 points (Fig. 2 uses
l = 8, i.e. 81 samples, on the product of the 5-variable family at n = 8);
the sorted distinct sample exponents, bracketed by the smallest exponent
gamma_11 and one past the largest, are the splitters S_k.  Section 2's
intervals [S_k, S_{k+1}) must then hold every exponent gamma_ij exactly once.
The kernels that sample and split on the device use the same grid function
as these host helpers."""
import numpy as np
import pytest

from paper_1303_7425_amd import polymul as pm
from paper_1303_7425_amd import workloads as W


def test_fig2_grid_has_81_samples():
    # Fig. 2: f, g = (1+x+y+2z^2+3t^3+5u^5)^8 and its mirror, 1287 terms each
    f, g = W.sparse_power(8, "f"), W.sparse_power(8, "g")
    assert len(f) == len(g) == 1287
    rows, cols = pm.ival_grid(len(f), len(g), 8)
    assert len(rows) == len(cols) == 81


@pytest.mark.parametrize("na,nb,l", [(1287, 1287, 8), (1001, 640, 5), (100, 7, 3), (64, 64, 63), (5, 9, 1)])
def test_grid_rows_and_staggered_columns(na, nb, l):
    rows, cols = pm.ival_grid(na, nb, l)
    assert len(rows) == (l + 1) ** 2
    di, dj, st = na // l, nb // l, nb // (2 * l)
    for t in range(len(rows)):
        r, c = divmod(t, l + 1)
        # sample row r sits at r * floor(na / l); odd sample rows start their
        # columns floor(nb / (2l)) later (the j_{0,i} offset), spacing floor(nb / l)
        assert rows[t] == min(r * di, na - 1)
        assert cols[t] == min((r % 2) * st + c * dj, nb - 1)
    assert rows.min() == 0 and cols.min() == 0
    assert rows.max() <= na - 1 and cols.max() <= nb - 1


def test_grid_l0_is_one_sample():
    rows, cols = pm.ival_grid(10, 20, 0)
    assert list(rows) == [0] and list(cols) == [0]


def test_grid_fig2_values():
    # l = 8 over a 1287 x 1287 matrix: spacing 160, odd-row offset 80
    rows, cols = pm.ival_grid(1287, 1287, 8)
    assert sorted(set(rows.tolist())) == [160 * r for r in range(9)]
    assert cols[:9].tolist() == [160 * c for c in range(9)]
    assert cols[9:18].tolist() == [min(80 + 160 * c, 1286) for c in range(9)]  # clamped to the last column


def _every_gamma_once(fk, gk, l):
    spl = pm.ival_splitters(fk, gk, l)
    assert np.all(np.diff(spl.astype(np.float64)) > 0) and np.all(spl[1:] > spl[:-1])
    gam = (fk[:, None] + gk[None, :]).ravel()
    assert spl[0] == gam.min() and spl[-1] == gam.max() + 1
    # the number of intervals [S_k, S_{k+1}) containing each gamma is exactly one
    lo = np.searchsorted(spl, gam, side="right") - 1
    assert np.all(lo >= 0) and np.all(lo < len(spl) - 1)
    assert np.all(spl[lo] <= gam) and np.all(gam < spl[lo + 1])
    inside = (spl[:-1, None] <= gam[None, :]) & (gam[None, :] < spl[1:, None])
    assert np.all(inside.sum(axis=0) == 1)
    return spl


def test_every_gamma_in_exactly_one_interval_fig2():
    f, g = W.sparse_power(8, "f"), W.sparse_power(8, "g")
    # the dense check below is (intervals x pairs); thin the operands to keep it small
    fk, gk = f.keys[::4].copy(), g.keys[::4].copy()
    spl = _every_gamma_once(fk, gk, 8)
    assert 2 <= len(spl) <= 81 + 2


@pytest.mark.parametrize("seed,na,nb,l", [(1, 1, 1, 0), (2, 1, 37, 4), (3, 50, 1, 8), (4, 200, 150, 8),
                                          (5, 300, 90, 63), (6, 17, 400, 12)])
def test_every_gamma_in_exactly_one_interval_random(seed, na, nb, l):
    rng = W.rng_for(seed)
    f = W.random_sparse(rng, na, nvars=3, bits=10)
    g = W.random_sparse(rng, nb, nvars=3, bits=10)
    _every_gamma_once(f.keys, g.keys, l)


def test_helpers_reject_bad_arguments():
    with pytest.raises(pm.PolymulError):
        pm.ival_grid(0, 5, 2)
    with pytest.raises(pm.PolymulError):
        pm.ival_grid(5, 5, 64)
