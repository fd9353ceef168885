"""Input generators: term counts fixed by the multinomial theorem and by the
paper's printed operand sizes (Section 6, Examples 1-3)."""
import json
import math
import os

import numpy as np
import pytest

from paper_1303_7425_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("n", [1, 4, 10, 20])
def test_dense_power_term_count(n):
    f = W.dense_power(n, 4, 16, "modp")
    assert len(f) == math.comb(n + 4, 4)
    assert np.all(f.keys[1:] > f.keys[:-1])
    assert int(f.keys[0]) == 0 and int(f.coefs[0]) == 1        # constant term


def test_config_sizes():
    f, g = W.config1()
    assert len(f) == len(g) == 1001 and int(g.coefs[0]) == 2
    f, g = W.config3()
    assert len(f) == len(g) == math.comb(12 + 5, 5) == 6188
    f, g = W.config3("f64")
    assert f.coefs.dtype == np.float64 and np.all(np.abs(f.coefs) <= 1) and np.all(f.coefs != 0)


def test_paper_operand_counts():
    gold = json.load(open(os.path.join(HERE, "golden", "paper_counts.json")))
    assert math.comb(40 + 4, 4) == gold["example1"]["input_terms"]
    # sparse families: 6 base terms -> C(n+5, 5) terms
    assert math.comb(25 + 5, 5) == gold["example2"]["input_terms"]
    assert math.comb(28 + 5, 5) == gold["example3"]["input_terms"]


@pytest.mark.slow
def test_paper_example3_operand_generated_count():
    gold = json.load(open(os.path.join(HERE, "golden", "paper_counts.json")))
    f, g = W.example3(28, 12, "modp")
    assert len(f) == gold["example3"]["input_terms"]
    assert len(g) == gold["example3"]["input_terms"]


def test_sparse_power_exact_coefs():
    # (1+x+y+2z^2+3t^3+5u^5)^2: the u^10 coefficient is 25, u^5 is 10, xu^5 is 10
    f = W.sparse_power(2, "f", 12, "modp")
    d = {tuple(e): c for e, c in zip(W.unpack(f.keys, 5, 12).tolist(), f.exact)}
    assert d[(0, 0, 0, 0, 10)] == 25 and d[(0, 0, 0, 0, 5)] == 10 and d[(1, 0, 0, 0, 5)] == 10
    assert d[(0, 0, 2, 3, 0)] == 12 and sum(d.values()) == 13 ** 2


def test_random_sparse_distinct_sorted():
    rng = W.rng_for(4)
    p = W.random_sparse(rng, 2000, 6, 10, 15, "f64")
    assert len(p) == 2000 and np.all(p.keys[1:] > p.keys[:-1])
    assert W.unpack(p.keys, 6, 10).max() <= 15


def test_config4_sizes_log_uniform():
    sizes, _ = W.config4_sizes()
    assert sizes.shape == (4096, 2) and sizes.min() >= 50 and sizes.max() < 20000
    # log-uniform: median near sqrt(50*20000) = 1000
    assert 700 < np.median(sizes) < 1400


def test_negative_coefficient_maps_to_residue():
    f, _ = W.example3(1, 12, "modp")
    d = {tuple(e): int(c) for e, c in zip(W.unpack(f.keys, 5, 12).tolist(), f.coefs)}
    assert d[(0, 0, 0, 0, 2)] == W.P61 - 1
