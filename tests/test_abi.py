"""C ABI without a GPU: the library loads, exports exactly what
include/polymul.h declares, rejects bad arguments before touching the device,
and its host planner computes the documented bounds."""
import ctypes

import numpy as np
import pytest

from paper_1303_7425_amd import polymul as pm
from paper_1303_7425_amd import workloads as W


@pytest.fixture(scope="module")
def L():
    return pm.lib()


def test_exports_match_header(L):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", pm.LIB_PATH], capture_output=True, text=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if ln.split()[-1].startswith("pm_")})
    assert exported == pm.header_symbols()
    for name in pm.header_symbols():
        assert hasattr(L, name)


def test_strerror_and_version(L):
    for code in range(0, -9, -1):
        assert L.pm_strerror(code)
    assert b"unknown" in L.pm_strerror(-99)
    assert L.pm_version().startswith(b"polymul")


def test_bad_arguments_rejected_on_host(L):
    f = pm.pm_cpoly(1, None, None)            # n = 1 with null pointers
    g = pm.pm_cpoly(0, None, None)
    mt, wb = ctypes.c_int64(0), ctypes.c_int64(0)
    good = pm.make_layout(2, 8, "modp")
    assert L.pm_mul_bound(None, ctypes.byref(g), ctypes.byref(g), ctypes.byref(mt), ctypes.byref(wb), None) == pm.PM_EINVAL
    assert L.pm_mul_bound(ctypes.byref(good), ctypes.byref(f), ctypes.byref(g), ctypes.byref(mt), ctypes.byref(wb),
                          None) == pm.PM_EINVAL
    for bad in (pm.make_layout(0, 8, "modp"), pm.make_layout(9, 8, "modp"), pm.pm_layout(2, 8, 7, 0),
                pm.pm_layout(2, 8, 0, 1), pm.make_layout(2, 0, "modp")):
        assert L.pm_mul_bound(ctypes.byref(bad), ctypes.byref(g), ctypes.byref(g), ctypes.byref(mt),
                              ctypes.byref(wb), None) == pm.PM_EINVAL
    h = pm.pm_poly(4, None, None, None)       # null n_out
    assert L.pm_mul(ctypes.byref(good), ctypes.byref(g), ctypes.byref(g), ctypes.byref(h), None, 0, None) == pm.PM_EINVAL
    assert L.pm_set_tuning(5, 0, 1) == pm.PM_EINVAL
    assert L.pm_set_tuning(-1, 4, 1) == pm.PM_EINVAL
    assert L.pm_set_tuning(-1, 3, 1) == pm.PM_OK
    assert L.pm_set_tuning(-1, 2, 1) == pm.PM_OK
    assert L.pm_set_tuning(-1, -1, 1) == pm.PM_OK
    assert L.pm_set_radix(2) == pm.PM_EINVAL
    assert L.pm_set_radix(-2) == pm.PM_EINVAL
    assert L.pm_set_radix(0) == pm.PM_OK
    assert L.pm_set_radix(-1) == pm.PM_OK
    lat = ctypes.c_double(0)
    assert L.pm_server_latency(None, 1, ctypes.byref(lat)) == pm.PM_EINVAL


def stats_of(f, g):
    nv = f.layout.nvars
    ef, eg = W.unpack(f.keys, nv, f.layout.bits), W.unpack(g.keys, nv, g.layout.bits)
    return np.concatenate([ef.min(0), ef.max(0), eg.min(0), eg.max(0)]).astype(np.uint64)


@pytest.mark.parametrize("case", ["dense10", "sparse6", "rand"])
def test_plan_bound_is_min_of_pairs_and_degree_box(case):
    if case == "dense10":
        f, g = W.config1()
    elif case == "sparse6":
        f, g = W.sparse_power(6, "f", 12, "modp"), W.sparse_power(6, "g", 12, "modp")
    else:
        rng = W.rng_for(1)
        f, g = W.random_sparse(rng, 300, 6, 10, 15, "modp"), W.random_sparse(rng, 200, 6, 10, 15, "modp")
    st = stats_of(f, g)
    nv = f.layout.nvars
    box = 1
    for v in range(nv):
        box *= int(st[nv + v]) + int(st[3 * nv + v]) - int(st[v]) - int(st[2 * nv + v]) + 1
    rc, mt, wb = pm.plan_from_stats((nv, f.layout.bits, f.layout.ring), [len(f)], [len(g)], st[None, :])
    assert rc == pm.PM_OK
    assert mt[0] == min(len(f) * len(g), box)
    assert wb > 0


def test_plan_batch_and_empty():
    f, g = W.config1()
    st = stats_of(f, g)
    rc, mt, wb = pm.plan_from_stats((4, 16, "i64"), [len(f), 0, len(f)], [len(g), 5, len(g)],
                                    np.stack([st, st, st]))
    assert rc == pm.PM_OK and mt[1] == 0 and mt[0] == mt[2]
    rc1, _, wb1 = pm.plan_from_stats((4, 16, "i64"), [len(f)], [len(g)], st[None, :])
    assert wb > wb1


def test_plan_overflow_detected():
    st = np.array([0, 200, 0, 100], dtype=np.uint64)   # 1 var, 8 bits: 200 + 100 > 255
    rc, _, _ = pm.plan_from_stats((1, 8, "modp"), [3], [3], st[None, :])
    assert rc == pm.PM_EOVERFLOW
    st = np.array([0, 200, 0, 55], dtype=np.uint64)    # 255 still fits
    rc, mt, _ = pm.plan_from_stats((1, 8, "modp"), [3], [3], st[None, :])
    assert rc == pm.PM_OK and mt[0] == 9


def test_plan_fp64_too_many_pairs():
    st = np.array([0, 1000, 0, 1000], dtype=np.uint64)
    rc, _, _ = pm.plan_from_stats((1, 32, "f64"), [1 << 17], [1 << 16], st[None, :])
    assert rc == pm.PM_ENOMEM                          # more than 2^32 - 1 FP64 term pairs in one product
    rc, _, _ = pm.plan_from_stats((1, 32, "modp"), [1 << 17], [1 << 16], st[None, :])
    assert rc == pm.PM_OK                              # a degree box this small takes the dense path


def test_plan_sparse_exact_too_many_pairs():
    # 2 variables x 32 bits, exponents up to 2^20: the degree box (about 2^42
    # cells) is far larger than the 2^33 term pairs, so the product is sparse;
    # its staged positions would not fit 32 bits, which the planner refuses
    st = np.array([0, 0, 1 << 20, 1 << 20, 0, 0, 1 << 20, 1 << 20], dtype=np.uint64)
    for ring in ("modp", "i64", "f64"):
        rc, _, _ = pm.plan_from_stats((2, 32, ring), [1 << 17], [1 << 16], st[None, :])
        assert rc == pm.PM_ENOMEM, ring
    rc, _, _ = pm.plan_from_stats((2, 32, "modp"), [1 << 16], [(1 << 16) - 1], st[None, :])
    assert rc == pm.PM_OK                              # 2^31 pairs still fit


def test_autotune_choices_save_and_load(tmp_path):
    # the autotuner's per-size-class choices survive the process as a text file
    src = tmp_path / "tune.txt"
    src.write_text("# tuned once\n0 0 25 -1 3 -1\n1 0 26 -1 0 1\n0 1 20 2 0 -1\n")
    pm.autotune_reset()
    pm.autotune_load(src)
    out = tmp_path / "out.txt"
    pm.autotune_save(out)
    lines = [ln for ln in out.read_text().splitlines() if not ln.startswith("#")]
    assert sorted(lines) == sorted(["0 0 25 -1 3 -1", "1 0 26 -1 0 1", "0 1 20 2 0 -1"])
    bad = tmp_path / "bad.txt"
    bad.write_text("0 0 25 -1 9 -1\n")            # sparse mode 9 does not exist
    with pytest.raises(pm.PolymulError):
        pm.autotune_load(bad)
    pm.autotune_save(out)                         # nothing of the bad file was taken
    assert sorted(ln for ln in out.read_text().splitlines() if not ln.startswith("#")) == sorted(lines)
    pm.autotune_reset()
    pm.autotune_save(out)
    assert [ln for ln in out.read_text().splitlines() if not ln.startswith("#")] == []


@pytest.mark.parametrize("example", [2, 3])
def test_plan_paper_examples_beyond_sparse_limits_take_degree_box(example):
    # Examples 2 and 3 of the paper: 2.03e10 and 5.63e10 term pairs, beyond the
    # sparse paths' 2^32 - 1; their degree boxes (2.35e10 and 7.36e9 cells)
    # take the products in the exact rings, with 8 bytes per cell of workspace
    from paper_1303_7425_amd import workloads as W
    f, g = W.config3("modp", n=25) if example == 2 else W.example3(28, 12, "modp")
    ef, eg = W.unpack(f.keys, 5, 12), W.unpack(g.keys, 5, 12)
    st = np.concatenate([ef.min(0), ef.max(0), eg.min(0), eg.max(0)]).astype(np.uint64)
    cells = int(np.prod((ef.max(0) + eg.max(0)) - (ef.min(0) + eg.min(0)) + 1, dtype=np.float64))
    rc, mt, wb = pm.plan_from_stats((5, 12, "modp"), [len(f)], [len(g)], st[None, :])
    assert rc == pm.PM_OK and mt[0] == min(cells, len(f) * len(g))
    assert 8 * cells <= wb < 8 * cells + (1 << 30)
    rc, _, _ = pm.plan_from_stats((5, 12, "f64"), [len(f)], [len(g)], st[None, :])
    assert rc == pm.PM_ENOMEM
