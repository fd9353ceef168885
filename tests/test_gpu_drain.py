"""Batched products drained to host memory wave by wave while the next wave
runs: every result handed to the callback equals the one-launch batch result
and the oracle, in product order, whatever the number of waves."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
from paper_1303_7425_amd import workloads as W
from test_gpu_batch import mixed_pairs


def _pm():
    from paper_1303_7425_amd import polymul
    return polymul


@pytest.mark.parametrize("ring", ["modp", "f64", "i64"])
@pytest.mark.parametrize("device_mib", [180, 1024])
def test_drain_matches_batch_and_oracle(ring, device_mib):
    pm = _pm()
    pairs = mixed_pairs(ring, count=24, seed=43)
    lay = (6, 10, ring)
    fs = [pm.to_device(f) for f, _ in pairs]
    gs = [pm.to_device(g) for _, g in pairs]
    ref = pm.mul_batch(lay, fs, gs)
    got = {}
    order = []

    def on_result(k, keys, coefs):
        order.append(k)
        got[k] = (keys.copy(), coefs.copy())

    waves = pm.mul_batch_drain(lay, fs, gs, on_result, device_bytes=device_mib << 20, host_bytes=128 << 20)
    print(f"[drain] ring={ring} device={device_mib} MiB waves={waves}", flush=True)
    assert order == list(range(len(pairs)))
    if device_mib == 180:
        assert waves > 1
    for k, ((f, g), (rk, rc)) in enumerate(zip(pairs, ref)):
        gk, gc = got[k]
        assert np.array_equal(gk, rk), k
        assert np.array_equal(np.asarray(gc).view(np.uint64), np.asarray(rc).view(np.uint64)), k
    for k in (0, 5, 11):
        wk, wc, _ = oracle.mul(*pairs[k])
        assert np.array_equal(got[k][0], wk) and np.array_equal(got[k][1].view(np.uint64), wc.view(np.uint64))


def test_drain_one_product_too_large():
    pm = _pm()
    f, g = W.config3("modp", n=8)
    with pytest.raises(pm.PolymulError) as ei:
        pm.mul_batch_drain((5, 12, "modp"), [pm.to_device(f)], [pm.to_device(g)], lambda *a: None,
                           device_bytes=1 << 20, host_bytes=1 << 20)
    assert ei.value.code == pm.PM_ENOMEM
