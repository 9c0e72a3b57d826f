"""The device generator reproduces the host generator's integer streams bit
for bit (so full-size inputs built on the device are the documented recipe)."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("s", [0.0, 0.8, 1.2])
def test_device_keys_and_values_match_host(s):
    import datagen.device as dgd
    n, d = 300_000, 50_000
    kh, vh, _ = datagen.plain_input(77, n, d, s)
    kd, vd, fd = dgd.plain_input(77, n, d, s, with_f64=True)
    assert np.array_equal(kd.cpu().numpy().view(np.uint64), kh)
    assert np.array_equal(vd.cpu().numpy(), vh)
    f = fd.cpu().numpy()
    assert np.isfinite(f).all() and abs(f.mean()) < 0.02 and abs(f.std() - 1) < 0.02


def test_device_segmented_matches_host():
    import datagen.device as dgd
    n = 400_000
    ah, bh, vh = datagen.segmented_input(55, n, n_a=50, b_per_a=1000)
    ad, bd, vd = dgd.segmented_input(55, n, n_a=50, b_per_a=1000)
    assert np.array_equal(ad.cpu().numpy(), ah)
    assert np.array_equal(bd.cpu().numpy(), bh)
    assert np.array_equal(vd.cpu().numpy(), vh)


@pytest.mark.parametrize("s", [0.0, 0.6, 1.0, 1.2])
def test_device_zipf_approx_domain_and_head(s):
    # keys stay in the d-value domain and the head rank's share matches the
    # continuous density x^-s on [1, d+1) it inverts
    import datagen.device as dgd
    n, d = 2_000_000, 1000
    k = dgd.zipf_approx_keys(91, n, d, s).cpu().numpy().view(np.uint64)
    dom = datagen.key_of_rank(np.arange(d, dtype=np.uint64))
    assert np.isin(k, dom).all()
    top = int((k == dom[0]).sum())
    dd = d + 1.0
    if abs(s - 1.0) < 1e-9:
        p0 = np.log(2.0) / np.log(dd)
    else:
        a = 1.0 - s
        p0 = (2.0 ** a - 1.0) / (dd ** a - 1.0)
    sigma = np.sqrt(n * p0 * (1 - p0))
    assert abs(top - n * p0) < 6 * sigma + 1, (top, n * p0)


def test_device_uniform_ranks_match_host():
    import datagen.device as dgd
    r = dgd.uniform_ranks(81, 500_000, 12_345).cpu().numpy()
    assert np.array_equal(r.astype(np.uint64), datagen.uniform_ranks(81, 500_000, 12_345))
