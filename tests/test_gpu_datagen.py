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
