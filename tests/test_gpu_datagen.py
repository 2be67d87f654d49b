"""The device generator of datagen's exactly reproducible fields gives the host
generator's float32 values bit for bit (the oracle consumes the host values, the
GPU tests and the benchmark the device ones)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import datagen  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("spec,k", [
    (datagen.FieldSpec(grid=(6, 5, 4), channels=3, terms=5, N=3, n_batches=2, drift=1e-3, seed=3, batch_seed0=30,
                       nu=1e-6), 1),
    (datagen.field_96_spec(N=2), 7),
    (datagen.field_48_spec(N=2), 0),
    (datagen.field_48_spec(N=2), 57),
])
def test_device_generator_matches_host_bitwise(spec, k):
    from datagen import gpu as G
    host = datagen.exact_field_batch(spec, k)
    dev = G.field_batch(spec, k).cpu().numpy()
    assert host.shape == dev.shape
    assert np.array_equal(host.view(np.uint32), dev.view(np.uint32))
