"""ht_project_static, the allocation-free variant of ht_project, through the C ABI:
its latent codes equal ht_project's bit for bit (the same kernels in the same order
on the same inputs), on two calls in a row with the second on a smaller input, for
a batch that the 256 MiB static scratch takes in one piece and one it takes in
several chunks."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import datagen  # noqa: E402
from paper_2412_16544_amd import htrise as H  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(y):
    return torch.from_numpy(np.ascontiguousarray(y)).to("cuda:0")


def both(st, y):
    r, _ = st.ranks()
    a = torch.full((y.shape[0], r[0], r[1]), float("nan"), dtype=torch.float64, device="cuda:0")
    b = torch.full_like(a, float("nan"))
    H.ht_project(st.h, y, a)
    H.ht_project_static(st.h, y, b)
    torch.cuda.synchronize()
    return a, b


def test_project_static_tiny_stream():
    ys = datagen.tiny_stream()
    st = H.HTStream(ys[0].shape[1:], 1e-4, 64, 8, 40)
    for y in ys[:4]:
        st.push(dev(y))
    for y in (dev(ys[4]), dev(ys[4][:3])):
        a, b = both(st, y)
        assert torch.equal(a, b)
    st.close()


def test_project_static_in_chunks():
    """96^3 x 3 field: one sample's chain needs ~13 MB, so a 32-sample batch is
    projected in two chunks; then a 5-sample batch in one."""
    from datagen import gpu as G
    spec = datagen.field_96_spec()
    st = H.HTStream(spec.n, 1e-4, 48, 32, 96)
    for k in range(2):
        st.push(G.field_batch(spec, k))
    y = G.field_batch(spec, 2)
    for yy in (y, y[:5].contiguous()):
        a, b = both(st, yy)
        assert torch.equal(a, b)
        assert torch.isfinite(b).all()
    st.close()
