"""GPU (MI355X) parity of the plain leaves-to-root hierarchical Tucker decomposition
(Sec. 2.3.1) with the oracle's PlainHT: the library's BHT-l2r on one sample whose
modes include the batch mode, with the plain-HT budget eps ||Y|| / sqrt(2d-3)
(HT_PLAIN_HT_BUDGET).  Ranks equal the oracle's (the root's two successors both
carry the rank of the final SVD), the reconstruction matches within 1e-10 ||Y||,
and the root is the diagonal of kept singular values (up to signs)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import datagen  # noqa: E402
from oracle import ht_oracle as ho  # noqa: E402
from paper_2412_16544_amd import htrise as H  # noqa: E402

pytestmark = pytest.mark.gpu


def plain_ht_gpu(y, eps, rank_cap=64):
    st = H.HTStream(y.shape, eps, rank_cap, 1, 1, flags=H.HT_PLAIN_HT_BUDGET)
    st.push(torch.from_numpy(np.ascontiguousarray(y[None])).to("cuda:0"))
    return st


def check(y, eps):
    y = y.astype(np.float32)
    st = plain_ht_gpu(y, eps)
    ref = ho.PlainHT(y, eps)
    assert st.ranks()[0] == ref.ranks, (st.ranks()[0], ref.ranks)
    rec = st.reconstruct(0, 1).cpu().numpy()[0]
    ny = np.linalg.norm(y.astype(np.float64))
    assert np.linalg.norm(rec - ref.reconstruct()) <= 1e-10 * ny
    assert np.linalg.norm(rec - y) <= eps * ny
    flat = st.export()
    r0 = ref.ranks[0]
    root = flat[-r0 * r0:].reshape(r0, r0)
    # the Gram route gives the kept singular vectors to ~u ||G|| / gap, so small near-equal
    # singular values leave off-diagonal entries of ~1e-11 ||Y||
    np.testing.assert_allclose(np.abs(root), np.abs(ref.root), atol=1e-10 * ny)
    return st, ref


@pytest.mark.parametrize("shape,rank", [((8, 9, 10, 7), 3), ((6, 5, 7, 4, 8), 2), ((12, 10, 9), 4)])
@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_plain_ht_model_tensors(shape, rank, eps):
    spec = datagen.HTModelSpec(n=shape[1:], rank=rank, N=shape[0], n_batches=1, seed=21, batch_seed0=2100, nu=1e-3)
    check(next(datagen.ht_model_stream(spec)), eps)


def test_plain_ht_tiny_batch_as_a_mode():
    """The first tiny-stream batch (8 samples of 16^4) as the 5-way tensor (8, 16, 16, 16, 16)."""
    check(datagen.tiny_stream(1)[0], 1e-4)


def test_plain_ht_small_field_batch_as_a_mode():
    spec = datagen.FieldSpec(grid=(24, 24, 24), channels=3, terms=6, N=8, n_batches=1, drift=2e-3, seed=9,
                             batch_seed0=900, nu=0.0, w_lo=0.2, w_hi=0.5)
    check(datagen.exact_field_batch(spec, 0), 1e-4)
