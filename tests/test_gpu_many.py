"""GPU (MI355X) tests of ht_rise_update_many: many independent streams in lock step.

Streams of uneven shapes (d = 3..5, so trees of depth 2 and 3 are aligned at their
leaves) advance together, one batch each per call.  The batched call runs the same
kernels as one ht_rise_update per stream (each eigen problem still gets a
workgroup of its own), so its results must equal the one-by-one updates bit for
bit, and the oracle's ranks and reconstructions as the single-stream tests demand.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import datagen  # noqa: E402
from oracle import ht_oracle as ho  # noqa: E402
from paper_2412_16544_amd import htrise as H  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(y):
    return torch.from_numpy(np.ascontiguousarray(y)).to("cuda:0")


def small_specs(count, n_batches=11, cap=1 << 17):
    """count - 1 streams of 3 or 4 modes under the cap, and one 16^5 stream (d = 5, a
    tree one layer deeper) with 4 samples."""
    specs = datagen.multi_stream_specs(count=count - 1, n_batches=n_batches, max_elements=cap, d_choices=(3, 4))
    specs.append(datagen.HTModelSpec(n=(16, 16, 16, 16, 16), rank=3, N=4, n_batches=n_batches, seed=4999,
                                     batch_seed0=499900, nu=1e-5, grow_at=(4, 8), grow_by=2, grow_scale=0.1))
    return specs


def make_streams(specs, data, prec, rank_cap=32):
    out = []
    for sp, ys in zip(specs, data):
        st = H.HTStream(sp.n, 1e-4, rank_cap, sp.N, sp.N * len(ys), prec=prec)
        st.push(dev(ys[0]))
        out.append(st)
    return out


@pytest.fixture(scope="module")
def six_streams():
    specs = small_specs(6)
    data = [list(datagen.ht_model_stream(sp)) for sp in specs]
    return specs, data


@pytest.mark.parametrize("prec", [H.HT_FP64, H.HT_FP32])
def test_many_equals_one_by_one(six_streams, prec):
    specs, data = six_streams
    a = make_streams(specs, data, prec)
    b = make_streams(specs, data, prec)
    nb = len(data[0])
    for k in range(1, nb):
        ia = [st.update(dev(ys[k])) for st, ys in zip(a, data)]
        st_code, ib = H.HTStream.update_many(b, [dev(ys[k]) for ys in data])
        assert st_code == H.HT_OK
        assert [i.skipped for i in ia] == [i.skipped for i in ib], k
        assert [i.status for i in ib] == [H.HT_OK] * len(b)
        for x, y in zip(a, b):
            assert x.ranks() == y.ranks(), k
    for x, y in zip(a, b):
        assert torch.equal(x.reconstruct(), y.reconstruct())


# reconstruction tolerance against the oracle (relative to the stream's norm): FP64
# arithmetic, and the mixed form's FP32 latent slices (relative error <~ sqrt(m) 2^-24
# per contraction level)
REC_TOL = {H.HT_FP64: 1e-10, H.HT_FP32: 5e-6}


@pytest.mark.parametrize("prec", [H.HT_FP64, H.HT_FP32])
def test_many_matches_oracle(six_streams, prec):
    """Every stream of the lock-step call against the oracle: skips and ranks after every
    batch, each batch's reconstruction error within eps ||Y_k|| (HT-RISE theorem), and
    the whole reconstruction against the oracle's."""
    specs, data = six_streams
    sts = make_streams(specs, data, prec)
    ors = []
    for ys in data:
        o = ho.BHT(ys[0].shape[1:], 1e-4)
        o.init_batch(ys[0])
        ors.append(o)
    for k in range(1, len(data[0])):
        code, infos = H.HTStream.update_many(sts, [dev(ys[k]) for ys in data])
        assert code == H.HT_OK
        oinfo = [o.update(ys[k]) for o, ys in zip(ors, data)]
        assert [i.skipped for i in infos] == [i.skipped for i in oinfo], k
        assert [s.ranks()[0] for s in sts] == [i.ranks for i in oinfo], k
    for s, o, ys, sp in zip(sts, ors, data, specs):
        rec_g = s.reconstruct().cpu().numpy()
        rec_o = o.reconstruct()
        yy = np.concatenate([y.astype(np.float64) for y in ys])
        assert np.linalg.norm(rec_g - rec_o) <= REC_TOL[prec] * np.linalg.norm(yy)
        for k in range(len(ys)):
            sl = slice(k * sp.N, (k + 1) * sp.N)
            err = np.linalg.norm(rec_g[sl] - yy[sl])
            assert err <= 1e-4 * (1 + 1e-3) * np.linalg.norm(yy[sl]), k


def test_many_rolls_back_only_the_failing_stream(six_streams):
    specs, data = six_streams
    # stream 0 gets a rank cap its growth at batch 4 cannot fit; the others are generous
    caps = [max(specs[0].rank, 1)] + [32] * 3
    sts = []
    for sp, ys, cap in zip(specs[:4], data[:4], caps):
        st = H.HTStream(sp.n, 1e-4, cap, sp.N, sp.N * len(ys))
        st.push(dev(ys[0]))
        sts.append(st)
    for k in range(1, 4):
        code, _ = H.HTStream.update_many(sts, [dev(ys[k]) for ys in data[:4]])
        assert code == H.HT_OK
    before = [s.ranks() for s in sts]
    before_rec0 = sts[0].reconstruct().cpu().numpy()
    code, infos = H.HTStream.update_many(sts, [dev(ys[4]) for ys in data[:4]])
    assert code == H.HT_ERANKCAP
    assert infos[0].status == H.HT_ERANKCAP
    assert [i.status for i in infos[1:]] == [H.HT_OK] * 3
    assert sts[0].ranks() == before[0]
    np.testing.assert_array_equal(sts[0].reconstruct().cpu().numpy(), before_rec0)
    for s, b, sp in zip(sts[1:], before[1:], specs[1:4]):
        assert s.ranks()[1] == b[1] + sp.N   # committed


@pytest.mark.parametrize("prec", [H.HT_FP64, H.HT_FP32])
def test_device_built_streams_match_oracle(prec):
    """Streams of the configured shapes' kind (3-5 modes, generating ranks up to 16),
    their batches built on the device (datagen.gpu.model_batches) and copied to the
    host for the oracle: ranks and skips after every batch and every batch's error bound."""
    from datagen import gpu as G
    specs = datagen.multi_stream_specs(count=3, seed0=4100, n_batches=11, max_elements=1 << 17,
                                       d_choices=(3, 4, 5), rank_hi=16)
    data = [list(G.model_batches(sp)) for sp in specs]
    host = [[y.cpu().numpy() for y in ys] for ys in data]
    sts = []
    ors = []
    for sp, ys, hs in zip(specs, data, host):
        st = H.HTStream(sp.n, 1e-4, 32, sp.N, sp.N * len(ys), prec=prec)
        st.push(ys[0])
        sts.append(st)
        o = ho.BHT(hs[0].shape[1:], 1e-4)
        o.init_batch(hs[0])
        ors.append(o)
    for k in range(1, len(data[0])):
        code, infos = H.HTStream.update_many(sts, [ys[k] for ys in data])
        assert code == H.HT_OK
        oinfo = [o.update(hs[k]) for o, hs in zip(ors, host)]
        assert [i.skipped for i in infos] == [i.skipped for i in oinfo], k
        assert [s.ranks()[0] for s in sts] == [i.ranks for i in oinfo], k
    for s, hs, sp in zip(sts, host, specs):
        rec = s.reconstruct().cpu().numpy()
        for k, y in enumerate(hs):
            yy = y.astype(np.float64)
            assert np.linalg.norm(rec[k * sp.N:(k + 1) * sp.N] - yy) <= 1e-4 * (1 + 1e-3) * np.linalg.norm(yy), k
