"""GPU (MI355X) parity of the adaptive error budget (App. C, HT_ADAPTIVE_BUDGET) with
the oracle's adaptive mode: after each layer the nodewise tolerance of the layers
above is recomputed from the energy lost so far.  Ranks and skips must equal the
oracle's at every batch, reconstructions match it (FP64 1e-10, mixed 5e-6 of ||Y||),
and every batch meets its error bound; the closed-form case of the oracle pins (a
pair a_0 (x) b_1 that only the adaptive budget drops) is checked in both forms."""

import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import datagen  # noqa: E402
from oracle import ht_oracle as ho  # noqa: E402
from paper_2412_16544_amd import htrise as H  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_oracle_pins import _triple_batches, _x_for  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(y):
    return torch.from_numpy(np.ascontiguousarray(y)).to("cuda:0")


def check(ys, eps, prec, tol, slack):
    N = max(y.shape[0] for y in ys)
    st = H.HTStream(ys[0].shape[1:], eps, 64, N, sum(y.shape[0] for y in ys), prec=prec,
                    flags=H.HT_ADAPTIVE_BUDGET)
    ost = ho.BHT(ys[0].shape[1:], eps, adaptive=True)
    for k, y in enumerate(ys):
        info = st.push(dev(y))
        oinfo = ost.init_batch(y) if k == 0 else ost.update(y)
        assert st.ranks()[0] == oinfo.ranks, (k, st.ranks()[0], oinfo.ranks)
        if k > 0:
            assert info.skipped == oinfo.skipped, k
    rec = st.reconstruct().cpu().numpy()
    ref = ost.reconstruct()
    yall = np.concatenate([y.astype(np.float64) for y in ys])
    assert np.linalg.norm(rec - ref) <= tol * np.linalg.norm(yall)
    off = 0
    for y in ys:
        yy = y.astype(np.float64)
        assert np.linalg.norm(rec[off:off + y.shape[0]] - yy) <= eps * (1 + slack) * np.linalg.norm(yy)
        off += y.shape[0]
    return st, ost


FORMS = [(H.HT_FP64, 1e-10, 0.0), (H.HT_FP32, 5e-6, 1e-3)]


@pytest.mark.parametrize("prec,tol,slack", FORMS)
def test_adaptive_closed_form(prec, tol, slack):
    eps = 1e-3
    base = [(1.0, 0, 0, 0), (0.5, 1, 1, 1)]
    y10 = _x_for(10.0 / 1.35, eps, 1.25)
    x = _x_for(0.35, eps, 1.25 + y10 ** 2)
    ys = [y.astype(np.float32) for y in _triple_batches([base, base + [(y10, 2, 0, 0), (x, 0, 1, 0)]])]
    st, ost = check(ys, eps, prec, tol, slack)
    assert st.ranks()[0] == [3, 2, 3, 2]


@pytest.mark.parametrize("prec,tol,slack", FORMS)
@pytest.mark.parametrize("eps", [1e-4, 1e-3])
def test_adaptive_tiny_stream(prec, tol, slack, eps):
    check(datagen.tiny_stream(), eps, prec, tol, slack)


@pytest.mark.parametrize("prec,tol,slack", FORMS)
def test_adaptive_small_field_stream(prec, tol, slack):
    spec = datagen.FieldSpec(grid=(24, 24, 24), channels=3, terms=6, N=8, n_batches=8, drift=2e-3, seed=9,
                             batch_seed0=900, nu=0.0, w_lo=0.2, w_hi=0.5)
    check(list(datagen.exact_field_stream(spec)), 1e-4, prec, tol, slack)
