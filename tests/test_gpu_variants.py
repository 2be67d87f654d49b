"""GPU (MI355X) parity of the method's variants with the oracle's: ST-HOSVD within a
layer (HT_ST_HOSVD, the footnote of Sec. 2.3.1) and dimension trees other than the
balanced one (ht_config.tree_parent, Sec. 2.3).  Ranks and skips equal the oracle's
at every batch, reconstructions match (FP64 1e-10, mixed 5e-6 of ||Y||), every batch
meets its error bound; the closed forms of the oracle pins (a node that keeps fewer
directions on its predecessors' contracted tensor) hold in both forms."""

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
from test_oracle_pins import _diag_pairs, _diag_stream  # noqa: E402

pytestmark = pytest.mark.gpu

FORMS = [(H.HT_FP64, 1e-10, 0.0), (H.HT_FP32, 5e-6, 1e-3)]


def dev(y):
    return torch.from_numpy(np.ascontiguousarray(y)).to("cuda:0")


def check(ys, eps, prec, tol, slack, flags, oracle_kw, tree_parent=None):
    N = max(y.shape[0] for y in ys)
    st = H.HTStream(ys[0].shape[1:], eps, 64, N, sum(y.shape[0] for y in ys), prec=prec, flags=flags,
                    tree_parent=tree_parent)
    d = ys[0].ndim - 1
    tree = None if tree_parent is None else ho.DimTree(d, parent=tree_parent)
    ost = ho.BHT(ys[0].shape[1:], eps, tree=tree, **oracle_kw)
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


ST = dict(flags=H.HT_ST_HOSVD, oracle_kw=dict(st_hosvd=True))


@pytest.mark.parametrize("prec,tol,slack", FORMS)
def test_st_hosvd_closed_forms(prec, tol, slack):
    ys, _, _ = _diag_stream([((1.0, 0.3, 0.05, 7e-5, 5.2e-5), _diag_pairs(5))])
    st, _ = check([ys[0].astype(np.float32)], 1e-4, prec, tol, slack, **ST)
    assert st.ranks()[0] == [4, 3]
    eps = 1e-4
    c = {k: eps * eps * v / 2.0 for k, v in {"x": 10.0, "z": 0.9, "w": 0.5}.items()}
    total = 1.09 / (1.0 - sum(c.values()))
    x, z, w = (math.sqrt(c[k] * total) for k in ("x", "z", "w"))
    ys, _, _ = _diag_stream([((1.0, 0.3), _diag_pairs(2)), ((1.0, 0.3, x, z, w), _diag_pairs(5))])
    st, _ = check([y.astype(np.float32) for y in ys], eps, prec, tol, slack, **ST)
    assert st.ranks()[0] == [4, 3]


@pytest.mark.parametrize("prec,tol,slack", FORMS)
def test_st_hosvd_tiny_stream(prec, tol, slack):
    check(datagen.tiny_stream(), 1e-4, prec, tol, slack, **ST)


@pytest.mark.parametrize("prec,tol,slack", FORMS)
def test_st_hosvd_small_field_stream(prec, tol, slack):
    spec = datagen.FieldSpec(grid=(24, 24, 24), channels=3, terms=6, N=8, n_batches=8, drift=2e-3, seed=9,
                             batch_seed0=900, nu=0.0, w_lo=0.2, w_hi=0.5)
    check(list(datagen.exact_field_stream(spec)), 1e-4, prec, tol, slack, **ST)


@pytest.mark.parametrize("prec,tol,slack", FORMS)
def test_st_hosvd_with_adaptive_budget_d5(prec, tol, slack):
    spec = datagen.HTModelSpec(n=(9, 8, 7, 6, 5), rank=2, N=4, n_batches=4, seed=77, batch_seed0=7700, nu=1e-7,
                               grow_at=(2,), grow_by=1, grow_scale=0.1)
    check(list(datagen.ht_model_stream(spec)), 1e-4, prec, tol, slack,
          flags=H.HT_ST_HOSVD | H.HT_ADAPTIVE_BUDGET, oracle_kw=dict(st_hosvd=True, adaptive=True))


# unbalanced trees over runs of consecutive modes (numbered layer by layer, left to right)
TREES4 = [[-1, 0, 0, 1, 1, 3, 3], [-1, 0, 0, 2, 2, 4, 4]]
TREE5 = [-1, 0, 0, 2, 2, 3, 3, 4, 4]
PLAIN = dict(flags=0, oracle_kw={})


@pytest.mark.parametrize("prec,tol,slack", FORMS)
@pytest.mark.parametrize("parent", TREES4)
def test_other_trees_tiny_stream(prec, tol, slack, parent):
    st, _ = check(datagen.tiny_stream(), 1e-4, prec, tol, slack, tree_parent=parent, **PLAIN)
    assert st.ranks()[0] != [8] * 6   # not the generating (balanced) tree's ranks


@pytest.mark.parametrize("prec,tol,slack", FORMS)
@pytest.mark.parametrize("parent", TREES4)
def test_other_trees_small_field_stream(prec, tol, slack, parent):
    spec = datagen.FieldSpec(grid=(24, 24, 24), channels=3, terms=6, N=8, n_batches=8, drift=2e-3, seed=9,
                             batch_seed0=900, nu=0.0, w_lo=0.2, w_hi=0.5)
    check(list(datagen.exact_field_stream(spec)), 1e-4, prec, tol, slack, tree_parent=parent, **PLAIN)


@pytest.mark.parametrize("prec,tol,slack", FORMS)
def test_other_tree_d5_with_variants(prec, tol, slack):
    spec = datagen.HTModelSpec(n=(8, 9, 8, 7, 8), rank=3, N=4, n_batches=6, seed=77, batch_seed0=7700, nu=1e-6,
                               grow_at=(3, 4), grow_by=2, grow_scale=0.1)
    ys = list(datagen.ht_model_stream(spec))
    check(ys, 1e-4, prec, tol, slack, tree_parent=TREE5, **PLAIN)
    check(ys, 1e-4, prec, tol, slack, tree_parent=TREE5, flags=H.HT_ST_HOSVD | H.HT_ADAPTIVE_BUDGET,
          oracle_kw=dict(st_hosvd=True, adaptive=True))
