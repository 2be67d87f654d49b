"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes from
a construction with a closed form, a theorem of the paper, an invariant, or a
brute-force computation written differently from the oracle's code path.
"""

import math

import numpy as np
import pytest

import datagen
from oracle import ht_oracle as ho


# --------------------------------------------------------------------------- #
# Dimension tree (Sec. 2.3, Fig. dimension_trees)
# --------------------------------------------------------------------------- #


@pytest.mark.parametrize("d", range(2, 10))
def test_tree_shape(d):
    t = ho.DimTree(d)
    assert len(t.nodes) == 2 * d - 1
    assert t.depth == math.ceil(math.log2(d))
    leaves = [nd for nd in t.nodes if nd.is_leaf]
    assert sorted(nd.dim for nd in leaves) == list(range(d))
    # balanced: leaves only on the last two layers
    assert {nd.layer for nd in leaves} <= {t.depth, t.depth - 1}
    # every transfer node's two successors cover adjacent mode ranges, first one first
    for nd in t.nodes:
        if nd.children:
            a, b = (t.nodes[c] for c in nd.children)
            assert (a.lo, a.hi, b.lo, b.hi) == (nd.lo, b.lo, a.hi, nd.hi)
            assert a.child_pos == 0 and b.child_pos == 1
            assert a.hi - a.lo == (nd.hi - nd.lo + 1) // 2
    # layer-major, left-to-right numbering
    keys = [(nd.layer, nd.lo) for nd in t.nodes]
    assert keys == sorted(keys)


def test_tree_d5_and_d3_groupings():
    # d=5: {1,2,3},{4,5} -> {1,2},{3},{4},{5} -> {1},{2}
    t = ho.DimTree(5)
    got = [(nd.layer, nd.lo + 1, nd.hi) for nd in t.nodes]
    assert got == [(0, 1, 5), (1, 1, 3), (1, 4, 5), (2, 1, 2), (2, 3, 3), (2, 4, 4), (2, 5, 5),
                   (3, 1, 1), (3, 2, 2)]
    t3 = ho.DimTree(3)
    assert [(nd.layer, nd.lo + 1, nd.hi) for nd in t3.nodes] == [(0, 1, 3), (1, 1, 2), (1, 3, 3), (2, 1, 1), (2, 2, 2)]


# Trees given by a parent array: unbalanced shapes hold the same runs of modes as the
# definition, and every node's rank on exact data is the rank of its unfolding (the
# node's modes against the batch and all other modes), computed here directly.
OTHER_TREES = {
    4: [[-1, 0, 0, 1, 1, 3, 3],            # {1,2,3},{4} -> {1,2},{3} -> {1},{2}
        [-1, 0, 0, 2, 2, 4, 4]],           # {1},{2,3,4} -> {2},{3,4} -> {3},{4}
    5: [[-1, 0, 0, 2, 2, 3, 3, 4, 4]],     # {1},{2,3,4,5} -> {2,3},{4,5} -> leaves
}


def test_tree_from_parent_array():
    t = ho.DimTree(4, parent=OTHER_TREES[4][1])
    assert [(nd.layer, nd.lo + 1, nd.hi, nd.children) for nd in t.nodes] == [
        (0, 1, 4, (1, 2)), (1, 1, 1, ()), (1, 2, 4, (3, 4)), (2, 2, 2, ()), (2, 3, 4, (5, 6)), (3, 3, 3, ()),
        (3, 4, 4, ())]
    for d in (2, 3, 4, 5, 6):
        b = ho.DimTree(d)
        assert ho.DimTree(d, parent=b.parents()).nodes == b.nodes
    for bad in ([-1, 0, 0, 0, 1, 1, 2], [-1, 0, 0, 1, 1, 1, 1], [-1, 0, 0, 2, 2, 1, 1], [0, 0, 0, 1, 1, 2, 2],
                [-1, 0, 0, 3, 3, 4, 4]):
        with pytest.raises(ValueError):
            ho.DimTree(4, parent=bad)


def _unfolding_rank(y, nd):
    """Rank of the batch's unfolding with the node's modes as rows (sample modes start at axis 1)."""
    axes = list(range(1 + nd.lo, 1 + nd.hi))
    rest = [a for a in range(y.ndim) if a not in axes]
    m = np.transpose(y, axes + rest).reshape(int(np.prod([y.shape[a] for a in axes])), -1)
    sv = np.linalg.svd(m.astype(np.float64), compute_uv=False)
    return int(np.sum(sv > 1e-5 * sv[0]))


@pytest.mark.parametrize("d,k", [(4, 0), (4, 1), (5, 0)])
def test_other_trees_rank_is_the_unfolding_rank(d, k):
    spec = datagen.HTModelSpec(n=(9, 8, 7, 6) if d == 4 else (5, 6, 5, 4, 5), rank=3, N=6, n_batches=1, seed=11 + d,
                               batch_seed0=1100 + d, nu=0.0)
    y = next(iter(datagen.ht_model_stream(spec)))
    tree = ho.DimTree(d, parent=OTHER_TREES[d][k])
    o = ho.BHT(y.shape[1:], 1e-6, tree=tree)
    o.init_batch(y)
    assert o.ranks == [_unfolding_rank(y, nd) for nd in tree.non_root]
    # the balanced tree of the generating model gives its own ranks, not these
    ob = ho.BHT(y.shape[1:], 1e-6)
    ob.init_batch(y)
    assert ob.ranks == [_unfolding_rank(y, nd) for nd in ob.tree.non_root]
    assert ob.ranks != o.ranks
    rec = o.reconstruct()
    assert np.linalg.norm(rec - y) <= 1e-6 * np.linalg.norm(y)


# --------------------------------------------------------------------------- #
# Closed-form d = 2 case: BHT-l2r is a truncated HOSVD of the two sample modes
# (Sec. 2.2 Tucker format; Eq. ht_leaf_svd) with the batch mode untouched.
# --------------------------------------------------------------------------- #


def _diag_batch(s, n1=7, n2=6, N=5, seed=3):
    """Y[n] = sum_i s_i w[n,i] a_i b_i^T with orthonormal a, b, w: both unfoldings have singular values s."""
    g = np.random.default_rng(seed)
    k = len(s)
    a = np.linalg.qr(g.standard_normal((n1, k)))[0]
    b = np.linalg.qr(g.standard_normal((n2, k)))[0]
    w = np.linalg.qr(g.standard_normal((N, k)))[0]
    y = np.einsum("i,ni,xi,yi->nxy", np.asarray(s), w, a, b)
    return y, a, b, w


S_DIAG = (1.0, 0.3, 0.05, 4e-5, 1e-6)


def test_d2_rank_rule_closed_form():
    y, a, b, w = _diag_batch(S_DIAG)
    st = ho.BHT(y.shape[1:], 1e-4)
    st.init_batch(y)
    # ||Y||^2 = sum s^2; eps_nw^2 = 1e-8 ||Y||^2 / 2 = 5.46e-9; tail after 3 = 1.6e-9 + 1e-12 -> rank 3
    assert st.ranks == [3, 3]
    err2 = ho.fro2(st.reconstruct() - y)
    assert err2 == pytest.approx(4e-5 ** 2 + 1e-6 ** 2, rel=1e-6)
    # the kept leaf bases span the first three a_i / b_i
    for u, f in ((st.core[1], a), (st.core[2], b)):
        assert np.linalg.norm(u @ (u.T @ f[:, :3]) - f[:, :3]) < 1e-12
    # root slices: |root[i,j,n]| = s_i |w[n,i]| on the diagonal, 0 elsewhere
    root = st.root
    for i in range(3):
        np.testing.assert_allclose(np.abs(root[i, i, :]), S_DIAG[i] * np.abs(w[:, i]), rtol=1e-10, atol=1e-14)
    off = root.copy()
    for i in range(3):
        off[i, i, :] = 0
    assert np.max(np.abs(off)) < 1e-12


def test_budget_denominator_is_2d_minus_2():
    """At eps = 5e-5 the tail after 3 lies between eps^2||Y||^2/2 and eps^2||Y||^2.

    With the sqrt(2d-2) = sqrt(2) share of the BHT-l2r corollary the rank is 4;
    the sqrt(2d-3) = 1 share of the plain-HT theorem would give 3.
    """
    y, *_ = _diag_batch(S_DIAG)
    st = ho.BHT(y.shape[1:], 5e-5)
    st.init_batch(y)
    assert st.ranks == [4, 4]


def test_rank_floor_is_one_for_bht_l2r():
    y, *_ = _diag_batch((1.0, 1e-9))
    st = ho.BHT(y.shape[1:], 0.5)
    st.init_batch(y)
    assert st.ranks == [1, 1]


# --------------------------------------------------------------------------- #
# Truncation: the reported discarded energy is the explicit projection residual
# (Eckart-Young), and the Gram branch agrees with the SVD branch.
# --------------------------------------------------------------------------- #


def test_truncation_tail_equals_explicit_residual():
    g = np.random.default_rng(11)
    m = g.standard_normal((9, 40)) * np.logspace(0, -6, 9)[:, None]
    for eps_nw in (1e-1, 1e-3, 1e-5):
        u, t = ho.truncated_svd(m, eps_nw, rmin=1)
        resid = m - u @ (u.T @ m)
        assert ho.fro2(resid) == pytest.approx(t.tail2, rel=1e-9, abs=1e-28)
        assert math.sqrt(t.tail2) <= eps_nw
        # one rank fewer would break the bound (minimality)
        if t.rank > 1:
            u1 = u[:, :-1]
            assert math.sqrt(ho.fro2(m - u1 @ (u1.T @ m))) > eps_nw


def test_gram_branch_matches_svd_branch(monkeypatch):
    g = np.random.default_rng(12)
    m = g.standard_normal((30, 500)) * np.logspace(0, -5, 30)[:, None]
    u1, t1 = ho.truncated_svd(m, 1e-3, rmin=1)
    monkeypatch.setattr(ho, "SVD_DIRECT_MAX_ENTRIES", 10)
    u2, t2 = ho.truncated_svd(m, 1e-3, rmin=1)
    assert t1.rank == t2.rank
    np.testing.assert_allclose(t2.sigma[: t1.rank], t1.sigma[: t1.rank], rtol=1e-12)
    np.testing.assert_allclose(np.abs(u1.T @ u2), np.eye(t1.rank), atol=1e-10)


def test_sign_normalisation():
    u = np.array([[0.1, -0.9], [-0.8, 0.2], [0.5, 0.3]])
    v = ho.sign_normalise(u)
    assert v[1, 0] > 0 and v[0, 1] > 0
    np.testing.assert_array_equal(np.abs(u), np.abs(v))


# --------------------------------------------------------------------------- #
# Exact-rank stream: 16^4, N=8, rank 4, +2 fresh directions at batches 3 and 4
# --------------------------------------------------------------------------- #


@pytest.fixture(scope="module")
def tiny_run():
    ys = datagen.tiny_stream()
    st = ho.BHT(ys[0].shape[1:], 1e-4)
    infos, recon0, snapshots = [], [], []
    for k, y in enumerate(ys):
        info = st.init_batch(y) if k == 0 else st.update(y)
        infos.append(info)
        recon0.append(st.reconstruct(0, ys[0].shape[0]))
        snapshots.append({i: c.copy() for i, c in st.core.items()})
    return ys, st, infos, recon0, snapshots


def test_exact_recovery_ranks_and_skips(tiny_run):
    ys, st, infos, _, _ = tiny_run
    # P6 / P7: ranks of the generating construction, skips where no direction is new
    assert [i.ranks for i in infos] == [[4] * 6, [4] * 6, [4] * 6, [6] * 6, [8] * 6]
    assert [i.skipped for i in infos] == [False, True, True, False, False]
    assert st.root.shape == (8, 8, 40)


def test_per_batch_error_bound_and_noise_level(tiny_run):
    ys, st, infos, _, _ = tiny_run
    off = 0
    for y, info in zip(ys, infos):
        y64 = y.astype(np.float64)
        rec = st.reconstruct(off, y.shape[0])
        err = math.sqrt(ho.fro2(rec - y64))
        assert err <= 1e-4 * math.sqrt(ho.fro2(y64))            # P2
        assert err / math.sqrt(ho.fro2(y64)) < 2e-6             # P6: noise level (nu = 1e-6)
        off += y.shape[0]


def test_orthonormal_cores(tiny_run):
    _, st, _, _, snapshots = tiny_run
    for snap in snapshots:                                      # P1
        for idx, u in snap.items():
            assert np.linalg.norm(u.T @ u - np.eye(u.shape[1])) < 1e-13


def test_norm_identity(tiny_run):
    ys, st, _, _, _ = tiny_run
    for y in ys:                                                # P3
        y64 = y.astype(np.float64)
        c1 = st.project(y64)
        rec = st.decode(c1)
        lhs = ho.fro2(y64 - rec)
        rhs = ho.fro2(y64) - ho.fro2(c1)
        assert abs(lhs - rhs) <= 1e-10 * ho.fro2(y64)


def test_layerwise_bound(tiny_run):
    ys, st, infos, _, _ = tiny_run
    off = 0
    for y, info in zip(ys, infos):                              # P4
        if not info.skipped:
            rec = st.reconstruct(off, y.shape[0])
            err2 = ho.fro2(rec - y.astype(np.float64))
            bound = sum(t.tail2 for t in info.decisions.values())
            assert err2 <= bound * (1 + 1e-9)
        off += y.shape[0]


def test_past_stream_invariance(tiny_run):
    _, _, _, recon0, _ = tiny_run
    for r in recon0[1:]:                                        # P5
        assert np.linalg.norm(r - recon0[0]) <= 1e-14 * np.linalg.norm(recon0[0])


def test_new_directions_span_the_fresh_leaf_columns(tiny_run):
    """After batch 3 every leaf basis contains the two fresh generating directions."""
    ys, st, _, _, snapshots = tiny_run
    # rebuild the generating frames of batch 3 with the generator's own seeds
    spec = datagen.HTModelSpec(n=(16, 16, 16, 16), rank=4, N=8, n_batches=5, seed=1, batch_seed0=100,
                               nu=1e-6, grow_at=(3, 4), grow_by=2, grow_scale=0.1)
    g = datagen.rng(spec.seed)
    base = datagen._build_frames(g, spec.n, datagen._feasible_ranks(spec.n, 4), [])
    fresh = datagen._build_frames(g, spec.n, datagen._feasible_ranks(spec.n, 2), [base])
    snap = snapshots[3]
    for leaf_idx, dim in ((3, 0), (4, 1), (5, 2), (6, 3)):
        u = snap[leaf_idx]
        for f in (base.leaf[dim], fresh.leaf[dim]):
            assert np.linalg.norm(f - u @ (u.T @ f)) < 1e-4


def test_zero_padding_of_parents_and_root(tiny_run):
    _, st, infos, _, snapshots = tiny_run
    # transfer node 1 (children 3, 4) after batch 3: old columns are zero outside the old 4x4 block
    g = snapshots[3][1].reshape(6, 6, 6)
    assert np.all(g[4:, :, :4] == 0) and np.all(g[:, 4:, :4] == 0)
    # root slices of the first 24 samples are zero outside the old 4x4 block
    assert np.all(st.root[4:, :, :24] == 0) and np.all(st.root[:, 4:, :24] == 0)
    assert np.all(st.root[6:, :, :32] == 0) and np.all(st.root[:, 6:, :32] == 0)


def test_duplicate_batch_skips_with_same_root_slice(tiny_run):
    ys, st, _, _, _ = tiny_run
    st2 = ho.BHT(ys[0].shape[1:], 1e-4)
    st2.init_batch(ys[0])
    info = st2.update(ys[0])                                     # P10
    assert info.skipped
    np.testing.assert_allclose(st2.root[:, :, 8:], st2.root[:, :, :8], rtol=0, atol=1e-12 * np.abs(st2.root).max())


# --------------------------------------------------------------------------- #
# Reconstruction against a dense network contraction (different code path)
# --------------------------------------------------------------------------- #


def test_reconstruction_equals_dense_network_contraction(tiny_run):
    _, st, _, _, _ = tiny_run
    g1 = st.core3(1)
    g2 = st.core3(2)
    u1, u2, u3, u4 = (st.core[i] for i in (3, 4, 5, 6))
    dense = np.einsum("ijn,abi,cdj,wa,xb,yc,zd->nwxyz", st.root, g1, g2, u1, u2, u3, u4, optimize=True)
    np.testing.assert_allclose(st.reconstruct(), dense, rtol=0, atol=1e-12 * np.abs(dense).max())


# --------------------------------------------------------------------------- #
# Other orders and trees: exact HT rank is recovered for d = 3 and d = 5
# --------------------------------------------------------------------------- #


@pytest.mark.parametrize("n,rank", [((9, 8, 7), 3), ((6, 5, 7, 4, 3), 2)])
def test_exact_recovery_other_orders(n, rank):
    spec = datagen.HTModelSpec(n=n, rank=rank, N=6, n_batches=3, seed=21, batch_seed0=2100, nu=1e-7,
                               grow_at=(2,), grow_by=1, grow_scale=0.1)
    ys = list(datagen.ht_model_stream(spec))
    st = ho.BHT(n, 1e-4)
    infos = [st.init_batch(ys[0])] + [st.update(y) for y in ys[1:]]
    t = st.tree
    expect0 = []
    for nd in t.non_root:
        if nd.is_leaf:
            expect0.append(min(rank, n[nd.dim]))
        else:
            expect0.append(rank)
    assert infos[0].ranks == expect0
    assert infos[1].skipped
    assert infos[2].ranks == [r + 1 for r in expect0]
    off = 0
    for y in ys:
        rec = st.reconstruct(off, y.shape[0])
        y64 = y.astype(np.float64)
        assert math.sqrt(ho.fro2(rec - y64)) <= 1e-6 * math.sqrt(ho.fro2(y64))
        off += y.shape[0]


def test_full_rank_at_tiny_tolerance_reproduces_input():
    g = np.random.default_rng(5)
    y = g.standard_normal((3, 3, 4, 2))
    st = ho.BHT(y.shape[1:], 1e-13)
    st.init_batch(y)
    np.testing.assert_allclose(st.reconstruct(), y, atol=1e-12)


def test_all_zero_update_skips_and_appends_zeros(tiny_run):
    ys, _, _, _, _ = tiny_run
    st = ho.BHT(ys[0].shape[1:], 1e-4)
    st.init_batch(ys[0])
    info = st.update(np.zeros_like(ys[0]))
    assert info.skipped and np.all(st.root[:, :, 8:] == 0)


def test_zero_initial_batch_rejected():
    with pytest.raises(ValueError):
        ho.BHT((3, 3), 1e-3).init_batch(np.zeros((2, 3, 3)))


# --------------------------------------------------------------------------- #
# Closed-form HT-RISE updates (d = 2, diagonal structure, known residual spectra)
# --------------------------------------------------------------------------- #


def _diag_stream(s_list, n1=9, n2=8, N=6, seed=31):
    """Batches Y_k[n] = sum_i s_k[i] w_k[n,i] a_i b_{pi(i)}^T sharing one set of orthonormal a, b."""
    g = np.random.default_rng(seed)
    k = max(len(s) for s, _ in s_list)
    a = np.linalg.qr(g.standard_normal((n1, k)))[0]
    b = np.linalg.qr(g.standard_normal((n2, k)))[0]
    out = []
    for s, pairs in s_list:
        w = np.linalg.qr(g.standard_normal((N, len(s))))[0]
        y = np.zeros((N, n1, n2))
        for col, (si, (ia, ib)) in enumerate(zip(s, pairs)):
            y += si * np.einsum("n,x,y->nxy", w[:, col], a[:, ia], b[:, ib])
        out.append(y)
    return out, a, b


def _diag_pairs(k):
    return [(i, i) for i in range(k)]


def test_rise_budget_is_2d_minus_2():
    """Residual spectrum (0.05, 4e-5, 1e-6) at eps = 5e-5: two new directions with sqrt(2d-2), one with 1."""
    ys, _, _ = _diag_stream([((1.0, 0.3), _diag_pairs(2)), ((1.0, 0.3, 0.05, 4e-5, 1e-6), _diag_pairs(5))])
    st = ho.BHT(ys[0].shape[1:], 5e-5)
    st.init_batch(ys[0])
    assert st.ranks == [2, 2]
    info = st.update(ys[1])
    assert not info.skipped
    assert st.ranks == [4, 4]


@pytest.mark.parametrize("factor,skips", [(1.5, False), (0.9, True)])
def test_skip_threshold_is_relative_to_new_batch(factor, skips):
    """A new direction of energy x^2 gives eps_proj = x exactly (Claim on orthogonal reconstructions)."""
    eps = 1e-4
    base2 = 1.0 + 0.09
    # x = factor * eps * ||Y2||, with ||Y2||^2 = base2 + x^2
    x = factor * eps * math.sqrt(base2 / (1 - (factor * eps) ** 2))
    ys, _, _ = _diag_stream([((1.0, 0.3), _diag_pairs(2)), ((1.0, 0.3, x), _diag_pairs(3))])
    st = ho.BHT(ys[0].shape[1:], eps)
    st.init_batch(ys[0] * 1e3)            # the scale of earlier batches must not matter
    info = st.update(ys[1])
    assert info.eps_proj == pytest.approx(x, rel=1e-6)
    assert info.skipped is skips
    assert st.ranks == ([2, 2] if skips else [3, 3])


def test_one_sided_growth_pads_the_right_root_axis():
    """The new direction a_2 x b_0 only grows leaf 1: the root is padded on its first axis."""
    ys, _, _ = _diag_stream([((1.0, 0.3), _diag_pairs(2)), ((1.0, 0.3, 0.2), [(0, 0), (1, 1), (2, 0)])])
    st = ho.BHT(ys[0].shape[1:], 1e-4)
    st.init_batch(ys[0])
    st.update(ys[1])
    assert st.ranks == [3, 2]
    assert st.root.shape == (3, 2, 12)
    assert np.all(st.root[2, :, :6] == 0)
    for k, y in enumerate(ys):
        rec = st.reconstruct(6 * k, 6)
        assert math.sqrt(ho.fro2(rec - y)) <= 1e-12 * math.sqrt(ho.fro2(y))


def test_layer_nodes_see_the_same_tensor():
    """HOSVD within a layer (not ST-HOSVD): s = (1, .3, .05, 7e-5, 5.2e-5) at eps = 1e-4.

    Leaf 1 keeps 4 (tail 0.50 thr); with HOSVD leaf 2 sees the same spectrum and keeps 4,
    whereas on the tensor already contracted with leaf 1 it would see (1, .3, .05, 7e-5)
    and keep 3 (tail 0.90 thr).
    """
    ys, _, _ = _diag_stream([((1.0, 0.3, 0.05, 7e-5, 5.2e-5), _diag_pairs(5))])
    st = ho.BHT(ys[0].shape[1:], 1e-4)
    st.init_batch(ys[0])
    assert st.ranks == [4, 4]


def test_scale_invariance_of_the_stream():
    ys = datagen.tiny_stream()
    st = ho.BHT(ys[0].shape[1:], 1e-4)
    infos = [st.init_batch(ys[0].astype(np.float64) * 1e3)]
    infos += [st.update(y.astype(np.float64) * 1e3) for y in ys[1:]]
    assert [i.ranks[0] for i in infos] == [4, 4, 4, 6, 8]
    assert [i.skipped for i in infos] == [False, True, True, False, False]


def test_first_layer_decisions_use_the_raw_batch():
    """Leaf decisions of the deepest layer carry the singular values of Y's own unfoldings."""
    ys = datagen.tiny_stream(1)
    y = ys[0].astype(np.float64)
    st = ho.BHT(y.shape[1:], 1e-4)
    info = st.init_batch(y)
    for idx, dim in ((3, 0), (4, 1), (5, 2), (6, 3)):
        m = np.moveaxis(y, 1 + dim, 0).reshape(16, -1)
        lam = np.sort(np.linalg.eigvalsh(m @ m.T))[::-1]
        np.testing.assert_allclose(info.decisions[idx].sigma[:4] ** 2, lam[:4], rtol=1e-10)


def test_relative_test_errors_closed_form():
    """Relative test error (Sec. 4.1, Eq. generalization_performance): a held-out sample
    y_n = sum_i s_i w_ni a_i b_i^T whose third direction lies outside the trained span
    {a_0, a_1} x {b_0, b_1} has error |s_2 w_n2| / sqrt(sum_i s_i^2 w_ni^2); a sample
    inside the span has none."""
    ys, _, _ = _diag_stream([((1.0, 0.3), _diag_pairs(2)), ((1.0, 0.3, 0.2), _diag_pairs(3)),
                             ((0.7, 0.4), _diag_pairs(2))])
    st = ho.BHT(ys[0].shape[1:], 1e-6)
    st.init_batch(ys[0])
    assert st.ranks == [2, 2]
    # the weights w of batch 1 are recovered from the data: w_ni = <y_n, a_i b_i^T> / s_i
    g = np.random.default_rng(31)
    a = np.linalg.qr(g.standard_normal((9, 3)))[0]
    b = np.linalg.qr(g.standard_normal((8, 3)))[0]
    s = np.array([1.0, 0.3, 0.2])
    w = np.array([[np.sum(yn * np.outer(a[:, i], b[:, i])) / s[i] for i in range(3)] for yn in ys[1]])
    expect = np.abs(s[2] * w[:, 2]) / np.sqrt(np.sum((s[None, :] * w) ** 2, axis=1))
    np.testing.assert_allclose(st.relative_test_errors(ys[1]), expect, rtol=1e-10)
    assert np.max(st.relative_test_errors(ys[2])) < 1e-13


# --------------------------------------------------------------------------- #
# Adaptive error budget (App. C)
# --------------------------------------------------------------------------- #


def _triple_batches(terms_list, n=(9, 8, 7), N=6, seed=5):
    """d = 3 batches y = sum_t s_t w_t (x) a_{i_t} (x) b_{j_t} (x) c_{k_t} with orthonormal
    a, b, c sets and orthonormal sample weights w (one per term).  Tree {1,2},{3}:
    the leaves see the a-, b- and c-directions, the (1,2) transfer node the pairs
    a_i (x) b_j."""
    g = np.random.default_rng(seed)
    a = np.linalg.qr(g.standard_normal((n[0], 4)))[0]
    b = np.linalg.qr(g.standard_normal((n[1], 4)))[0]
    c = np.linalg.qr(g.standard_normal((n[2], 4)))[0]
    out = []
    for terms in terms_list:
        w = np.linalg.qr(g.standard_normal((N, len(terms))))[0]
        y = np.zeros((N,) + n)
        for t, (st, i, j, k) in enumerate(terms):
            y += st * np.einsum("n,x,y,z->nxyz", w[:, t], a[:, i], b[:, j], c[:, k])
        out.append(y)
    return out


def _x_for(frac, eps, base2):
    """x with x^2 = frac * eps^2 * (base2 + x^2)."""
    c = frac * eps * eps
    return math.sqrt(c * base2 / (1.0 - c))


def test_adaptive_budget_bht_l2r_closed_form():
    """The pair a_0 (x) b_1 carries x^2 = 0.35 eps^2 ||Y||^2 at the (1,2) node only: the
    leaves lose nothing, so App. C's tolerance for layer 1 is eps_abs^2 / 2 (two SVDs
    left) instead of eps_abs^2 / 4: the fixed budget keeps the pair (rank 3), the
    adaptive one drops it (rank 2), and the error is exactly x."""
    eps = 1e-3
    x = _x_for(0.35, eps, 1.25)
    (y,) = _triple_batches([[(1.0, 0, 0, 0), (0.5, 1, 1, 1), (x, 0, 1, 0)]])
    fixed = ho.BHT(y.shape[1:], eps)
    fixed.init_batch(y)
    adapt = ho.BHT(y.shape[1:], eps, adaptive=True)
    adapt.init_batch(y)
    assert fixed.ranks == [3, 2, 2, 2]
    assert adapt.ranks == [2, 2, 2, 2]
    err = math.sqrt(ho.fro2(adapt.reconstruct() - y))
    assert err == pytest.approx(x, rel=1e-8)
    assert err <= eps * math.sqrt(ho.fro2(y))
    # d = 2 has a single layer: nothing to adapt
    ys, _, _ = _diag_stream([((1.0, 0.3, 0.05, 4e-5, 1e-6), _diag_pairs(5))])
    for e in (1e-4, 5e-5):
        f2, a2 = ho.BHT(ys[0].shape[1:], e), ho.BHT(ys[0].shape[1:], e, adaptive=True)
        f2.init_batch(ys[0])
        a2.init_batch(ys[0])
        assert f2.ranks == a2.ranks


def test_adaptive_budget_ht_rise_closed_form():
    """HT-RISE: a new leaf direction a_2 (x) b_0 of energy 10 eps^2 ||Y||^2 forces an
    update that the leaves absorb exactly; the pair a_0 (x) b_1 of energy
    0.35 eps_des^2 is kept at the (1,2) node by the fixed budget (eps_des^2 / 4) and
    dropped by the adaptive one (eps_des^2 / 2)."""
    eps = 1e-3
    base = [(1.0, 0, 0, 0), (0.5, 1, 1, 1)]
    y10 = _x_for(10.0 / 1.35, eps, 1.25)  # rough size; the exact fractions follow from the norms
    x = _x_for(0.35, eps, 1.25 + y10 ** 2)
    y0, y1 = _triple_batches([base, base + [(y10, 2, 0, 0), (x, 0, 1, 0)]])
    ny2 = ho.fro2(y1)
    assert x * x == pytest.approx(0.35 * eps * eps * ny2, rel=1e-9)
    fixed = ho.BHT(y0.shape[1:], eps)
    adapt = ho.BHT(y0.shape[1:], eps, adaptive=True)
    for st in (fixed, adapt):
        st.init_batch(y0)
        assert st.ranks == [2, 2, 2, 2]
        info = st.update(y1)
        assert not info.skipped
    assert fixed.ranks == [4, 2, 3, 2]
    assert adapt.ranks == [3, 2, 3, 2]
    err = math.sqrt(ho.fro2(adapt.reconstruct(6, 6) - y1))
    assert err == pytest.approx(x, rel=1e-6)
    assert err <= eps * math.sqrt(ny2)


def test_adaptive_budget_meets_the_bound_on_the_tiny_stream():
    ys = datagen.tiny_stream()
    st = ho.BHT(ys[0].shape[1:], 1e-4, adaptive=True)
    for k, y in enumerate(ys):
        (st.init_batch if k == 0 else st.update)(y)
    for k, y in enumerate(ys):
        yy = y.astype(np.float64)
        assert math.sqrt(ho.fro2(st.reconstruct(8 * k, 8) - yy)) <= 1e-4 * math.sqrt(ho.fro2(yy))


# --------------------------------------------------------------------------- #
# Plain leaves-to-root HT (Sec. 2.3.1), the baseline of the format comparison
# --------------------------------------------------------------------------- #


def test_plain_ht_of_a_matrix_is_the_truncated_svd():
    """d = 2: one SVD with eps_nw = eps ||Y|| / sqrt(2*2-3) = eps ||Y||: the rank is the
    smallest r whose tail of squared singular values is <= eps^2 ||Y||^2, the root holds
    the kept singular values and the error is the tail."""
    g = np.random.default_rng(3)
    s = np.array([1.0, 0.5, 0.1, 0.03, 0.009, 0.001])
    u = np.linalg.qr(g.standard_normal((9, 6)))[0]
    v = np.linalg.qr(g.standard_normal((7, 6)))[0]
    y = (u * s) @ v.T
    for eps, r in ((0.05, 3), (0.02, 4), (0.005, 5)):
        ht = ho.PlainHT(y, eps)
        tail = np.sum(s[r:] ** 2)
        assert tail <= (eps * np.linalg.norm(s)) ** 2 < np.sum(s[r - 1:] ** 2)
        assert ht.ranks == [r, r]
        np.testing.assert_allclose(np.diag(ht.root), s[:r], rtol=1e-12)
        assert math.sqrt(ho.fro2(ht.reconstruct() - y)) == pytest.approx(math.sqrt(tail), rel=1e-8)


def test_plain_ht_budget_is_2d_minus_3():
    """d = 3 diagonal tensor s_t a_t (x) b_t (x) c_t with x^2 = 0.3 eps^2 ||Y||^2 on its last
    term: the plain-HT tolerance eps^2 ||Y||^2 / 3 drops it at the leaves (rank 2), the
    batch format's eps^2 ||Y||^2 / 4 would keep it (rank 3); the error is exactly x."""
    g = np.random.default_rng(8)
    a, b, c = (np.linalg.qr(g.standard_normal((n, 3)))[0] for n in (8, 7, 6))
    eps = 1e-3
    x = _x_for(0.3, eps, 1.09)
    s = (1.0, 0.3, x)
    y = sum(st * np.einsum("i,j,k->ijk", a[:, t], b[:, t], c[:, t]) for t, st in enumerate(s))
    ht = ho.PlainHT(y, eps)
    assert ht.ranks == [2, 2, 2, 2]
    assert math.sqrt(ho.fro2(ht.reconstruct() - y)) == pytest.approx(x, rel=1e-6)
    bht = ho.BHT(y.shape, eps)
    bht.init_batch(y[None])
    assert bht.ranks[2:] == [3, 3]


@pytest.mark.parametrize("shape,rank", [((8, 9, 10, 7), 3), ((6, 5, 7, 4, 8), 2), ((12, 10, 9), 4)])
def test_plain_ht_bound_orthonormal_cores_and_diagonal_root(shape, rank):
    """Thm. ht_nodewise_error: ||Y - Y_hat|| <= eps ||Y||; every core orthonormal; the
    root is diagonal and non-increasing; exact low-rank data is recovered."""
    spec = datagen.HTModelSpec(n=shape[1:], rank=rank, N=shape[0], n_batches=1, seed=21, batch_seed0=2100,
                               nu=1e-3)
    y = next(datagen.ht_model_stream(spec)).astype(np.float64)
    for eps in (1e-2, 1e-4):
        ht = ho.PlainHT(y, eps)
        assert math.sqrt(ho.fro2(ht.reconstruct() - y)) <= eps * math.sqrt(ho.fro2(y))
        for u in ht.core.values():
            np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-12)
        sv = np.diag(ht.root)
        assert np.all(np.diff(sv) <= 0) and np.allclose(ht.root, np.diag(sv))


# --------------------------------------------------------------------------- #
# ST-HOSVD within a layer (the footnote of Sec. 2.3.1)
# --------------------------------------------------------------------------- #


def test_st_hosvd_bht_l2r_closed_form():
    """The spectrum of the HOSVD pin: with ST-HOSVD leaf 2 sees the tensor leaf 1 has
    contracted, (1, .3, .05, 7e-5) at tail 0.90 thr, and keeps 3."""
    ys, _, _ = _diag_stream([((1.0, 0.3, 0.05, 7e-5, 5.2e-5), _diag_pairs(5))])
    st = ho.BHT(ys[0].shape[1:], 1e-4, st_hosvd=True)
    st.init_batch(ys[0])
    assert st.ranks == [4, 3]
    assert math.sqrt(ho.fro2(st.reconstruct() - ys[0])) <= 1e-4 * math.sqrt(ho.fro2(ys[0]))


def test_st_hosvd_ht_rise_closed_form():
    """A residual spectrum (x, z, w) with z^2 = 0.9 thr, w^2 = 0.5 thr (thr = eps_des^2 / 2):
    leaf 1 keeps x and z (dropping z too would leave 1.4 thr); with HOSVD leaf 2 sees the
    same and keeps 2, with ST-HOSVD it sees the tensor leaf 1 contracted, where w is
    gone, and keeps only x."""
    eps = 1e-4
    fr = {"x": 10.0, "z": 0.9, "w": 0.5}
    c = {k: eps * eps * v / 2.0 for k, v in fr.items()}
    total = 1.09 / (1.0 - sum(c.values()))
    x, z, w = (math.sqrt(c[k] * total) for k in ("x", "z", "w"))
    ys, _, _ = _diag_stream([((1.0, 0.3), _diag_pairs(2)), ((1.0, 0.3, x, z, w), _diag_pairs(5))])
    hosvd, st = ho.BHT(ys[0].shape[1:], eps), ho.BHT(ys[0].shape[1:], eps, st_hosvd=True)
    for s in (hosvd, st):
        s.init_batch(ys[0])
        assert not s.update(ys[1]).skipped
    assert hosvd.ranks == [4, 4]
    assert st.ranks == [4, 3]
    err = math.sqrt(ho.fro2(st.reconstruct(6, 6) - ys[1]))
    assert err == pytest.approx(math.sqrt(z * z + w * w), rel=1e-6)
    assert err <= eps * math.sqrt(ho.fro2(ys[1]))


def test_st_hosvd_meets_the_bound_on_the_tiny_stream():
    ys = datagen.tiny_stream()
    st = ho.BHT(ys[0].shape[1:], 1e-4, st_hosvd=True)
    for k, y in enumerate(ys):
        (st.init_batch if k == 0 else st.update)(y)
    assert st.ranks == [8] * 6
    for k, y in enumerate(ys):
        yy = y.astype(np.float64)
        assert math.sqrt(ho.fro2(st.reconstruct(8 * k, 8) - yy)) <= 1e-4 * math.sqrt(ho.fro2(yy))


# --------------------------------------------------------------------------- #
# Decision bookkeeping: the near-tie flag, the residual rank cap, the stream helper
# --------------------------------------------------------------------------- #


def test_near_tie_flags_a_tail_at_the_threshold():
    """d = 2 closed form (both unfoldings have singular values s): with s_3 placed so
    that the tail of rank 2 is eps_nw^2 (1 + delta), the decision keeps 3 directions
    and is a near tie for a band wider than delta, not for a narrower one."""
    eps = 1e-3
    base = np.array([1.0, 0.5])
    for delta, band, expect in ((1e-7, 1e-5, True), (1e-7, 1e-9, False), (1e-3, 1e-5, False)):
        # ||Y||^2 = 1.25 + s3^2 and eps_nw^2 = eps^2 ||Y||^2 / 2; s3^2 = eps_nw^2 (1 + delta)
        c = eps * eps * (1.0 + delta) / 2.0
        s3 = math.sqrt(c * 1.25 / (1.0 - c))
        y, _, _, _ = _diag_batch(np.concatenate([base, [s3]]))
        o = ho.BHT(y.shape[1:], eps)
        info = o.init_batch(y)
        assert o.ranks == [3, 3]
        assert info.any_near_tie(band) is expect, (delta, band)
        t = info.decisions[1]
        thr = t.eps_nw ** 2
        assert abs(t.tail2_prev - thr) == pytest.approx(delta * thr, rel=1e-3)


def test_residual_rank_cap_is_the_complement_of_the_old_basis():
    """At eps = 1e-17 the truncation of a residual would also keep the rounding noise
    left along the old basis (~1e-16 of the batch, far above eps_nw); the cap
    alpha - r_old keeps each node to its mode size, and the cores stay orthonormal."""
    g = np.random.default_rng(5)
    n1, n2, N = 4, 5, 12
    a = np.linalg.qr(g.standard_normal((n1, n1)))[0]
    b = np.linalg.qr(g.standard_normal((n2, n2)))[0]
    y0 = np.einsum("ni,xi,yi->nxy", g.standard_normal((N, 2)), a[:, :2], b[:, :2])
    y1 = g.standard_normal((N, n1, n2))            # full rank: every direction is new
    o = ho.BHT((n1, n2), 1e-17)
    o.init_batch(y0)
    r_old = list(o.ranks)        # at this tolerance the first batch's noise is kept too
    info = o.update(y1)
    assert not info.skipped
    assert o.ranks == [n1, n2]   # never beyond the mode size
    for idx, r0 in zip((1, 2), r_old):
        u = o.core[idx]
        assert np.allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-12)
        assert info.decisions[idx].rmax == u.shape[0] - r0


def test_compress_stream_is_init_then_updates():
    ys = datagen.tiny_stream()
    a = ho.compress_stream(ys, 1e-4)
    b = ho.BHT(ys[0].shape[1:], 1e-4)
    b.init_batch(ys[0])
    for y in ys[1:]:
        b.update(y)
    assert a.ranks == b.ranks and a.n_accum == b.n_accum
    assert np.array_equal(a.reconstruct(), b.reconstruct())
