"""Kernel-level parity of the HIP library with NumPy FP64, through the C ABI test entry points."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2412_16544_amd import htrise as H  # noqa: E402

pytestmark = pytest.mark.gpu


def rng(seed):
    return np.random.default_rng(seed)


def unfold_np(x, P, m, S):
    return x.reshape(P, m, S).transpose(1, 0, 2).reshape(m, P * S)


@pytest.mark.parametrize("n,dtype", [(1, np.float32), (1000, np.float64), (1 << 20, np.float32), (3_000_001, np.float64)])
def test_sumsq(n, dtype):
    x = rng(1).standard_normal(n).astype(dtype)
    got = H.ht_test_sumsq(torch.from_numpy(x).cuda()).item()
    ref = float(np.sum(x.astype(np.float64) ** 2))
    assert got == pytest.approx(ref, rel=1e-13)


GRAM_SHAPES = [(1, 1, 1), (3, 8, 1), (2, 9, 31), (6, 33, 32), (3, 96, 1000), (5, 3, 7), (100, 16, 1), (2, 200, 33), (1, 130, 40), (7, 17, 5),
               (4, 256, 3), (9, 40, 64), (1, 300, 2),
               # register-direct blocks (FP32 input): runs in blocks of 32, and runs of 1-4 columns
               (3, 96, 1024), (2, 128, 64), (5, 40, 96), (64, 12, 16384), (100, 96, 3), (37, 64, 1), (50, 48, 2),
               (19, 96, 4), (3, 120, 32), (4, 108, 64),
               # above 128 rows (waves owning two tile rows of a block pair): three block rows
               # with a ragged last one and many column ranges, four block rows, slices of fewer
               # than 32 columns, eight block rows with an odd tile count in the last one
               (1, 306, 4608), (2, 500, 333), (40, 200, 7), (1, 1000, 97)]


@pytest.mark.parametrize("P,m,S", GRAM_SHAPES)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_gram(P, m, S, dtype):
    x = rng(P * 1000 + m + S).standard_normal(P * m * S).astype(dtype)
    G = H.ht_test_gram(torch.from_numpy(x).cuda(), P, m, S).cpu().numpy()
    M = unfold_np(x.astype(np.float64), P, m, S)
    ref = M @ M.T
    assert np.max(np.abs(G - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("P,m,S,R", [(3, 96, 1000, 12), (5, 9, 7, 3), (100, 16, 1, 5), (2, 128, 33, 64), (7, 17, 5, 1),
                                     (4, 64, 300, 16), (50, 40, 2, 20), (1, 96, 31, 47),
                                     (3, 96, 1024, 12), (2, 128, 64, 64), (5, 40, 96, 20), (2, 96, 288, 47),
                                     (100, 96, 3, 14), (37, 64, 1, 5), (50, 48, 2, 20), (19, 96, 4, 32),
                                     # three row tiles (33-48 rows): per-tile wave ownership of the FP64 Gram
                                     (4, 48, 2048, 18), (3, 44, 64, 40), (2, 48, 96, 47), (37, 48, 1, 5),
                                     (21, 36, 3, 17), (19, 48, 4, 30),
                                     # runs not in whole blocks of 32; rows not in steps of four
                                     (3, 76, 330, 20), (5, 40, 34, 12), (9, 103, 62, 33)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_resid_gram(P, m, S, R, dtype):
    g = rng(P * 7 + m + S + R)
    x = g.standard_normal(P * m * S).astype(dtype)
    U = np.linalg.qr(g.standard_normal((m, R)))[0]
    G = H.ht_test_resid_gram(torch.from_numpy(x).cuda(), P, m, S, torch.from_numpy(U).cuda()).cpu().numpy()
    M = unfold_np(x.astype(np.float64), P, m, S)
    Rr = M - U @ (U.T @ M)
    ref = Rr @ Rr.T
    assert np.max(np.abs(G - ref)) <= 1e-12 * max(1.0, np.max(np.abs(M @ M.T)))


# Direct contraction of modes above 128 rows with lent scratch: few column blocks are
# split into row chunks (partial products summed in chunk order); with the energies
# ||X||^2 and ||Z||^2.  No scratch, or too little, runs it unsplit; the results agree.
@pytest.mark.parametrize("P,m,S,R", [(16, 600, 68, 32), (4, 480, 100, 24), (2, 129, 50, 5), (3, 1000, 7, 64),
                                     (1, 131, 1, 1),
                                     # column-tiled kernel (1024 blocks or more) on fewer than 256
                                     # workgroups; a ragged last block
                                     (16, 480, 1088, 24), (3, 300, 5999, 20)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_ttm_contract_split(P, m, S, R, dtype):
    g = rng(P + m + S + R + 5)
    x = g.standard_normal(P * m * S).astype(dtype)
    U = g.standard_normal((m, R))
    xt, Ut = torch.from_numpy(x).cuda(), torch.from_numpy(U).cuda()
    ref = np.einsum("ar,pas->prs", U, x.astype(np.float64).reshape(P, m, S))
    for ws in (8 * P * R * S, 0):
        Z, nx, nz = H.ht_test_ttm_contract_split(xt, P, m, S, Ut, ws)
        Z = Z.cpu().numpy()
        assert np.max(np.abs(Z - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
        assert nx == pytest.approx(float(np.sum(x.astype(np.float64) ** 2)), rel=1e-12)
        assert nz == pytest.approx(float(np.sum(ref ** 2)), rel=1e-12)


# The residual Gram as (I - U U^T) M M^T (I - U U^T) from the FP64 Gram of M
# (register-direct shapes; 128 rows with 64 basis columns; runs of 1-4 columns;
# eight row tiles).  M near the span of U, as in HT-RISE, so the residual is small next
# to M: the explicit FP64 residual Gram is exact to ~u ||R|| ||M||, and the comparison
# sees the rounding of M M^T, relative to ||M||^2 (u = 2^-53).
PROJ_SHAPES = [(3, 96, 1024, 12), (2, 128, 64, 64), (5, 40, 96, 20), (4, 48, 2048, 6), (64, 12, 512, 3),
               (50, 40, 2, 20), (100, 36, 4, 12), (7, 64, 3, 30), (9, 92, 1, 32), (3, 120, 32, 40),
               (8, 48, 65536, 6)]


def proj_inputs(P, m, S, R, seed):
    g = rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((m, m)))
    scale = np.where(np.arange(m) < R, 1.0, 1e-3)
    M = Q @ (scale[:, None] * g.standard_normal((m, P * S)))
    x = np.ascontiguousarray(M.reshape(m, P, S).transpose(1, 0, 2), dtype=np.float32)
    return x, Q[:, :R].copy()


@pytest.mark.parametrize("P,m,S,R", PROJ_SHAPES)
def test_resid_gram_proj(P, m, S, R):
    x, U = proj_inputs(P, m, S, R, 11 * P + m + S + R)
    G = H.ht_test_resid_gram_proj(torch.from_numpy(x).cuda(), P, m, S, torch.from_numpy(U).cuda()).cpu().numpy()
    M = unfold_np(x.astype(np.float64), P, m, S)
    Rr = M - U @ (U.T @ M)
    ref = Rr @ Rr.T
    unit = 2.0 ** -53 * float(np.sum(M * M))
    assert np.array_equal(G, G.T)
    err = np.max(np.abs(G - ref)) / unit
    # tail sums (the quantities the rank rule reads) of the two Grams
    lg, lr = np.linalg.eigvalsh(G)[::-1], np.linalg.eigvalsh(ref)[::-1]
    terr = np.max(np.abs(np.cumsum(lg[::-1])[::-1] - np.cumsum(lr[::-1])[::-1])) / unit
    assert err <= 16.0 and terr <= 16.0, (err, terr)


# modes of more than 128 rows (transfer nodes): the Gram of M by the large-mode Gram
# kernel, FP32 or FP64 data, and the projection in four launches
@pytest.mark.parametrize("P,m,S,R", [(2, 200, 1000, 30), (16, 400, 256, 24), (3, 576, 100, 64), (1, 129, 4000, 1)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_resid_gram_proj_large_modes(P, m, S, R, dtype):
    x, U = proj_inputs(P, m, S, R, 13 * P + m + S + R)
    x = x.astype(dtype)
    G = H.ht_test_resid_gram_proj(torch.from_numpy(x).cuda(), P, m, S, torch.from_numpy(U).cuda()).cpu().numpy()
    M = unfold_np(x.astype(np.float64), P, m, S)
    Rr = M - U @ (U.T @ M)
    ref = Rr @ Rr.T
    unit = 2.0 ** -53 * float(np.sum(M * M))
    assert np.array_equal(G, G.T)
    err = np.max(np.abs(G - ref)) / unit
    lg, lr = np.linalg.eigvalsh(G)[::-1], np.linalg.eigvalsh(ref)[::-1]
    terr = np.max(np.abs(np.cumsum(lg[::-1])[::-1] - np.cumsum(lr[::-1])[::-1])) / unit
    assert err <= 16.0 and terr <= 16.0, (err, terr)


# ... and the shapes outside the register-direct blocks (rows not in steps of four,
# runs not in blocks of 32): the LDS-panel FP64 Gram of the data
@pytest.mark.parametrize("P,m,S,R", [(3, 50, 33, 4), (7, 47, 100, 12), (40, 17, 5, 6), (2, 126, 70, 64)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_resid_gram_proj_panel_shapes(P, m, S, R, dtype):
    x, U = proj_inputs(P, m, S, R, 17 * P + m + S + R)
    x = x.astype(dtype)
    G = H.ht_test_resid_gram_proj(torch.from_numpy(x).cuda(), P, m, S, torch.from_numpy(U).cuda()).cpu().numpy()
    M = unfold_np(x.astype(np.float64), P, m, S)
    Rr = M - U @ (U.T @ M)
    ref = Rr @ Rr.T
    unit = 2.0 ** -53 * float(np.sum(M * M))
    assert np.array_equal(G, G.T)
    err = np.max(np.abs(G - ref)) / unit
    lg, lr = np.linalg.eigvalsh(G)[::-1], np.linalg.eigvalsh(ref)[::-1]
    terr = np.max(np.abs(np.cumsum(lg[::-1])[::-1] - np.cumsum(lr[::-1])[::-1])) / unit
    assert err <= 16.0 and terr <= 16.0, (err, terr)


def test_resid_gram_proj_rejects_bad_arguments():
    x = torch.zeros(3 * 50 * 33, dtype=torch.float32).cuda()
    U = torch.zeros((50, 65), dtype=torch.float64).cuda()
    with pytest.raises(H.HTError):
        H.ht_test_resid_gram_proj(x, 3, 50, 33, U)


@pytest.mark.parametrize("P,m,S,R", [(3, 96, 1000, 12), (5, 3, 7, 3), (100, 16, 1, 5), (2, 200, 33, 64),
                                     (1, 130, 40, 17), (7, 17, 5, 1), (4, 64, 300, 16), (50, 9, 1, 9),
                                     # column runs in whole blocks of 32, m % 4 == 0: register-direct FP64
                                     (3, 96, 1024, 12), (2, 128, 64, 64), (5, 40, 96, 20), (2, 96, 288, 47),
                                     (64, 8, 16384, 3), (3, 4, 32, 1), (4, 48, 2048, 18), (3, 44, 64, 40),
                                     # modes of more than 128 rows: U staged once, or in chunks (m = 600)
                                     (16, 182, 42, 40), (3, 600, 50, 40), (2, 131, 1, 64),
                                     # ... and with 1024 column blocks of 16 or more, whole blocks per
                                     # wave (a ragged last block; U in two chunks for m = 300; 1024 to
                                     # 4096 blocks, fewer tiles of eight than workgroups could run)
                                     (64, 160, 1100, 24), (5, 131, 13109, 17), (7, 300, 10000, 46),
                                     (16, 400, 1600, 30), (3, 200, 5999, 20), (1, 144, 16384, 16),
                                     # LDS-panel kernel (42 and 47 rows, runs not in blocks of 32)
                                     (5824, 42, 1, 30), (3, 47, 9, 47),
                                     # modes of at most 8 rows: one column per thread (S > 1 with
                                     # 33 columns, outside the register kernel's blocks of 32)
                                     (1000, 3, 1, 3), (7, 5, 33, 4)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_ttm_contract(P, m, S, R, dtype):
    g = rng(P + m + S + R)
    x = g.standard_normal(P * m * S).astype(dtype)
    U = g.standard_normal((m, R))
    Z = H.ht_test_ttm_contract(torch.from_numpy(x).cuda(), P, m, S, torch.from_numpy(U).cuda()).cpu().numpy()
    ref = np.einsum("ar,pas->prs", U, x.astype(np.float64).reshape(P, m, S))
    assert np.max(np.abs(Z - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


# Mixed form (FP32 matrix cores).  Inputs near a rank-R subspace, as in HT-RISE:
# X = U C + noise of relative size 1e-3, so the residual is small next to X.
# FP32 error model: each product entry carries a relative error <~ sqrt(m) 2^-24
# ~ 1e-6 of its column's magnitude (Frobenius), so |delta R| <~ 1e-6 ||X|| and a
# residual energy or residual Gram entry moves by <= 2 ||R|| |delta R| + |delta R|^2.
F32_REL = 2e-6

MIXED_SHAPES = [(3, 96, 1000, 12), (5, 9, 7, 3), (100, 16, 1, 5), (2, 128, 33, 64), (7, 17, 5, 1),
                (4, 64, 300, 16), (50, 40, 2, 20), (1, 96, 31, 47),
                # column runs in whole blocks of 32 with m % 4 == 0: the register-direct FP32 contraction
                (3, 96, 1024, 12), (2, 128, 64, 64), (5, 40, 96, 20), (3, 4, 32, 1), (2, 96, 288, 47),
                (64, 8, 16384, 3),
                # runs of 1-4 columns: 16 slabs per register block (partial last block, several per wave)
                (100, 96, 3, 14), (37, 64, 1, 5), (50, 48, 2, 20), (19, 96, 4, 32), (300000, 40, 1, 3),
                # three row tiles (33-48 rows), runs in blocks of 32 and short runs
                (4, 48, 2048, 18), (3, 44, 64, 40), (2, 48, 96, 47), (37, 48, 1, 5), (21, 36, 3, 17),
                (19, 48, 4, 30),
                # runs that are not whole blocks of 32 and row counts that are not
                # multiples of four (LDS-panel kernel)
                (3, 76, 330, 20), (5, 40, 34, 12), (2, 124, 100, 64), (9, 103, 62, 33), (4, 17, 2050, 5),
                # outside the register kernels: the LDS-panel kernel (42 and 47 rows) and one
                # column per thread (modes of at most 8 rows)
                (5824, 42, 1, 30), (33, 47, 5, 47), (220000, 3, 1, 3), (3000, 1, 2, 1)]


def near_subspace(P, m, S, R, seed, dtype=np.float32):
    g = rng(seed)
    U = np.linalg.qr(g.standard_normal((m, R)))[0]
    C = g.standard_normal((P, R, S))
    X = np.einsum("ar,prs->pas", U, C) + 1e-3 * g.standard_normal((P, m, S))
    return X.astype(dtype).reshape(-1), U


@pytest.mark.parametrize("P,m,S,R", MIXED_SHAPES)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_ttm_contract_f32(P, m, S, R, dtype):
    x, U = near_subspace(P, m, S, R, P * 3 + m + S + R, dtype)
    Z, n2, r2 = H.ht_test_ttm_contract_f32(torch.from_numpy(x).cuda(), P, m, S, torch.from_numpy(U).cuda())
    X = x.astype(np.float64).reshape(P, m, S)
    ref = np.einsum("ar,pas->prs", U, X)
    nX = np.linalg.norm(X)
    assert Z.dtype == torch.float32
    assert np.linalg.norm(Z.cpu().numpy() - ref) <= F32_REL * nX
    assert n2 == pytest.approx(float(np.sum(X ** 2)), rel=1e-13)
    Rr = X - np.einsum("ar,prs->pas", U, ref)
    nR = np.linalg.norm(Rr)
    dR = F32_REL * nX
    assert abs(r2 - nR ** 2) <= 2 * nR * dR + dR ** 2


@pytest.mark.parametrize("P,m,S,R", MIXED_SHAPES)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_resid_gram_f32(P, m, S, R, dtype):
    x, U = near_subspace(P, m, S, R, P * 5 + m + S + R, dtype)
    G = H.ht_test_resid_gram_f32(torch.from_numpy(x).cuda(), P, m, S, torch.from_numpy(U).cuda()).cpu().numpy()
    M = unfold_np(x.astype(np.float64), P, m, S)
    Rr = M - U @ (U.T @ M)
    ref = Rr @ Rr.T
    nR, dR = np.linalg.norm(Rr), F32_REL * np.linalg.norm(M)
    assert np.linalg.norm(G - ref) <= 2 * nR * dR + dR ** 2
    assert np.allclose(G, G.T, rtol=0, atol=1e-15 * np.abs(ref).max())


@pytest.mark.parametrize("P,R,S,m", [(3, 12, 1000, 96), (5, 3, 7, 3), (100, 5, 1, 16), (2, 64, 33, 200),
                                     (1, 17, 40, 130), (7, 1, 5, 17),
                                     # enough column groups that a workgroup runs several row blocks
                                     (2, 17, 40000, 150), (3, 46, 25000, 306)])
@pytest.mark.parametrize("with_m", [False, True])
def test_ttm_expand(P, R, S, m, with_m):
    g = rng(P + m + S + R + 7)
    Z = g.standard_normal((P, R, S))
    U = g.standard_normal((m, R))
    M = g.standard_normal((P, m, S)).astype(np.float32) if with_m else None
    out = H.ht_test_ttm_expand(torch.from_numpy(Z).cuda(), torch.from_numpy(U).cuda(),
                               None if M is None else torch.from_numpy(M).cuda()).cpu().numpy()
    ref = np.einsum("ar,prs->pas", U, Z)
    if with_m:
        ref = M.astype(np.float64) - ref
    assert np.max(np.abs(out - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_ttm_expand_float32_output():
    g = rng(3)
    Z = g.standard_normal((4, 6, 50))
    U = g.standard_normal((20, 6))
    out = H.ht_test_ttm_expand(torch.from_numpy(Z).cuda(), torch.from_numpy(U).cuda(), out_dtype=torch.float32)
    ref = np.einsum("ar,prs->pas", U, Z).astype(np.float32)
    np.testing.assert_array_equal(out.cpu().numpy(), ref)


def psd_with_spectrum(k, lam, seed):
    q = np.linalg.qr(rng(seed).standard_normal((k, k)))[0]
    return (q * lam[None, :]) @ q.T, q


@pytest.mark.parametrize("k", [1, 2, 3, 16, 40, 96, 132, 133, 200, 300])
def test_eig_spectrum_and_vectors(k):
    lam = np.logspace(0, -12, k) if k > 1 else np.array([2.0])
    G, q = psd_with_spectrum(k, lam, k)
    thr = 0.5 * np.sum(lam[k // 2:]) + 0.5 * np.sum(lam[k // 2 + 1:]) if k > 1 else 0.0
    ev, vecs, r, tail = H.ht_test_eig(torch.from_numpy(G).cuda(), 1, k, thr)
    ev = ev.cpu().numpy()
    ref = np.sort(np.linalg.eigvalsh(G))[::-1]
    # the leading eigenvalues the rule needed are returned (at least r), the rest untouched
    m = int(np.argmax(np.isnan(np.append(ev, np.nan))))
    assert m >= min(k, (k // 2 + 1 if k > 1 else 1)) and np.all(np.isnan(ev[m:]))
    assert np.max(np.abs(ev[:m] - ref[:m])) <= 1e-13 * ref[0] * max(1, k / 16)
    # truncation rule against the reference spectrum: tail after k//2 is <= thr < tail after k//2 - 1
    assert r == (k // 2 + 1 if k > 1 else 1)
    v = vecs.cpu().numpy()
    assert np.linalg.norm(v.T @ v - np.eye(r)) < 1e-12
    resid = G @ v - v * ev[:r][None, :]
    assert np.max(np.abs(resid)) <= 1e-12 * ref[0]
    piv = np.argmax(np.abs(v), axis=0)
    assert np.all(v[piv, np.arange(r)] > 0)


@pytest.mark.parametrize("k", [8, 96, 150])
def test_eig_rank_rule_exact_boundary(k):
    lam = np.concatenate([np.linspace(10, 1, 5), np.full(k - 5, 1e-6)])
    G, _ = psd_with_spectrum(k, lam, 5 + k)
    thr = (k - 5) * 1e-6 * 1.5
    _, _, r, tail = H.ht_test_eig(torch.from_numpy(G).cuda(), 1, k, thr)
    assert r == 5
    assert tail == pytest.approx((k - 5) * 1e-6, rel=1e-6)
    _, _, r0, _ = H.ht_test_eig(torch.from_numpy(G * 0).cuda() + 0.0, 0, k, 1.0)
    assert r0 == 0


def test_eig_degenerate_cluster_spans_the_eigenspace():
    k = 60
    lam = np.concatenate([np.full(4, 3.0), np.full(3, 1.0), np.full(k - 7, 1e-9)])
    G, q = psd_with_spectrum(k, lam, 17)
    _, vecs, r, _ = H.ht_test_eig(torch.from_numpy(G).cuda(), 1, k, 1e-6)
    assert r == 7
    v = vecs.cpu().numpy()
    P = v @ v.T
    Pref = q[:, :7] @ q[:, :7].T
    assert np.linalg.norm(P - Pref) < 1e-10


def exact_rank(lam, thr, rmin, rmax):
    """The truncation rule on a reference spectrum (descending): minimal r in
    [rmin, rmax] whose discarded energy, summed from the smallest value up, is <= thr."""
    tail = np.concatenate([np.cumsum(np.clip(lam[::-1], 0, None))[::-1], [0.0]])
    for r in range(rmin, rmax + 1):
        if tail[r] <= thr:
            return r
    return rmax


def lowrank_gram(k, r0, seed, noise=1e-5, cols=3000):
    g = rng(seed)
    X = g.standard_normal((k, r0)) @ g.standard_normal((r0, cols)) + noise * g.standard_normal((k, cols))
    return X @ X.T


# Gram matrices shaped like the method's: a few strong directions over a floor.  The
# Krylov basis sits in LDS up to k = 224 and in global scratch beyond.
@pytest.mark.parametrize("k,r0,rmin", [(40, 3, 0), (96, 3, 0), (96, 12, 1), (182, 5, 0), (224, 30, 0),
                                       (300, 12, 0), (768, 20, 1)])
def test_eig_lanczos_certified_matches_householder(k, r0, rmin):
    G = lowrank_gram(k, r0, k + r0)
    thr = 1e-6 * np.trace(G)
    rmax = min(k, 64)
    lam = np.sort(np.linalg.eigvalsh(G))[::-1]
    r_ref = exact_rank(lam, thr, rmin, rmax)
    Gd = torch.from_numpy(G).cuda()
    evh, vh, rh, th = H.ht_test_eig(Gd, rmin, rmax, thr, method=H.EIG_HOUSEHOLDER)
    evl, vl, rl, tl, steps = H.ht_test_eig(Gd, rmin, rmax, thr, method=H.EIG_LANCZOS, info=True)
    eva, va, ra, ta, sa = H.ht_test_eig(Gd, rmin, rmax, thr, info=True)
    print("k %d: rank %d, Lanczos steps %d" % (k, rl, steps))
    assert rh == rl == ra == r_ref
    assert 0 < steps <= 64 and sa == steps  # the automatic choice took the proven decision
    VL, VH = vl.cpu().numpy(), vh.cpu().numpy()
    assert np.linalg.norm(VL.T @ VL - np.eye(rl)) < 1e-12
    assert np.linalg.norm(VL @ VL.T - VH @ VH.T) < 1e-11
    ev = evl.cpu().numpy()[:rl]
    assert np.max(np.abs(ev - lam[:rl])) <= 1e-13 * lam[0]
    assert np.max(np.abs(G @ VL - VL * ev[None, :])) <= 1e-12 * lam[0]
    assert tl == pytest.approx(th, rel=1e-6, abs=1e-12 * lam[0])
    piv = np.argmax(np.abs(VL), axis=0)
    assert np.all(VL[piv, np.arange(rl)] > 0)
    np.testing.assert_array_equal(va.cpu().numpy(), VL)


def test_eig_lanczos_refuses_unprovable_decisions():
    """A degenerate cluster (a single Krylov sequence sees one vector per eigenspace)
    and a slowly decaying spectrum that needs more than 64 steps are left to the
    Householder path, which the automatic choice then takes."""
    lam = np.concatenate([np.full(4, 3.0), np.full(3, 1.0), np.full(53, 1e-9)])
    G1, _ = psd_with_spectrum(60, lam, 17)
    lam2 = np.logspace(0, -12, 150)
    G2, _ = psd_with_spectrum(150, lam2, 150)
    thr2 = 0.5 * np.sum(lam2[75:]) + 0.5 * np.sum(lam2[76:])
    for G, thr, r_ref in ((G1, 1e-6, 7), (G2, thr2, 76)):
        Gd = torch.from_numpy(G).cuda()
        k = G.shape[0]
        _, _, rl, _, steps = H.ht_test_eig(Gd, 1, k, thr, method=H.EIG_LANCZOS, info=True)
        assert rl == -1 and steps < 0
        _, va, ra, _ = H.ht_test_eig(Gd, 1, k, thr)
        _, vh, rh, _ = H.ht_test_eig(Gd, 1, k, thr, method=H.EIG_HOUSEHOLDER)
        assert ra == rh == r_ref
        np.testing.assert_array_equal(va.cpu().numpy(), vh.cpu().numpy())


def test_eig_lanczos_budget_edges():
    """Exact low rank (the Krylov space becomes invariant), a threshold the trace
    already meets with rmin = 1, and the rank capped below the rule's choice (the
    Householder path then reports the capped rank with its larger tail)."""
    G = lowrank_gram(96, 6, 5, noise=0.0)
    Gd = torch.from_numpy(G).cuda()
    lam = np.sort(np.linalg.eigvalsh(G))[::-1]
    thr = 1e-9 * np.trace(G)
    _, v, r, _, steps = H.ht_test_eig(Gd, 0, 64, thr, method=H.EIG_LANCZOS, info=True)
    assert r == exact_rank(lam, thr, 0, 64) == 6 and 0 < steps <= 8
    _, _, r1, t1, s1 = H.ht_test_eig(Gd, 1, 64, 2.0 * np.trace(G), info=True)
    assert r1 == 1 and s1 > 0 and t1 == pytest.approx(np.sum(lam[1:]), rel=1e-9)
    _, _, r2, t2, s2 = H.ht_test_eig(Gd, 0, 3, thr, info=True)
    assert r2 == 3 and s2 < 0 and t2 == pytest.approx(np.sum(lam[3:]), rel=1e-9)


@pytest.mark.parametrize("alpha,r_old,rR", [(96, 12, 3), (16, 0, 4), (200, 40, 8), (9, 4, 5), (400, 30, 8)])
def test_orth_expand(alpha, r_old, rR):
    g = rng(alpha + r_old)
    U = np.linalg.qr(g.standard_normal((alpha, r_old)))[0] if r_old else None
    V = g.standard_normal((alpha, rR))
    if U is not None:
        V = V - U @ (U.T @ V) + 1e-9 * (U @ g.standard_normal((r_old, rR)))
    core = H.ht_test_orth_expand(None if U is None else torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda())
    core = core.cpu().numpy()
    assert np.linalg.norm(core.T @ core - np.eye(r_old + rR)) < 1e-13
    if U is not None:
        np.testing.assert_array_equal(core[:, :r_old], U)
    new = core[:, r_old:]
    # same span as V projected off U
    Vp = V if U is None else V - U @ (U.T @ V)
    Q = np.linalg.qr(Vp)[0]
    assert np.linalg.norm(Q @ (Q.T @ new) - new) < 1e-12
    piv = np.argmax(np.abs(new), axis=0)
    assert np.all(new[piv, np.arange(rR)] > 0)
