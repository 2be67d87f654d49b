"""BF16x3 residuals emulated on the CPU: why the library rejects HT_BF16X3.

A BF16x3 product splits each FP32 operand x into hi = bf16(x) and lo = bf16(x - hi)
and sums hi*hi' + hi*lo' + lo*hi' with FP32 accumulation on the BF16 matrix cores.
Products of two BF16 values are exact in FP32, so the emulation below (round to
nearest even BF16 by bit manipulation, exact products, FP32 sums through a float32
matrix product) is the arithmetic of those matrix cores up to the order of the FP32
sums.  HT-RISE's Step 2 residual R = M - U (U^T M) (Sec. 3.2, Eq. compute_residual)
is formed that way and in plain FP32 on leaf unfoldings of the two field streams, and
both are compared with the FP64 residual.  The leaf basis U is the oracle's truncated
SVD of the first batch's leaf unfolding with the nodewise tolerance of Alg. 1, i.e.
the leaf core BHT-l2r computes for a leaf of the deepest layer; M is a later batch's
leaf unfolding.  The streams run with fewer samples per batch than the benchmark so
that the test stays within seconds; the errors are relative to ||M|| and do not depend
on the sample count.

What the numbers show, against the library's error model of the FP32 residual
(2 u sqrt(r + 1) ||Y||, u = 2^-24) and its certificates:

* the FP32 residual error stays inside that model;
* the BF16x3 residual error is 20-30 times larger and reaches a tenth of eps_nw
  itself, so a decision's tail sums near the threshold move by a fifth of the
  threshold (2 sqrt(thr) dR): most decisions of the stored traces lie closer to their
  threshold than that and could not be certified;
* every growing node would fail the kept-vector criterion (1 % of the threshold) and
  be recomputed in FP64, and the precision gate fails at eps = 1e-4 for both streams:
  a BF16x3 form could take no decision of its own.
"""

import json
import math
import os

import numpy as np
import pytest

import datagen
from oracle.ht_oracle import truncated_svd

HERE = os.path.dirname(os.path.abspath(__file__))
U32 = 2.0 ** -24
EPS = 1e-4


def bf16(x: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 (round to nearest, ties to even), returned as FP32 values."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    r = (b + np.uint32(0x7FFF) + ((b >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return r.view(np.float32)


def mm_bf16x3(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    ah, bh = bf16(a), bf16(b)
    al, bl = bf16(a - ah), bf16(b - bh)   # a - ah is exact in FP32
    return (ah @ bh + ah @ bl) + al @ bh


def mm_f32(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.float32) @ np.asarray(b, dtype=np.float32)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9, -3.0e-5, 0.0], dtype=np.float32)
    got = bf16(x)
    # 8 significant bits: 1 + 2^-8 is a tie (even -> 1), 1 + 3 * 2^-9 rounds up to 1 + 2^-7
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 and got[3] == np.float32(1.0 + 2.0 ** -7)
    assert abs(got[4] + 3.0e-5) <= 2.0 ** -8 * 3.0e-5 and got[5] == 0.0
    a = np.random.default_rng(0).standard_normal((16, 64)).astype(np.float32)
    hi = bf16(a)
    assert np.all(np.abs(a - hi) <= 2.0 ** -8 * np.abs(a))   # 8 significant bits
    # the split keeps 16 significant bits: x - hi - lo is at most 2^-16 |x|
    lo = bf16(a - hi)
    assert np.all(np.abs(a.astype(np.float64) - hi - lo) <= 2.0 ** -16 * np.abs(a))


def residual_errors(spec, k):
    """(r_old, ||M||, eps_nw, dR_f32, dR_bf16x3, d) for the mode-1 leaf of batch k."""
    y0 = datagen.exact_field_batch(spec, 0)
    yk = datagen.exact_field_batch(spec, k)
    d = y0.ndim - 1
    m0 = np.moveaxis(y0, 1, 0).reshape(y0.shape[1], -1).astype(np.float64)
    u, _ = truncated_svd(m0, EPS * np.linalg.norm(m0) / math.sqrt(2 * d - 2), rmin=1)
    M = np.moveaxis(yk, 1, 0).reshape(yk.shape[1], -1)
    M64 = M.astype(np.float64)
    nM = float(np.linalg.norm(M64))
    R64 = M64 - u @ (u.T @ M64)
    errs = []
    for mm in (mm_f32, mm_bf16x3):
        c = mm(u.T, M)
        r = M.astype(np.float32) - mm(u, c)
        errs.append(float(np.linalg.norm(r.astype(np.float64) - R64)))
    return u.shape[1], nM, EPS * nM / math.sqrt(2 * d - 2), errs[0], errs[1], d


def gate(u_eff, eps, d, rank_cap):
    """The library's precision gate with a residual error of u_eff sqrt(r + 1) ||Y||."""
    return 2.0 * u_eff * math.sqrt((2 * d - 2) * (rank_cap + 1.0)) <= 0.5 * eps / math.sqrt(2 * d - 2)


def undecidable_share(trace_file, delta_rel):
    """Share of the trace's update batches with a decision closer to its threshold than delta_rel."""
    rows = json.load(open(os.path.join(HERE, "golden", trace_file)))["batches"][1:]
    margins = [b["min_decision_margin_rel"] for b in rows if b.get("min_decision_margin_rel") is not None]
    return sum(1 for m in margins if m < delta_rel) / len(margins), len(margins)


@pytest.mark.parametrize("stream,k,rank_cap,trace", [
    ("field96", 5, 48, "field96_trace.json"),
    ("field48", 14, 64, "field48_trace.json"),
])
def test_bf16x3_residual_cannot_be_certified(stream, k, rank_cap, trace):
    spec = datagen.field_96_spec(N=2) if stream == "field96" else datagen.field_48_spec(N=1)
    r, nM, eps_nw, d32, dbf, d = residual_errors(spec, k)
    model32 = 2.0 * U32 * math.sqrt(r + 1) * nM
    # FP32: inside the library's error model, a few thousandths of eps_nw
    assert d32 <= model32
    assert d32 <= 0.01 * eps_nw
    # BF16x3: 20-30x the FP32 error, a tenth of eps_nw
    assert dbf >= 15.0 * d32
    assert dbf >= 0.08 * eps_nw
    # a tail sum near the threshold thr = eps_nw^2 moves by up to 2 sqrt(thr) dR
    delta_rel = 2.0 * dbf / eps_nw
    assert delta_rel >= 0.16
    share, n = undecidable_share(trace, delta_rel)
    assert n > 5 and share >= 0.4, (share, n)
    # the kept-vector criterion (1 % of thr) fails for every growing node
    assert 2.0 * dbf / eps_nw > 0.01
    # the precision gate with the measured error per sqrt(r + 1): FP32 passes, BF16x3 fails
    u32_eff = d32 / (math.sqrt(r + 1) * nM)
    ubf_eff = dbf / (math.sqrt(r + 1) * nM)
    assert gate(max(u32_eff, U32), EPS, d, rank_cap)
    assert not gate(ubf_eff, EPS, d, rank_cap)
