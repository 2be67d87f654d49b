"""Seeded synthetic tensor streams for the batch hierarchical Tucker method.

This module only *synthesises inputs*: it holds none of the method's arithmetic
(no truncation, no projection onto learned bases, no rank decision).  Both the
FP64 oracle and the HIP path consume its output, so it sits in a module of its
own that imports neither of them.

Every batch is generated in float64 from ``numpy.random.Generator(PCG64(seed))``
and rounded once to float32.  All consumers see the same float32 values (the
oracle promotes them exactly to float64).  Layout is C order ``[N][n1]...[nd]``:
each sample is contiguous, the batch index is the slowest.

Stream families (sizes are the paper's workload shapes, see the experiments
section's dataset table; the paper's datasets themselves are not used):

* ``ht_model_stream`` - exact hierarchical-Tucker-rank tensors built from
  random orthonormal frames on a balanced dimension tree, plus relative
  Gaussian noise, optionally growing by fresh orthogonal directions at chosen
  batches.  The 16x16x16x16, N=8, rank-4 instance is ``tiny_stream``.
* ``separable_field_stream`` - smooth drifting fields, a sum of separable
  Gaussian-bump x sine terms over the spatial modes times a channel vector,
  standing in for the paper's PDE snapshots.  ``field_96_stream`` is the
  96x96x96x3, N=32, 20-batch instance; ``field_48_stream`` the 48^4x4 one.
* ``multi_stream_specs`` - 64 independent small exact-rank streams of uneven
  shapes for the many-streams batched form.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Iterator, List, Sequence, Tuple

import numpy as np

__all__ = [
    "rng",
    "HTModelSpec",
    "ht_model_stream",
    "tiny_stream",
    "FieldSpec",
    "separable_field_stream",
    "field_96_spec",
    "field_48_spec",
    "field_96_stream",
    "field_48_stream",
    "multi_stream_specs",
]


def rng(seed: int) -> np.random.Generator:
    """The one seeded generator every stream draws from (PCG64)."""
    return np.random.Generator(np.random.PCG64(int(seed)))


def _orthonormal(g: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Q factor of a Gaussian rows x cols matrix (orthonormal columns)."""
    q, r = np.linalg.qr(g.standard_normal((rows, cols)))
    # make the factor unique so the stream does not depend on LAPACK's sign choice
    q = q * np.where(np.diag(r) < 0, -1.0, 1.0)[None, :]
    return q


def _fresh_orthonormal(g: np.random.Generator, existing: np.ndarray, cols: int) -> np.ndarray:
    """``cols`` orthonormal columns orthogonal to the columns of ``existing``."""
    rows = existing.shape[0]
    k = existing.shape[1]
    if k + cols > rows:
        raise ValueError("no room for %d fresh directions in dimension %d (have %d)" % (cols, rows, k))
    m = np.concatenate([existing, g.standard_normal((rows, cols))], axis=1)
    q, r = np.linalg.qr(m)
    q = q * np.where(np.diag(r) < 0, -1.0, 1.0)[None, :]
    return q[:, k:]


def _split(lo: int, hi: int) -> Tuple[Tuple[int, int], Tuple[int, int]]:
    """Generating-tree split of the mode range [lo, hi): the first half gets ceil(q/2)."""
    q = hi - lo
    mid = lo + (q + 1) // 2
    return (lo, mid), (mid, hi)


# --------------------------------------------------------------------------- #
# Exact-HT-rank streams
# --------------------------------------------------------------------------- #


@dataclass
class HTModelSpec:
    """An exact-rank generating model on the balanced first-half-split tree.

    ``rank`` gives the generating rank of every non-root node (one int for all
    nodes, capped per node by feasibility).  ``grow_at`` lists batch indices
    (0 = initial batch) at which ``grow_by`` fresh orthogonal directions are
    added at every node; the new component's root slices have standard
    deviation ``grow_scale``.
    """

    n: Tuple[int, ...]
    rank: int
    N: int
    n_batches: int
    seed: int
    batch_seed0: int
    nu: float
    grow_at: Tuple[int, ...] = ()
    grow_by: int = 2
    grow_scale: float = 0.1

    @property
    def elements_per_batch(self) -> int:
        return self.N * int(np.prod(self.n))


class _Frames:
    """Orthonormal frames of one direction set on every node of the generating tree.

    A node is a mode range (lo, hi).  Its frame F has prod(n[lo:hi]) rows (C-order
    flattening of those modes) and r columns.  A leaf frame is a random
    orthonormal n_i x r matrix; an interior frame is (F_a kron F_b) B with B a
    random orthonormal (r_a r_b) x r matrix, so it is orthonormal too.  Only the
    two children of the root are ever materialised as full frames.
    """

    def __init__(self, n: Sequence[int]):
        self.n = tuple(int(x) for x in n)
        self.leaf: dict = {}
        self.mix: dict = {}
        self.rank: dict = {}

    def frame(self, lo: int, hi: int) -> np.ndarray:
        if hi - lo == 1:
            return self.leaf[lo]
        (a0, a1), (b0, b1) = _split(lo, hi)
        fa = self.frame(a0, a1)
        fb = self.frame(b0, b1)
        b = self.mix[(lo, hi)]  # (r_a*r_b, r)
        ra, rb = fa.shape[1], fb.shape[1]
        r = b.shape[1]
        t = (fa @ b.reshape(ra, rb * r)).reshape(fa.shape[0], rb, r)
        out = np.einsum("xbr,yb->xyr", t, fb)
        return out.reshape(fa.shape[0] * fb.shape[0], r)


def _node_ranges(lo: int, hi: int, out: list) -> None:
    out.append((lo, hi))
    if hi - lo > 1:
        a, b = _split(lo, hi)
        _node_ranges(*a, out)
        _node_ranges(*b, out)


def _feasible_ranks(n: Sequence[int], rank: int) -> dict:
    """Generating rank per node range: min(rank, n_i) at leaves, min(rank, r_a r_b) above."""
    d = len(n)
    ranks: dict = {}

    def visit(lo, hi):
        if hi - lo == 1:
            ranks[(lo, hi)] = min(rank, n[lo])
            return ranks[(lo, hi)]
        a, b = _split(lo, hi)
        ra = visit(*a)
        rb = visit(*b)
        ranks[(lo, hi)] = min(rank, ra * rb)
        return ranks[(lo, hi)]

    visit(0, d)
    return ranks


def _build_frames(g: np.random.Generator, n: Sequence[int], ranks: dict, previous: List[_Frames]) -> _Frames:
    f = _Frames(n)
    d = len(n)
    nodes: list = []
    _node_ranges(0, d, nodes)
    for (lo, hi) in nodes:
        if (lo, hi) == (0, d):
            continue
        r = ranks[(lo, hi)]
        f.rank[(lo, hi)] = r
        if hi - lo == 1:
            if previous:
                existing = np.concatenate([p.leaf[lo] for p in previous], axis=1)
                f.leaf[lo] = _fresh_orthonormal(g, existing, r)
            else:
                f.leaf[lo] = _orthonormal(g, n[lo], r)
    # interior mixing matrices (children ranks are known now)
    for (lo, hi) in nodes:
        if (lo, hi) == (0, d) or hi - lo == 1:
            continue
        a, b = _split(lo, hi)
        ra, rb = f.rank[a], f.rank[b]
        f.mix[(lo, hi)] = _orthonormal(g, ra * rb, f.rank[(lo, hi)])
    return f


def ht_model_parts(spec: HTModelSpec) -> Iterator[Tuple[List[Tuple[np.ndarray, np.ndarray, np.ndarray]],
                                                            np.random.Generator]]:
    """Per batch k: the terms (F_L, S, F_R) of its signal, sum_terms F_L S_n F_R^T per
    sample n, and the batch's generator, positioned for the noise draw.

    F_L, F_R are the frames of the root's two children of each direction set
    introduced so far and S (N x r_L x r_R) holds fresh Gaussian root slices scaled
    by the set's scale."""
    n = tuple(spec.n)
    d = len(n)
    if d < 2:
        raise ValueError("need at least two modes")
    g = rng(spec.seed)
    base_ranks = _feasible_ranks(n, spec.rank)
    sets: List[_Frames] = [_build_frames(g, n, base_ranks, [])]
    scales = [1.0]
    left, right = _split(0, d)
    for k in range(spec.n_batches):
        if k in spec.grow_at:
            grow = _feasible_ranks(n, spec.grow_by)
            sets.append(_build_frames(g, n, grow, sets))
            scales.append(spec.grow_scale)
        gb = rng(spec.batch_seed0 + k)
        terms = []
        for fr, sc in zip(sets, scales):
            fl = fr.frame(*left)
            fright = fr.frame(*right)
            terms.append((fl, sc * gb.standard_normal((spec.N, fl.shape[1], fright.shape[1])), fright))
        yield terms, gb


def ht_model_stream(spec: HTModelSpec) -> Iterator[np.ndarray]:
    """Yield ``spec.n_batches`` float32 batches of shape (N, *n).

    Batch k is sum over the direction sets introduced so far of
    F_L S_k F_R^T (per sample), where F_L, F_R are the frames of the root's two
    children and S_k holds fresh Gaussian root slices, plus relative noise of
    standard deviation ``nu * rms(signal)``.
    """
    n = tuple(spec.n)
    for terms, gb in ht_model_parts(spec):
        y = np.zeros((spec.N, terms[0][0].shape[0], terms[0][2].shape[0]))
        for fl, s, fright in terms:
            y += np.einsum("xi,nij,yj->nxy", fl, s, fright, optimize=True)
        if spec.nu > 0:
            rms = math.sqrt(float(np.mean(y * y)))
            y += spec.nu * rms * gb.standard_normal(y.shape)
        yield y.reshape((spec.N,) + n).astype(np.float32)


def tiny_stream(n_batches: int = 5, nu: float = 1e-6) -> List[np.ndarray]:
    """16x16x16x16 samples, N=8, exact HT rank 4, fresh +2 directions at batches 3 and 4.

    Model seed 1, batch seeds 100+k.  Expected ranks at eps=1e-4 (every
    non-root node): 4, 4, 4, 6, 8; batches 1 and 2 add no direction.
    """
    spec = HTModelSpec(n=(16, 16, 16, 16), rank=4, N=8, n_batches=n_batches, seed=1,
                       batch_seed0=100, nu=nu, grow_at=(3, 4), grow_by=2, grow_scale=0.1)
    return list(ht_model_stream(spec))


# --------------------------------------------------------------------------- #
# Drifting separable fields
# --------------------------------------------------------------------------- #


@dataclass
class FieldSpec:
    """Sum of ``terms`` separable Gaussian-bump x sine terms on a uniform [0,1] grid.

    Sample s of batch k is
      sum_t a[s,t] * prod_m exp(-(x_m - mu[t,m](k))^2 / (2 w[t,m]^2))
                          * sin(2 pi om[t,m](k) x_m + phi[t,m]) * v[t, c]
    over ``len(grid)`` spatial modes and a channel mode of size ``channels``.
    mu drifts by ``drift * k * delta`` (delta = +-1), om by a factor
    (1 + drift * k); with ``reflect`` both are reflected into [mu_lo, mu_hi]
    and [om_lo, om_hi].  With ``period`` > 0 the drift oscillates instead:
    mu = mu0 + drift * delta * sin(2 pi k / period), om = om0 (1 + drift *
    sin(2 pi k / period)).  With ``active0`` > 0 only the first ``active0`` terms
    are present at batch 0 and term t >= active0 switches on at batch
    (t - active0 + 1) * ``onset_every`` (its coefficients are zero before).
    """

    grid: Tuple[int, ...]
    channels: int
    terms: int
    N: int
    n_batches: int
    drift: float
    seed: int
    batch_seed0: int
    nu: float = 0.0
    w_lo: float = 0.05
    w_hi: float = 0.2
    reflect: bool = False
    mu_lo: float = 0.1
    mu_hi: float = 0.9
    om_lo: float = 1.0
    om_hi: float = 6.0
    period: int = 0
    active0: int = 0
    onset_every: int = 0

    @property
    def n(self) -> Tuple[int, ...]:
        return tuple(self.grid) + (self.channels,)

    @property
    def elements_per_batch(self) -> int:
        return self.N * int(np.prod(self.n))


def _reflect(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    span = hi - lo
    y = np.mod(x - lo, 2.0 * span)
    return lo + np.where(y > span, 2.0 * span - y, y)


def _field_params(spec: FieldSpec) -> dict:
    g = rng(spec.seed)
    m = len(spec.grid)
    t = spec.terms
    return {
        "mu0": g.uniform(0.2, 0.8, size=(t, m)),
        "w": g.uniform(spec.w_lo, spec.w_hi, size=(t, m)),
        "om0": g.uniform(1.0, 4.0, size=(t, m)),
        "phi": g.uniform(0.0, 2.0 * math.pi, size=(t, m)),
        "v": g.standard_normal((t, spec.channels)),
        "delta": np.where(g.uniform(size=(t, m)) < 0.5, -1.0, 1.0),
    }


def field_mode_functions(spec: FieldSpec, k: int) -> List[np.ndarray]:
    """Per spatial mode m, the (terms x n_m) matrix of 1-D factors at batch k."""
    p = _field_params(spec)
    if spec.period > 0:
        ph = math.sin(2.0 * math.pi * k / spec.period)
        mu = p["mu0"] + spec.drift * ph * p["delta"]
        om = p["om0"] * (1.0 + spec.drift * ph)
    else:
        mu = p["mu0"] + spec.drift * k * p["delta"]
        om = p["om0"] * (1.0 + spec.drift * k)
    if spec.reflect:
        mu = _reflect(mu, spec.mu_lo, spec.mu_hi)
        om = _reflect(om, spec.om_lo, spec.om_hi)
    out = []
    for mi, nm in enumerate(spec.grid):
        x = np.linspace(0.0, 1.0, nm)[None, :]
        f = np.exp(-((x - mu[:, mi:mi + 1]) ** 2) / (2.0 * p["w"][:, mi:mi + 1] ** 2))
        f = f * np.sin(2.0 * math.pi * om[:, mi:mi + 1] * x + p["phi"][:, mi:mi + 1])
        out.append(f)
    return out


def separable_field_stream(spec: FieldSpec, batches: Sequence[int] | None = None) -> Iterator[np.ndarray]:
    """Yield float32 batches (N, *grid, channels) of the drifting field."""
    p = _field_params(spec)
    m = len(spec.grid)
    split = (m + 1) // 2
    ks = range(spec.n_batches) if batches is None else batches
    for k in ks:
        fs = field_mode_functions(spec, k)
        t = spec.terms
        # left factor: outer product of the first `split` spatial modes, per term
        left = fs[0]
        for f in fs[1:split]:
            left = (left[:, :, None] * f[:, None, :]).reshape(t, -1)
        right = p["v"]  # (t, C)
        for f in reversed(fs[split:]):
            right = (f[:, :, None] * right[:, None, :]).reshape(t, -1)
        a = rng(spec.batch_seed0 + k).standard_normal((spec.N, t))
        y = np.empty((spec.N, left.shape[1], right.shape[1]))
        for s in range(spec.N):
            y[s] = (left.T * a[s][None, :]) @ right
        if spec.nu > 0:
            gn = rng(10_000_000 + spec.batch_seed0 + k)
            rms = math.sqrt(float(np.mean(y * y)))
            y += spec.nu * rms * gn.standard_normal(y.shape)
        yield y.reshape((spec.N,) + spec.n).astype(np.float32)


def field_96_spec(n_batches: int = 20, N: int = 32, drift: float = 3e-4) -> FieldSpec:
    """96x96x96 grid x 3 channels, 12 terms, no noise (seeds 2, 200+k).

    Drift defaults to 0.03% of the domain per batch with bump widths in
    [0.2, 0.5]: at eps = 1e-4 every rank then stays <= 48 over 20 batches.  At
    1% per batch (widths [0.05, 0.2]) the (1,2) transfer rank reaches 194 and no
    batch is ever skipped; that setting is kept available through ``drift``.
    Generated with ``exact_field_batch`` (host) or ``datagen.gpu`` (device).
    """
    return FieldSpec(grid=(96, 96, 96), channels=3, terms=12, N=N, n_batches=n_batches,
                     drift=drift, seed=2, batch_seed0=200, nu=0.0, w_lo=0.2, w_hi=0.5)


def field_48_spec(n_batches: int = 100, N: int = 16, nu: float = 1e-6) -> FieldSpec:
    """48^4 grid x 4 channels, 16 terms, relative noise nu (seeds 5, 500+k).

    Six terms are present from the first batch and one more switches on every
    nine batches (the last at batch 90); centres and frequencies oscillate with
    amplitude 0.1% and a period of 25 batches; bump widths in [0.2, 0.5].  At
    eps = 1e-4 the ranks then stay below 64 over 100 batches with about a quarter
    of the batches updating.  A drift that keeps growing (0.01% per batch and up,
    24 terms) passes rank 64 at the (1,2,3) transfer node within 12 batches.
    Generated with ``exact_field_batch`` (host) or ``datagen.gpu`` (device)."""
    return FieldSpec(grid=(48, 48, 48, 48), channels=4, terms=16, N=N, n_batches=n_batches,
                     drift=1e-3, seed=5, batch_seed0=500, nu=nu, w_lo=0.2, w_hi=0.5,
                     period=25, active0=6, onset_every=9)


def field_96_stream(n_batches: int = 20, N: int = 32) -> Iterator[np.ndarray]:
    return exact_field_stream(field_96_spec(n_batches, N))


def field_48_stream(n_batches: int = 100, N: int = 16, nu: float = 1e-6) -> Iterator[np.ndarray]:
    return exact_field_stream(field_48_spec(n_batches, N, nu))


# --------------------------------------------------------------------------- #
# Many independent small streams
# --------------------------------------------------------------------------- #


def multi_stream_specs(count: int = 64, seed0: int = 4000, n_batches: int = 11,
                       max_elements: int = 1 << 25, nu: float = 1e-5,
                       d_choices: Sequence[int] = (3, 4, 5), rank_hi: int = 12) -> List[HTModelSpec]:
    """``count`` exact-rank streams: d from ``d_choices``, n_i in [16,128], N in [4,32].

    Mode sizes are drawn uniformly; while N * prod(n) exceeds ``max_elements`` the
    largest mode is redrawn uniformly below its current size (at least 16), which
    ends quickly even for d = 5 (plain redrawing of all modes almost never meets
    the cap there).  A cap below N * 16^d cannot be met; smaller caps therefore
    come with fewer modes in ``d_choices``.  The generating rank r0 is drawn from
    [2, rank_hi] and capped by what the modes allow; batches 4 and 8 add 2 fresh
    directions at every node.  ``n_batches`` counts the initial batch, so 11 means
    10 updates.
    """
    specs = []
    for s in range(count):
        g = rng(seed0 + s)
        d = int(d_choices[int(g.integers(0, len(d_choices)))])
        N = int(g.integers(4, 33))
        n = [int(x) for x in g.integers(16, 129, size=d)]
        while N * int(np.prod(n)) > max_elements:
            i = int(np.argmax(n))
            if n[i] <= 16:
                break
            n[i] = int(g.integers(16, n[i]))
        r0 = int(g.integers(2, rank_hi + 1))
        r0 = min(r0, min(n) - 4)
        specs.append(HTModelSpec(n=tuple(n), rank=r0, N=N, n_batches=n_batches, seed=seed0 + s,
                                 batch_seed0=(seed0 + s) * 100, nu=nu, grow_at=(4, 8),
                                 grow_by=2, grow_scale=0.1))
    return specs


# --------------------------------------------------------------------------- #
# Separable fields that the host and the GPU generate bit for bit alike
# --------------------------------------------------------------------------- #
#
# A batch of the drifting field is sum_t A_t (x) B_t with A_t[s, p1] the sample's
# coefficient times the 1-D factors of the first half of the spatial modes and
# B_t[p2] the factors of the rest times the channel vector.  A_t and B_t are
# rounded to 24-bit fixed point (a power-of-two scale per batch), so every product
# A_t[s, p1] B_t[p2] and every partial sum over the T <= 32 terms is an exact
# FP64 number: the signal is the same in any summation order (a BLAS product on
# the host, a loop on the GPU).  The noise is a counter-based generator: SplitMix64
# (Steele, Lea & Flood, "Fast splittable pseudorandom number generators", 2014) of
# the element's counter, whose four 16-bit fields give an Irwin-Hall sum
# g = (n0 + n1 + n2 + n3 - 131070) 2^-16 (mean 0, variance ~1/3), again exact.  The
# element is float32(signal + scale * g) with one FP64 multiply and one add.

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB
FIXED_BITS = 24


def splitmix64(counter: np.ndarray) -> np.ndarray:
    """SplitMix64 output for state (counter + 1) * gamma (uint64 arithmetic mod 2^64)."""
    with np.errstate(over="ignore"):
        z = (counter.astype(np.uint64) + np.uint64(1)) * np.uint64(GOLDEN_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_MIX2)
        return z ^ (z >> np.uint64(31))


def noise_unit(key: int, start: int, count: int) -> np.ndarray:
    """Irwin-Hall noise g for elements [start, start + count) of the batch with this key."""
    c = np.arange(start, start + count, dtype=np.uint64) + np.uint64((int(key) << 40) & (2 ** 64 - 1))
    z = splitmix64(c)
    m = np.uint64(0xFFFF)
    s = (z & m) + ((z >> np.uint64(16)) & m) + ((z >> np.uint64(32)) & m) + (z >> np.uint64(48))
    return (s.astype(np.int64) - 131070).astype(np.float64) * 2.0 ** -16


def _fixed(x: np.ndarray) -> np.ndarray:
    """x rounded to FIXED_BITS-bit fixed point with a power-of-two scale above max |x|."""
    mx = float(np.max(np.abs(x)))
    if mx == 0.0:
        return np.zeros_like(x)
    e = math.frexp(mx)[1]               # mx < 2^e
    q = 2.0 ** (e - FIXED_BITS)
    return np.round(x / q) * q


def term_mask(spec: FieldSpec, k: int) -> np.ndarray:
    """1 for the terms present at batch k, 0 for those not yet switched on."""
    m = np.ones(spec.terms)
    if spec.active0 > 0:
        for t in range(spec.active0, spec.terms):
            if k < (t - spec.active0 + 1) * spec.onset_every:
                m[t] = 0.0
    return m


@dataclass
class FieldFactors:
    """One batch of an exactly reproducible field: A (T, N, P1), B (T, P2), noise scale and key."""
    A: np.ndarray
    B: np.ndarray
    scale: float
    key: int
    shape: Tuple[int, ...]


def exact_field_factors(spec: FieldSpec, k: int) -> FieldFactors:
    p = _field_params(spec)
    fs = field_mode_functions(spec, k)
    t = spec.terms
    m = len(spec.grid)
    split = (m + 1) // 2
    left = fs[0]
    for f in fs[1:split]:
        left = (left[:, :, None] * f[:, None, :]).reshape(t, -1)
    right = p["v"]
    for f in reversed(fs[split:]):
        right = (f[:, :, None] * right[:, None, :]).reshape(t, -1)
    a = rng(spec.batch_seed0 + k).standard_normal((spec.N, t))
    a = a * term_mask(spec, k)[None, :]
    A = np.ascontiguousarray(_fixed(a.T[:, :, None] * left[:, None, :]))   # (T, N, P1), C order
    B = np.ascontiguousarray(_fixed(right))                                 # (T, P2), C order
    # ||signal||^2 = sum_s sum_{t,t'} <A_t[s], A_t'[s]> <B_t, B_t'>  (for the noise scale)
    gb = B @ B.T
    e2 = 0.0
    for s in range(spec.N):
        ga = A[:, s, :] @ A[:, s, :].T
        e2 += float(np.sum(ga * gb))
    E = spec.N * left.shape[1] * right.shape[1]
    rms = math.sqrt(max(e2, 0.0) / E)
    scale = spec.nu * rms * math.sqrt(3.0)
    return FieldFactors(A, B, scale, spec.batch_seed0 + k, (spec.N,) + spec.n)


def exact_field_batch(spec: FieldSpec, k: int, chunk: int = 1 << 22, workers: int = 4) -> np.ndarray:
    """Batch k of the exactly reproducible field as float32 (N, *grid, channels), on the host.

    The signal is one BLAS product (exact, so its blocking is immaterial); only the
    noise and the rounding run in worker threads, which call no BLAS (concurrent
    BLAS calls from several threads are not safe in every BLAS build)."""
    ff = exact_field_factors(spec, k)
    T, N, P1 = ff.A.shape
    P2 = ff.B.shape[1]
    sig = (ff.A.reshape(T, N * P1).T @ ff.B).reshape(-1)      # exact in any order
    out = np.empty(N * P1 * P2, dtype=np.float32)

    def one(c0):
        c1 = min(sig.size, c0 + chunk)
        y = sig[c0:c1] + ff.scale * noise_unit(ff.key, c0, c1 - c0) if ff.scale != 0.0 else sig[c0:c1]
        out[c0:c1] = y.astype(np.float32)

    starts = range(0, sig.size, chunk)
    if workers > 1 and sig.size > chunk:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, starts))
    else:
        for c0 in starts:
            one(c0)
    return out.reshape(ff.shape)


def checksum(y: np.ndarray) -> int:
    """Exact checksum of a float32 array: the sum of its bit patterns as integers."""
    return int(np.sum(np.ascontiguousarray(y, dtype=np.float32).view(np.uint32), dtype=np.uint64))


def exact_field_stream(spec: FieldSpec, batches: Sequence[int] | None = None) -> Iterator[np.ndarray]:
    ks = range(spec.n_batches) if batches is None else batches
    for k in ks:
        yield exact_field_batch(spec, k)
