"""FP64 NumPy oracle of BHT-l2r and HT-RISE (Aksoy & Gorodetsky, arXiv 2412.16544).

TEST INFRASTRUCTURE.  This module is the slow, obviously correct reference the
HIP library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
never does, and it imports nothing from the product package.

Everything is float64.  Each step follows the paper in its own order and
notation:

* dimension tree: balanced binary tree, depth ceil(log2 d), leaves on the last
  two layers (Sec. 2.3, "Hierarchical Tucker Format"); the first half of a node's
  modes gets ceil(q/2) of them; or any binary tree over runs of consecutive modes
  given by its parent array;
* BHT-l2r: Algorithm 1 (Sec. 3.1) - HOSVD layer by layer from the leaves, the
  batch mode kept intact and absorbed into the root;
* HT-RISE: Algorithm 2 (Sec. 3.2) - Step 1 projection and the skip test
  (Eq. relative_error_threshold), Step 2 residual (Eq. compute_residual),
  Step 3 truncated SVD of the residual (Eq. svd_on_residual), basis
  concatenation (Eq. concatenating_orthonormal_vectors), parent zero padding
  (Eq. incremental_zero_padding1, App. B padWithZeros), projection onto the
  updated cores (Eq. incremental_projection_onto_updated_cores) and root
  concatenation (Eq. incremental_root_concatenate);
* reconstruction: root-to-leaves contraction (Eq. htucker_reconstruction).

Readings taken where the paper is silent or garbled (each one is listed in
the design notes of the repository):

* truncation: minimal r with ||E||_F <= eps_nw (<=), tail energies summed from
  the smallest singular value up; r >= 1 in BHT-l2r, r >= 0 for a residual
  and at most alpha - r_old;
* budget: eps_nw = eps * ||Y|| / sqrt(2d-2) (Alg. 1, Alg. 2 and the BHT-l2r
  corollary in App. A; the sqrt(2d-3) of the plain-HT theorem does not apply);
  with ``adaptive`` (App. C) it is recomputed after every layer from the error
  incurred so far and the number of SVDs left (every non-root node of the layers
  still to come);
* eps_des uses the norm of the *new* batch;
* skip test with <=, radicand clamped at 0;
* C-order reshapes; a merged sibling index is i_a * r_b + i_b, so a transfer
  core U (alpha x r) folds to (r_a, r_b, r);
* the transfer-node basis of Step 2 is the core already zero-padded by the
  growth of its children in this batch (alpha = r_a^k r_b^k);
* "unfold(C, l)" in Alg. 2's inner loop is read as the unfolding along the mode
  of node j;
* leaves on layer p-1 are processed on the partially projected tensor;
* within a layer every node sees the same tensor (HOSVD, not ST-HOSVD); with
  ``st_hosvd`` (the variant of the footnote in Sec. 2.3.1) the nodes of a layer are
  truncated left to right, each on the tensor its predecessors contracted;
* the new residual directions get one classical Gram-Schmidt pass against the
  old basis and a QR (a no-op in exact arithmetic, where they are orthogonal
  already);
* singular vectors are sign-normalised: the entry of largest magnitude (lowest
  index on ties) is made positive.

Truncated SVD: ``numpy.linalg.svd`` of the explicit unfolding when it has at most
5e7 entries, else eigen-decomposition (``numpy.linalg.eigh``) of its FP64 Gram
matrix with sigma^2 = max(lambda, 0).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

SVD_DIRECT_MAX_ENTRIES = 50_000_000


# --------------------------------------------------------------------------- #
# Dimension tree (Sec. 2.3)
# --------------------------------------------------------------------------- #


@dataclass
class Node:
    idx: int                 # position in layer-major, left-to-right order (root = 0)
    layer: int
    lo: int                  # modes [lo, hi) of the sample tensor (0-based)
    hi: int
    parent: int = -1
    children: Tuple[int, ...] = ()
    child_pos: int = -1      # 0 = first successor, 1 = second successor

    @property
    def is_leaf(self) -> bool:
        return not self.children

    @property
    def dim(self) -> int:    # valid for leaves: the mode this leaf refers to
        return self.lo


class DimTree:
    """Binary dimension tree over d modes (Sec. 2.3).

    By default balanced: a node over q > 1 modes has two successors, the first
    ceil(q/2) modes and the rest.  Any other binary tree whose nodes hold runs of
    consecutive modes can be given as ``parent`` (2d - 1 entries, -1 for the root):
    a node's successors are the nodes naming it as parent, the lower index first,
    and the leaves, read left to right, are modes 0 .. d-1.  Either way nodes are
    numbered layer by layer from the root, left to right (``parent`` must already be
    in that order), so ``nodes[1:]`` is the order of the HT rank vector
    R = [r_{1,1}, r_{1,2}, r_{2,1}, ...].
    """

    def __init__(self, d: int, parent: Optional[Sequence[int]] = None):
        if d < 2:
            raise ValueError("a dimension tree needs d >= 2")
        self.d = d
        raw: List[Tuple[int, int, int, int, int]] = []  # (layer, lo, hi, parent_raw, pos)

        def build(lo, hi, layer, parent, pos):
            me = len(raw)
            raw.append((layer, lo, hi, parent, pos))
            if hi - lo > 1:
                mid = lo + (hi - lo + 1) // 2
                build(lo, mid, layer + 1, me, 0)
                build(mid, hi, layer + 1, me, 1)

        if parent is None:
            build(0, d, 0, -1, -1)
        else:
            raw = self._from_parent(d, [int(p) for p in parent])
        order = sorted(range(len(raw)), key=lambda i: (raw[i][0], raw[i][1]))
        new_of = {old: new for new, old in enumerate(order)}
        self.nodes: List[Node] = []
        for new, old in enumerate(order):
            layer, lo, hi, par, pos = raw[old]
            self.nodes.append(Node(new, layer, lo, hi, new_of[par] if par >= 0 else -1, (), pos))
        kids: Dict[int, List[int]] = {}
        for nd in self.nodes:
            if nd.parent >= 0:
                kids.setdefault(nd.parent, []).append(nd.idx)
        for p_idx, ch in kids.items():
            ch.sort(key=lambda i: self.nodes[i].lo)
            self.nodes[p_idx].children = tuple(ch)
        self.depth = max(nd.layer for nd in self.nodes)

    @staticmethod
    def _from_parent(d: int, parent: List[int]) -> List[Tuple[int, int, int, int, int]]:
        """(layer, lo, hi, parent, pos) per node of a tree given by its parent array."""
        if len(parent) != 2 * d - 1 or parent[0] != -1:
            raise ValueError("a tree over d modes has 2d - 1 nodes, node 0 the root (parent -1)")
        kids: List[List[int]] = [[] for _ in parent]
        for i in range(1, len(parent)):
            if not 0 <= parent[i] < i:
                raise ValueError("every node's parent must precede it")
            kids[parent[i]].append(i)
        if any(len(k) not in (0, 2) for k in kids):
            raise ValueError("every inner node needs exactly two successors")
        lo = [0] * len(parent)
        hi = [0] * len(parent)
        layer = [0] * len(parent)
        nxt = [0]

        def walk(i):
            if not kids[i]:
                lo[i], hi[i] = nxt[0], nxt[0] + 1
                nxt[0] += 1
                return
            for c in kids[i]:
                layer[c] = layer[i] + 1
                walk(c)
            lo[i], hi[i] = lo[kids[i][0]], hi[kids[i][1]]

        walk(0)
        if nxt[0] != d:
            raise ValueError("the tree must have d leaves")
        key = [(layer[i], lo[i]) for i in range(len(parent))]
        if key != sorted(key):
            raise ValueError("nodes must be numbered layer by layer, left to right")
        pos = [-1] + [kids[parent[i]].index(i) for i in range(1, len(parent))]
        return [(layer[i], lo[i], hi[i], parent[i], pos[i]) for i in range(len(parent))]

    def parents(self) -> List[int]:
        return [nd.parent for nd in self.nodes]

    def layer(self, ell: int) -> List[Node]:
        return [nd for nd in self.nodes if nd.layer == ell]

    def frontier(self, ell: int) -> List[Node]:
        """Modes of the level tensor entering layer ell, in mode order.

        The nodes of layer ell, plus leaves of shallower layers (whose modes pass
        through untouched until their own layer is processed).
        """
        f = [nd for nd in self.nodes if nd.layer == ell or (nd.is_leaf and nd.layer < ell)]
        return sorted(f, key=lambda nd: nd.lo)

    @property
    def non_root(self) -> List[Node]:
        return self.nodes[1:]


# --------------------------------------------------------------------------- #
# Tensor primitives (Sec. 2.1)
# --------------------------------------------------------------------------- #


def fro2(x: np.ndarray) -> float:
    """Squared Frobenius norm in float64 (NumPy's pairwise summation)."""
    x = np.asarray(x, dtype=np.float64)
    return float(np.sum(x * x))


def unfold(c: np.ndarray, k: int) -> np.ndarray:
    """Mode-k unfolding: mode k becomes the rows, every other mode the columns."""
    return np.moveaxis(c, k, 0).reshape(c.shape[k], -1)


def contract_mode_t(c: np.ndarray, k: int, u: np.ndarray) -> np.ndarray:
    """C x_k U^T: mode k of size alpha is contracted with U (alpha x r) -> size r."""
    out = np.tensordot(c, u, axes=([k], [0]))
    return np.moveaxis(out, -1, k)


def contract_mode(c: np.ndarray, k: int, u: np.ndarray) -> np.ndarray:
    """C x_k U: mode k of size r is expanded with U (alpha x r) -> size alpha."""
    out = np.tensordot(c, u, axes=([k], [1]))
    return np.moveaxis(out, -1, k)


def sign_normalise(u: np.ndarray) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry is positive."""
    u = np.array(u, dtype=np.float64, copy=True)
    if u.size == 0:
        return u
    piv = np.argmax(np.abs(u), axis=0)
    s = np.sign(u[piv, np.arange(u.shape[1])])
    s[s == 0] = 1.0
    return u * s[None, :]


@dataclass
class Truncation:
    """One error-truncated SVD decision (Eq. ht_leaf_svd / svd_on_residual)."""

    rank: int
    sigma: np.ndarray        # all singular values, descending
    tail2: float             # sum of sigma_i^2 over the discarded i
    eps_nw: float
    tail2_prev: float        # tail energy one rank lower (inf when rank == rmin)
    rmin: int
    rmax: int

    def near_tie(self, rel: float = 1e-9, abs_tol: float = 0.0) -> bool:
        """True when the decision sits within max(rel * eps_nw^2, abs_tol) of the threshold."""
        thr = self.eps_nw ** 2
        band = max(rel * thr, abs_tol)
        close_keep = abs(self.tail2 - thr) <= band
        close_drop = math.isfinite(self.tail2_prev) and abs(self.tail2_prev - thr) <= band
        return close_keep or close_drop


def truncated_svd(m: np.ndarray, eps_nw: float, rmin: int, rmax: Optional[int] = None):
    """Left singular vectors of M kept by the minimal-rank rule ||E||_F <= eps_nw.

    Returns (U_r, Truncation).  ``rmax`` caps the rank (used for residuals).
    """
    a, b = m.shape
    if a * b <= SVD_DIRECT_MAX_ENTRIES:
        u, s, _ = np.linalg.svd(m, full_matrices=False)
    else:
        lam, v = np.linalg.eigh(m @ m.T)
        order = np.argsort(lam)[::-1]
        lam = lam[order]
        u = v[:, order]
        s = np.sqrt(np.clip(lam, 0.0, None))
    kmax = len(s) if rmax is None else min(len(s), rmax)
    sq = s.astype(np.float64) ** 2
    # tail[r] = sum_{i >= r} sigma_i^2 (0-based), accumulated from the smallest value up
    tail = np.zeros(len(s) + 1)
    acc = 0.0
    for i in range(len(s) - 1, -1, -1):
        acc += sq[i]
        tail[i] = acc
    thr = eps_nw * eps_nw
    r = None
    for cand in range(rmin, kmax + 1):
        if tail[cand] <= thr:
            r = cand
            break
    if r is None:
        r = kmax
    prev = tail[r - 1] if r - 1 >= rmin else math.inf
    info = Truncation(rank=r, sigma=s, tail2=float(tail[r]), eps_nw=eps_nw,
                      tail2_prev=float(prev), rmin=rmin, rmax=kmax)
    return sign_normalise(u[:, :r]), info


# --------------------------------------------------------------------------- #
# Batch hierarchical Tucker state
# --------------------------------------------------------------------------- #


@dataclass
class BatchInfo:
    skipped: bool
    norm_y: float
    eps_des: float
    eps_proj: float
    ranks: List[int]
    decisions: Dict[int, Truncation] = field(default_factory=dict)

    def any_near_tie(self, rel: float = 1e-9, abs_tol: float = 0.0) -> bool:
        return any(t.near_tie(rel, abs_tol) for t in self.decisions.values())


class BHT:
    """Batch-HT representation (tree, cores) of an accumulation (Sec. 3.1).

    ``core[i]`` is node i's basis as a matrix: n_i x r for a leaf, (r_a r_b) x r
    for a transfer node (row index i_a * r_b + i_b).  ``root`` has shape
    (r_{1,1}, r_{1,2}, N_acc).
    """

    def __init__(self, n: Sequence[int], eps: float, tree: Optional[DimTree] = None, adaptive: bool = False,
                 st_hosvd: bool = False):
        self.n = tuple(int(x) for x in n)
        self.d = len(self.n)
        self.tree = tree if tree is not None else DimTree(self.d)
        if not (0.0 < eps < 1.0):
            raise ValueError("eps must lie in (0, 1)")
        self.eps = float(eps)
        # App. C: after each layer the nodewise tolerance is recomputed from the error
        # actually incurred so far, eps_nw = sqrt(eps_abs^2 - eps_l^2) / sqrt(svd_rem)
        self.adaptive = bool(adaptive)
        # the footnote of Sec. 2.3.1: the nodes of a layer may instead be truncated one
        # after the other (ST-HOSVD), each on the tensor its predecessors in the layer
        # (left to right) have already contracted
        self.st_hosvd = bool(st_hosvd)
        self.core: Dict[int, np.ndarray] = {}
        self.root: Optional[np.ndarray] = None
        self.history: List[BatchInfo] = []

    # ---- bookkeeping (updateIndexSet, App. B) -------------------------------
    def rank(self, idx: int) -> int:
        return int(self.core[idx].shape[1])

    @property
    def ranks(self) -> List[int]:
        return [self.rank(nd.idx) for nd in self.tree.non_root]

    @property
    def n_accum(self) -> int:
        return 0 if self.root is None else int(self.root.shape[2])

    def mode_size(self, nd: Node, processed: bool) -> int:
        """Size of node nd's mode in a level tensor (before or after its own layer)."""
        if processed:
            return self.rank(nd.idx)
        if nd.is_leaf:
            return self.n[nd.dim]
        a, b = nd.children
        return self.rank(a) * self.rank(b)

    def _merge_to(self, c: np.ndarray, ell: int) -> np.ndarray:
        """Reshape a tensor whose layer-ell nodes are contracted to the layer ell-1 frontier.

        Adjacent sibling modes fuse into one mode of size r_a * r_b (Eq.
        ht_index_set_construction); C order gives the index i_a * r_b + i_b.
        """
        n_b = c.shape[0]
        if ell == 1:
            r11 = self.rank(self.tree.nodes[0].children[0])
            r12 = self.rank(self.tree.nodes[0].children[1])
            return c.reshape(n_b, r11, r12)
        sizes = [self.mode_size(nd, processed=False) for nd in self.tree.frontier(ell - 1)]
        return c.reshape((n_b,) + tuple(sizes))

    # ---- Step 1: projection onto the cores ------------------------------------
    def project(self, y: np.ndarray) -> np.ndarray:
        """Latent code C1 (N, r11, r12) of a batch: contract leaves-to-root with U^T."""
        c = np.asarray(y, dtype=np.float64)
        for ell in range(self.tree.depth, 0, -1):
            front = self.tree.frontier(ell)
            for k, nd in enumerate(front):
                if nd.layer == ell:
                    c = contract_mode_t(c, 1 + k, self.core[nd.idx])
            c = self._merge_to(c, ell)
        return c

    # ---- root-to-leaves reconstruction (Eq. htucker_reconstruction) ---------
    def decode(self, latent: np.ndarray) -> np.ndarray:
        """Full tensors (N, *n) from latent codes (N, r11, r12)."""
        c = np.asarray(latent, dtype=np.float64)
        n_b = c.shape[0]
        for ell in range(1, self.tree.depth + 1):
            front = self.tree.frontier(ell)
            # split every merged mode of the previous layer into the ell-layer modes
            c = c.reshape((n_b,) + tuple(self.mode_size(nd, processed=(nd.layer == ell)) for nd in front))
            for k, nd in enumerate(front):
                if nd.layer == ell:
                    c = contract_mode(c, 1 + k, self.core[nd.idx])
        return c.reshape((n_b,) + self.n)

    def relative_test_errors(self, y: np.ndarray) -> np.ndarray:
        """Per-sample ||Y_i - decode(project(Y_i))|| / ||Y_i|| of held-out samples: the
        summands of the relative test error (Sec. 4.1, Eq. generalization_performance)."""
        y = np.asarray(y, dtype=np.float64)
        rec = self.decode(self.project(y))
        d = (y - rec).reshape(y.shape[0], -1)
        n = y.reshape(y.shape[0], -1)
        return np.sqrt(np.sum(d * d, axis=1)) / np.sqrt(np.sum(n * n, axis=1))

    def reconstruct(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = self.n_accum - first
        lat = np.moveaxis(self.root[:, :, first:first + count], 2, 0)
        return self.decode(lat)

    def _adapted_eps_nw(self, eps_abs: float, ny2: float, c: np.ndarray, ell: int) -> float:
        """App. C: the nodewise tolerance for the layers above ell, from the error of
        the approximation so far, eps_l^2 = ||Y||^2 - ||C_l||^2, the remaining budget
        eps_rem^2 = eps_abs^2 - eps_l^2 and the number of SVDs still to come."""
        eps_l2 = ny2 - fro2(c)
        rem2 = max(0.0, eps_abs * eps_abs - eps_l2)
        svd_rem = sum(1 for nd in self.tree.non_root if nd.layer < ell)
        return math.sqrt(rem2 / svd_rem)

    # ---- BHT-l2r (Algorithm 1) -----------------------------------------------
    def init_batch(self, y: np.ndarray) -> BatchInfo:
        y = np.asarray(y, dtype=np.float64)
        self._check_batch(y)
        d = self.d
        ny = math.sqrt(fro2(y))
        if ny == 0.0:
            raise ValueError("the initial batch must not be all zeros")
        eps_nw = self.eps * ny / math.sqrt(2 * d - 2)
        self.core = {}
        decisions: Dict[int, Truncation] = {}
        c = y
        for ell in range(self.tree.depth, 0, -1):
            front = self.tree.frontier(ell)
            here = [(k, nd) for k, nd in enumerate(front) if nd.layer == ell]
            if self.st_hosvd:
                for k, nd in here:  # each node on the tensor its predecessors contracted
                    u, t = truncated_svd(unfold(c, 1 + k), eps_nw, rmin=1)
                    decisions[nd.idx] = t
                    self.core[nd.idx] = u
                    c = contract_mode_t(c, 1 + k, u)
            else:
                bases = {}
                for k, nd in here:  # every node of the layer sees the same tensor
                    u, t = truncated_svd(unfold(c, 1 + k), eps_nw, rmin=1)
                    bases[nd.idx] = u
                    decisions[nd.idx] = t
                for k, nd in here:
                    self.core[nd.idx] = bases[nd.idx]
                    c = contract_mode_t(c, 1 + k, bases[nd.idx])
            c = self._merge_to(c, ell)
            if self.adaptive and ell > 1:
                eps_nw = self._adapted_eps_nw(self.eps * ny, ny * ny, c, ell)
        self.root = np.ascontiguousarray(np.moveaxis(c, 0, 2))
        c2 = fro2(c)
        info = BatchInfo(False, ny, self.eps * ny, math.sqrt(max(0.0, ny * ny - c2)), self.ranks, decisions)
        self.history.append(info)
        return info

    # ---- HT-RISE (Algorithm 2) -----------------------------------------------
    def update(self, y: np.ndarray) -> BatchInfo:
        y = np.asarray(y, dtype=np.float64)
        self._check_batch(y)
        if self.root is None:
            raise RuntimeError("update before the initial batch")
        d = self.d
        ny2 = fro2(y)
        ny = math.sqrt(ny2)
        eps_des = self.eps * ny
        c1 = self.project(y)
        eps_proj = math.sqrt(max(0.0, ny2 - fro2(c1)))
        if eps_proj <= eps_des:
            self._append_root(c1)
            info = BatchInfo(True, ny, eps_des, eps_proj, self.ranks, {})
            self.history.append(info)
            return info
        eps_nw = eps_des / math.sqrt(2 * d - 2)
        decisions: Dict[int, Truncation] = {}
        c = y
        for ell in range(self.tree.depth, 0, -1):
            front = self.tree.frontier(ell)
            here = [(k, nd) for k, nd in enumerate(front) if nd.layer == ell]
            grown = {}
            for k, nd in here:
                u_old = self.core[nd.idx]
                alpha, r_old = u_old.shape
                m = unfold(c, 1 + k)
                resid = m - u_old @ (u_old.T @ m)                           # Step 2
                u_r, t = truncated_svd(resid, eps_nw, rmin=0, rmax=alpha - r_old)  # Step 3
                decisions[nd.idx] = t
                if u_r.shape[1] > 0:
                    u_r = u_r - u_old @ (u_old.T @ u_r)
                    q, rr = np.linalg.qr(u_r)
                    u_r = sign_normalise(q)
                grown[nd.idx] = np.concatenate([u_old, u_r], axis=1)
                if self.st_hosvd:   # this node's expansion, then its contraction, before the next
                    self._pad_parent(nd, grown[nd.idx].shape[1] - r_old)
                    self.core[nd.idx] = grown[nd.idx]
                    c = contract_mode_t(c, 1 + k, grown[nd.idx])
            if not self.st_hosvd:
                for k, nd in here:
                    r_new = grown[nd.idx].shape[1] - self.rank(nd.idx)
                    self._pad_parent(nd, r_new)
                    self.core[nd.idx] = grown[nd.idx]
                for k, nd in here:
                    c = contract_mode_t(c, 1 + k, self.core[nd.idx])
            c = self._merge_to(c, ell)
            if self.adaptive and ell > 1:
                eps_nw = self._adapted_eps_nw(eps_des, ny2, c, ell)
        self._append_root(c)
        info = BatchInfo(False, ny, eps_des, eps_proj, self.ranks, decisions)
        self.history.append(info)
        return info

    # ---- padWithZeros (App. B) and root concatenation -------------------------
    def _pad_parent(self, nd: Node, r_new: int) -> None:
        if r_new == 0:
            return
        par = self.tree.nodes[nd.parent]
        if par.idx == 0:
            widths = [(0, 0), (0, 0), (0, 0)]
            widths[nd.child_pos] = (0, r_new)
            self.root = np.pad(self.root, widths)
            return
        a, b = par.children
        ra, rb = self.rank(a), self.rank(b)
        g = self.core[par.idx].reshape(ra, rb, -1)
        widths = [(0, 0), (0, 0), (0, 0)]
        widths[nd.child_pos] = (0, r_new)
        g = np.pad(g, widths)
        self.core[par.idx] = g.reshape(g.shape[0] * g.shape[1], g.shape[2])

    def _append_root(self, c1: np.ndarray) -> None:
        self.root = np.concatenate([self.root, np.moveaxis(c1, 0, 2)], axis=2)

    def _check_batch(self, y: np.ndarray) -> None:
        if y.ndim != self.d + 1 or tuple(y.shape[1:]) != self.n:
            raise ValueError("batch shape %r does not match (N, %r)" % (y.shape, self.n))
        if y.shape[0] < 1:
            raise ValueError("empty batch")

    # ---- the transfer core as a 3-way tensor (Eq. ht_tucker_core_reshape) ----
    def core3(self, idx: int) -> np.ndarray:
        nd = self.tree.nodes[idx]
        if nd.is_leaf:
            return self.core[idx]
        a, b = nd.children
        return self.core[idx].reshape(self.rank(a), self.rank(b), self.rank(idx))


class PlainHT:
    """Leaves-to-root error truncated hierarchical Tucker decomposition of ONE d-way
    tensor (Sec. 2.3.1, the algorithm the paper takes from Grasedyck's leaves-to-root
    method), the baseline the batch format is compared with (App. D.1).

    Layers p..2: an error truncated SVD of every node's unfolding of the same level
    tensor (Eq. ht_leaf_svd, HOSVD within a layer), contraction with the kept left
    singular vectors (Eq. ht_leaf_contraction) and the reshape to the next frontier
    (Eq. ht_index_set_construction); transfer cores are the reshaped vectors (Eq.
    ht_tucker_core_reshape).  Layer 1: one truncated SVD of the matrix C_1 (Eq.
    ht_last_svd): U_1 and V_1 become the cores of the root's two successors and the
    kept singular values the (diagonal) root.  Every truncation uses
    eps_nw = eps ||Y|| / sqrt(2d - 3) (Thm. ht_nodewise_error).
    """

    def __init__(self, y: np.ndarray, eps: float, tree: Optional[DimTree] = None):
        y = np.asarray(y, dtype=np.float64)
        self.n = tuple(y.shape)
        self.d = y.ndim
        if self.d < 2:
            raise ValueError("a dimension tree needs d >= 2")
        self.tree = tree if tree is not None else DimTree(self.d)
        self.eps = float(eps)
        ny = math.sqrt(fro2(y))
        eps_nw = self.eps * ny / math.sqrt(2 * self.d - 3)
        self.core: Dict[int, np.ndarray] = {}
        self.decisions: Dict[int, Truncation] = {}
        c = y
        for ell in range(self.tree.depth, 1, -1):
            front = self.tree.frontier(ell)
            here = [(k, nd) for k, nd in enumerate(front) if nd.layer == ell]
            bases = {}
            for k, nd in here:          # every node of the layer sees the same tensor
                u, t = truncated_svd(unfold(c, k), eps_nw, rmin=1)
                bases[nd.idx] = u
                self.decisions[nd.idx] = t
            for k, nd in here:
                self.core[nd.idx] = bases[nd.idx]
                c = contract_mode_t(c, k, bases[nd.idx])
            c = c.reshape(tuple(self._size(nd) for nd in self.tree.frontier(ell - 1)))
        # layer 1: the final SVD of C_1 (alpha_11 x alpha_12)
        root = self.tree.nodes[0]
        a, b = root.children
        c1 = c.reshape(self._size(self.tree.nodes[a]), self._size(self.tree.nodes[b]))
        u, sv, vt = np.linalg.svd(c1, full_matrices=False)
        tail = np.concatenate([np.cumsum((sv ** 2)[::-1])[::-1], [0.0]])
        r0 = next(r for r in range(1, len(sv) + 1) if tail[r] <= eps_nw * eps_nw)
        self.core[a] = u[:, :r0]
        self.core[b] = vt[:r0].T
        self.root = np.diag(sv[:r0])
        self.decisions[a] = Truncation(rank=r0, sigma=sv, tail2=float(tail[r0]), eps_nw=eps_nw,
                                       tail2_prev=float(tail[r0 - 1]) if r0 > 1 else math.inf, rmin=1,
                                       rmax=len(sv))

    def _size(self, nd: Node) -> int:
        """Size of nd's mode in the level tensor entering its layer."""
        if nd.is_leaf:
            return self.n[nd.dim]
        ca, cb = nd.children
        return self.core[ca].shape[1] * self.core[cb].shape[1]

    @property
    def ranks(self) -> List[int]:
        return [int(self.core[nd.idx].shape[1]) for nd in self.tree.non_root]

    def _frame(self, idx: int) -> np.ndarray:
        """The node's basis over its modes: (prod of its mode sizes) x r, C order."""
        nd = self.tree.nodes[idx]
        if nd.is_leaf:
            return self.core[idx]
        ca, cb = nd.children
        fa, fb = self._frame(ca), self._frame(cb)
        g = self.core[idx].reshape(fa.shape[1], fb.shape[1], -1)
        return np.einsum("ia,jb,abr->ijr", fa, fb, g).reshape(fa.shape[0] * fb.shape[0], -1)

    def reconstruct(self) -> np.ndarray:
        a, b = self.tree.nodes[0].children
        return (self._frame(a) @ self.root @ self._frame(b).T).reshape(self.n)

    def num_elements(self) -> int:
        """Entries of all cores and the root (the denominator of the compression ratio)."""
        return int(sum(u.size for u in self.core.values()) + self.root.size)


def compress_stream(batches, eps: float, tree: Optional[DimTree] = None) -> BHT:
    """BHT-l2r on the first batch, HT-RISE on every later one."""
    it = iter(batches)
    first = np.asarray(next(it), dtype=np.float64)
    st = BHT(first.shape[1:], eps, tree)
    st.init_batch(first)
    for y in it:
        st.update(y)
    return st
