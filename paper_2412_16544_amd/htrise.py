"""Python binding of the C ABI in include/ht_rise.h (argument marshalling only).

The functions below carry the C names and pass raw device pointers of torch
tensors to ``libhtrise.so``; every step of BHT-l2r / HT-RISE runs in the
library's HIP kernels.  PyTorch only supplies device memory and the stream.
The library must be built (``python -m paper_2412_16544_amd.build``); loading
fails loudly otherwise - there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhtrise.so")

HT_OK, HT_EINVAL, HT_ESHAPE, HT_ENOMEM, HT_ERANKCAP, HT_EDEVICE, HT_ENUMERIC = range(7)
HT_FP64, HT_FP32, HT_BF16X3 = 0, 1, 2
HT_F32, HT_F64 = 0, 1
HT_ADAPTIVE_BUDGET, HT_PLAIN_HT_BUDGET, HT_ST_HOSVD = 1, 2, 4

STATUS_NAMES = {0: "HT_OK", 1: "HT_EINVAL", 2: "HT_ESHAPE", 3: "HT_ENOMEM", 4: "HT_ERANKCAP",
                5: "HT_EDEVICE", 6: "HT_ENUMERIC"}


class ht_config(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n", ctypes.POINTER(ctypes.c_int64)), ("eps_rel", ctypes.c_double),
                ("rank_cap", ctypes.c_int32), ("max_batch", ctypes.c_int64), ("n_cap", ctypes.c_int64),
                ("prec", ctypes.c_int32), ("in_dtype", ctypes.c_int32), ("flags", ctypes.c_uint64),
                ("tree_parent", ctypes.POINTER(ctypes.c_int32))]


class ht_update_info(ctypes.Structure):
    _fields_ = [("skipped", ctypes.c_int32), ("rank_growth", ctypes.c_int32), ("norm_y", ctypes.c_double),
                ("eps_proj", ctypes.c_double), ("eps_des", ctypes.c_double), ("device_ms", ctypes.c_float),
                ("status", ctypes.c_int32), ("prec_used", ctypes.c_int32), ("recomputed", ctypes.c_int32)]


class HTError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhtrise.so is not built; run `python -m paper_2412_16544_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        L.ht_workspace_bytes.argtypes = [ctypes.POINTER(ht_config), ctypes.POINTER(sz)]
        L.ht_update_precision.argtypes = [ctypes.POINTER(ht_config), ctypes.POINTER(i32)]
        L.ht_init_batch.argtypes = [ctypes.POINTER(ht_config), vp, sz, vp, i64, vp, ctypes.POINTER(vp),
                                    ctypes.POINTER(ht_update_info)]
        L.ht_rise_update.argtypes = [vp, vp, i64, vp, ctypes.POINTER(ht_update_info)]
        L.ht_rise_update_many.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64), i32, vp,
                                          ctypes.POINTER(ht_update_info)]
        L.ht_project.argtypes = [vp, vp, i64, vp, vp]
        L.ht_project_static.argtypes = [vp, vp, i64, vp, vp]
        L.ht_reconstruct.argtypes = [vp, i64, i64, vp, i32, vp]
        L.ht_decode.argtypes = [vp, vp, i64, vp, i32, vp]
        L.ht_rte.argtypes = [vp, vp, i64, ctypes.POINTER(ctypes.c_double), vp]
        L.ht_query_ranks.argtypes = [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.ht_export_cores.argtypes = [vp, ctypes.POINTER(ctypes.c_double), sz, ctypes.POINTER(sz)]
        L.ht_destroy.argtypes = [vp]
        L.ht_destroy.restype = None
        L.ht_status_str.argtypes = [ctypes.c_int]
        L.ht_status_str.restype = ctypes.c_char_p
        L.ht_last_error.argtypes = []
        L.ht_last_error.restype = ctypes.c_char_p
        for name in ("ht_workspace_bytes", "ht_update_precision", "ht_init_batch", "ht_rise_update",
                     "ht_rise_update_many", "ht_project", "ht_project_static", "ht_decode", "ht_rte",
                     "ht_reconstruct", "ht_query_ranks", "ht_export_cores"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st: int, where: str) -> None:
    if st != HT_OK:
        raise HTError(st, where, lib().ht_last_error().decode())


def make_config(n: Sequence[int], eps: float, rank_cap: int, max_batch: int, n_cap: int,
                prec: int = HT_FP64, in_dtype: int = HT_F32, flags: int = 0,
                tree_parent: Optional[Sequence[int]] = None) -> Tuple[ht_config, object]:
    arr = (ctypes.c_int64 * len(n))(*[int(x) for x in n])
    par = None if tree_parent is None else (ctypes.c_int32 * len(tree_parent))(*[int(x) for x in tree_parent])
    cfg = ht_config(len(n), ctypes.cast(arr, ctypes.POINTER(ctypes.c_int64)), float(eps), int(rank_cap),
                    int(max_batch), int(n_cap), int(prec), int(in_dtype), int(flags),
                    None if par is None else ctypes.cast(par, ctypes.POINTER(ctypes.c_int32)))
    return cfg, (arr, par)  # keep the arrays alive with cfg


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream) -> int:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(stream)


# ---- the C entry points, same names ------------------------------------------------------------
def ht_workspace_bytes(cfg: ht_config) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().ht_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)), "ht_workspace_bytes")
    return int(out.value)


def ht_update_precision(cfg: ht_config) -> int:
    out = ctypes.c_int32(0)
    _check(lib().ht_update_precision(ctypes.byref(cfg), ctypes.byref(out)), "ht_update_precision")
    return int(out.value)


def ht_init_batch(cfg: ht_config, ws, Y, stream=None) -> Tuple[int, ht_update_info]:
    h = ctypes.c_void_p(0)
    info = ht_update_info()
    st = lib().ht_init_batch(ctypes.byref(cfg), _ptr(ws), ws.numel() * ws.element_size(), _ptr(Y), Y.shape[0],
                             _stream(stream), ctypes.byref(h), ctypes.byref(info))
    _check(st, "ht_init_batch")
    return h.value, info


def ht_rise_update(h: int, Y, stream=None) -> ht_update_info:
    info = ht_update_info()
    _check(lib().ht_rise_update(h, _ptr(Y), Y.shape[0], _stream(stream), ctypes.byref(info)), "ht_rise_update")
    return info


def ht_rise_update_many(handles: Sequence[int], Ys, stream=None):
    """HT-RISE on several handles in lock step; returns (status, [ht_update_info]).

    Raises HTError for argument errors; a handle whose update failed is rolled back
    and reported through its info's status (the call's status is the first failure).
    """
    n = len(handles)
    hs = (ctypes.c_void_p * n)(*[ctypes.c_void_p(h) for h in handles])
    ys = (ctypes.c_void_p * n)(*[ctypes.c_void_p(_ptr(y)) for y in Ys])
    ns = (ctypes.c_int64 * n)(*[int(y.shape[0]) for y in Ys])
    infos = (ht_update_info * n)()
    st = lib().ht_rise_update_many(hs, ys, ns, n, _stream(stream), infos)
    if st not in (HT_OK, HT_ERANKCAP, HT_ENUMERIC):
        _check(st, "ht_rise_update_many")
    return st, list(infos)


def ht_project(h: int, Y, latent, stream=None) -> None:
    _check(lib().ht_project(h, _ptr(Y), Y.shape[0], _ptr(latent), _stream(stream)), "ht_project")


def ht_project_static(h: int, Y, latent, stream=None) -> None:
    _check(lib().ht_project_static(h, _ptr(Y), Y.shape[0], _ptr(latent), _stream(stream)), "ht_project_static")


def ht_reconstruct(h: int, first: int, count: int, out, dtype: int, stream=None) -> None:
    _check(lib().ht_reconstruct(h, first, count, _ptr(out), dtype, _stream(stream)), "ht_reconstruct")


def ht_decode(h: int, latent, out, dtype: int, stream=None) -> None:
    _check(lib().ht_decode(h, _ptr(latent), latent.shape[0], _ptr(out), dtype, _stream(stream)), "ht_decode")


def ht_rte(h: int, Y, stream=None) -> List[float]:
    n = int(Y.shape[0])
    buf = (ctypes.c_double * n)()
    _check(lib().ht_rte(h, _ptr(Y), n, buf, _stream(stream)), "ht_rte")
    return [float(buf[i]) for i in range(n)]


def ht_query_ranks(h: int) -> Tuple[List[int], int]:
    buf = (ctypes.c_int32 * 256)()
    nr = ctypes.c_int32(0)
    nacc = ctypes.c_int64(0)
    _check(lib().ht_query_ranks(h, buf, 256, ctypes.byref(nr), ctypes.byref(nacc)), "ht_query_ranks")
    return [int(buf[i]) for i in range(nr.value)], int(nacc.value)


def ht_export_cores(h: int):
    import numpy as np
    need = ctypes.c_size_t(0)
    _check(lib().ht_export_cores(h, None, 0, ctypes.byref(need)), "ht_export_cores")
    out = np.zeros(need.value // 8, dtype=np.float64)
    _check(lib().ht_export_cores(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), need.value,
                                 ctypes.byref(need)), "ht_export_cores")
    return out


def ht_destroy(h: int) -> None:
    if h:
        lib().ht_destroy(h)


def ht_status_str(st: int) -> str:
    return lib().ht_status_str(st).decode()


# ---- a handle object that owns the workspace tensor -----------------------------------------
@dataclass
class UpdateInfo:
    skipped: bool
    rank_growth: int
    norm_y: float
    eps_proj: float
    eps_des: float
    device_ms: float
    status: int = HT_OK
    prec_used: int = HT_FP64
    recomputed: int = 0

    @staticmethod
    def of(i: ht_update_info) -> "UpdateInfo":
        return UpdateInfo(bool(i.skipped), int(i.rank_growth), float(i.norm_y), float(i.eps_proj),
                          float(i.eps_des), float(i.device_ms), int(i.status), int(i.prec_used),
                          int(i.recomputed))


class HTStream:
    """One tensor stream in batch-HT form: the workspace tensor plus the library handle."""

    def __init__(self, n: Sequence[int], eps: float, rank_cap: int, max_batch: int, n_cap: int,
                 in_dtype: str = "float32", prec: int = HT_FP64, device: str = "cuda:0", flags: int = 0,
                 tree_parent: Optional[Sequence[int]] = None):
        import torch
        self.n = tuple(int(x) for x in n)
        self.d = len(self.n)
        self.device = torch.device(device)
        self._cfg, self._keep = make_config(self.n, eps, rank_cap, max_batch, n_cap, prec,
                                            HT_F32 if in_dtype == "float32" else HT_F64, flags, tree_parent)
        self.ws_bytes = ht_workspace_bytes(self._cfg)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.h = 0

    def init_batch(self, Y, stream=None) -> UpdateInfo:
        if self.h:
            raise RuntimeError("stream already initialised")
        self.h, info = ht_init_batch(self._cfg, self.ws, Y, stream)
        return UpdateInfo.of(info)

    def update(self, Y, stream=None) -> UpdateInfo:
        return UpdateInfo.of(ht_rise_update(self.h, Y, stream))

    def push(self, Y, stream=None) -> UpdateInfo:
        return self.init_batch(Y, stream) if not self.h else self.update(Y, stream)

    @staticmethod
    def update_many(streams: Sequence["HTStream"], Ys, stream=None) -> Tuple[int, List[UpdateInfo]]:
        """HT-RISE on several initialised streams at once (ht_rise_update_many)."""
        st, infos = ht_rise_update_many([s.h for s in streams], Ys, stream)
        return st, [UpdateInfo.of(i) for i in infos]

    def ranks(self) -> Tuple[List[int], int]:
        return ht_query_ranks(self.h)

    def project(self, Y, stream=None):
        import torch
        r, _ = self.ranks()
        lat = torch.empty((Y.shape[0], r[0], r[1]), dtype=torch.float64, device=self.device)
        ht_project(self.h, Y, lat, stream)
        return lat

    def reconstruct(self, first: int = 0, count: Optional[int] = None, dtype: str = "float64", stream=None):
        import torch
        _, nacc = self.ranks()
        if count is None:
            count = nacc - first
        td = torch.float64 if dtype == "float64" else torch.float32
        out = torch.empty((count,) + self.n, dtype=td, device=self.device)
        ht_reconstruct(self.h, first, count, out, HT_F64 if dtype == "float64" else HT_F32, stream)
        return out

    def decode(self, latent, dtype: str = "float64", stream=None):
        """Tensors of latent codes [N][r11][r12] (float64 CUDA tensor), root-to-leaves."""
        import torch
        td = torch.float64 if dtype == "float64" else torch.float32
        out = torch.empty((latent.shape[0],) + self.n, dtype=td, device=self.device)
        ht_decode(self.h, latent.contiguous(), out, HT_F64 if dtype == "float64" else HT_F32, stream)
        return out

    def rte(self, Y, stream=None) -> List[float]:
        """Per-sample relative errors of encode -> decode on held-out samples."""
        return ht_rte(self.h, Y, stream)

    def export(self):
        """Cores (rank-vector order, rows x r) and root (N_acc, r11, r12) as float64 NumPy arrays."""
        flat = ht_export_cores(self.h)
        return flat

    def reset(self) -> None:
        """Drops the representation; the workspace is kept for the next init_batch."""
        if self.h:
            ht_destroy(self.h)
            self.h = 0

    def close(self) -> None:
        if self.h:
            ht_destroy(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- kernel-level entry points of include/ht_rise_testing.h -----------------------------------
def _tlib():
    L = lib()
    if not getattr(L, "_ht_testing_ready", False):
        vp, i64, i32, sz, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double
        L.ht_test_sumsq.argtypes = [vp, i32, i64, vp, vp, vp]
        L.ht_test_gram_scratch_doubles.argtypes = [i64, i64, i64]
        L.ht_test_gram_scratch_doubles.restype = sz
        L.ht_test_gram.argtypes = [vp, i32, i64, i64, i64, vp, vp, vp]
        L.ht_test_ttm_contract.argtypes = [vp, i32, i64, i64, i64, vp, i32, vp, vp]
        L.ht_test_resid_gram.argtypes = [vp, i32, i64, i64, i64, vp, i32, vp, vp, vp]
        L.ht_test_resid_gram_f32.argtypes = [vp, i32, i64, i64, i64, vp, i32, vp, vp, vp]
        L.ht_test_resid_gram_proj.argtypes = [vp, i32, i64, i64, i64, vp, i32, vp, vp, vp]
        L.ht_test_ttm_contract_split.argtypes = [vp, i32, i64, i64, i64, vp, i32, vp, vp, sz, vp, vp]
        L.ht_test_ttm_partials_doubles.argtypes = []
        L.ht_test_ttm_partials_doubles.restype = sz
        L.ht_test_ttm_contract_f32.argtypes = [vp, i32, i64, i64, i64, vp, i32, vp, vp, vp, vp, vp]
        L.ht_test_ttm_expand.argtypes = [vp, i64, i32, i64, vp, i64, vp, i32, vp, i32, vp]
        L.ht_test_eig_scratch_doubles.argtypes = [i32, i32]
        L.ht_test_eig_scratch_doubles.restype = sz
        L.ht_test_eig.argtypes = [vp, i32, i32, i32, dbl, vp, vp, vp, vp, vp, vp]
        L.ht_test_eig_method.argtypes = [vp, i32, i32, i32, dbl, i32, vp, vp, vp, vp, vp, vp]
        L.ht_test_orth_expand.argtypes = [vp, i64, i32, vp, i32, vp, vp]
        L.ht_test_decision_certified.argtypes = [i32, i32, i32, dbl, dbl, dbl, dbl, dbl]
        L.ht_test_decision_certified.restype = i32
        for name in ("ht_test_sumsq", "ht_test_gram", "ht_test_resid_gram", "ht_test_resid_gram_f32",
                     "ht_test_resid_gram_proj", "ht_test_ttm_contract_split",
                     "ht_test_ttm_contract", "ht_test_ttm_contract_f32", "ht_test_ttm_expand", "ht_test_eig",
                     "ht_test_eig_method", "ht_test_orth_expand"):
            getattr(L, name).restype = ctypes.c_int
        L._ht_testing_ready = True
    return L


def _dt(t) -> int:
    import torch
    return HT_F32 if t.dtype == torch.float32 else HT_F64


def ht_test_sumsq(x, stream=None):
    import torch
    out = torch.empty(1, dtype=torch.float64, device=x.device)
    sc = torch.empty(1024, dtype=torch.float64, device=x.device)
    _check(_tlib().ht_test_sumsq(_ptr(x), _dt(x), x.numel(), _ptr(out), _ptr(sc), _stream(stream)), "ht_test_sumsq")
    return out


def ht_test_gram(x, P: int, m: int, S: int, stream=None):
    import torch
    L = _tlib()
    sc = torch.empty(max(1, L.ht_test_gram_scratch_doubles(P, m, S)), dtype=torch.float64, device=x.device)
    G = torch.empty((m, m), dtype=torch.float64, device=x.device)
    _check(L.ht_test_gram(_ptr(x), _dt(x), P, m, S, _ptr(G), _ptr(sc), _stream(stream)), "ht_test_gram")
    return G


def ht_test_resid_gram(x, P: int, m: int, S: int, U, stream=None):
    import torch
    L = _tlib()
    sc = torch.empty(max(1, L.ht_test_gram_scratch_doubles(P, m, S)), dtype=torch.float64, device=x.device)
    G = torch.empty((m, m), dtype=torch.float64, device=x.device)
    Ucm = U.t().contiguous()
    _check(L.ht_test_resid_gram(_ptr(x), _dt(x), P, m, S, _ptr(Ucm), U.shape[1], _ptr(G), _ptr(sc),
                                _stream(stream)), "ht_test_resid_gram")
    return G


def ht_test_resid_gram_f32(x, P: int, m: int, S: int, U, stream=None):
    import torch
    L = _tlib()
    sc = torch.empty(max(1, L.ht_test_gram_scratch_doubles(P, m, S)), dtype=torch.float64, device=x.device)
    G = torch.empty((m, m), dtype=torch.float64, device=x.device)
    Ucm = U.t().contiguous()
    _check(L.ht_test_resid_gram_f32(_ptr(x), _dt(x), P, m, S, _ptr(Ucm), U.shape[1], _ptr(G), _ptr(sc),
                                    _stream(stream)), "ht_test_resid_gram_f32")
    return G


def ht_test_resid_gram_proj(x, P: int, m: int, S: int, U, stream=None):
    import torch
    L = _tlib()
    sc = torch.empty(max(1, L.ht_test_gram_scratch_doubles(P, m, S)), dtype=torch.float64, device=x.device)
    G = torch.empty((m, m), dtype=torch.float64, device=x.device)
    Ucm = U.t().contiguous()
    _check(L.ht_test_resid_gram_proj(_ptr(x), _dt(x), P, m, S, _ptr(Ucm), U.shape[1], _ptr(G), _ptr(sc),
                                     _stream(stream)), "ht_test_resid_gram_proj")
    return G


def ht_test_ttm_contract_f32(x, P: int, m: int, S: int, U, stream=None):
    """Returns (Z float32 [P][R][S], ||X||^2, ||X - U U^T X||^2)."""
    import torch
    L = _tlib()
    R = U.shape[1]
    Ucm = U.t().contiguous()
    Z = torch.empty((P, R, S), dtype=torch.float32, device=x.device)
    sc = torch.empty(2 * L.ht_test_ttm_partials_doubles(), dtype=torch.float64, device=x.device)
    out = torch.zeros(2, dtype=torch.float64, device=x.device)
    _check(L.ht_test_ttm_contract_f32(_ptr(x), _dt(x), P, m, S, _ptr(Ucm), R, _ptr(Z), _ptr(out), _ptr(out) + 8,
                                      _ptr(sc), _stream(stream)), "ht_test_ttm_contract_f32")
    torch.cuda.synchronize()
    return Z, float(out[0].item()), float(out[1].item())


def ht_test_ttm_contract_split(x, P: int, m: int, S: int, U, scratch_doubles: int, stream=None):
    """Returns (Z float64 [P][R][S], ||X||^2, ||Z||^2) of the direct contraction with
    scratch_doubles of lent scratch (row chunks when it has few column blocks)."""
    import torch
    R = U.shape[1]
    Ucm = U.t().contiguous()
    Z = torch.empty((P, R, S), dtype=torch.float64, device=x.device)
    sc = torch.empty(max(1, scratch_doubles), dtype=torch.float64, device=x.device)
    sq = torch.zeros(2 + 2048, dtype=torch.float64, device=x.device)
    _check(_tlib().ht_test_ttm_contract_split(_ptr(x), _dt(x), P, m, S, _ptr(Ucm), R, _ptr(Z), _ptr(sc),
                                              scratch_doubles, _ptr(sq), _stream(stream)), "ht_test_ttm_contract_split")
    torch.cuda.synchronize()
    return Z, float(sq[0].item()), float(sq[1].item())


def ht_test_ttm_contract(x, P: int, m: int, S: int, U, stream=None):
    import torch
    R = U.shape[1]
    Ucm = U.t().contiguous()  # column-major m x R
    Z = torch.empty((P, R, S), dtype=torch.float64, device=x.device)
    _check(_tlib().ht_test_ttm_contract(_ptr(x), _dt(x), P, m, S, _ptr(Ucm), R, _ptr(Z), _stream(stream)),
           "ht_test_ttm_contract")
    return Z


def ht_test_ttm_expand(Z, U, M=None, out_dtype=None, stream=None):
    import torch
    P, R, S = Z.shape
    m = U.shape[0]
    Ucm = U.t().contiguous()
    od = out_dtype or torch.float64
    out = torch.empty((P, m, S), dtype=od, device=Z.device)
    _check(_tlib().ht_test_ttm_expand(_ptr(Z), P, R, S, _ptr(Ucm), m, _ptr(M), _dt(M) if M is not None else HT_F64,
                                      _ptr(out), HT_F32 if od == torch.float32 else HT_F64, _stream(stream)),
           "ht_test_ttm_expand")
    return out


EIG_AUTO, EIG_HOUSEHOLDER, EIG_LANCZOS = 0, 1, 2


def ht_test_eig(G, rmin: int, rmax: int, thr: float, stream=None, method: int = EIG_AUTO, info: bool = False):
    """Eigen-decomposition with the truncation rule (ht_test_eig_method).  Returns
    (evals, vecs, rank, tail), plus the Lanczos step count when info is set."""
    import torch
    k = G.shape[0]
    L = _tlib()
    sc = torch.empty(L.ht_test_eig_scratch_doubles(k, max(rmax, 1)), dtype=torch.float64, device=G.device)
    ev = torch.full((k,), float('nan'), dtype=torch.float64, device=G.device)
    vecs = torch.zeros((max(rmax, 1), k), dtype=torch.float64, device=G.device)
    rank = torch.zeros(1, dtype=torch.int32, device=G.device)
    tail = torch.zeros(1, dtype=torch.float64, device=G.device)
    _check(L.ht_test_eig_method(_ptr(G.contiguous()), k, rmin, rmax, float(thr), int(method), _ptr(ev), _ptr(vecs),
                                _ptr(rank), _ptr(tail), _ptr(sc), _stream(stream)), "ht_test_eig_method")
    torch.cuda.synchronize()
    r = int(rank.item())
    out = (ev, vecs[:max(r, 0)].t(), r, float(tail.item()))
    if info:
        return out + (int(sc[-56].item()),)
    return out


def ht_test_orth_expand(U_old, V, stream=None):
    import torch
    alpha = V.shape[0]
    r_old = 0 if U_old is None else U_old.shape[1]
    rR = V.shape[1]
    core = torch.zeros((r_old + rR, alpha), dtype=torch.float64, device=V.device)
    if U_old is not None:
        core[:r_old] = U_old.t()
    Vcm = V.t().contiguous()
    _check(_tlib().ht_test_orth_expand(_ptr(core), alpha, r_old, _ptr(Vcm), rR, _ptr(core), _stream(stream)),
           "ht_test_orth_expand")
    return core.t()


def ht_test_decision_certified(r: int, rmin: int, room: int, t_r: float, lam_r: float, thr: float, dR: float,
                               gerr: float) -> bool:
    """Host-only certificate of one mixed-form rank decision (ht_rise_testing.h)."""
    return bool(_tlib().ht_test_decision_certified(r, rmin, room, t_r, lam_r, thr, dR, gerr))


# ---- optional per-kernel timing (include/ht_rise_profile.h) --------------------------------------
class ht_kernel_stats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


def _plib():
    L = lib()
    if not getattr(L, "_ht_profile_ready", False):
        L.ht_profile_enable.argtypes = [ctypes.c_int32]
        L.ht_profile_enable.restype = ctypes.c_int
        L.ht_profile_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ht_kernel_stats)]
        L.ht_profile_read.restype = ctypes.c_int
        L.ht_profile_kind_count.restype = ctypes.c_int32
        L.ht_profile_kind_name.argtypes = [ctypes.c_int32]
        L.ht_profile_kind_name.restype = ctypes.c_char_p
        L._ht_profile_ready = True
    return L


def ht_profile_enable(on: bool) -> None:
    _check(_plib().ht_profile_enable(1 if on else 0), "ht_profile_enable")


def ht_profile_read_all() -> dict:
    L = _plib()
    out = {}
    for k in range(L.ht_profile_kind_count()):
        st = ht_kernel_stats()
        _check(L.ht_profile_read(k, ctypes.byref(st)), "ht_profile_read")
        out[L.ht_profile_kind_name(k).decode()] = {"launches": int(st.launches), "ms": float(st.ms),
                                                   "flops": float(st.flops), "bytes": float(st.bytes)}
    return out
