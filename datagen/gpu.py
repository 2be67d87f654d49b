"""Device-side generation of datagen's streams.

``field_batch_into(spec, k, out)`` writes batch k of a field straight into a float32
CUDA tensor (``libhtgen.so``); the values equal ``datagen.exact_field_batch(spec, k)``
bit for bit.  ``model_batches(spec)`` yields the batches of an exact-rank model stream
built on the device from the same frames and root slices as
``datagen.ht_model_stream``, with the noise drawn on the device: the same model, not
the same bits (a test that compares with the oracle copies these batches to the host).
"""

from __future__ import annotations

import ctypes
import os

from . import FieldSpec, HTModelSpec, exact_field_factors, ht_model_parts

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhtgen.so")
_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhtgen.so is not built; run `python -m datagen.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.htgen_field.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        L.htgen_field.restype = ctypes.c_int
        _lib = L
    return _lib


def field_batch_into(spec: FieldSpec, k: int, out, stream=None) -> None:
    """Generates batch k of the field into out (float32 CUDA tensor of spec's batch shape)."""
    import torch
    ff = exact_field_factors(spec, k)
    if tuple(out.shape) != ff.shape or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of shape %r" % (ff.shape,))
    A = torch.from_numpy(ff.A).to(out.device).contiguous()
    B = torch.from_numpy(ff.B).to(out.device).contiguous()
    T, N, P1 = ff.A.shape
    s = int(torch.cuda.current_stream(out.device).cuda_stream) if stream is None else int(stream)
    st = lib().htgen_field(A.data_ptr(), B.data_ptr(), T, N, P1, ff.B.shape[1], ff.key, ff.scale, out.data_ptr(), s)
    if st != 0:
        raise RuntimeError("htgen_field failed (%d)" % st)
    torch.cuda.current_stream(out.device).synchronize()


def field_batch(spec: FieldSpec, k: int, device: str = "cuda:0"):
    import torch
    out = torch.empty((spec.N,) + spec.n, dtype=torch.float32, device=device)
    field_batch_into(spec, k, out)
    return out


def checksum(t) -> int:
    """datagen.checksum of a float32 CUDA tensor (the sum of its bit patterns), on the device."""
    import torch
    return int((t.contiguous().view(torch.int32).to(torch.int64) & 0xFFFFFFFF).sum().item())


def model_batches(spec: HTModelSpec, device: str = "cuda:0"):
    """Yield the spec.n_batches float32 batches (N, *n) of the exact-rank model stream on
    the device: sum over the stream's direction sets of F_L S_n F_R^T per sample in
    FP64, plus relative noise nu * rms(signal) from a device generator seeded per batch."""
    import torch
    dev = torch.device(device)
    for k, (terms, _) in enumerate(ht_model_parts(spec)):
        y = None
        for fl, sl, fr in terms:
            a = torch.from_numpy(fl).to(dev)                               # nl x rl
            b = torch.from_numpy(sl).to(dev)                               # N x rl x rr
            c = torch.from_numpy(fr.T.copy()).to(dev)                      # rr x nr
            t = torch.matmul(torch.matmul(a, b), c)                        # N x nl x nr
            y = t if y is None else y + t
        if spec.nu > 0:
            rms = torch.sqrt(torch.mean(y * y))
            gen = torch.Generator(device=dev)
            gen.manual_seed(int(spec.batch_seed0 + k) * 1000003 + 17)
            y = y + spec.nu * rms * torch.randn(y.shape, generator=gen, dtype=torch.float64, device=dev)
        yield y.reshape((spec.N,) + tuple(spec.n)).to(torch.float32).contiguous()
