"""Device-side generation of datagen's exactly reproducible fields (``libhtgen.so``).

``field_batch_into(spec, k, out)`` writes batch k straight into a float32 CUDA
tensor; the values equal ``datagen.exact_field_batch(spec, k)`` bit for bit.
"""

from __future__ import annotations

import ctypes
import os

from . import FieldSpec, exact_field_factors

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
