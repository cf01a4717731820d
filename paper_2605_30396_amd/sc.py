"""Python binding of libsc (the C ABI declared in include/sc.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libsc.so.  PyTorch provides the device memory and the stream.
There is no fallback: if libsc.so is missing or a call fails, an exception
is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsc.so")

SC_OK = 0
SC_EINVAL = -1
SC_ENORM = -2
SC_ENONFINITE = -3
SC_EDEVICE = -4
SC_ENOMEM = -5
SC_ENODEV = -6

EPS_RELATIVE = 0x1
PREC_BF16 = 0x2
NO_FP64_REFIT = 0x4
NORMALIZE = 0x8

DIRS_PER_SIGNAL = 0
DIRS_SHARED = 1


class ScError(RuntimeError):
    def __init__(self, fn, code, lib):
        msg = lib.sc_strerror(code).decode()
        detail = lib.sc_last_error().decode() if code == SC_EDEVICE or code == SC_EINVAL else ""
        super().__init__(f"{fn} failed: {msg} ({code}) {detail}".strip())
        self.code = code


_lib = None
P = C.c_void_p
I32 = C.c_int
I64 = C.c_int64
F32 = C.c_float


def load():
    """Load libsc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                           "or python -m paper_2605_30396_amd.build")
    lib = C.CDLL(LIB_PATH)
    sig = {
        "sc_strerror": (C.c_char_p, [I32]),
        "sc_last_error": (C.c_char_p, []),
        "sc_gram_precompute": (I32, [P, I32, I32, I32, P, C.POINTER(P)]),
        "sc_dict_destroy": (I32, [P]),
        "sc_dict_dims": (I32, [P, C.POINTER(I32), C.POINTER(I32)]),
        "sc_dict_gram": (I32, [P, P, P]),
        "sc_omp_encode": (I32, [P, P, I64, I32, F32, I32, P, P, P, P, P]),
        "sc_omp_stats": (I32, [P, C.POINTER(I64), I32, P]),
        "sc_sh_eval_sparse": (I32, [P, P, P, P, I64, I32, P, I64, I32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(fn, rc):
    if rc != SC_OK:
        raise ScError(fn, rc, load())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_f32(t, name, ndim):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.dim() == ndim
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {ndim}-d float32 CUDA tensor")


def _dev_i32(t, name, ndim):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32 and t.dim() == ndim
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {ndim}-d int32 CUDA tensor")


class Dictionary:
    """Owns an sc_dict handle (device copies of D, its layouts and G)."""

    def __init__(self, handle, d, K, device):
        self._h = handle
        self.d, self.K, self.device = d, K, device

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("dictionary handle already destroyed")
        return self._h

    def gram(self, stream=None):
        """The handle's FP32 Gram matrix G = D^T D as a new (K, K) tensor."""
        out = torch.empty((self.K, self.K), dtype=torch.float32, device=self.device)
        _check("sc_dict_gram", load().sc_dict_gram(self.handle, _ptr(out), _stream(stream)))
        return out

    def destroy(self):
        if self._h is not None:
            load().sc_dict_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def gram_precompute(D, flags=0, stream=None) -> Dictionary:
    """Set up dictionary D ((K, d) float32 CUDA tensor, atom-major)."""
    _dev_f32(D, "D", 2)
    K, d = D.shape
    h = C.c_void_p()
    _check("sc_gram_precompute", load().sc_gram_precompute(_ptr(D), d, K, flags, _stream(stream), C.byref(h)))
    return Dictionary(h, d, K, D.device)


def omp_encode(h: Dictionary, X, k, eps=0.0, flags=0, out=None, stream=None):
    """Sparse-code the rows of X ((N, d) float32 CUDA).  Returns (idx, coef,
    count, resid) device tensors; `out` may supply them preallocated."""
    _dev_f32(X, "X", 2)
    N = X.shape[0]
    if out is None:
        idx = torch.empty((N, k), dtype=torch.int32, device=X.device)
        coef = torch.empty((N, k), dtype=torch.float32, device=X.device)
        count = torch.empty((N,), dtype=torch.int32, device=X.device)
        resid = torch.empty((N,), dtype=torch.float32, device=X.device)
    else:
        idx, coef, count, resid = out
    _check("sc_omp_encode", load().sc_omp_encode(h.handle, _ptr(X), N, int(k), float(eps), int(flags), _ptr(idx),
                                                 _ptr(coef), _ptr(count), _ptr(resid), _stream(stream)))
    return idx, coef, count, resid


def omp_stats(h: Dictionary, reset=False, stream=None):
    v = (C.c_int64 * 4)()
    _check("sc_omp_stats", load().sc_omp_stats(h.handle, v, int(bool(reset)), _stream(stream)))
    return dict(signals=v[0], atoms=v[1], fp64_refits=v[2], fallbacks=v[3])


def sh_eval_sparse(h: Dictionary, idx, coef, count, dirs, dir_mode=DIRS_PER_SIGNAL, out=None, stream=None):
    """Radiance from codes.  dirs (N,3) per signal or (M,3) shared; returns
    rgb (N,3) or (N,M,3)."""
    _dev_i32(idx, "idx", 2)
    _dev_f32(coef, "coef", 2)
    _dev_i32(count, "count", 1)
    _dev_f32(dirs, "dirs", 2)
    N, k = idx.shape
    M = dirs.shape[0]
    if out is None:
        shape = (N, 3) if dir_mode == DIRS_PER_SIGNAL else (N, M, 3)
        out = torch.empty(shape, dtype=torch.float32, device=idx.device)
    _check("sc_sh_eval_sparse", load().sc_sh_eval_sparse(h.handle, _ptr(idx), _ptr(coef), _ptr(count), N, k,
                                                         _ptr(dirs), M, int(dir_mode), _ptr(out), _stream(stream)))
    return out
