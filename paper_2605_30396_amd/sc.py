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

TRAIN_FP32 = 0x1
TRAIN_GRAD_ONLY = 0x2

TUNE_FP32_CORRELATION = 1
TUNE_ROW_CACHE = 2
TUNE_RESTRICTED_CAP = 3
TUNE_ROW_CACHE_BF16 = 4
CORR_VALU = 0
CORR_MFMA = 1

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


MAX_SCENES = 32
ORDER_COST = 0
ORDER_GIVEN = 1


class Scene(C.Structure):
    """sc_scene: one scene of a batched launch."""
    _fields_ = [("dict", C.c_void_p), ("X", C.c_void_p), ("N", C.c_int64), ("k", C.c_int32), ("eps", C.c_float),
                ("flags", C.c_int32), ("idx", C.c_void_p), ("coef", C.c_void_p), ("count", C.c_void_p),
                ("resid", C.c_void_p)]


class BatchTuning(C.Structure):
    """sc_batch_tuning: launch shape of the batched encoder."""
    _fields_ = [("tile", C.c_int32), ("row_cache", C.c_int32), ("wg_per_cu", C.c_int32), ("order", C.c_int32),
                ("corr", C.c_int32)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        return cls(**{n: int(d[n]) for n, _ in cls._fields_})


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
        "sc_dict_set_tuning": (I32, [P, I32, I32]),
        "sc_dict_get_tuning": (I32, [P, I32, C.POINTER(I32)]),
        "sc_sh_eval_sparse": (I32, [P, P, P, P, I64, I32, P, I64, I32, P, P]),
        "sc_proposer_num_params": (I64, [I32, I32, I32]),
        "sc_proposer_create": (I32, [I32, I32, I32, C.POINTER(P)]),
        "sc_proposer_destroy": (I32, [P]),
        "sc_proposer_dims": (I32, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), C.POINTER(I64)]),
        "sc_proposer_set_params": (I32, [P, P, P]),
        "sc_proposer_get_params": (I32, [P, P, P]),
        "sc_proposer_forward": (I32, [P, P, I64, I32, P, P, P]),
        "sc_omp_encode_learned_workspace": (C.c_size_t, [I64, I32]),
        "sc_omp_encode_learned": (I32, [P, P, P, I64, I32, F32, I32, I32, P, P, P, P, P, C.c_size_t, P]),
        "sc_omp_encode_learned_noalloc": (I32, [P, P, P, I64, I32, F32, I32, I32, P, P, P, P, P]),
        "sc_omp_encode_restricted": (I32, [P, P, I64, I32, F32, I32, P, I32, P, P, P, P, P, P, P]),
        "sc_screen_topk": (I32, [P, P, I64, I32, P, P]),
        "sc_omp_encode_rows": (I32, [P, P, P, P, I64, I32, F32, I32, P, P, P, P, P]),
        "sc_mod_workspace": (C.c_size_t, [I32, I32]),
        "sc_mod_update": (I32, [P, I64, I32, I32, P, P, P, I32, P, P, C.POINTER(I32), P, C.c_size_t, P]),
        "sc_csc_workspace": (C.c_size_t, [I64]),
        "sc_omp_encode_csc_workspace": (C.c_size_t, [I64, I32]),
        "sc_omp_encode_csc": (I32, [P, P, I64, I32, F32, I32, P, P, P, I64, C.POINTER(I64), P, P, C.c_size_t, P]),
        "sc_csc_colptr": (I32, [P, I64, P, P, C.c_size_t, P]),
        "sc_csc_fill": (I32, [P, P, P, I64, I32, P, P, P, P]),
        "sc_sh_eval_csc": (I32, [P, P, P, P, I64, P, I64, I32, P, P]),
        "sc_gaussian_rgb_csc": (I32, [P, P, P, P, I64, P, P, C.POINTER(F32), P, P]),
        "sc_omp_encode_batched_workspace": (C.c_size_t, []),
        "sc_omp_encode_batched": (I32, [C.POINTER(Scene), I32, C.POINTER(BatchTuning), P, C.c_size_t, P]),
        "sc_batch_autotune": (I32, [C.POINTER(Scene), I32, I64, P, C.c_size_t, C.POINTER(BatchTuning),
                                    C.POINTER(F32), P]),
        "sc_proposer_train_workspace": (C.c_size_t, [P, I64]),
        "sc_proposer_train_step": (I32, [P, P, P, I64, P, P, I32, F32, F32, F32, F32, F32, I32, P, P, P,
                                         C.c_size_t, P]),
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


def _addr(t):
    return None if t is None else int(t.data_ptr())


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

    def set_tuning(self, key, value):
        _check("sc_dict_set_tuning", load().sc_dict_set_tuning(self.handle, int(key), int(value)))

    def get_tuning(self, key):
        v = C.c_int()
        _check("sc_dict_get_tuning", load().sc_dict_get_tuning(self.handle, int(key), C.byref(v)))
        return v.value

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


# ----------------------------------------------------------------------------
# learned support proposer
# ----------------------------------------------------------------------------

PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def pack_params(params: dict) -> torch.Tensor:
    """Flatten a {W1, b1, W2, b2, W3, b3} dict (arrays or tensors) into the
    library's FP32 parameter vector (that order, row-major)."""
    parts = [torch.as_tensor(params[n], dtype=torch.float32).reshape(-1) for n in PARAM_ORDER]
    return torch.cat(parts)


def unpack_params(vec, d, H, K) -> dict:
    shapes = {"W1": (H, d), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (K, H), "b3": (K,)}
    out, o = {}, 0
    for n in PARAM_ORDER:
        sz = int(torch.tensor(shapes[n]).prod())
        out[n] = vec[o:o + sz].reshape(shapes[n])
        o += sz
    return out


class Proposer:
    """Owns an sc_proposer handle (FP32 master weights, BF16 copies, Adam state)."""

    def __init__(self, handle, d, H, K, device):
        self._h = handle
        self.d, self.H, self.K, self.device = d, H, K, device
        self.nparams = int(load().sc_proposer_num_params(d, H, K))

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("proposer handle already destroyed")
        return self._h

    def set_params(self, params, stream=None):
        vec = params if isinstance(params, torch.Tensor) else pack_params(params)
        vec = vec.to(device=self.device, dtype=torch.float32).contiguous()
        if vec.numel() != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {vec.numel()}")
        _check("sc_proposer_set_params", load().sc_proposer_set_params(self.handle, _ptr(vec), _stream(stream)))
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()

    def get_params(self, stream=None):
        out = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _check("sc_proposer_get_params", load().sc_proposer_get_params(self.handle, _ptr(out), _stream(stream)))
        return out

    def destroy(self):
        if self._h is not None:
            load().sc_proposer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def proposer_create(d, H, K, device="cuda:0") -> Proposer:
    h = C.c_void_p()
    _check("sc_proposer_create", load().sc_proposer_create(d, H, K, C.byref(h)))
    return Proposer(h, d, H, K, torch.device(device))


def proposer_forward(p: Proposer, X, n_cand=24, want_logits=False, cand=None, stream=None):
    """Candidate atoms (N, n_cand) int32 sorted by index (row of -1 = none) and,
    if asked, the FP32 logits (N, K).  `cand` may be a preallocated output."""
    _dev_f32(X, "X", 2)
    N = X.shape[0]
    if cand is None:
        cand = torch.empty((N, n_cand), dtype=torch.int32, device=X.device)
    else:
        _dev_i32(cand, "cand", 2)
        if tuple(cand.shape) != (N, n_cand):
            raise ValueError(f"cand must have shape {(N, n_cand)}")
    logits = torch.empty((N, p.K), dtype=torch.float32, device=X.device) if want_logits else None
    _check("sc_proposer_forward", load().sc_proposer_forward(p.handle, _ptr(X), N, int(n_cand), _ptr(cand),
                                                             _ptr(logits), _stream(stream)))
    return cand, logits


def screen_topk(h: Dictionary, X, n_cand=24, cand=None, stream=None):
    """The n_cand atoms of largest |<a_j, x>| per signal (N, n_cand) int32,
    sorted by atom index (row of -1 = not finite)."""
    _dev_f32(X, "X", 2)
    N = X.shape[0]
    if cand is None:
        cand = torch.empty((N, n_cand), dtype=torch.int32, device=X.device)
    else:
        _dev_i32(cand, "cand", 2)
        if tuple(cand.shape) != (N, n_cand):
            raise ValueError(f"cand must have shape {(N, n_cand)}")
    _check("sc_screen_topk", load().sc_screen_topk(h.handle, _ptr(X), N, int(n_cand), _ptr(cand), _stream(stream)))
    return cand


def learned_workspace_bytes(N, n_cand=24):
    return int(load().sc_omp_encode_learned_workspace(int(N), int(n_cand)))


def omp_encode_learned(h: Dictionary, p: Proposer, X, k, eps, n_cand=24, flags=0, out=None, workspace=None,
                       stream=None):
    """Proposer-guided OMP with full-OMP fallback.  Returns (idx, coef, count, resid)."""
    _dev_f32(X, "X", 2)
    N = X.shape[0]
    if out is None:
        idx = torch.empty((N, k), dtype=torch.int32, device=X.device)
        coef = torch.empty((N, k), dtype=torch.float32, device=X.device)
        count = torch.empty((N,), dtype=torch.int32, device=X.device)
        resid = torch.empty((N,), dtype=torch.float32, device=X.device)
    else:
        idx, coef, count, resid = out
    need = learned_workspace_bytes(N, n_cand)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    _check("sc_omp_encode_learned", load().sc_omp_encode_learned(
        h.handle, p.handle, _ptr(X), N, int(k), float(eps), int(flags), int(n_cand), _ptr(idx), _ptr(coef),
        _ptr(count), _ptr(resid), _ptr(workspace), workspace.numel(), _stream(stream)))
    return idx, coef, count, resid


# device scratch of sc_omp_encode_learned_noalloc (SC_STATIC_SCRATCH_BYTES in sc.h)
STATIC_SCRATCH_BYTES = 32 << 20


def noalloc_max_signals(n_cand=24):
    """Largest N that sc_omp_encode_learned_noalloc accepts with n_cand candidates."""
    lo, hi = 0, STATIC_SCRATCH_BYTES
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if learned_workspace_bytes(mid, n_cand) <= STATIC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid - 1
    return lo


def omp_encode_learned_noalloc(h: Dictionary, p: Proposer, X, k, eps, n_cand=24, flags=0, out=None, stream=None):
    """sc_omp_encode_learned with the library's static device scratch in place
    of a workspace (no allocation inside the call; the outputs are allocated
    here unless `out` is given).  Returns (idx, coef, count, resid)."""
    _dev_f32(X, "X", 2)
    N = X.shape[0]
    if out is None:
        out = (torch.empty((N, k), dtype=torch.int32, device=X.device),
               torch.empty((N, k), dtype=torch.float32, device=X.device),
               torch.empty((N,), dtype=torch.int32, device=X.device),
               torch.empty((N,), dtype=torch.float32, device=X.device))
    idx, coef, count, resid = out
    _check("sc_omp_encode_learned_noalloc", load().sc_omp_encode_learned_noalloc(
        h.handle, p.handle, _ptr(X), N, int(k), float(eps), int(flags), int(n_cand), _ptr(idx), _ptr(coef),
        _ptr(count), _ptr(resid), _stream(stream)))
    return idx, coef, count, resid


def train_workspace_bytes(p: Proposer, B):
    return int(load().sc_proposer_train_workspace(p.handle, int(B)))


def proposer_train_step(p: Proposer, X, sup_idx, sup_count, B, rows=None, lr=1e-3, beta1=0.9, beta2=0.999,
                        adam_eps=1e-8, pos_weight=1.0, flags=0, loss=None, grads=None, workspace=None, stream=None):
    """One training step on the batch X[rows] (or X[:B]).  `loss` (1-element
    float32 tensor) and `grads` (nparams) receive the batch loss and gradient
    if given."""
    _dev_f32(X, "X", 2)
    _dev_i32(sup_idx, "sup_idx", 2)
    _dev_i32(sup_count, "sup_count", 1)
    if rows is not None:
        _dev_i32(rows, "rows", 1)
    if workspace is None:
        workspace = torch.empty(train_workspace_bytes(p, B), dtype=torch.uint8, device=X.device)
    _check("sc_proposer_train_step", load().sc_proposer_train_step(
        p.handle, _ptr(X), _ptr(rows), int(B), _ptr(sup_idx), _ptr(sup_count), sup_idx.shape[1], float(lr),
        float(beta1), float(beta2), float(adam_eps), float(pos_weight), int(flags), _ptr(loss), _ptr(grads),
        _ptr(workspace), workspace.numel(), _stream(stream)))


def omp_encode_restricted(h: Dictionary, X, k, eps, cand, flags=0, out=None, miss_rows=None, miss_count=None,
                          stream=None):
    """Restricted OMP over candidate lists; returns (codes..., miss_rows, miss_count)."""
    _dev_f32(X, "X", 2)
    _dev_i32(cand, "cand", 2)
    N = X.shape[0]
    if out is None:
        out = (torch.empty((N, k), dtype=torch.int32, device=X.device),
               torch.empty((N, k), dtype=torch.float32, device=X.device),
               torch.empty((N,), dtype=torch.int32, device=X.device),
               torch.empty((N,), dtype=torch.float32, device=X.device))
    idx, coef, count, resid = out
    if miss_rows is None:
        miss_rows = torch.empty((max(N, 1),), dtype=torch.int32, device=X.device)
    if miss_count is None:
        miss_count = torch.zeros((1,), dtype=torch.int32, device=X.device)
    _check("sc_omp_encode_restricted", load().sc_omp_encode_restricted(
        h.handle, _ptr(X), N, int(k), float(eps), int(flags), _ptr(cand), cand.shape[1], _ptr(idx), _ptr(coef),
        _ptr(count), _ptr(resid), _ptr(miss_rows), _ptr(miss_count), _stream(stream)))
    return idx, coef, count, resid, miss_rows, miss_count


def omp_encode_rows(h: Dictionary, X, rows, nrows, max_rows, k, eps, out, flags=0, stream=None):
    """Plain FP32 encoder on X[rows[:*nrows]] (nrows: 1-element device int32)."""
    idx, coef, count, resid = out
    _check("sc_omp_encode_rows", load().sc_omp_encode_rows(
        h.handle, _ptr(X), _ptr(rows), _ptr(nrows), int(max_rows), int(k), float(eps), int(flags), _ptr(idx),
        _ptr(coef), _ptr(count), _ptr(resid), _stream(stream)))
    return out


# ----------------------------------------------------------------------------
# many scenes in one launch
# ----------------------------------------------------------------------------

def _scene_array(scenes):
    """scenes: list of dicts {dict: Dictionary, X, k, eps, flags=0, out=(idx, coef, count, resid)}
    (outputs allocated when absent).  Returns the ctypes array and the list
    of output tuples."""
    if not 1 <= len(scenes) <= MAX_SCENES:
        raise ValueError(f"1..{MAX_SCENES} scenes")
    arr = (Scene * len(scenes))()
    outs = []
    for q, sc_ in enumerate(scenes):
        X = sc_["X"]
        _dev_f32(X, "X", 2)
        N, k = X.shape[0], int(sc_["k"])
        out = sc_.get("out")
        if out is None:
            out = (torch.empty((N, k), dtype=torch.int32, device=X.device),
                   torch.empty((N, k), dtype=torch.float32, device=X.device),
                   torch.empty((N,), dtype=torch.int32, device=X.device),
                   torch.empty((N,), dtype=torch.float32, device=X.device))
        idx, coef, count, resid = out
        h = sc_["dict"].handle
        arr[q] = Scene(h.value if isinstance(h, C.c_void_p) else h, _addr(X), N, k, float(sc_.get("eps", 0.0)),
                       int(sc_.get("flags", 0)), _addr(idx), _addr(coef), _addr(count), _addr(resid))
        outs.append(out)
    return arr, outs


def batched_workspace_bytes():
    return int(load().sc_omp_encode_batched_workspace())


def omp_encode_batched(scenes, tuning=None, workspace=None, stream=None):
    """Encode several scenes (each with its own dictionary, k and eps) in one
    persistent launch.  tuning: BatchTuning, dict or None.  Returns the list
    of (idx, coef, count, resid) per scene."""
    arr, outs = _scene_array(scenes)
    dev = scenes[0]["X"].device
    if workspace is None:
        workspace = torch.empty(batched_workspace_bytes(), dtype=torch.uint8, device=dev)
    if isinstance(tuning, dict):
        tuning = BatchTuning.from_dict(tuning)
    tp = C.byref(tuning) if tuning is not None else None
    _check("sc_omp_encode_batched", load().sc_omp_encode_batched(arr, len(scenes), tp, _ptr(workspace),
                                                                 workspace.numel(), _stream(stream)))
    return outs


def batch_autotune(scenes, sample=65536, workspace=None, stream=None):
    """The library's autotuner for omp_encode_batched on the first `sample`
    signals of each scene.  Returns (BatchTuning, best time in ms)."""
    arr, _ = _scene_array(scenes)
    dev = scenes[0]["X"].device
    if workspace is None:
        workspace = torch.empty(batched_workspace_bytes(), dtype=torch.uint8, device=dev)
    best = BatchTuning()
    ms = C.c_float(0.0)
    _check("sc_batch_autotune", load().sc_batch_autotune(arr, len(scenes), int(sample), _ptr(workspace),
                                                         workspace.numel(), C.byref(best), C.byref(ms),
                                                         _stream(stream)))
    return best, float(ms.value)


# ----------------------------------------------------------------------------
# CSC storage of the codes
# ----------------------------------------------------------------------------

def pack_csc(idx, coef, count, stream=None):
    """Codes (N x k padded) -> (colptr int64[N+1], rows int32[nnz], vals
    float32[nnz]) on the device.  Synchronises once to read nnz."""
    _dev_i32(idx, "idx", 2)
    _dev_f32(coef, "coef", 2)
    _dev_i32(count, "count", 1)
    N, k = idx.shape
    lib = load()
    colptr = torch.empty((N + 1,), dtype=torch.int64, device=idx.device)
    ws = torch.empty(max(int(lib.sc_csc_workspace(N)), 1), dtype=torch.uint8, device=idx.device)
    _check("sc_csc_colptr", lib.sc_csc_colptr(_ptr(count), N, _ptr(colptr), _ptr(ws), ws.numel(), _stream(stream)))
    nnz = int(colptr[N].item())
    rows = torch.empty((max(nnz, 1),), dtype=torch.int32, device=idx.device)
    vals = torch.empty((max(nnz, 1),), dtype=torch.float32, device=idx.device)
    _check("sc_csc_fill", lib.sc_csc_fill(_ptr(idx), _ptr(coef), _ptr(count), N, k, _ptr(colptr), _ptr(rows),
                                          _ptr(vals), _stream(stream)))
    return colptr, rows[:nnz], vals[:nnz]


def omp_encode_csc(h: Dictionary, X, k, eps=0.0, flags=0, cap=None, stream=None):
    """Encode straight to CSC: returns (colptr int64[N+1], rows int32[nnz],
    vals float32[nnz], resid float32[N])."""
    _dev_f32(X, "X", 2)
    N = X.shape[0]
    lib = load()
    ws = torch.empty(max(int(lib.sc_omp_encode_csc_workspace(N, k)), 1), dtype=torch.uint8, device=X.device)
    colptr = torch.empty((N + 1,), dtype=torch.int64, device=X.device)
    resid = torch.empty((max(N, 1),), dtype=torch.float32, device=X.device)
    cap = N * k if cap is None else int(cap)
    rows = torch.empty((max(cap, 1),), dtype=torch.int32, device=X.device)
    vals = torch.empty((max(cap, 1),), dtype=torch.float32, device=X.device)
    nnz = C.c_int64(0)
    _check("sc_omp_encode_csc", lib.sc_omp_encode_csc(h.handle, _ptr(X), N, int(k), float(eps), int(flags),
                                                      _ptr(colptr), _ptr(rows), _ptr(vals), cap, C.byref(nnz),
                                                      _ptr(resid), _ptr(ws), ws.numel(), _stream(stream)))
    n = int(nnz.value)
    return colptr, rows[:n], vals[:n], resid[:N]


def sh_eval_csc(h: Dictionary, colptr, rows, vals, dirs, dir_mode=DIRS_PER_SIGNAL, out=None, stream=None):
    N = colptr.shape[0] - 1
    M = dirs.shape[0]
    if out is None:
        shape = (N, 3) if dir_mode == DIRS_PER_SIGNAL else (N, M, 3)
        out = torch.empty(shape, dtype=torch.float32, device=dirs.device)
    _check("sc_sh_eval_csc", load().sc_sh_eval_csc(h.handle, _ptr(colptr), _ptr(rows), _ptr(vals), N, _ptr(dirs), M,
                                                   int(dir_mode), _ptr(out), _stream(stream)))
    return out


def gaussian_rgb_csc(h: Dictionary, colptr, rows, vals, pos, dc, cam, out=None, stream=None):
    """Per-Gaussian colour max(0, C0 dc + SH_rest(view dir) + 0.5) from CSC codes."""
    N = colptr.shape[0] - 1
    _dev_f32(pos, "pos", 2)
    _dev_f32(dc, "dc", 2)
    if out is None:
        out = torch.empty((N, 3), dtype=torch.float32, device=pos.device)
    c = (C.c_float * 3)(*[float(v) for v in cam])
    _check("sc_gaussian_rgb_csc", load().sc_gaussian_rgb_csc(h.handle, _ptr(colptr), _ptr(rows), _ptr(vals), N,
                                                             _ptr(pos), _ptr(dc), c, _ptr(out), _stream(stream)))
    return out


# ----------------------------------------------------------------------------
# dictionary learning
# ----------------------------------------------------------------------------

def mod_update(X, idx, coef, count, resid, K, out=None, workspace=None, stream=None):
    """One dictionary update from fixed codes; returns ((K, d) float32 CUDA
    tensor of unit atoms, number of atoms replaced)."""
    _dev_f32(X, "X", 2)
    _dev_i32(idx, "idx", 2)
    _dev_f32(coef, "coef", 2)
    _dev_i32(count, "count", 1)
    _dev_f32(resid, "resid", 1)
    N, d = X.shape
    lib = load()
    if out is None:
        out = torch.empty((K, d), dtype=torch.float32, device=X.device)
    if workspace is None:
        workspace = torch.empty(max(int(lib.sc_mod_workspace(d, K)), 1), dtype=torch.uint8, device=X.device)
    nrep = C.c_int32(0)
    _check("sc_mod_update", lib.sc_mod_update(_ptr(X), N, d, int(K), _ptr(idx), _ptr(coef), _ptr(count),
                                              idx.shape[1], _ptr(resid), _ptr(out), C.byref(nrep), _ptr(workspace),
                                              workspace.numel(), _stream(stream)))
    return out, int(nrep.value)
