"""ctypes wrappers around the plain-C FP64 oracle (sc_oracle.c).

TEST INFRASTRUCTURE: see the package docstring.  The shared object is built
with gcc next to this file by `build()` (and on first use if it is missing).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.c")
# SC_ORACLE_LIB points the wrappers at another build of the same source (the
# sanitizer build of sanitize_check.sh)
_SO = os.environ.get("SC_ORACLE_LIB") or os.path.join(_HERE, "libsc_oracle.so")
_lib = None


def lib_path() -> str:
    return _SO


def build() -> str:
    """Compile sc_oracle.c with gcc into oracle/libsc_oracle.so."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread", _SRC,
                           "-lm", "-o", tmp])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = C.CDLL(_SO)
    P = C.c_void_p
    lib.orc_omp.argtypes = [P, C.c_int, C.c_int, P, C.c_int64, C.c_int, C.c_double, C.c_int,
                            P, C.c_int, P, P, P, P, P, P, P, P, P, C.c_int]
    lib.orc_omp.restype = C.c_int
    lib.orc_sh_basis.argtypes = [P, C.c_int64, C.c_int, P]
    lib.orc_sh_basis.restype = None
    lib.orc_radiance.argtypes = [P, C.c_int, C.c_int, P, P, P, C.c_int64, C.c_int, P, C.c_int64,
                                 C.c_int, P]
    lib.orc_radiance.restype = C.c_int
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _threads(n):
    if n is not None:
        return int(n)
    return max(1, len(os.sched_getaffinity(0)))


def omp(D, X, k, eps=0.0, relative=False, nthreads=None, with_margin=False, cand=None, with_path=False):
    """Orthogonal Matching Pursuit of every row of X over the atoms (rows) of D.

    D: (K, d) float32 atom-major; X: (N, d) float32.  Returns dict with
    idx (N,k) int32 in selection order (-1 padded), coef (N,k) float64,
    count (N,) int32, resid (N,) float64 = ||x - D_I gamma||_2 and, if asked,
    margin (N,) = min over steps of (|c|_(1) - |c|_(2)) / ||r|| and gap (N,)
    = min over steps of |c|_(1) - |c|_(2), and rpath
    (N, k+1): the residual norm before each selection and at the end, with
    mpath and gpath (N, k): each step's relative margin and absolute gap
    (NaN past the end).
    cand: optional (N, n_cand) int32 -- restrict each signal's pursuit to
    its listed atoms."""
    lib = _load()
    D = np.ascontiguousarray(D, np.float32)
    X = np.ascontiguousarray(X, np.float32)
    K, d = D.shape
    N = X.shape[0]
    assert X.shape[1] == d
    idx = np.empty((N, k), np.int32)
    coef = np.empty((N, k), np.float64)
    count = np.empty(N, np.int32)
    resid = np.empty(N, np.float64)
    margin = np.empty(N, np.float64) if with_margin else None
    gap = np.empty(N, np.float64) if with_margin else None
    rpath = np.empty((N, k + 1), np.float64) if with_path else None
    mpath = np.empty((N, k), np.float64) if with_path else None
    gpath = np.empty((N, k), np.float64) if with_path else None
    n_cand = 0
    if cand is not None:
        cand = np.ascontiguousarray(cand, np.int32)
        assert cand.shape[0] == N
        n_cand = cand.shape[1]
    rc = lib.orc_omp(_p(D), d, K, _p(X), N, int(k), float(eps), int(bool(relative)), _p(cand), n_cand,
                     _p(idx), _p(coef), _p(count), _p(resid), _p(margin), _p(rpath), _p(gap), _p(mpath), _p(gpath),
                     _threads(nthreads))
    if rc != 0:
        raise ValueError("orc_omp: invalid arguments")
    out = dict(idx=idx, coef=coef, count=count, resid=resid)
    if with_margin:
        out["margin"] = margin
        out["gap"] = gap
    if with_path:
        out["rpath"] = rpath
        out["mpath"] = mpath
        out["gpath"] = gpath
    return out


def omp_restricted(D, X, cand, k, eps=0.0, relative=False, nthreads=None):
    """OMP restricted to per-signal candidate atoms (the proposer's list)."""
    return omp(D, X, k, eps, relative, nthreads, cand=cand)


def sh_basis(dirs, L=3):
    """Real SH basis of degree 1..L at the given directions: (M, (L+1)^2-1)
    float64, ordered band by band with m = -l..l."""
    lib = _load()
    dd = np.ascontiguousarray(dirs, np.float64)
    M = dd.shape[0]
    nb = (L + 1) ** 2 - 1
    Y = np.empty((M, nb), np.float64)
    lib.orc_sh_basis(_p(dd), M, int(L), _p(Y))
    return Y


def radiance(D, idx, coef, count, dirs, shared_dirs):
    """View-dependent radiance of sparse codes (dense reconstruction, then the
    SH sum).  shared_dirs=False: dirs (N,3) -> (N,3); True: dirs (M,3) ->
    (N,M,3).  float64."""
    lib = _load()
    D = np.ascontiguousarray(D, np.float32)
    idx = np.ascontiguousarray(idx, np.int32)
    coef = np.ascontiguousarray(coef, np.float32)
    count = np.ascontiguousarray(count, np.int32)
    dirs = np.ascontiguousarray(dirs, np.float32)
    K, d = D.shape
    N, kcap = idx.shape
    M = dirs.shape[0]
    out = np.empty((N, M, 3) if shared_dirs else (N, 3), np.float64)
    rc = lib.orc_radiance(_p(D), d, K, _p(idx), _p(coef), _p(count), N, kcap, _p(dirs), M,
                          int(bool(shared_dirs)), _p(out))
    if rc != 0:
        raise ValueError("orc_radiance: invalid arguments")
    return out


def gram(D):
    """G = D^T D of the paper's d x K dictionary (atoms are rows of D here)."""
    Dd = np.asarray(D, np.float64)
    return Dd @ Dd.T
