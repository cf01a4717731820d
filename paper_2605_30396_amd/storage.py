"""Storage accounting of compressed SH coefficients (Sec. 2.2, Sec. 3).

Uncompressed, a Gaussian's view-dependent SH coefficients are d = 45 FP32
values (the DC term is not compressed).  Compressed, they are one CSC
column -- each non-zero as an FP32 value plus an atom index -- and one
column pointer, and the scene shares one dictionary of K atoms.  The
compression ratio is the first size over the second.  Index and pointer
widths are parameters (4 bytes each by default: int32 indices, int32
column offsets within a scene).
"""
from __future__ import annotations


def dense_bytes(N, d=45, value_bytes=4):
    return int(N) * int(d) * value_bytes


def csc_bytes(N, nnz, value_bytes=4, index_bytes=4, ptr_bytes=4):
    return int(nnz) * (value_bytes + index_bytes) + (int(N) + 1) * ptr_bytes


def dictionary_bytes(K, d=45, value_bytes=4):
    return int(K) * int(d) * value_bytes


def compression_ratio(N, nnz, K, d=45, value_bytes=4, index_bytes=4, ptr_bytes=4):
    """Dense rest-coefficient bytes over (CSC codes + shared dictionary) bytes."""
    return dense_bytes(N, d, value_bytes) / (csc_bytes(N, nnz, value_bytes, index_bytes, ptr_bytes) +
                                            dictionary_bytes(K, d, value_bytes))
