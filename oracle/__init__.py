"""Merge Path oracle: TEST INFRASTRUCTURE ONLY.

Plain CPU implementations of what the GPU path computes, written from the
paper (Green, Odeh, Birk, "Merge Path - A Visually Intuitive Approach to
Parallel Merging").  The merge, split, sort and batched oracles are plain C
(``mp_oracle.c``, compiled with gcc); the split-predictor network oracle is
float64 numpy (``mlp.py``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library and never calls it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mp_oracle.c")
_LIB = os.path.join(_HERE, "libmp_oracle.so")

_NAME = {np.dtype(np.uint32): "u32", np.dtype(np.int32): "i32",
         np.dtype(np.uint64): "u64", np.dtype(np.float32): "f32"}

_lib = None


def build(out: str = _LIB, extra_flags=()) -> str:
    """Compile the C oracle with gcc into a shared library and return its path."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           *extra_flags, "-o", out, _SRC]
    subprocess.run(cmd, check=True)
    return out


def load(path: str | None = None):
    """Load (building first if absent) the oracle library."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _declare(lib):
    p, i64 = ctypes.c_void_p, ctypes.c_int64
    for n in _NAME.values():
        getattr(lib, f"oracle_merge_{n}").argtypes = [p, i64, p, i64, p, p]
        getattr(lib, f"oracle_merge_{n}").restype = None
        getattr(lib, f"oracle_merge_kv_{n}").argtypes = [p, p, i64, p, p, i64, p, p]
        getattr(lib, f"oracle_partition_{n}").argtypes = [p, i64, p, i64, p, i64, p]
        getattr(lib, f"oracle_sort_{n}").argtypes = [p, p, i64]
        getattr(lib, f"oracle_merge_batched_{n}").argtypes = [p, p, p, p, i64, p]
        getattr(lib, f"oracle_set_op_{n}").argtypes = [ctypes.c_int, p, i64, p, i64, p]
        getattr(lib, f"oracle_join_{n}").argtypes = [p, i64, p, i64, p, p, i64]
        getattr(lib, f"oracle_join_{n}").restype = i64
        getattr(lib, f"oracle_set_op_{n}").restype = i64
    return lib


def _ptr(x):
    return ctypes.c_void_p(x.ctypes.data) if x is not None else ctypes.c_void_p(0)


def _key_name(a: np.ndarray, b: np.ndarray | None = None) -> str:
    if b is not None and a.dtype != b.dtype:
        raise TypeError("A and B must share a key dtype")
    return _NAME[a.dtype]


def merge(A, B, with_src: bool = False, lib=None):
    """Sequential merge along the Merge Path (section 2.1); ties take A first."""
    lib = lib or load()
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    n = _key_name(A, B)
    S = np.empty(len(A) + len(B), dtype=A.dtype)
    src = np.empty(len(S), dtype=np.int64) if with_src else None
    getattr(lib, f"oracle_merge_{n}")(_ptr(A), len(A), _ptr(B), len(B), _ptr(S), _ptr(src))
    return (S, src) if with_src else S


def merge_kv(Ak, Av, Bk, Bv, lib=None):
    lib = lib or load()
    Ak, Bk = np.ascontiguousarray(Ak), np.ascontiguousarray(Bk)
    Av = np.ascontiguousarray(Av).view(np.uint32)
    Bv = np.ascontiguousarray(Bv).view(np.uint32)
    n = _key_name(Ak, Bk)
    Sk = np.empty(len(Ak) + len(Bk), dtype=Ak.dtype)
    Sv = np.empty(len(Sk), dtype=np.uint32)
    rc = getattr(lib, f"oracle_merge_kv_{n}")(_ptr(Ak), _ptr(Av), len(Ak), _ptr(Bk),
                                              _ptr(Bv), len(Bk), _ptr(Sk), _ptr(Sv))
    if rc != 0:
        raise MemoryError("oracle_merge_kv failed")
    return Sk, Sv


def partition(A, B, diag, lib=None):
    """Split on each cross diagonal (Lemma 8, Theorem 9): A-count of the first d outputs."""
    lib = lib or load()
    A, B = np.ascontiguousarray(A), np.ascontiguousarray(B)
    diag = np.ascontiguousarray(diag, dtype=np.int64)
    out = np.empty(len(diag), dtype=np.int64)
    rc = getattr(lib, f"oracle_partition_{_key_name(A, B)}")(
        _ptr(A), len(A), _ptr(B), len(B), _ptr(diag), len(diag), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_partition failed ({rc})")
    return out


def sort(keys, vals=None, lib=None):
    """Stable bottom-up merge sort (left run = A).  Returns new arrays."""
    lib = lib or load()
    k = np.array(keys, copy=True)
    v = None if vals is None else np.array(vals, copy=True).view(np.uint32)
    rc = getattr(lib, f"oracle_sort_{_key_name(k)}")(_ptr(k), _ptr(v), len(k))
    if rc != 0:
        raise MemoryError("oracle_sort failed")
    return k if vals is None else (k, v)


def merge_batched(A, a_off, B, b_off, lib=None):
    lib = lib or load()
    A, B = np.ascontiguousarray(A), np.ascontiguousarray(B)
    a_off = np.ascontiguousarray(a_off, dtype=np.int64)
    b_off = np.ascontiguousarray(b_off, dtype=np.int64)
    S = np.empty(len(A) + len(B), dtype=A.dtype)
    rc = getattr(lib, f"oracle_merge_batched_{_key_name(A, B)}")(
        _ptr(A), _ptr(a_off), _ptr(B), _ptr(b_off), len(a_off) - 1, _ptr(S))
    if rc != 0:
        raise ValueError(f"oracle_merge_batched failed ({rc})")
    return S


SET_OPS = {"intersection": 0, "union": 1, "difference": 2, "symmetric_difference": 3}


def set_op(op: str, A, B, lib=None):
    """Multiset intersection / union / difference / symmetric difference of
    sorted A and B, in merged order (A's copies before B's)."""
    lib = lib or load()
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    n = _key_name(A, B)
    S = np.empty(len(A) + len(B), dtype=A.dtype)
    k = getattr(lib, f"oracle_set_op_{n}")(SET_OPS[op], _ptr(A), len(A), _ptr(B), len(B), _ptr(S))
    return S[:k].copy()


def join(A, B, cap: int | None = None, lib=None):
    """Inner join of A and B: (I, J, count), the pairs with A[i] == B[j] in
    (i, j) order (a nested loop: O(|A| |B|), for small inputs).  With cap,
    only the first cap pairs are returned; count is always the total."""
    lib = lib or load()
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    name = _key_name(A, B)
    fn = getattr(lib, f"oracle_join_{name}")
    if cap is None:
        cap = fn(_ptr(A), len(A), _ptr(B), len(B), None, None, 0)
    I = np.empty(max(cap, 1), dtype=np.int64)
    J = np.empty(max(cap, 1), dtype=np.int64)
    k = fn(_ptr(A), len(A), _ptr(B), len(B), _ptr(I), _ptr(J), cap)
    m = min(k, cap)
    return I[:m].copy(), J[:m].copy(), int(k)
