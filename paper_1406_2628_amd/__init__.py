"""Merge Path on MI355X (gfx950): Python binding of ``libmergepath.so``.

Argument marshalling only: every step of every operation runs in the HIP
kernels of the C-ABI library (``include/mergepath.h``).  PyTorch supplies
device memory and the current stream; it computes nothing here.  If the
library is not built, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmergepath.so")

MP_NONE, MP_U32, MP_I32, MP_U64, MP_F32 = 0, 1, 2, 3, 4
_STATUS = {0: "MP_OK", -1: "MP_ERR_INVALID_ARG", -2: "MP_ERR_UNSUPPORTED",
           -3: "MP_ERR_OVERLAP", -4: "MP_ERR_WORKSPACE", -5: "MP_ERR_HIP",
           -6: "MP_ERR_STATE"}
TORCH_TO_MP = {torch.uint32: MP_U32, torch.int32: MP_I32, torch.uint64: MP_U64,
               torch.float32: MP_F32}

_lib = None


class MergePathError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1406_2628_amd.build` (no CPU fallback exists)")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _declare(L):
    p, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    sig = {
        "mp_last_error": ([], ctypes.c_char_p),
        "mp_version": ([], i32),
        "mp_partition": ([i32, p, i64, p, i64, p, i64, p, p], i32),
        "mp_partition_lanes": ([i32], i32),
        "mp_merge": ([i32, p, i64, p, i64, p, p], i32),
        "mp_merge_checksum": ([i32, p, i64, p, i64, p, p], i32),
        "mp_merge_split": ([i32, p, i64, p, i64, p, i32, p, p], i32),
        "mp_set_op_workspace_bytes": ([i64, i64], ctypes.c_size_t),
        "mp_set_op": ([i32, i32, p, i64, p, i64, p, p, p, ctypes.c_size_t, p], i32),
        "mp_set_op_noalloc": ([i32, i32, p, i64, p, i64, p, p, p], i32),
        "mp_join_workspace_bytes": ([i64, i64], ctypes.c_size_t),
        "mp_join": ([i32, p, i64, p, i64, p, p, i64, p, p, ctypes.c_size_t, p], i32),
        "mp_merge_kv": ([i32, i32, p, p, i64, p, p, i64, p, p, p], i32),
        "mp_merge_batched_workspace_bytes": ([i32, i64, i64], sz),
        "mp_merge_batched": ([i32, p, p, p, p, i64, i64, i64, p, p, sz, p], i32),
        "mp_sort_block_keys": ([ctypes.c_int, ctypes.c_int], i64),
        "mp_sort_workspace_bytes": ([i32, i32, i64], sz),
        "mp_sort": ([i32, i32, p, p, i64, p, sz, p], i32),
        "mp_set_config": ([ctypes.c_char_p, ctypes.c_void_p], i32),
        "mp_get_config": ([ctypes.c_char_p, ctypes.c_void_p], i32),
        "mp_graph_enable": ([i32], i32),
        "mp_graph_clear": ([], i32),
        "mp_graph_count": ([], i64),
        "mp_autotune_merge": ([i32, i32, p, p, i64, p, p, i64, p, p, i32, p, p], i32),
        "mp_autotune_batched": ([i32, p, p, p, p, i64, i64, i64, p, i32, p, p], i32),
        "mp_autotune_sort": ([i32, i32, p, p, p, p, i64, p, sz, i32, p, p], i32),
        "mp_copy": ([p, p, i64, i32, i32, p], i32),
        "mp_bw_probe": ([i32, p, p, i64, i32, i32, p], i32),
        "mp_timing_enable": ([i32], i32),
        "mp_timing_reset": ([], i32),
        "mp_timing_query": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_int64)], i32),
        "mp_stats_query": ([ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], i32),
        "mp_stats_workgroups": ([ctypes.POINTER(ctypes.c_int64)], i32),
        "mp_lp_create": ([ctypes.POINTER(p), i32, i32, ctypes.c_uint64], i32),
        "mp_lp_destroy": ([p], None),
        "mp_lp_num_params": ([p], i32),
        "mp_lp_shape": ([p, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "mp_lp_get_params": ([p, p, i32], i32),
        "mp_lp_set_params": ([p, p, i32], i32),
        "mp_lp_set_window": ([p, i64], i32),
        "mp_lp_window": ([p], i64),
        "mp_lp_windows": ([p, ctypes.POINTER(ctypes.c_int64), i32], i32),
        "mp_lp_examples": ([p, i32, p, i64, p, i64, i64, ctypes.c_uint64, p, p, p, p, p], i32),
        "mp_lp_forward": ([p, p, i64, p, p], i32),
        "mp_lp_grad": ([p, p, p, i64, p, p, p], i32),
        "mp_lp_adam_step": ([p, p, p, i64, ctypes.c_float, p], i32),
        "mp_lp_train": ([p, i32, p, p, p, p, i32, i64, i32, ctypes.c_float,
                         ctypes.POINTER(ctypes.c_float), p], i32),
        "mp_lp_calibrate": ([p, i32, p, i64, p, i64, i64, ctypes.POINTER(ctypes.c_int64), p], i32),
        "mp_partition_learned": ([p, i32, p, i64, p, i64, p, i64, p, p, p], i32),
        "mp_lp_save": ([p, ctypes.c_char_p], i32),
        "mp_lp_load": ([ctypes.POINTER(p), ctypes.c_char_p], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes, f.restype = args, res
    return L


class Config(ctypes.Structure):
    """Kernel variant (mp_config): mode 1 = per-tile, 2 = persistent."""
    _fields_ = [("mode", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("vt", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("margin", ctypes.c_int32)]


def set_config(op: str, mode: int | None = None, nt: int = 256, vt: int = 16, grid: int = 0,
               margin: int = 0):
    """Select the kernel variant of ``op`` ('merge', 'batched', 'sort'); mode None resets."""
    if mode is None:
        _check(lib().mp_set_config(op.encode(), None))
    else:
        cfg = Config(mode, nt, vt, grid, margin)
        _check(lib().mp_set_config(op.encode(), ctypes.cast(ctypes.byref(cfg), ctypes.c_void_p)))


def graph_mode(on: bool = True):
    """Record sort and batched launches into cached hipGraphs (see mp_graph_enable)."""
    _check(lib().mp_graph_enable(1 if on else 0))


def graph_clear():
    _check(lib().mp_graph_clear())


def graph_count() -> int:
    return lib().mp_graph_count()


def get_config(op: str):
    """(mode, nt, vt, grid, margin) that ``op`` currently uses."""
    cfg = Config()
    _check(lib().mp_get_config(op.encode(), ctypes.cast(ctypes.byref(cfg), ctypes.c_void_p)))
    return (cfg.mode, cfg.nt, cfg.vt, cfg.grid, cfg.margin)


def copy(src: torch.Tensor, dst: torch.Tensor, unroll: int = 0, grid: int = 0):
    """Reference streaming copy of src's bytes into dst (bandwidth probe)."""
    n = src.numel() * src.element_size()
    _check(lib().mp_copy(_ptr(src), _ptr(dst), n, unroll, grid, _stream(src.device)))


BW_KINDS = {"copy": 0, "read": 1, "write": 2}


def bw_probe(kind: str, src: torch.Tensor | None, dst: torch.Tensor, n_bytes: int,
             unroll: int = 0, grid: int = 0):
    """Bandwidth reference: copy, read-only or write-only pass over n_bytes
    (for 'read', dst is the small per-wavefront sink)."""
    dev_ = dst.device
    _check(lib().mp_bw_probe(BW_KINDS[kind], _ptr(src), _ptr(dst), n_bytes, unroll, grid,
                             _stream(dev_)))


def timing_enable(on: bool = True):
    _check(lib().mp_timing_enable(1 if on else 0))
    _check(lib().mp_timing_reset())


def timing_query(name: str):
    """(total_ms, launches) of kernel family ``name`` since the last reset."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().mp_timing_query(name.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def stats_query():
    """(tiles, window reloads) of the persistent kernels since the last reset."""
    t, r = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().mp_stats_query(ctypes.byref(t), ctypes.byref(r)))
    return t.value, r.value


def stats_workgroups() -> int:
    """Workgroups of the persistent kernels that had a tile, since the last reset."""
    g = ctypes.c_int64()
    _check(lib().mp_stats_workgroups(ctypes.byref(g)))
    return g.value


def last_error() -> str:
    return lib().mp_last_error().decode()


def _check(status: int):
    if status != 0:
        raise MergePathError(status, last_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _key_dtype(*ts) -> int:
    dt = ts[0].dtype
    for t in ts:
        if t.dtype != dt:
            raise TypeError("key arrays must share one dtype")
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("arrays must be contiguous device tensors")
    if dt not in TORCH_TO_MP:
        raise TypeError(f"unsupported key dtype {dt}")
    return TORCH_TO_MP[dt]


def _val_dtype(*ts) -> int:
    dt = ts[0].dtype
    for t in ts:
        if t.dtype != dt or t.element_size() != 4:
            raise TypeError("values must share one 4-byte dtype")
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("arrays must be contiguous device tensors")
    return {torch.uint32: MP_U32, torch.int32: MP_I32, torch.float32: MP_F32}[dt]


def partition(A: torch.Tensor, B: torch.Tensor, diag: torch.Tensor,
              out: torch.Tensor | None = None) -> torch.Tensor:
    """Split (count of A elements) on each cross diagonal in ``diag`` (int64)."""
    kt = _key_dtype(A, B)
    if out is None:
        out = torch.empty(diag.numel(), dtype=torch.int64, device=A.device)
    _check(lib().mp_partition(kt, _ptr(A), A.numel(), _ptr(B), B.numel(), _ptr(diag),
                              diag.numel(), _ptr(out), _stream(A.device)))
    return out


SET_OPS = {"intersection": 0, "union": 1, "difference": 2, "symmetric_difference": 3}


def set_op(op: str, A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None,
           count: torch.Tensor | None = None, ws: torch.Tensor | None = None,
           sync: bool = True):
    """Multiset intersection / union / difference / symmetric_difference of
    sorted A and B.  With sync (default) returns the output trimmed to its
    length; otherwise returns (out, count) with count an int64 device scalar."""
    kt = _key_dtype(A, B)
    code = SET_OPS[op]
    cap = A.numel() if code in (0, 2) else A.numel() + B.numel()
    if out is None:
        out = torch.empty(max(cap, 1), dtype=A.dtype, device=A.device)
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=A.device)
    need = lib().mp_set_op_workspace_bytes(A.numel(), B.numel())
    if ws is None:
        ws = torch.empty(max(need, 8), dtype=torch.uint8, device=A.device)
    _check(lib().mp_set_op(code, kt, _ptr(A), A.numel(), _ptr(B), B.numel(), _ptr(out), _ptr(count),
                           _ptr(ws), ws.numel(), _stream(A.device)))
    if not sync:
        return out, count
    k = int(count.item())
    if k < 0:
        raise RuntimeError("mp_set_op: a tile's wait for the tiles before it gave up")
    return out[:k]


def join(A: torch.Tensor, B: torch.Tensor, cap: int | None = None, I=None, J=None, count=None,
         ws=None, sync: bool = True):
    """Inner join of sorted A and B: pairs (i, j) with A[i] == B[j] in
    (i, j) order.  With sync (default) and cap None, counts first and
    returns (I, J) trimmed to the count; otherwise returns (I, J, count)
    with count an int64 device scalar (the total, which may exceed cap)."""
    kt = _key_dtype(A, B)
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=A.device)
    need = lib().mp_join_workspace_bytes(A.numel(), B.numel())
    if ws is None:
        ws = torch.empty(max(need, 8), dtype=torch.uint8, device=A.device)
    if cap is None and sync:
        _check(lib().mp_join(kt, _ptr(A), A.numel(), _ptr(B), B.numel(), None, None, 0,
                             _ptr(count), _ptr(ws), ws.numel(), _stream(A.device)))
        cap = int(count.item())
    cap = 0 if cap is None else cap
    if I is None:
        I = torch.empty(max(cap, 1), dtype=torch.int64, device=A.device)
    if J is None:
        J = torch.empty(max(cap, 1), dtype=torch.int64, device=A.device)
    _check(lib().mp_join(kt, _ptr(A), A.numel(), _ptr(B), B.numel(), _ptr(I), _ptr(J), cap,
                         _ptr(count), _ptr(ws), ws.numel(), _stream(A.device)))
    if not sync:
        return I, J, count
    k = min(int(count.item()), cap)
    return I[:k], J[:k]


def set_op_noalloc(op: str, A: torch.Tensor, B: torch.Tensor, out: torch.Tensor,
                   count: torch.Tensor):
    """mp_set_op_noalloc: the set operation with the library's fixed device
    scratch instead of a workspace.  ``out`` must hold the operation's room
    and ``count`` is an int64 device scalar; nothing is allocated and
    nothing synchronised.  Returns (out, count)."""
    kt = _key_dtype(A, B)
    _check(lib().mp_set_op_noalloc(SET_OPS[op], kt, _ptr(A), A.numel(), _ptr(B), B.numel(),
                                   _ptr(out), _ptr(count), _stream(A.device)))
    return out, count


def merge_split(A: torch.Tensor, B: torch.Tensor, a_split: torch.Tensor, tile: int = 4096,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """Merge tile by tile from given splits on the diagonals min(k * tile, N)
    (ceil(N / tile) + 1 int64 values, as ``partition`` returns them)."""
    kt = _key_dtype(A, B)
    if out is None:
        out = torch.empty(A.numel() + B.numel(), dtype=A.dtype, device=A.device)
    _check(lib().mp_merge_split(kt, _ptr(A), A.numel(), _ptr(B), B.numel(), _ptr(a_split), tile,
                                _ptr(out), _stream(A.device)))
    return out


def merge_checksum(A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Merge without writing it: adds sum(S[i] * (i + 1)) mod 2^64 (keys as
    unsigned bits) to ``out`` (a zeroed uint64 device scalar when None)."""
    kt = _key_dtype(A, B)
    if out is None:
        out = torch.zeros(1, dtype=torch.uint64, device=A.device)
    _check(lib().mp_merge_checksum(kt, _ptr(A), A.numel(), _ptr(B), B.numel(), _ptr(out),
                                   _stream(A.device)))
    return out


def set_partition_lanes(lanes: int = 0):
    """Lanes that search one diagonal together in ``partition`` and the
    learned partition: 0 = chosen per call, else a power of two up to 64."""
    _check(lib().mp_partition_lanes(lanes))


def merge(A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    kt = _key_dtype(A, B)
    if out is None:
        out = torch.empty(A.numel() + B.numel(), dtype=A.dtype, device=A.device)
    _check(lib().mp_merge(kt, _ptr(A), A.numel(), _ptr(B), B.numel(), _ptr(out),
                          _stream(A.device)))
    return out


def merge_kv(Ak, Av, Bk, Bv, out_k=None, out_v=None):
    kt = _key_dtype(Ak, Bk)
    vt = _val_dtype(Av, Bv)
    if Av.numel() != Ak.numel() or Bv.numel() != Bk.numel():
        raise ValueError("each value array must match its key array")
    n = Ak.numel() + Bk.numel()
    if out_k is None:
        out_k = torch.empty(n, dtype=Ak.dtype, device=Ak.device)
    if out_v is None:
        out_v = torch.empty(n, dtype=Av.dtype, device=Ak.device)
    _check(lib().mp_merge_kv(kt, vt, _ptr(Ak), _ptr(Av), Ak.numel(), _ptr(Bk), _ptr(Bv),
                             Bk.numel(), _ptr(out_k), _ptr(out_v), _stream(Ak.device)))
    return out_k, out_v


def merge_batched_workspace_bytes(dtype: torch.dtype, n_pairs: int, total: int) -> int:
    return lib().mp_merge_batched_workspace_bytes(TORCH_TO_MP[dtype], n_pairs, total)


def merge_batched(A, a_off, B, b_off, total_a: int | None = None, total_b: int | None = None,
                  out=None, ws=None):
    """Independent merges of (A[a_off[k]:a_off[k+1]], B[b_off[k]:b_off[k+1]])."""
    kt = _key_dtype(A, B)
    n_pairs = a_off.numel() - 1
    total_a = A.numel() if total_a is None else total_a
    total_b = B.numel() if total_b is None else total_b
    if out is None:
        out = torch.empty(total_a + total_b, dtype=A.dtype, device=A.device)
    need = merge_batched_workspace_bytes(A.dtype, n_pairs, total_a + total_b)
    if ws is None and need:
        ws = torch.empty(need, dtype=torch.uint8, device=A.device)
    _check(lib().mp_merge_batched(kt, _ptr(A), _ptr(a_off), _ptr(B), _ptr(b_off), n_pairs,
                                  total_a, total_b, _ptr(out), _ptr(ws),
                                  0 if ws is None else ws.numel(), _stream(A.device)))
    return out


def sort_block_keys(key_dtype: torch.dtype, val_dtype: torch.dtype | None = None) -> int:
    """Length of the blocks the sort orders first (its first runs)."""
    vt = MP_NONE if val_dtype is None else {torch.uint32: MP_U32, torch.int32: MP_I32,
                                             torch.float32: MP_F32}[val_dtype]
    return int(lib().mp_sort_block_keys(TORCH_TO_MP[key_dtype], vt))


def sort_workspace_bytes(key_dtype: torch.dtype, val_dtype: torch.dtype | None, n: int) -> int:
    vt = MP_NONE if val_dtype is None else {torch.uint32: MP_U32, torch.int32: MP_I32,
                                             torch.float32: MP_F32}[val_dtype]
    return lib().mp_sort_workspace_bytes(TORCH_TO_MP[key_dtype], vt, n)


def sort(keys: torch.Tensor, vals: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """Stable in-place merge sort of ``keys`` (and ``vals`` with them)."""
    kt = _key_dtype(keys)
    vt = MP_NONE if vals is None else _val_dtype(vals)
    need = sort_workspace_bytes(keys.dtype, None if vals is None else vals.dtype, keys.numel())
    if ws is None and need:
        ws = torch.empty(need, dtype=torch.uint8, device=keys.device)
    _check(lib().mp_sort(kt, vt, _ptr(keys), _ptr(vals), keys.numel(), _ptr(ws),
                         0 if ws is None else ws.numel(), _stream(keys.device)))
    return keys if vals is None else (keys, vals)


class LearnedPartitioner:
    """Handle of the learned split predictor (mp_lp_*): an FP32 MLP whose
    prediction bounds the exact split search; outputs equal ``partition``."""

    def __init__(self, hidden: int = 32, features: int = 5, seed: int = 0, _handle=None):
        self._h = ctypes.c_void_p()
        if _handle is not None:
            self._h = _handle
        else:
            _check(lib().mp_lp_create(ctypes.byref(self._h), hidden, features, seed))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and h.value and _lib is not None:
            _lib.mp_lp_destroy(h)
            self._h = ctypes.c_void_p()

    @property
    def num_params(self) -> int:
        return lib().mp_lp_num_params(self._h)

    @property
    def window(self) -> int:
        return lib().mp_lp_window(self._h)

    @window.setter
    def window(self, w: int):
        _check(lib().mp_lp_set_window(self._h, w))

    def windows(self):
        """Per-bucket (lo, hi) window offsets as an (n, 2) int64 numpy array,
        or an empty (0, 2) array when one symmetric window is set."""
        import numpy as np
        n = lib().mp_lp_windows(self._h, None, 0)
        out = np.zeros((max(n, 0), 2), dtype=np.int64)
        if n > 0:
            lib().mp_lp_windows(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n)
        return out

    def get_params(self):
        import numpy as np
        out = np.empty(self.num_params, dtype=np.float32)
        _check(lib().mp_lp_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p), len(out)))
        return out

    def set_params(self, params):
        import numpy as np
        arr = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().mp_lp_set_params(self._h, arr.ctypes.data_as(ctypes.c_void_p), len(arr)))

    def examples(self, A, B, K: int, seed: int = 1):
        """(X, r, diag, split) device tensors for K stratified diagonals of (A, B)."""
        kt = _key_dtype(A, B)
        F = self.shape[0]
        X = torch.empty((K, F), dtype=torch.float32, device=A.device)
        r = torch.empty(K, dtype=torch.float32, device=A.device)
        d = torch.empty(K, dtype=torch.int64, device=A.device)
        s = torch.empty(K, dtype=torch.int64, device=A.device)
        _check(lib().mp_lp_examples(self._h, kt, _ptr(A), A.numel(), _ptr(B), B.numel(), K, seed,
                                    _ptr(X), _ptr(r), _ptr(d), _ptr(s), _stream(A.device)))
        return X, r, d, s

    @property
    def shape(self):
        """(features, hidden units)."""
        f, h = ctypes.c_int(), ctypes.c_int()
        _check(lib().mp_lp_shape(self._h, ctypes.byref(f), ctypes.byref(h)))
        return f.value, h.value

    def forward(self, X):
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(lib().mp_lp_forward(self._h, _ptr(X), X.shape[0], _ptr(y), _stream(X.device)))
        return y

    def grad(self, X, r):
        g = torch.empty(self.num_params, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(lib().mp_lp_grad(self._h, _ptr(X), _ptr(r), X.shape[0], _ptr(g), _ptr(loss),
                                _stream(X.device)))
        return g, loss

    def adam_step(self, X, r, lr: float):
        _check(lib().mp_lp_adam_step(self._h, _ptr(X), _ptr(r), X.shape[0], lr, _stream(X.device)))

    def train(self, sets, k_diag: int = 1 << 14, epochs: int = 4000, lr: float = 1e-2) -> float:
        """Train on a list of (A, B) device tensor pairs; returns the final loss."""
        kt = _key_dtype(*[t for ab in sets for t in ab])
        n = len(sets)
        As = (ctypes.c_void_p * n)(*[a.data_ptr() for a, _ in sets])
        Bs = (ctypes.c_void_p * n)(*[b.data_ptr() for _, b in sets])
        nas = (ctypes.c_int64 * n)(*[a.numel() for a, _ in sets])
        nbs = (ctypes.c_int64 * n)(*[b.numel() for _, b in sets])
        loss = ctypes.c_float()
        _check(lib().mp_lp_train(self._h, kt, As, nas, Bs, nbs, n, k_diag, epochs, lr,
                                 ctypes.byref(loss), _stream(sets[0][0].device)))
        return loss.value

    def calibrate(self, A, B, n_diag: int = 1 << 16) -> int:
        """Set the window from a held-out pair; returns the largest validation error."""
        kt = _key_dtype(A, B)
        err = ctypes.c_int64()
        _check(lib().mp_lp_calibrate(self._h, kt, _ptr(A), A.numel(), _ptr(B), B.numel(), n_diag,
                                     ctypes.byref(err), _stream(A.device)))
        return err.value

    def partition(self, A, B, diag, out=None, fallbacks=None):
        """Same result as ``partition``; ``fallbacks`` (uint64 device scalar) counts misses."""
        kt = _key_dtype(A, B)
        if out is None:
            out = torch.empty(diag.numel(), dtype=torch.int64, device=A.device)
        _check(lib().mp_partition_learned(self._h, kt, _ptr(A), A.numel(), _ptr(B), B.numel(),
                                          _ptr(diag), diag.numel(), _ptr(out), _ptr(fallbacks),
                                          _stream(A.device)))
        return out

    def save(self, path: str):
        _check(lib().mp_lp_save(self._h, path.encode()))

    @classmethod
    def load(cls, path: str) -> "LearnedPartitioner":
        h = ctypes.c_void_p()
        _check(lib().mp_lp_load(ctypes.byref(h), path.encode()))
        return cls(_handle=h)
