"""Autotuning: the library's native tuner plus a JSON cache of its choices.

The tuner itself runs in the library (mp_autotune_*): it times every
compiled (lanes, outputs-per-lane) variant of an operation on the caller's
inputs with HIP events and installs the fastest.  This module calls it and
keeps the winners in a JSON file keyed by GPU architecture, operation, key
type and size class (log2 of the number of keys), so later processes can
apply them without re-timing.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import torch

from . import (Config, MP_NONE, TORCH_TO_MP, _check, _key_dtype, _ptr, _stream, _val_dtype,
               lib, set_config, sort_workspace_bytes)

_choices: dict[str, list[int]] = {}


def _arch() -> str:
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def _key(op: str, dtype: torch.dtype, n: int) -> str:
    return f"{_arch()}/{op}/{str(dtype).replace('torch.', '')}/{int(math.log2(max(1, n)))}"


def _record(op, dtype, n, cfg: Config):
    _choices[_key(op, dtype, n)] = [cfg.mode, cfg.nt, cfg.vt, cfg.grid, cfg.margin]
    return (cfg.mode, cfg.nt, cfg.vt, cfg.grid, cfg.margin)


def tune_merge(A, B, out, reps: int = 5, Av=None, Bv=None, out_v=None):
    kt = _key_dtype(A, B)
    vt = MP_NONE if Av is None else _val_dtype(Av, Bv)
    cfg = Config()
    _check(lib().mp_autotune_merge(kt, vt, _ptr(A), _ptr(Av), A.numel(), _ptr(B), _ptr(Bv),
                                   B.numel(), _ptr(out), _ptr(out_v), reps,
                                   ctypes.cast(ctypes.byref(cfg), ctypes.c_void_p),
                                   _stream(A.device)))
    return _record("merge", A.dtype, A.numel() + B.numel(), cfg)


def tune_batched(A, a_off, B, b_off, out, reps: int = 5):
    kt = _key_dtype(A, B)
    cfg = Config()
    _check(lib().mp_autotune_batched(kt, _ptr(A), _ptr(a_off), _ptr(B), _ptr(b_off),
                                     a_off.numel() - 1, A.numel(), B.numel(), _ptr(out), reps,
                                     ctypes.cast(ctypes.byref(cfg), ctypes.c_void_p),
                                     _stream(A.device)))
    return _record("batched", A.dtype, A.numel() + B.numel(), cfg)


def tune_sort(keys_in, keys, reps: int = 3, vals_in=None, vals=None, ws=None):
    kt = _key_dtype(keys_in, keys)
    vt = MP_NONE if vals is None else _val_dtype(vals_in, vals)
    n = keys.numel()
    need = sort_workspace_bytes(keys.dtype, None if vals is None else vals.dtype, n)
    if ws is None and need:
        ws = torch.empty(need, dtype=torch.uint8, device=keys.device)
    cfg = Config()
    _check(lib().mp_autotune_sort(kt, vt, _ptr(keys_in), _ptr(vals_in), _ptr(keys), _ptr(vals),
                                  n, _ptr(ws), 0 if ws is None else ws.numel(), reps,
                                  ctypes.cast(ctypes.byref(cfg), ctypes.c_void_p),
                                  _stream(keys.device)))
    return _record("sort", keys.dtype, n, cfg)


def save(path: str):
    """Write every choice made in this process (merged with the file's)."""
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.update(_choices)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def apply(path: str, op: str, dtype: torch.dtype, n: int) -> bool:
    """Install the cached choice for (op, dtype, size class) if there is one."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        data = json.load(f)
    c = data.get(_key(op, dtype, n))
    if c is None:
        return False
    set_config(op, *c)
    return True


__all__ = ["tune_merge", "tune_batched", "tune_sort", "save", "apply", "TORCH_TO_MP"]
