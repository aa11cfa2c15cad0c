"""Thin ctypes binding of liblabs.so (include/labs.h).

Only argument marshalling lives here: torch supplies device buffers and the
current stream, every computation runs in the library's HIP kernels.  If the
library has not been built the calls raise instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblabs.so")

LABS_OK = 0
LABS_PENDING = 1
LABS_EINVAL = -1
LABS_ENOMEM = -2
LABS_EDEVICE = -3
LABS_EBUSY = -4
LABS_ENOTFOUND = -5

I32 = ctypes.c_int32
I64 = ctypes.c_int64
U64 = ctypes.c_uint64
VP = ctypes.c_void_p


class LabsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"labs error {code}: {msg}")
        self.code = code


class WalkOut(ctypes.Structure):
    _fields_ = [("best_seq", VP), ("best_E", VP), ("steps_done", VP), ("digest", VP),
                ("trace_j", VP), ("trace_E", VP), ("n_trace", I64)]


class Plan(ctypes.Structure):
    _fields_ = [("lanes_per_walk", I32), ("load_factor", ctypes.c_double),
                ("max_concurrent", I64)]


_lib = None


def lib():
    """Load liblabs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        L.labs_last_error.restype = ctypes.c_char_p
        L.labs_l_max.restype = I32
        L.labs_key_words.argtypes = [I32]
        L.labs_key_words.restype = I32
        L.labs_energy.argtypes = [VP, I32, I64, VP, VP]
        L.labs_energy.restype = I32
        L.labs_pack_skew.argtypes = [VP, I32, I64, VP]
        L.labs_pack_skew.restype = I32
        L.labs_unpack_skew.argtypes = [VP, I32, I64, VP]
        L.labs_unpack_skew.restype = I32
        L.labs_expand_skew.argtypes = [VP, I32, I64, VP]
        L.labs_expand_skew.restype = I32
        L.labs_starts.argtypes = [I32, I64, U64, VP, VP]
        L.labs_starts.restype = I32
        L.labs_walks_workspace_bytes.argtypes = [I32, I64, I64, ctypes.POINTER(Plan),
                                                 ctypes.POINTER(U64)]
        L.labs_walks_workspace_bytes.restype = I32
        L.labs_walks_min_workspace_bytes.argtypes = [I32, I64, ctypes.POINTER(Plan),
                                                     ctypes.POINTER(U64)]
        L.labs_walks_min_workspace_bytes.restype = I32
        L.labs_walks.argtypes = [VP, I32, I64, I64, U64, ctypes.POINTER(WalkOut), VP, U64,
                                 ctypes.POINTER(Plan), VP]
        L.labs_walks.restype = I32
        _lib = L
    return _lib


def _check(rc: int):
    if rc < 0:
        raise LabsError(rc, lib().labs_last_error().decode())
    return rc


def _stream_handle(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def l_max() -> int:
    return int(lib().labs_l_max())


def key_words(L: int) -> int:
    return int(lib().labs_key_words(L))


def free_bits(L: int) -> int:
    return (L + 1) // 2


# ---------------------------------------------------------------- host helpers
def pack_skew(x: np.ndarray, L: int) -> np.ndarray:
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.int8).reshape(-1, free_bits(L)))
    out = np.zeros((xa.shape[0], key_words(L)), dtype=np.uint64)
    _check(lib().labs_pack_skew(xa.ctypes.data, L, xa.shape[0], out.ctypes.data))
    return out


def unpack_skew(keys: np.ndarray, L: int) -> np.ndarray:
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64).reshape(-1, key_words(L)))
    out = np.zeros((k.shape[0], free_bits(L)), dtype=np.int8)
    _check(lib().labs_unpack_skew(k.ctypes.data, L, k.shape[0], out.ctypes.data))
    return out


def expand_skew(x: np.ndarray, L: int) -> np.ndarray:
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.int8).reshape(-1, free_bits(L)))
    out = np.zeros((xa.shape[0], L), dtype=np.int8)
    _check(lib().labs_expand_skew(xa.ctypes.data, L, xa.shape[0], out.ctypes.data))
    return out


# -------------------------------------------------------------- device calls
def energy(seqs, stream=None):
    """Eq. 1 energies of an int8 [n, L] CUDA tensor of +-1 values -> int32 [n]."""
    import torch
    if seqs.dtype != torch.int8 or seqs.dim() != 2 or not seqs.is_cuda:
        raise ValueError("seqs must be a 2-D int8 CUDA tensor")
    seqs = seqs.contiguous()
    n, L = seqs.shape
    if n and not bool(((seqs == 1) | (seqs == -1)).all()):
        raise ValueError("sequence elements must be +1 or -1")
    out = torch.empty(n, dtype=torch.int32, device=seqs.device)
    _check(lib().labs_energy(_dptr(seqs), L, n, _dptr(out), _stream_handle(stream)))
    return out


def starts(L: int, n_walks: int, seed: int, device="cuda", stream=None):
    import torch
    out = torch.empty((n_walks, max(key_words(L), 1)), dtype=torch.int64, device=device)
    _check(lib().labs_starts(L, n_walks, seed & 0xFFFFFFFFFFFFFFFF, _dptr(out),
                             _stream_handle(stream)))
    return out


def make_plan(lanes_per_walk: int = 0, load_factor: float = 0.0, max_concurrent: int = 0) -> Plan:
    return Plan(lanes_per_walk, load_factor, max_concurrent)


def workspace_bytes(L: int, n_walks: int, walk_len: int, plan: Optional[Plan] = None) -> int:
    b = U64(0)
    _check(lib().labs_walks_workspace_bytes(L, n_walks, walk_len,
                                            ctypes.byref(plan) if plan else None, ctypes.byref(b)))
    return int(b.value)


def min_workspace_bytes(L: int, walk_len: int, plan: Optional[Plan] = None) -> int:
    b = U64(0)
    _check(lib().labs_walks_min_workspace_bytes(L, walk_len, ctypes.byref(plan) if plan else None,
                                                ctypes.byref(b)))
    return int(b.value)


def alloc_workspace(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=device)


def walks(L: int, n_walks: int, walk_len: int, seed: int = 0, starts_t=None, n_trace: int = 0,
          plan: Optional[Plan] = None, workspace=None, digest: bool = True, stream=None,
          device="cuda"):
    """Run n_walks self-avoiding walks; returns a dict of CUDA tensors.

    Keys: best_seq int64 [n, W] (bit patterns of the uint64 key words), best_E
    int32 [n], steps_done int64 [n], digest int64 [n] (uint64 bit patterns), and
    trace_j int16 / trace_E int32 [n_trace, walk_len] when n_trace > 0.
    """
    import torch
    W = key_words(L)
    if W == 0:
        raise LabsError(LABS_EINVAL, f"invalid L={L}")
    if starts_t is not None:
        if starts_t.dtype != torch.int64 or tuple(starts_t.shape) != (n_walks, W) or not starts_t.is_cuda:
            raise ValueError("starts must be an int64 CUDA tensor of shape (n_walks, W)")
        starts_t = starts_t.contiguous()
    if workspace is None:
        workspace = alloc_workspace(workspace_bytes(L, n_walks, walk_len, plan), device=device)
    res = {
        "best_seq": torch.empty((n_walks, W), dtype=torch.int64, device=device),
        "best_E": torch.empty(n_walks, dtype=torch.int32, device=device),
        "steps_done": torch.empty(n_walks, dtype=torch.int64, device=device),
        "digest": torch.empty(n_walks, dtype=torch.int64, device=device) if digest else None,
    }
    if n_trace:
        res["trace_j"] = torch.zeros((n_trace, walk_len), dtype=torch.int16, device=device)
        res["trace_E"] = torch.zeros((n_trace, walk_len), dtype=torch.int32, device=device)
    out = WalkOut(_dptr(res["best_seq"]), _dptr(res["best_E"]), _dptr(res["steps_done"]),
                  _dptr(res["digest"]), _dptr(res.get("trace_j")), _dptr(res.get("trace_E")),
                  n_trace)
    _check(lib().labs_walks(_dptr(starts_t), L, n_walks, walk_len, seed & 0xFFFFFFFFFFFFFFFF,
                            ctypes.byref(out), _dptr(workspace), workspace.numel(),
                            ctypes.byref(plan) if plan else None, _stream_handle(stream)))
    return res
