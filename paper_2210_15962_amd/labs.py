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
                ("trace_j", VP), ("trace_E", VP), ("n_trace", I64), ("cap_steps", VP)]


class Plan(ctypes.Structure):
    _fields_ = [("lanes_per_walk", I32), ("load_factor", ctypes.c_double),
                ("max_concurrent", I64)]


class Instance(ctypes.Structure):
    _fields_ = [("L", I32), ("lanes_per_walk", I32), ("n_walks", I64), ("walk_len", I64),
                ("seed", U64), ("starts", VP), ("load_factor", ctypes.c_double),
                ("out", WalkOut)]


class SolveCfg(ctypes.Structure):
    _fields_ = [("walks_per_round", I64), ("walk_len", I64), ("seed", U64),
                ("time_limit_s", ctypes.c_double), ("nses_limit", ctypes.c_double),
                ("target_E", I32), ("pad", I32), ("max_rounds", I64), ("plan", Plan),
                ("first_round", I64)]


class SolveResult(ctypes.Structure):
    _fields_ = [("best_E", I32), ("reached_target", I32), ("best_seq", U64 * 3), ("rounds", I64),
                ("nfes", ctypes.c_double), ("walk_steps", ctypes.c_double),
                ("seconds", ctypes.c_double), ("target_seconds", ctypes.c_double),
                ("target_nfes", ctypes.c_double)]


class ServeCfg(ctypes.Structure):
    _fields_ = [("pool_bytes", U64), ("max_pending", I32), ("lanes_per_walk", I32),
                ("chunk_steps", I64), ("load_factor", ctypes.c_double), ("whole_space", I32)]


class ServeResult(ctypes.Structure):
    _fields_ = [("best_seq", VP), ("best_E", VP), ("steps_done", VP), ("digest", VP),
                ("t_submit_ns", I64), ("t_admit_ns", I64), ("t_done_ns", I64),
                ("total_steps", I64)]


class ServeCounters(ctypes.Structure):
    _fields_ = [("submitted", I64), ("admitted", I64), ("completed", I64), ("pending", I64),
                ("active", I64), ("launches", I64), ("walk_steps", I64), ("busy_ns", I64),
                ("pool_bytes", U64), ("pool_used", U64), ("pool_peak", U64)]


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
        L.labs_walks_noalloc.argtypes = [VP, I32, I64, I64, U64, ctypes.POINTER(WalkOut),
                                         ctypes.POINTER(Plan), VP]
        L.labs_walks_noalloc.restype = I32
        L.labs_full_l_max.restype = I32
        L.labs_full_key_words.argtypes = [I32]
        L.labs_full_key_words.restype = I32
        L.labs_full_walks_workspace_bytes.argtypes = [I32, I64, I64, ctypes.POINTER(Plan),
                                                      ctypes.POINTER(U64)]
        L.labs_full_walks_workspace_bytes.restype = I32
        L.labs_full_walks.argtypes = [VP, I32, I64, I64, U64, ctypes.POINTER(WalkOut), VP, U64,
                                      ctypes.POINTER(Plan), VP]
        L.labs_full_walks.restype = I32
        L.labs_batch_workspace_bytes.argtypes = [ctypes.POINTER(Instance), I32, ctypes.POINTER(U64)]
        L.labs_batch_workspace_bytes.restype = I32
        L.labs_walks_batch.argtypes = [ctypes.POINTER(Instance), I32, VP, U64, VP]
        L.labs_walks_batch.restype = I32
        L.labs_full_batch_workspace_bytes.argtypes = [ctypes.POINTER(Instance), I32, ctypes.POINTER(U64)]
        L.labs_full_batch_workspace_bytes.restype = I32
        L.labs_full_walks_batch.argtypes = [ctypes.POINTER(Instance), I32, VP, U64, VP]
        L.labs_full_walks_batch.restype = I32
        L.labs_batch_graph_create.argtypes = [ctypes.POINTER(Instance), I32, VP, U64,
                                              ctypes.POINTER(VP)]
        L.labs_batch_graph_create.restype = I32
        L.labs_batch_graph_launch.argtypes = [VP, VP]
        L.labs_batch_graph_launch.restype = I32
        L.labs_batch_graph_destroy.argtypes = [VP]
        L.labs_batch_graph_destroy.restype = I32
        L.labs_tune_set.argtypes = [I32, I32, ctypes.c_double]
        L.labs_tune_set.restype = I32
        L.labs_tune_get.argtypes = [I32, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_double)]
        L.labs_tune_get.restype = I32
        L.labs_autotune.argtypes = [I32, I64, I64, VP, U64, VP, ctypes.POINTER(I32),
                                    ctypes.POINTER(ctypes.c_double)]
        L.labs_autotune.restype = I32
        L.labs_solve_workspace_bytes.argtypes = [I32, ctypes.POINTER(SolveCfg), ctypes.POINTER(U64)]
        L.labs_solve_workspace_bytes.restype = I32
        L.labs_solve.argtypes = [I32, ctypes.POINTER(SolveCfg), VP, U64, VP, ctypes.POINTER(SolveResult)]
        L.labs_solve.restype = I32
        L.labs_lambda_model.argtypes = [I32]
        L.labs_lambda_model.restype = ctypes.c_double
        L.labs_nses_limit.argtypes = [I32, ctypes.c_double, I32]
        L.labs_nses_limit.restype = ctypes.c_double
        L.labs_optimality_probability.argtypes = [I32, ctypes.c_double]
        L.labs_optimality_probability.restype = ctypes.c_double
        L.labs_serve_create.argtypes = [ctypes.POINTER(ServeCfg), ctypes.POINTER(VP)]
        L.labs_serve_create.restype = I32
        L.labs_serve_destroy.argtypes = [VP]
        L.labs_serve_destroy.restype = I32
        L.labs_serve_submit.argtypes = [VP, I32, I64, I64, U64, VP, ctypes.POINTER(U64)]
        L.labs_serve_submit.restype = I32
        L.labs_serve_poll.argtypes = [VP, U64, ctypes.POINTER(ServeResult)]
        L.labs_serve_poll.restype = I32
        L.labs_serve_wait.argtypes = [VP, U64, I64, ctypes.POINTER(ServeResult)]
        L.labs_serve_wait.restype = I32
        L.labs_serve_stats.argtypes = [VP, ctypes.POINTER(ServeCounters)]
        L.labs_serve_stats.restype = I32
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


def _in_use_on(stream, *tensors):
    """Tensors a call hands to the library stay reserved for the caller's stream:
    they were allocated on torch's current stream, so without this the caching
    allocator could give them to current-stream work while the kernels still run."""
    if stream is None:
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


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
    _in_use_on(stream, seqs, out)
    return out


def starts(L: int, n_walks: int, seed: int, device="cuda", stream=None):
    import torch
    out = torch.empty((n_walks, max(key_words(L), 1)), dtype=torch.int64, device=device)
    _check(lib().labs_starts(L, n_walks, seed & 0xFFFFFFFFFFFFFFFF, _dptr(out),
                             _stream_handle(stream)))
    _in_use_on(stream, out)
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
          device="cuda", cap_steps: bool = False):
    """Run n_walks self-avoiding walks; returns a dict of CUDA tensors.

    Keys: best_seq int64 [n, W] (bit patterns of the uint64 key words), best_E
    int32 [n], steps_done int64 [n], digest int64 [n] (uint64 bit patterns),
    trace_j int16 / trace_E int32 [n_trace, walk_len] when n_trace > 0, and
    cap_steps int32 [n, 4] (scans on 4, 5, 6 or all C planes) when requested.
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
    if cap_steps:
        res["cap_steps"] = torch.zeros((n_walks, 4), dtype=torch.int32, device=device)
    out = WalkOut(_dptr(res["best_seq"]), _dptr(res["best_E"]), _dptr(res["steps_done"]),
                  _dptr(res["digest"]), _dptr(res.get("trace_j")), _dptr(res.get("trace_E")),
                  n_trace, _dptr(res.get("cap_steps")))
    _check(lib().labs_walks(_dptr(starts_t), L, n_walks, walk_len, seed & 0xFFFFFFFFFFFFFFFF,
                            ctypes.byref(out), _dptr(workspace), workspace.numel(),
                            ctypes.byref(plan) if plan else None, _stream_handle(stream)))
    _in_use_on(stream, workspace, starts_t, *res.values())
    return res


NOALLOC_SCRATCH_BYTES = 64 << 20


def walks_noalloc(L: int, n_walks: int, walk_len: int, seed: int = 0, starts_t=None,
                  n_trace: int = 0, plan: Optional[Plan] = None, stream=None, device="cuda"):
    """labs_walks_noalloc: walks() without a workspace (the library's fixed
    64 MiB device array holds the visited tables).  Only the result tensors
    are allocated, here, by the caller's side; the library allocates nothing."""
    import torch
    W = key_words(L)
    if W == 0:
        raise LabsError(LABS_EINVAL, f"invalid L={L}")
    if starts_t is not None:
        if starts_t.dtype != torch.int64 or tuple(starts_t.shape) != (n_walks, W) or not starts_t.is_cuda:
            raise ValueError("starts must be an int64 CUDA tensor of shape (n_walks, W)")
        starts_t = starts_t.contiguous()
    res = {
        "best_seq": torch.empty((n_walks, W), dtype=torch.int64, device=device),
        "best_E": torch.empty(n_walks, dtype=torch.int32, device=device),
        "steps_done": torch.empty(n_walks, dtype=torch.int64, device=device),
        "digest": torch.empty(n_walks, dtype=torch.int64, device=device),
    }
    if n_trace:
        res["trace_j"] = torch.zeros((n_trace, walk_len), dtype=torch.int16, device=device)
        res["trace_E"] = torch.zeros((n_trace, walk_len), dtype=torch.int32, device=device)
    out = WalkOut(_dptr(res["best_seq"]), _dptr(res["best_E"]), _dptr(res["steps_done"]),
                  _dptr(res["digest"]), _dptr(res.get("trace_j")), _dptr(res.get("trace_E")),
                  n_trace, None)
    _check(lib().labs_walks_noalloc(_dptr(starts_t), L, n_walks, walk_len, seed & 0xFFFFFFFFFFFFFFFF,
                                    ctypes.byref(out), ctypes.byref(plan) if plan else None,
                                    _stream_handle(stream)))
    _in_use_on(stream, starts_t, *res.values())
    return res


# ------------------------------------------------------------- whole space
def full_l_max() -> int:
    return int(lib().labs_full_l_max())


def full_key_words(L: int) -> int:
    return int(lib().labs_full_key_words(L))


def full_workspace_bytes(L: int, n_walks: int, walk_len: int, plan: Optional[Plan] = None) -> int:
    b = U64(0)
    _check(lib().labs_full_walks_workspace_bytes(L, n_walks, walk_len,
                                                 ctypes.byref(plan) if plan else None, ctypes.byref(b)))
    return int(b.value)


def full_walks(L: int, n_walks: int, walk_len: int, seed: int = 0, starts_t=None, n_trace: int = 0,
               plan: Optional[Plan] = None, workspace=None, digest: bool = True, stream=None,
               device="cuda", cap_steps: bool = False):
    """Self-avoiding walks over all 2^L sequences of length L (labs_full_walks);
    returns a dict of CUDA tensors laid out as walks() does, with W = ceil(L/64)
    key words holding the whole sequence and trace_j the position flipped."""
    import torch
    W = full_key_words(L)
    if W == 0:
        raise LabsError(LABS_EINVAL, f"invalid L={L}")
    if starts_t is not None:
        if starts_t.dtype != torch.int64 or tuple(starts_t.shape) != (n_walks, W) or not starts_t.is_cuda:
            raise ValueError("starts must be an int64 CUDA tensor of shape (n_walks, W)")
        starts_t = starts_t.contiguous()
    if workspace is None:
        workspace = alloc_workspace(full_workspace_bytes(L, n_walks, walk_len, plan), device=device)
    res = {
        "best_seq": torch.empty((n_walks, W), dtype=torch.int64, device=device),
        "best_E": torch.empty(n_walks, dtype=torch.int32, device=device),
        "steps_done": torch.empty(n_walks, dtype=torch.int64, device=device),
        "digest": torch.empty(n_walks, dtype=torch.int64, device=device) if digest else None,
    }
    if n_trace:
        res["trace_j"] = torch.zeros((n_trace, walk_len), dtype=torch.int16, device=device)
        res["trace_E"] = torch.zeros((n_trace, walk_len), dtype=torch.int32, device=device)
    if cap_steps:
        res["cap_steps"] = torch.zeros((n_walks, 4), dtype=torch.int32, device=device)
    out = WalkOut(_dptr(res["best_seq"]), _dptr(res["best_E"]), _dptr(res["steps_done"]),
                  _dptr(res["digest"]), _dptr(res.get("trace_j")), _dptr(res.get("trace_E")),
                  n_trace, _dptr(res.get("cap_steps")))
    _check(lib().labs_full_walks(_dptr(starts_t), L, n_walks, walk_len, seed & 0xFFFFFFFFFFFFFFFF,
                                 ctypes.byref(out), _dptr(workspace), workspace.numel(),
                                 ctypes.byref(plan) if plan else None, _stream_handle(stream)))
    _in_use_on(stream, workspace, starts_t, *res.values())
    return res


# ----------------------------------------------------------- mixed-L batches
def _alloc_outputs(L, n_walks, walk_len, n_trace, device="cuda", cap_steps=False, full=False):
    import torch
    W = full_key_words(L) if full else key_words(L)
    res = {
        "best_seq": torch.empty((n_walks, W), dtype=torch.int64, device=device),
        "best_E": torch.empty(n_walks, dtype=torch.int32, device=device),
        "steps_done": torch.empty(n_walks, dtype=torch.int64, device=device),
        "digest": torch.empty(n_walks, dtype=torch.int64, device=device),
    }
    if n_trace:
        res["trace_j"] = torch.zeros((n_trace, walk_len), dtype=torch.int16, device=device)
        res["trace_E"] = torch.zeros((n_trace, walk_len), dtype=torch.int32, device=device)
    if cap_steps:
        res["cap_steps"] = torch.zeros((n_walks, 4), dtype=torch.int32, device=device)
    return res


def make_instances(specs, results):
    """ctypes array of labs_instance from dicts (L, n_walks, walk_len, seed, starts_t,
    lanes_per_walk, load_factor, n_trace, cap_steps) and their output tensors."""
    arr = (Instance * max(len(specs), 1))()
    for i, (sp, res) in enumerate(zip(specs, results)):
        st = sp.get("starts_t")
        out = WalkOut(_dptr(res["best_seq"]), _dptr(res["best_E"]), _dptr(res["steps_done"]),
                      _dptr(res["digest"]), _dptr(res.get("trace_j")), _dptr(res.get("trace_E")),
                      int(sp.get("n_trace", 0)), _dptr(res.get("cap_steps")))
        arr[i] = Instance(int(sp["L"]), int(sp.get("lanes_per_walk", 0)), int(sp["n_walks"]),
                          int(sp["walk_len"]), int(sp.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF,
                          _dptr(st), float(sp.get("load_factor", 0.0)), out)
    return arr


def batch_workspace_bytes(specs, results=None) -> int:
    """labs_batch_workspace_bytes for the instances (output buffers of their
    size are allocated for the call when results is None)."""
    results = results or [_alloc_outputs(sp["L"], sp["n_walks"], 0, 0) for sp in specs]
    arr = make_instances(specs, results)
    b = U64(0)
    _check(lib().labs_batch_workspace_bytes(arr, len(specs), ctypes.byref(b)))
    return int(b.value)


def walks_batch(specs, workspace=None, stream=None, device="cuda"):
    """Run several instances (list of dicts, see make_instances) in one launch.
    Returns one result dict per instance, like walks()."""
    results = [_alloc_outputs(sp["L"], sp["n_walks"], sp["walk_len"], sp.get("n_trace", 0), device,
                              sp.get("cap_steps", False))
               for sp in specs]
    arr = make_instances(specs, results)
    if workspace is None:
        b = U64(0)
        _check(lib().labs_batch_workspace_bytes(arr, len(specs), ctypes.byref(b)))
        workspace = alloc_workspace(b.value, device=device)
    _check(lib().labs_walks_batch(arr, len(specs), _dptr(workspace), workspace.numel(),
                                  _stream_handle(stream)))
    _in_use_on(stream, workspace, *[t for r in results for t in r.values()],
               *[sp.get("starts_t") for sp in specs])
    return results


def full_batch_workspace_bytes(specs, results=None) -> int:
    """labs_full_batch_workspace_bytes for whole-space instances (as
    batch_workspace_bytes)."""
    results = results or [_alloc_outputs(sp["L"], sp["n_walks"], 0, 0, full=True) for sp in specs]
    arr = make_instances(specs, results)
    b = U64(0)
    _check(lib().labs_full_batch_workspace_bytes(arr, len(specs), ctypes.byref(b)))
    return int(b.value)


def full_walks_batch(specs, workspace=None, stream=None, device="cuda"):
    """Whole-space instances (list of dicts as for walks_batch, L in [3, 255])
    in persistent launches (labs_full_walks_batch).  Returns one result dict
    per instance, like full_walks()."""
    results = [_alloc_outputs(sp["L"], sp["n_walks"], sp["walk_len"], sp.get("n_trace", 0), device,
                              sp.get("cap_steps", False), full=True)
               for sp in specs]
    arr = make_instances(specs, results)
    if workspace is None:
        b = U64(0)
        _check(lib().labs_full_batch_workspace_bytes(arr, len(specs), ctypes.byref(b)))
        workspace = alloc_workspace(b.value, device=device)
    _check(lib().labs_full_walks_batch(arr, len(specs), _dptr(workspace), workspace.numel(),
                                       _stream_handle(stream)))
    _in_use_on(stream, workspace, *[t for r in results for t in r.values()],
               *[sp.get("starts_t") for sp in specs])
    return results


class BatchGraph:
    """hipGraph of one mixed-L batch: create once, replay with launch()."""

    def __init__(self, specs, workspace=None, device="cuda"):
        self.specs = specs
        self.results = [_alloc_outputs(sp["L"], sp["n_walks"], sp["walk_len"], sp.get("n_trace", 0),
                                       device, sp.get("cap_steps", False)) for sp in specs]
        self._arr = make_instances(specs, self.results)
        if workspace is None:
            b = U64(0)
            _check(lib().labs_batch_workspace_bytes(self._arr, len(specs), ctypes.byref(b)))
            workspace = alloc_workspace(b.value, device=device)
        self.workspace = workspace
        h = VP()
        _check(lib().labs_batch_graph_create(self._arr, len(specs), _dptr(workspace),
                                             workspace.numel(), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().labs_batch_graph_launch(self._h, _stream_handle(stream)))
        return self.results

    def close(self):
        if self._h:
            lib().labs_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_set(L: int, lanes_per_walk: int, load_factor: float):
    _check(lib().labs_tune_set(L, lanes_per_walk, load_factor))


def tune_get(L: int):
    g, lf = I32(0), ctypes.c_double(0)
    rc = lib().labs_tune_get(L, ctypes.byref(g), ctypes.byref(lf))
    if rc not in (LABS_OK, LABS_ENOTFOUND):
        _check(rc)
    return int(g.value), float(lf.value), rc == LABS_OK


def save_tuning(path: str):
    """Write the per-L tuning table (every odd L with an entry) as JSON:
    {"L": {"lanes_per_walk": G, "load_factor": a}}."""
    import json
    table = {}
    for L in range(3, l_max() + 1, 2):
        g, lf, found = tune_get(L)
        if found:
            table[str(L)] = {"lanes_per_walk": g, "load_factor": lf}
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    return table


def load_tuning(path: str) -> int:
    """Enter every entry of a JSON table written by save_tuning; returns the count."""
    import json
    with open(path) as f:
        table = json.load(f)
    for L, e in table.items():
        tune_set(int(L), int(e["lanes_per_walk"]), float(e["load_factor"]))
    return len(table)


def autotune(L: int, n_walks: int = 131072, walk_len: int = 512, stream=None, device="cuda"):
    """Time lanes per walk / load factor for L on a short run; stores and returns the best.

    The run must fill the GPU at every candidate lane count (131,072 walks do
    at 2 lanes per walk), otherwise it measures fill rather than cost per step.
    """
    W = key_words(L)
    need = workspace_bytes(L, n_walks, walk_len, make_plan(2, 0.5)) + \
        ((n_walks * (8 * W + 12) + 255) // 256) * 256
    ws = alloc_workspace(need, device=device)
    g, lf = I32(0), ctypes.c_double(0)
    _check(lib().labs_autotune(L, n_walks, walk_len, _dptr(ws), ws.numel(), _stream_handle(stream),
                               ctypes.byref(g), ctypes.byref(lf)))
    return int(g.value), float(lf.value)


class Server:
    """Continuous-batching walk server (labs_serve_* in include/labs.h).

    submit() queues one request and returns its id; poll()/wait() return None
    while it runs and a dict of host arrays (best_seq, best_E, steps_done,
    digest) plus submit/admit/done times once it is done.  whole_space=True
    makes a server of whole-space requests (keys as for full_walks).
    """

    def __init__(self, pool_bytes: int = 0, max_pending: int = 0, lanes_per_walk: int = 0,
                 chunk_steps: int = 0, load_factor: float = 0.0, whole_space: bool = False):
        cfg = ServeCfg(pool_bytes, max_pending, lanes_per_walk, chunk_steps, load_factor,
                       1 if whole_space else 0)
        h = VP()
        _check(lib().labs_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._shape = {}
        self._key_words = full_key_words if whole_space else key_words

    def submit(self, L: int, n_walks: int, walk_len: int, seed: int = 0, starts=None) -> int:
        st = None
        if starts is not None:
            st = np.ascontiguousarray(np.asarray(starts, dtype=np.uint64).reshape(n_walks, self._key_words(L)))
        rid = U64(0)
        _check(lib().labs_serve_submit(self._h, L, n_walks, walk_len, seed,
                                       None if st is None else st.ctypes.data, ctypes.byref(rid)))
        self._shape[rid.value] = (L, n_walks)
        return int(rid.value)

    def _result(self, rid, call):
        L, n = self._shape.get(rid, (3, 0))      # unknown ids: the library reports them
        W = self._key_words(L)
        out = dict(best_seq=np.zeros((n, W), np.uint64), best_E=np.zeros(n, np.int32),
                   steps_done=np.zeros(n, np.int64), digest=np.zeros(n, np.uint64))
        res = ServeResult(out["best_seq"].ctypes.data, out["best_E"].ctypes.data,
                          out["steps_done"].ctypes.data, out["digest"].ctypes.data, 0, 0, 0, 0)
        rc = _check(call(ctypes.byref(res)))
        if rc == LABS_PENDING:
            return None
        self._shape.pop(rid, None)
        out.update(t_submit_ns=res.t_submit_ns, t_admit_ns=res.t_admit_ns, t_done_ns=res.t_done_ns,
                   total_steps=res.total_steps)
        return out

    def poll(self, rid: int):
        return self._result(rid, lambda r: lib().labs_serve_poll(self._h, rid, r))

    def wait(self, rid: int, timeout_s: Optional[float] = None):
        t = -1 if timeout_s is None else int(timeout_s * 1e9)
        return self._result(rid, lambda r: lib().labs_serve_wait(self._h, rid, t, r))

    def stats(self) -> dict:
        c = ServeCounters()
        _check(lib().labs_serve_stats(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in ServeCounters._fields_}

    def close(self):
        if self._h:
            lib().labs_serve_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------ solver and stopping model
def solve(L: int, walks_per_round: int, walk_len: int = 0, seed: int = 0, time_limit_s: float = 0.0,
          nses_limit: float = 0.0, target_E: int = 0, max_rounds: int = 0,
          plan: Optional[Plan] = None, workspace=None, stream=None, device="cuda",
          first_round: int = 0) -> dict:
    """Alg. 1: rounds of walks_per_round fresh walks until a stopping condition
    holds (labs_solve).  walk_len 0 = 8 D.  first_round > 0 resumes a run that
    stopped after that many rounds.  Returns the global best and counts."""
    cfg = SolveCfg(walks_per_round, walk_len, seed & 0xFFFFFFFFFFFFFFFF, time_limit_s, nses_limit,
                   target_E, 0, max_rounds, plan if plan is not None else Plan(0, 0.0, 0),
                   first_round)
    if workspace is None:
        nb = U64(0)
        _check(lib().labs_solve_workspace_bytes(L, ctypes.byref(cfg), ctypes.byref(nb)))
        workspace = alloc_workspace(nb.value, device=device)
    res = SolveResult()
    _check(lib().labs_solve(L, ctypes.byref(cfg), _dptr(workspace), workspace.numel(),
                            _stream_handle(stream), ctypes.byref(res)))
    W = key_words(L)
    return {"best_E": res.best_E, "best_seq": np.array(res.best_seq[:W], dtype=np.uint64),
            "rounds": res.rounds, "nfes": res.nfes, "walk_steps": res.walk_steps,
            "seconds": res.seconds, "reached_target": bool(res.reached_target),
            "target_seconds": res.target_seconds, "target_nfes": res.target_nfes}


def lambda_model(L: int) -> float:
    return lib().labs_lambda_model(L)


def nses_limit(L: int, P: float = 0.99, N: int = 100) -> float:
    return lib().labs_nses_limit(L, P, N)


def optimality_probability(L: int, nses_total: float) -> float:
    return lib().labs_optimality_probability(L, nses_total)
