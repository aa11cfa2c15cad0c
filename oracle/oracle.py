"""CPU oracle for the skew-symmetric LABS self-avoiding walk -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It wraps ``liblabs_oracle.so`` (built from
``labs_oracle.cpp`` with g++) through ctypes and adds the paper's I/O
conventions.  It shares no code with the GPU library.

Functions and the passage each follows (Boskovic, Herzog & Brest, arXiv
2210.15962):

* ``energy(s)``             -- Eq. 1, direct O(L^2) sum of squared C_k.
* ``expand_skew(x, L)``     -- Eq. 2, skew-symmetric expansion of D free bits.
* ``merit_factor(L, E)``    -- Eq. 1, F = L^2 / (2E).
* ``walk(...)`` / ``walks`` -- Eq. 3 (self-avoiding walk) and Alg. 2 (walk
  length counts moves, best tracked with strict "<" from the first pivot).
* ``bruteforce(L)``         -- exhaustive enumeration of all 2^D skew sequences.
* ``starts(L, n, seed)``    -- seeded uniform +-1 first pivots (Eq. 3 draws them
  uniformly; the generator is SplitMix64).
* ``decode_table_hex(hex, L)`` -- Sec. 4.2 / Table 1 hexadecimal code of the
  first half of a sequence (first free bit = most significant of D bits).
* ``nses_limit`` / ``optimality_probability`` -- Eq. 6 and Eq. 7 with the
  lambda model of Sec. 4.1.
* ``full_walk`` / ``full_walks`` / ``full_starts`` / ``full_bruteforce`` --
  the whole search space (the sokol_full solver of Sec. 5's future work):
  the same walk rules (Eq. 3, Alg. 2) over all 2^L sequences of any length L,
  a neighbour negating one of the L positions, energies from Eq. 1.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "labs_oracle.cpp")
_LIB = os.path.join(_HERE, "liblabs_oracle.so")

U64 = ctypes.c_uint64
I64 = ctypes.c_int64
I32 = ctypes.c_int32
P = ctypes.c_void_p


def build_library(force: bool = False) -> str:
    """Compile ``liblabs_oracle.so`` with g++ (portable x86-64-v3 code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-march=x86-64-v3", "-std=c++17", "-fPIC", "-shared",
               "-pthread", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build_library()
        L = ctypes.CDLL(path)
        L.orc_l_max.restype = I32
        L.orc_energy.argtypes = [P, I32]
        L.orc_energy.restype = I64
        L.orc_expand_skew.argtypes = [P, I32, P]
        L.orc_expand_skew.restype = I32
        L.orc_energy_packed.argtypes = [P, I32]
        L.orc_energy_packed.restype = I64
        L.orc_mix64.argtypes = [U64]
        L.orc_mix64.restype = U64
        L.orc_starts.argtypes = [I32, I64, U64, P]
        L.orc_starts.restype = I32
        L.orc_walk.argtypes = [I32, P, I64, P, P, P, P, P, P]
        L.orc_walk.restype = I32
        L.orc_walks.argtypes = [I32, P, I64, I64, P, P, P, P, I32]
        L.orc_walks.restype = I32
        L.orc_bruteforce.argtypes = [I32, P, P, P, P]
        L.orc_bruteforce.restype = I32
        L.orc_full_l_max.restype = I32
        L.orc_full_starts.argtypes = [I32, I64, U64, P]
        L.orc_full_starts.restype = I32
        L.orc_full_energy_packed.argtypes = [P, I32]
        L.orc_full_energy_packed.restype = I64
        L.orc_full_walk.argtypes = [I32, P, I64, P, P, P, P, P, P]
        L.orc_full_walk.restype = I32
        L.orc_full_walks.argtypes = [I32, P, I64, I64, P, P, P, P, I32]
        L.orc_full_walks.restype = I32
        L.orc_full_bruteforce.argtypes = [I32, P, P, P, P]
        L.orc_full_bruteforce.restype = I32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def free_bits(L: int) -> int:
    return (L + 1) // 2


def key_words(L: int) -> int:
    return (free_bits(L) + 63) // 64


def l_max() -> int:
    return int(lib().orc_l_max())


def energy(s) -> int:
    """Eq. 1 energy of one full +-1 sequence."""
    a = np.ascontiguousarray(np.asarray(s, dtype=np.int8))
    e = lib().orc_energy(_ptr(a), int(a.size))
    if e < 0:
        raise ValueError("invalid sequence")
    return int(e)


def expand_skew(x, L: int) -> np.ndarray:
    """Eq. 2: full sequence (int8 +-1, length L) from D free bits."""
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.int8))
    if xa.size != free_bits(L):
        raise ValueError("need D=(L+1)/2 free bits")
    s = np.zeros(L, dtype=np.int8)
    if lib().orc_expand_skew(_ptr(xa), L, _ptr(s)) != 0:
        raise ValueError("invalid L")
    return s


def energy_packed(key, L: int) -> int:
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64).reshape(-1))
    if k.size < key_words(L):
        raise ValueError("key too short")
    e = lib().orc_energy_packed(_ptr(k), L)
    if e < 0:
        raise ValueError("invalid L")
    return int(e)


def merit_factor(L: int, E: int) -> float:
    return L * L / (2.0 * E)


def mix64(z: int) -> int:
    return int(lib().orc_mix64(z & 0xFFFFFFFFFFFFFFFF))


def starts(L: int, n_walks: int, seed: int) -> np.ndarray:
    out = np.zeros((n_walks, key_words(L)), dtype=np.uint64)
    if lib().orc_starts(L, n_walks, seed & 0xFFFFFFFFFFFFFFFF, _ptr(out)) != 0:
        raise ValueError("invalid arguments")
    return out


def pack(x) -> np.ndarray:
    """Pack +-1 free bits into the key layout (bit j-1 = x_j, 1 means -1)."""
    xa = np.asarray(x, dtype=np.int8).reshape(-1)
    D = xa.size
    W = (D + 63) // 64
    out = np.zeros(W, dtype=np.uint64)
    for j in range(D):
        if xa[j] < 0:
            out[j // 64] |= np.uint64(1) << np.uint64(j % 64)
    return out


def unpack(key, L: int) -> np.ndarray:
    D = free_bits(L)
    k = np.asarray(key, dtype=np.uint64).reshape(-1)
    x = np.ones(D, dtype=np.int8)
    for j in range(D):
        if (int(k[j // 64]) >> (j % 64)) & 1:
            x[j] = -1
    return x


class WalkResult:
    __slots__ = ("best_E", "best_seq", "steps", "digest", "trace_j", "trace_E")

    def __init__(self, best_E, best_seq, steps, digest, trace_j=None, trace_E=None):
        self.best_E = best_E
        self.best_seq = best_seq
        self.steps = steps
        self.digest = digest
        self.trace_j = trace_j
        self.trace_E = trace_E


def walk(L: int, start, walk_len: int, trace: bool = True) -> WalkResult:
    """One self-avoiding walk (Eq. 3 / Alg. 2) from a packed start key."""
    W = key_words(L)
    st = np.ascontiguousarray(np.asarray(start, dtype=np.uint64).reshape(-1)[:W])
    bE = np.zeros(1, dtype=np.int64)
    bs = np.zeros(W, dtype=np.uint64)
    sd = np.zeros(1, dtype=np.int64)
    dg = np.zeros(1, dtype=np.uint64)
    tj = np.zeros(max(walk_len, 1), dtype=np.int16) if trace else None
    tE = np.zeros(max(walk_len, 1), dtype=np.int32) if trace else None
    rc = lib().orc_walk(L, _ptr(st), walk_len, _ptr(bE), _ptr(bs), _ptr(sd), _ptr(dg),
                        _ptr(tj) if trace else None, _ptr(tE) if trace else None)
    if rc != 0:
        raise ValueError("invalid walk arguments")
    steps = int(sd[0])
    return WalkResult(int(bE[0]), bs, steps, int(dg[0]),
                      tj[:steps].copy() if trace else None,
                      tE[:steps].copy() if trace else None)


def walks(L: int, starts_arr: np.ndarray, walk_len: int, n_threads: Optional[int] = None):
    """Independent walks (Eq. 4) over host threads.  Returns a dict of arrays."""
    W = key_words(L)
    st = np.ascontiguousarray(np.asarray(starts_arr, dtype=np.uint64).reshape(-1, W))
    n = st.shape[0]
    bE = np.zeros(n, dtype=np.int64)
    bs = np.zeros((n, W), dtype=np.uint64)
    sd = np.zeros(n, dtype=np.int64)
    dg = np.zeros(n, dtype=np.uint64)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    rc = lib().orc_walks(L, _ptr(st), n, walk_len, _ptr(bE), _ptr(bs), _ptr(sd), _ptr(dg),
                         int(n_threads))
    if rc != 0:
        raise ValueError("invalid walk arguments")
    return {"best_E": bE, "best_seq": bs, "steps_done": sd, "digest": dg}


def bruteforce(L: int):
    """(min E, number of minimisers, first minimiser key, sum of all E)."""
    mn = np.zeros(1, dtype=np.int64)
    cnt = np.zeros(1, dtype=np.int64)
    first = np.zeros(1, dtype=np.uint64)
    tot = np.zeros(1, dtype=np.int64)
    if lib().orc_bruteforce(L, _ptr(mn), _ptr(cnt), _ptr(first), _ptr(tot)) != 0:
        raise ValueError("L out of brute-force range")
    return int(mn[0]), int(cnt[0]), int(first[0]), int(tot[0])


def decode_table_hex(code: str, L: int) -> np.ndarray:
    """Free bits (+-1) from the hexadecimal code used in Table 1.

    Sec. 4.2 codes the first half of the sequence in hexadecimal, one nibble per
    four bits, leading zeros dropped down to D bits.  The bit string is read
    most-significant first: its first bit is x_1.  0 maps to +1 and 1 to -1 (the
    opposite mapping gives the negated sequence, which has the same energy).
    """
    D = free_bits(L)
    v = int(code, 16)
    if v >> D:
        raise ValueError("code wider than D bits")
    bits = [(v >> (D - 1 - i)) & 1 for i in range(D)]
    return np.array([-1 if b else 1 for b in bits], dtype=np.int8)


# Sec. 4.1: lambda(L) = 0.006753 * 0.8617^L (rate of the exponential law of
# the number of solution evaluations needed to reach the optimum).
LAMBDA_A = 0.006753
LAMBDA_B = 0.8617


def lambda_model(L: int) -> float:
    return LAMBDA_A * LAMBDA_B ** L


def nses_limit(L: int, P: float = 0.99, N: int = 100) -> float:
    """Eq. 6: evaluations per run so that N runs reach the optimum with prob. P."""
    return math.log(1.0 - P) / (-lambda_model(L) * N)


def optimality_probability(L: int, nses_total: float) -> float:
    """Eq. 7: P(S_best) = 1 - exp(-lambda * sum of NSEs over the runs)."""
    return 1.0 - math.exp(-lambda_model(L) * nses_total)


# ---- the whole search space --------------------------------------------------

def full_key_words(L: int) -> int:
    return (L + 63) // 64


def full_l_max() -> int:
    return int(lib().orc_full_l_max())


def full_starts(L: int, n_walks: int, seed: int) -> np.ndarray:
    """Seeded uniform whole sequences: W = ceil(L/64) words per walk."""
    out = np.zeros((n_walks, full_key_words(L)), dtype=np.uint64)
    if lib().orc_full_starts(L, n_walks, seed & 0xFFFFFFFFFFFFFFFF, _ptr(out)) != 0:
        raise ValueError("invalid arguments")
    return out


def full_energy_packed(key, L: int) -> int:
    """Eq. 1 energy of a packed whole sequence (bit i-1 = s_i, 1 means -1)."""
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64).reshape(-1))
    if k.size < full_key_words(L):
        raise ValueError("key too short")
    e = lib().orc_full_energy_packed(_ptr(k), L)
    if e < 0:
        raise ValueError("invalid L")
    return int(e)


def full_pack(s) -> np.ndarray:
    """Pack a +-1 sequence (bit i-1 = s_i, 1 means -1)."""
    return pack(s)


def full_unpack(key, L: int) -> np.ndarray:
    k = np.asarray(key, dtype=np.uint64).reshape(-1)
    s = np.ones(L, dtype=np.int8)
    for i in range(L):
        if (int(k[i // 64]) >> (i % 64)) & 1:
            s[i] = -1
    return s


def full_walk(L: int, start, walk_len: int, trace: bool = True) -> WalkResult:
    """One self-avoiding walk over the whole space from a packed sequence."""
    W = full_key_words(L)
    st = np.ascontiguousarray(np.asarray(start, dtype=np.uint64).reshape(-1)[:W])
    bE = np.zeros(1, dtype=np.int64)
    bs = np.zeros(W, dtype=np.uint64)
    sd = np.zeros(1, dtype=np.int64)
    dg = np.zeros(1, dtype=np.uint64)
    tj = np.zeros(max(walk_len, 1), dtype=np.int16) if trace else None
    tE = np.zeros(max(walk_len, 1), dtype=np.int32) if trace else None
    rc = lib().orc_full_walk(L, _ptr(st), walk_len, _ptr(bE), _ptr(bs), _ptr(sd), _ptr(dg),
                             _ptr(tj) if trace else None, _ptr(tE) if trace else None)
    if rc != 0:
        raise ValueError("invalid walk arguments")
    steps = int(sd[0])
    return WalkResult(int(bE[0]), bs, steps, int(dg[0]),
                      tj[:steps].copy() if trace else None,
                      tE[:steps].copy() if trace else None)


def full_walks(L: int, starts_arr: np.ndarray, walk_len: int, n_threads: Optional[int] = None):
    """Independent whole-space walks over host threads.  Returns a dict of arrays."""
    W = full_key_words(L)
    st = np.ascontiguousarray(np.asarray(starts_arr, dtype=np.uint64).reshape(-1, W))
    n = st.shape[0]
    bE = np.zeros(n, dtype=np.int64)
    bs = np.zeros((n, W), dtype=np.uint64)
    sd = np.zeros(n, dtype=np.int64)
    dg = np.zeros(n, dtype=np.uint64)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    rc = lib().orc_full_walks(L, _ptr(st), n, walk_len, _ptr(bE), _ptr(bs), _ptr(sd), _ptr(dg),
                              int(n_threads))
    if rc != 0:
        raise ValueError("invalid walk arguments")
    return {"best_E": bE, "best_seq": bs, "steps_done": sd, "digest": dg}


def full_bruteforce(L: int):
    """All 2^L sequences: (min E, number of minimisers, first minimiser, sum of all E)."""
    mn = np.zeros(1, dtype=np.int64)
    cnt = np.zeros(1, dtype=np.int64)
    first = np.zeros(1, dtype=np.uint64)
    tot = np.zeros(1, dtype=np.int64)
    if lib().orc_full_bruteforce(L, _ptr(mn), _ptr(cnt), _ptr(first), _ptr(tot)) != 0:
        raise ValueError("L out of brute-force range")
    return int(mn[0]), int(cnt[0]), int(first[0]), int(tot[0])
