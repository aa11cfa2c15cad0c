"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws random numbers only; it contains none of the method's
arithmetic (no energies, no walks).  Both the GPU path and the CPU oracle are
fed from here, so a parity test compares the two on identical inputs.

Workload shapes follow the paper: first pivots are uniform i.i.d. +-1 free
bits (Eq. 3); lengths are odd (Eq. 2 defines the skew-symmetric space for odd
L only).
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def free_bits(L: int) -> int:
    return (L + 1) // 2


def key_words(L: int) -> int:
    return (free_bits(L) + 63) // 64


def random_pm1(n: int, L: int, seed: int) -> np.ndarray:
    """n uniform +-1 sequences of length L (int8 [n, L])."""
    b = _rng(seed).integers(0, 2, size=(n, L), dtype=np.int8)
    return (1 - 2 * b).astype(np.int8)


def random_start_keys(L: int, n: int, seed: int) -> np.ndarray:
    """n uniform packed skew-symmetric start keys (uint64 [n, W], bits above D zero)."""
    D, W = free_bits(L), key_words(L)
    words = _rng(seed).integers(0, 2**63, size=(n, W), dtype=np.int64).astype(np.uint64)
    words |= _rng(seed + 1).integers(0, 2, size=(n, W), dtype=np.int64).astype(np.uint64) << np.uint64(63)
    for t in range(W):
        bits = D - 64 * t
        if bits < 64:
            words[:, t] &= np.uint64((1 << bits) - 1)
    return words


def random_full_keys(L: int, n: int, seed: int) -> np.ndarray:
    """n uniform packed whole sequences of length L (uint64 [n, ceil(L/64)], bits above L zero)."""
    W = (L + 63) // 64
    words = _rng(seed).integers(0, 2**63, size=(n, W), dtype=np.int64).astype(np.uint64)
    words |= _rng(seed + 1).integers(0, 2, size=(n, W), dtype=np.int64).astype(np.uint64) << np.uint64(63)
    for t in range(W):
        bits = L - 64 * t
        if bits < 64:
            words[:, t] &= np.uint64((1 << bits) - 1)
    return words


def odd_lengths(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """n odd lengths drawn uniformly from {lo, lo+2, ..., hi} (lo, hi odd)."""
    k = (hi - lo) // 2 + 1
    return lo + 2 * _rng(seed).integers(0, k, size=n)


def lengths(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """n lengths drawn uniformly from {lo, lo+1, ..., hi}."""
    return lo + _rng(seed).integers(0, hi - lo + 1, size=n)


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of n requests of a Poisson process of the given rate."""
    u = _rng(seed).random(n)
    return np.cumsum(-np.log1p(-u) / rate)


def sample_indices(n_total: int, n_first: int, n_random: int, seed: int) -> np.ndarray:
    """Walk indices to spot-check: the first n_first plus n_random seeded others."""
    first = np.arange(min(n_first, n_total))
    rest = np.arange(len(first), n_total)
    if len(rest) and n_random:
        pick = _rng(seed).choice(rest, size=min(n_random, len(rest)), replace=False)
        return np.concatenate([first, np.sort(pick)])
    return first


def as_int64_keys(keys: np.ndarray) -> np.ndarray:
    """uint64 key words reinterpreted as int64 (the dtype torch tensors carry)."""
    return np.ascontiguousarray(keys, dtype=np.uint64).view(np.int64)
