"""Pins of the whole-space oracle (the sokol_full solver of Sec. 5's future
work): the walk of Eq. 3 / Alg. 2 over all 2^L sequences of any length L, a
neighbour negating one of the L positions.

Each test checks the oracle against something other than itself: a walk
derived by hand, Barker codes (textbook sequences whose every |C_k| <= 1),
the lower bound E >= floor(L/2) (a lag with L - k odd has an odd C_k), the
closed form of the mean energy, numpy.correlate, invariants of Eq. 1 under
negation and alternation, and an independent step-by-step re-check of walks
from the definition.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
import labs_inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

BARKER = {
    3: [1, 1, -1],
    4: [1, 1, -1, 1],
    5: [1, 1, 1, -1, 1],
    7: [1, 1, 1, -1, -1, 1, -1],
    11: [1, 1, 1, -1, -1, -1, 1, -1, -1, 1, -1],
    13: [1, 1, 1, 1, 1, -1, -1, 1, 1, -1, 1, -1, 1],
}


def np_energy(s) -> int:
    """Eq. 1 via numpy.correlate (independent of the oracle's loops)."""
    s = np.asarray(s, dtype=np.int64)
    r = np.correlate(s, s, mode="full")[len(s):]
    return int(np.sum(r * r))


def pack(s) -> np.ndarray:
    s = np.asarray(s).reshape(-1)
    out = np.zeros((len(s) + 63) // 64, dtype=np.uint64)
    for i, v in enumerate(s):
        if v < 0:
            out[i // 64] |= np.uint64(1) << np.uint64(i % 64)
    return out


def unpack(key, L):
    k = np.asarray(key, dtype=np.uint64).reshape(-1)
    return np.array([-1 if (int(k[i // 64]) >> (i % 64)) & 1 else 1 for i in range(L)], dtype=np.int8)


def test_walk_L3_by_hand():
    rows = [tuple(map(int, l.split())) for l in open(os.path.join(GOLDEN, "full_walk_L3_by_hand.txt"))
            if l.strip() and not l.startswith("#")]
    r = O.full_walk(3, pack([1, 1, 1]), 100)
    assert r.steps == len(rows) == 7                    # trapped after visiting all 8 states
    assert list(r.trace_j) == [j for _, j, _ in rows]
    assert list(r.trace_E) == [e for _, _, e in rows]
    assert r.best_E == 1 and int(r.best_seq[0]) == 0b001   # first pivot with E = 1: -++


@pytest.mark.parametrize("L", sorted(BARKER))
def test_barker_lengths_attain_the_lower_bound(L):
    # E >= floor(L/2): C_k is odd whenever L - k is odd.  Barker codes attain it,
    # so the exhaustive minimum at a Barker length is exactly floor(L/2).
    assert O.full_energy_packed(pack(BARKER[L]), L) == L // 2 == np_energy(BARKER[L])
    mn, cnt, first, total = O.full_bruteforce(L)
    assert mn == L // 2
    assert O.full_energy_packed(np.array([first], dtype=np.uint64), L) == mn


@pytest.mark.parametrize("L", [6, 8, 9, 10, 12, 14])
def test_no_barker_code_at_other_lengths(L):
    # No Barker sequence exists at these lengths, so the minimum exceeds the bound.
    mn, cnt, first, total = O.full_bruteforce(L)
    assert mn > L // 2
    assert np_energy(unpack([first], L)) == mn


@pytest.mark.parametrize("L", [3, 6, 9, 12, 15])
def test_mean_energy_closed_form(L):
    # E[C_k^2] = L - k for uniform +-1 sequences: sum over 2^L sequences is
    # 2^L * L (L - 1) / 2.
    mn, cnt, first, total = O.full_bruteforce(L)
    assert total == (1 << L) * L * (L - 1) // 2


@pytest.mark.parametrize("L", [3, 4, 7, 8, 10])
def test_bruteforce_against_numpy_enumeration(L):
    Es = []
    for v in range(1 << L):
        s = np.array([-1 if (v >> i) & 1 else 1 for i in range(L)])
        Es.append(np_energy(s))
    Es = np.array(Es)
    mn, cnt, first, total = O.full_bruteforce(L)
    assert mn == Es.min() and cnt == int((Es == mn).sum())
    assert first == int(np.argmax(Es == mn)) and total == int(Es.sum())


@pytest.mark.parametrize("L", [5, 16, 33, 64, 65, 100, 128, 129, 192, 193, 247, 255])
def test_energy_packed_matches_numpy(L):
    for key in I.random_full_keys(L, 4, seed=L):
        s = unpack(key, L)
        E = O.full_energy_packed(key, L)
        assert E == np_energy(s)
        assert E % 4 == (L // 2) % 4                    # odd C_k^2 = 1 (mod 8), even = 0 (mod 4)
        alt = np.array([(-1) ** i for i in range(L)], dtype=np.int8)
        assert O.full_energy_packed(pack(-s), L) == E
        assert O.full_energy_packed(pack(alt * s), L) == E
        assert O.full_energy_packed(pack(s[::-1]), L) == E


def test_starts_layout_and_mask():
    for L in (3, 64, 65, 127, 128, 129, 192, 193, 255):
        st = O.full_starts(L, 5, seed=7)
        W = (L + 63) // 64
        assert st.shape == (5, W)
        for w in range(5):
            for t in range(W):
                v = O.mix64((7 + 0x9E3779B97F4A7C15 * (w * W + t + 1)) & 0xFFFFFFFFFFFFFFFF)
                bits = L - 64 * t
                if bits < 64:
                    v &= (1 << bits) - 1
                assert int(st[w, t]) == v


def check_full_walk(L, start, walk_len, r):
    """Independent re-check of a whole-space walk from the definition."""
    s = unpack(start, L)
    visited = {tuple(s)}
    E = np_energy(s)
    best, best_s, h = E, s.copy(), 0
    for t in range(r.steps):
        cand = []
        for i in range(L):
            y = s.copy()
            y[i] = -y[i]
            if tuple(y) not in visited:
                cand.append((np_energy(y), i + 1))
        assert cand, "moved although every neighbour was visited"
        e_min, i_min = min(cand)
        assert r.trace_j[t] == i_min and r.trace_E[t] == e_min
        assert (e_min - E) % 4 == 0                       # every C_k changes by 0, +-2 or +-4
        s[i_min - 1] = -s[i_min - 1]
        visited.add(tuple(s))
        E = e_min
        if E < best:
            best, best_s = E, s.copy()
        h = O.mix64(h ^ ((i_min << 32) | (E & 0xFFFFFFFF)))
    if r.steps < walk_len:
        for i in range(L):
            y = s.copy()
            y[i] = -y[i]
            assert tuple(y) in visited
    assert r.best_E == best and np.array_equal(unpack(r.best_seq, L), best_s)
    assert r.digest == O.mix64(h ^ r.steps)
    assert len(visited) == r.steps + 1


@pytest.mark.parametrize("L,walk_len,n", [(4, 40, 4), (6, 100, 3), (9, 200, 3), (20, 200, 2),
                                          (33, 120, 2), (64, 60, 1), (70, 50, 1), (200, 8, 1),
                                          (255, 6, 1)])
def test_walk_semantics(L, walk_len, n):
    for start in I.random_full_keys(L, n, seed=200 + L):
        r = O.full_walk(L, start, walk_len)
        check_full_walk(L, start, walk_len, r)


def test_walk_traps_at_small_L():
    for L in (3, 4, 5):
        for start in I.random_full_keys(L, 4, seed=L):
            r = O.full_walk(L, start, 200)
            assert r.steps < (1 << L)
            check_full_walk(L, start, 200, r)


@pytest.mark.parametrize("L", [16, 27, 50, 101])
def test_walk_metamorphic_symmetries(L):
    # Negation and alternation (s_i -> (-1)^i s_i) keep every energy and map
    # position i to position i, so the traces are identical.
    alt = np.array([(-1) ** i for i in range(L)], dtype=np.int8)
    for start in I.random_full_keys(L, 2, seed=L + 1):
        s = unpack(start, L)
        ref = O.full_walk(L, start, 150)
        for y in (-s, alt * s, -alt * s):
            r = O.full_walk(L, pack(y), 150)
            assert np.array_equal(r.trace_j, ref.trace_j) and np.array_equal(r.trace_E, ref.trace_E)
            assert r.best_E == ref.best_E and r.digest == ref.digest


def test_skew_start_walks_the_whole_space():
    # A skew-symmetric start (Eq. 2) is an ordinary point of the whole space:
    # same energy as in the skew oracle, and no walk goes below the
    # exhaustive minimum, which is at most the skew minimum.
    L = 13
    mn = O.full_bruteforce(L)[0]
    assert mn <= O.bruteforce(L)[0]
    for key in I.random_start_keys(L, 4, seed=5):
        s = O.expand_skew(O.unpack(key, L), L)
        assert O.full_energy_packed(pack(s), L) == O.energy_packed(key, L)
        r = O.full_walk(L, pack(s), 300)
        assert r.best_E >= mn


def test_walks_threads_agree_with_single_walk():
    L = 57
    st = I.random_full_keys(L, 5, seed=13)
    res = O.full_walks(L, st, 200, n_threads=3)
    for i in range(5):
        r = O.full_walk(L, st[i], 200, trace=False)
        assert res["best_E"][i] == r.best_E and res["digest"][i] == r.digest
        assert res["steps_done"][i] == r.steps


def test_walk_len_zero_and_domain():
    st = I.random_full_keys(100, 1, seed=9)[0]
    r = O.full_walk(100, st, 0)
    assert r.steps == 0 and r.digest == 0
    assert r.best_E == O.full_energy_packed(st, 100)
    for bad in (2, 256):
        with pytest.raises(ValueError):
            O.full_walk(bad, np.zeros(4, dtype=np.uint64), 5)
    # the longest whole-space length: four key words, the top bit free
    assert O.full_l_max() == 255 and O.full_key_words(255) == 4
    st = I.random_full_keys(255, 1, seed=11)[0]
    r = O.full_walk(255, st, 3)
    assert r.steps == 3 and len(r.best_seq) == 4
