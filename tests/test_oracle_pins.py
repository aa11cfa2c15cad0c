"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: values the
paper prints (Table 1), textbook sequences (Barker codes), closed forms,
invariants of the skew-symmetric space (Eq. 2), a library routine
(numpy.correlate), hand-derived walks, and brute force on tiny inputs.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
import labs_inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def np_energy(s) -> int:
    """Eq. 1 via numpy.correlate (independent of the oracle's loops)."""
    s = np.asarray(s, dtype=np.int64)
    r = np.correlate(s, s, mode="full")[len(s):]      # lags 1..L-1
    return int(np.sum(r * r))


def np_autocorr(s) -> np.ndarray:
    s = np.asarray(s, dtype=np.int64)
    return np.correlate(s, s, mode="full")[len(s) - 1:]  # lags 0..L-1


def load_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_new_best_sequences.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            L, E, F, code = line.split()
            rows.append((int(L), int(E), float(F), code))
    return rows


# ------------------------------------------------------------------ Eq. 1
BARKER = {
    3: [1, 1, -1],
    5: [1, 1, 1, -1, 1],
    7: [1, 1, 1, -1, -1, 1, -1],
    11: [1, 1, 1, -1, -1, -1, 1, -1, -1, 1, -1],
    13: [1, 1, 1, 1, 1, -1, -1, 1, 1, -1, 1, -1, 1],
}


def test_barker13_energy_and_merit_factor():
    E = O.energy(BARKER[13])
    assert E == 6
    assert O.merit_factor(13, E) == pytest.approx(169 / 12, abs=1e-12)


@pytest.mark.parametrize("L", sorted(BARKER))
def test_barker_codes_attain_the_bound(L):
    # Barker codes have |C_k| <= 1; for odd L, C_k = 0 (odd k), +-1 (even k).
    assert O.energy(BARKER[L]) == (L - 1) // 2


@pytest.mark.parametrize("L", [1, 2, 3, 8, 31, 64, 101])
def test_constant_sequence_closed_form(L):
    # All-ones: C_k = L - k, so E = sum_{k=1}^{L-1} k^2 = (L-1) L (2L-1) / 6.
    assert O.energy(np.ones(L, dtype=np.int8)) == (L - 1) * L * (2 * L - 1) // 6


@pytest.mark.parametrize("L", [2, 5, 16, 27, 64, 151, 301])
def test_energy_matches_numpy_correlate(L):
    for s in I.random_pm1(20, L, seed=L):
        assert O.energy(s) == np_energy(s)


# ------------------------------------------------------------------ Eq. 2
def test_barker13_is_skew_symmetric():
    b = np.array(BARKER[13], dtype=np.int8)
    assert np.array_equal(O.expand_skew(b[:7], 13), b)


@pytest.mark.parametrize("L", [3, 5, 7, 27, 101, 151, 223, 301, 383])
def test_skew_invariants(L):
    D, m = (L + 1) // 2, (L - 1) // 2
    for key in I.random_start_keys(L, 12, seed=L):
        x = O.unpack(key, L)
        s = O.expand_skew(x, L)
        assert np.array_equal(s[:D], x)
        C = np_autocorr(s)
        assert np.all(C[1::2] == 0)                  # odd lags vanish
        E = O.energy(s)
        assert E == np_energy(s)
        assert E % 8 == m % 8                        # even-lag C_k odd => C_k^2 = 1 mod 8
        assert E >= m
        assert O.energy_packed(key, L) == E


@pytest.mark.parametrize("L", [5, 9, 27, 101, 151])
def test_symmetries_preserve_energy(L):
    D = (L + 1) // 2
    sign = np.array([(-1) ** (j + 1) for j in range(D)], dtype=np.int8)  # (-1)^j, j 1-based
    for key in I.random_start_keys(L, 10, seed=2 * L):
        x = O.unpack(key, L)
        E = O.energy(O.expand_skew(x, L))
        assert O.energy(O.expand_skew(-x, L)) == E
        assert O.energy(O.expand_skew(sign * x, L)) == E
        assert O.energy(O.expand_skew(-sign * x, L)) == E


# ------------------------------------------------------------------ Table 1
@pytest.mark.parametrize("row", load_table1(), ids=lambda r: f"L{r[0]}")
def test_table1_energies_and_merit_factors(row):
    L, E_printed, F_printed, code = row
    x = O.decode_table_hex(code, L)
    s = O.expand_skew(x, L)
    E = O.energy(s)
    assert E == E_printed
    assert np_energy(s) == E_printed
    assert O.merit_factor(L, E) == pytest.approx(F_printed, abs=1e-4)
    assert np.all(np_autocorr(s)[1::2] == 0)
    assert E % 8 == ((L - 1) // 2) % 8


# ------------------------------------------------------------------ brute force
@pytest.mark.parametrize("L", [3, 5, 7, 11, 13])
def test_bruteforce_minimum_at_barker_lengths(L):
    mn, cnt, first, total = O.bruteforce(L)
    assert mn == (L - 1) // 2
    assert cnt >= 1
    assert O.energy_packed(np.array([first], dtype=np.uint64), L) == mn


@pytest.mark.parametrize("L", list(range(3, 30, 2)))
def test_bruteforce_mean_energy_closed_form(L):
    # E[C_k^2] = 2(L-k) - 1 for even k on uniform skew sequences, which sums to
    # (L-1)(L-2)/2 over the even lags.
    D = (L + 1) // 2
    mn, cnt, first, total = O.bruteforce(L)
    assert total == (2 ** D) * (L - 1) * (L - 2) // 2


@pytest.mark.parametrize("L", [9, 15, 19, 21])
def test_bruteforce_against_numpy_enumeration(L):
    D = (L + 1) // 2
    energies = []
    for v in range(2 ** D):
        x = np.array([-1 if (v >> j) & 1 else 1 for j in range(D)], dtype=np.int8)
        energies.append(np_energy(O.expand_skew(x, L)))
    energies = np.array(energies)
    mn, cnt, first, total = O.bruteforce(L)
    assert mn == energies.min()
    assert cnt == int(np.sum(energies == mn))
    assert first == int(np.argmin(energies))
    assert total == int(energies.sum())


# ------------------------------------------------------------------ SplitMix64
def test_splitmix64_reference_outputs():
    # SplitMix64 seeded with 0 emits mix64(k * 0x9E3779B97F4A7C15), k = 1, 2, 3:
    # the published first outputs of the reference generator.
    g = 0x9E3779B97F4A7C15
    assert O.mix64(g) == 0xE220A8397B1DCDAF
    assert O.mix64((2 * g) % 2 ** 64) == 0x6E789E6AA1B965F4
    assert O.mix64((3 * g) % 2 ** 64) == 0x06C45D188009454F


def test_seeded_starts_layout():
    for L in [3, 27, 127, 129, 151, 255, 301, 383]:
        st = O.starts(L, 5, seed=7)
        D, W = (L + 1) // 2, (L + 127) // 128
        assert st.shape == (5, (D + 63) // 64)
        g = 0x9E3779B97F4A7C15
        for w in range(5):
            for t in range(st.shape[1]):
                v = O.mix64((7 + g * (w * st.shape[1] + t + 1)) % 2 ** 64)
                bits = D - 64 * t
                if bits < 64:
                    v &= (1 << bits) - 1
                assert int(st[w, t]) == v


# ------------------------------------------------------------------ walks
def test_walk_L3_by_hand():
    # L = 3: s = (x1, x2, -x1), C_1 = 0, C_2 = -1, so every sequence has E = 1.
    # From (+,+) all neighbours tie; lowest j wins until every state is visited:
    # (+,+) -1-> (-,+) -2-> (-,-) -1-> (+,-), then both neighbours are visited.
    r = O.walk(3, O.pack([1, 1]), 10)
    assert list(r.trace_j) == [1, 2, 1]
    assert list(r.trace_E) == [1, 1, 1]
    assert r.steps == 3 and r.best_E == 1
    assert int(r.best_seq[0]) == 0


def test_walk_L5_by_hand():
    # L = 5: s = (x1, x2, x3, -x2, x1), C_2 = 2 x1 x3 - 1, C_4 = 1, odd lags 0,
    # so E = 2 if x1 == x3 else 10.  Walking from (+,+,+) with lowest-j ties:
    # +++ -2-> +-+ (2) -1-> --+ (10) -3-> --- (2) -2-> -+- (2) -1-> ++- (10)
    # -2-> +-- (10); all three neighbours of +-- are then visited (trapped).
    r = O.walk(5, O.pack([1, 1, 1]), 50)
    assert list(r.trace_j) == [2, 1, 3, 2, 1, 2]
    assert list(r.trace_E) == [2, 10, 2, 2, 10, 10]
    assert r.steps == 6
    assert r.best_E == 2 and int(r.best_seq[0]) == 0   # the start itself (strict <)


def _check_walk_semantics(L, start, walk_len, r):
    """Independent re-check of a walk trace from the definition (Eq. 3)."""
    D = (L + 1) // 2
    x = O.unpack(start, L).astype(np.int8)
    visited = {tuple(x)}
    E = np_energy(O.expand_skew(x, L))
    best, best_x = E, x.copy()
    h = 0
    for t in range(r.steps):
        cand = []
        for j in range(D):
            y = x.copy()
            y[j] = -y[j]
            if tuple(y) in visited:
                continue
            cand.append((np_energy(O.expand_skew(y, L)), j + 1))
        assert cand, "the oracle moved although every neighbour was visited"
        e_min, j_min = min(cand)
        assert r.trace_j[t] == j_min and r.trace_E[t] == e_min
        x[j_min - 1] = -x[j_min - 1]
        visited.add(tuple(x))
        E = e_min
        if E < best:
            best, best_x = E, x.copy()
        h = O.mix64(h ^ ((j_min << 32) | (E & 0xFFFFFFFF)))
    if r.steps < walk_len:   # trapped: every neighbour must be visited
        for j in range(D):
            y = x.copy()
            y[j] = -y[j]
            assert tuple(y) in visited
    assert r.best_E == best
    assert np.array_equal(O.unpack(r.best_seq, L), best_x)
    assert r.digest == O.mix64(h ^ r.steps)
    assert len(visited) == r.steps + 1               # no pivot repeats


@pytest.mark.parametrize("L,walk_len,n", [(7, 100, 4), (9, 300, 4), (13, 500, 3), (27, 300, 2),
                                          (41, 200, 2), (63, 150, 1)])
def test_walk_semantics(L, walk_len, n):
    for start in I.random_start_keys(L, n, seed=100 + L):
        r = O.walk(L, start, walk_len)
        _check_walk_semantics(L, start, walk_len, r)


def test_walk_traps_at_L7():
    # 16 states: a 100-move walk must stop early with all neighbours visited.
    for start in I.random_start_keys(7, 8, seed=3):
        r = O.walk(7, start, 100)
        assert r.steps < 16
        _check_walk_semantics(7, start, 100, r)


@pytest.mark.parametrize("L", [27, 51, 101])
def test_walk_metamorphic_symmetries(L):
    D = (L + 1) // 2
    sign = np.array([(-1) ** (j + 1) for j in range(D)], dtype=np.int8)
    for start in I.random_start_keys(L, 3, seed=L + 5):
        x = O.unpack(start, L)
        ref = O.walk(L, start, 400)
        for y in (-x, sign * x, -sign * x):
            r = O.walk(L, O.pack(y), 400)
            assert np.array_equal(r.trace_j, ref.trace_j)
            assert np.array_equal(r.trace_E, ref.trace_E)
            assert r.best_E == ref.best_E and r.digest == ref.digest


def test_walk_len_zero_returns_start():
    st = I.random_start_keys(101, 1, seed=9)[0]
    r = O.walk(101, st, 0)
    assert r.steps == 0
    assert r.best_E == O.energy_packed(st, 101)
    assert np.array_equal(r.best_seq, st)
    assert r.digest == 0


def test_config1_walks_never_beat_bruteforce_minimum():
    L = 27
    mn, cnt, first, total = O.bruteforce(L)
    res = O.walks(L, O.starts(L, 64, seed=0), 4096)
    assert np.all(res["best_E"] >= mn)
    assert np.all(res["steps_done"] <= 4096)
    # reaching the optimum in 64 walks of 4096 moves over 2^14 states is expected
    assert res["best_E"].min() == mn


def test_walks_threads_agree_with_single_walk():
    L = 51
    st = I.random_start_keys(L, 6, seed=11)
    res = O.walks(L, st, 300, n_threads=3)
    for i in range(6):
        r = O.walk(L, st[i], 300, trace=False)
        assert res["best_E"][i] == r.best_E and res["digest"][i] == r.digest
        assert res["steps_done"][i] == r.steps


# ------------------------------------------------------------------ Eq. 6 / 7
@pytest.mark.parametrize("L", [71, 121, 171, 247])
def test_stopping_condition_consistent_with_probability(L):
    # N runs of NSEs_lmt evaluations each (Eq. 6) reach the optimum with P (Eq. 7).
    n = O.nses_limit(L, P=0.99, N=100)
    assert O.optimality_probability(L, 100 * n) == pytest.approx(0.99, abs=1e-12)
    assert O.lambda_model(L) == pytest.approx(0.006753 * 0.8617 ** L, rel=1e-15)
    assert O.nses_limit(L + 2) > n                      # harder as L grows
