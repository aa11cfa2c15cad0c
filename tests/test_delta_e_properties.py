"""Property tests (hypothesis) of the incremental energy changes the kernels
evaluate, against the oracle's direct Eq. 1 recomputation.

Skew-symmetric space (Eq. 2): negating free bit j changes the even-lag
correlations by 4 u_k with u_k = -s_j (MF_k s_{j+k} + MB_k s_{j-k}), MF the
forward lags inside the sequence without the lag k0 = L + 1 - 2j (the pair
(j, L+1-j) keeps its product), MB the backward lags; dE = 8 sum u C + 16 sum u^2
and every odd-lag C stays 0.  Whole space: negating position i changes C_k by
2 u_k with the plain forward and backward lags; dE = 4 sum u C + 4 sum u^2.
Also: the symmetry group {x, -x, alt x, -alt x} leaves E unchanged, and
dE = 0 (mod 8) on skew sequences, 0 (mod 4) on any sequence.
"""
import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import oracle as O


def corr(s):
    s = np.asarray(s, dtype=np.int64)
    L = len(s)
    return np.array([int(np.dot(s[: L - k], s[k:])) for k in range(L)])   # C_0..C_{L-1}


def skew_delta(x, L, j):
    """dE of negating free bit j (1-based), from the even-lag C of x."""
    D = (L + 1) // 2
    s = O.expand_skew(x, L).astype(np.int64)
    C = corr(s)
    tot_uc, tot_u2 = 0, 0
    for k in range(2, L, 2):
        a = s[j - 1 + k] if (j + k <= L and k != L + 1 - 2 * j and j < D) else 0
        b = s[j - 1 - k] if j - k >= 1 else 0
        u = -s[j - 1] * (a + b)
        tot_uc += u * C[k]
        tot_u2 += u * u
    return 8 * tot_uc + 16 * tot_u2


def full_delta(s, i):
    s = np.asarray(s, dtype=np.int64)
    L = len(s)
    C = corr(s)
    tot_uc, tot_u2 = 0, 0
    for k in range(1, L):
        a = s[i - 1 + k] if i + k <= L else 0
        b = s[i - 1 - k] if i - k >= 1 else 0
        u = -s[i - 1] * (a + b)
        tot_uc += u * C[k]
        tot_u2 += u * u
    return 4 * tot_uc + 4 * tot_u2


odd_L = st.integers(min_value=1, max_value=40).map(lambda t: 2 * t + 1)


@settings(max_examples=60, deadline=None)
@given(L=odd_L, data=st.data())
def test_skew_delta_matches_direct_recompute(L, data):
    D = (L + 1) // 2
    x = np.array(data.draw(st.lists(st.sampled_from([-1, 1]), min_size=D, max_size=D)), dtype=np.int8)
    E0 = O.energy(O.expand_skew(x, L))
    assert (E0 - (L - 1) // 2) % 8 == 0
    assert all(c == 0 for c in corr(O.expand_skew(x, L))[1::2])       # odd lags vanish
    for j in range(1, D + 1):
        y = x.copy()
        y[j - 1] = -y[j - 1]
        dE = O.energy(O.expand_skew(y, L)) - E0
        assert skew_delta(x, L, j) == dE
        assert dE % 8 == 0


@settings(max_examples=60, deadline=None)
@given(data=st.data(), L=st.integers(min_value=3, max_value=70))
def test_full_delta_matches_direct_recompute(L, data):
    s = np.array(data.draw(st.lists(st.sampled_from([-1, 1]), min_size=L, max_size=L)), dtype=np.int8)
    E0 = O.energy(s)
    for i in range(1, L + 1):
        y = s.copy()
        y[i - 1] = -y[i - 1]
        dE = O.energy(y) - E0
        assert full_delta(s, i) == dE
        assert dE % 4 == 0


@settings(max_examples=80, deadline=None)
@given(L=odd_L, data=st.data())
def test_symmetry_group_keeps_skew_energy(L, data):
    D = (L + 1) // 2
    x = np.array(data.draw(st.lists(st.sampled_from([-1, 1]), min_size=D, max_size=D)), dtype=np.int8)
    alt = np.array([(-1) ** (j + 1) for j in range(D)], dtype=np.int8)
    E = O.energy(O.expand_skew(x, L))
    for y in (-x, alt * x, -alt * x):
        assert O.energy(O.expand_skew(y, L)) == E
