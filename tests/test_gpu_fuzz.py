"""Randomised parity (hypothesis, derandomised so reruns are reproducible):
lengths, walk counts, walk lengths, seeds and lanes per walk drawn at random,
every walk's best energy, best sequence, move count and digest compared
bit-exactly with the oracle, for both the skew-symmetric space and the whole
space.  Oracle work per example is bounded (walks x moves x D x L^2)."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BUDGET = 4e9          # oracle multiply-adds per example


def _labs():
    from paper_2210_15962_amd import labs
    return labs


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


@settings(max_examples=30, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow])
@given(L=st.integers(1, 191).map(lambda t: 2 * t + 1), n=st.integers(1, 300),
       walk_len=st.integers(0, 400), seed=st.integers(0, 2**64 - 1),
       lanes=st.sampled_from([0, 1, 2, 4, 8]))
def test_skew_walks_random_shapes(L, n, walk_len, seed, lanes):
    D = (L + 1) // 2
    per_walk = max(walk_len, 1) * D * L * L / 2
    n = max(1, min(n, int(BUDGET / per_walk)))
    print(f"[fuzz skew] L={L} n={n} walk_len={walk_len} lanes={lanes} seed={seed}", flush=True)
    labs = _labs()
    res = labs.walks(L, n, walk_len, seed=seed, plan=labs.make_plan(lanes_per_walk=lanes))
    torch.cuda.synchronize()
    ref = O.walks(L, O.starts(L, n, seed), walk_len)
    np.testing.assert_array_equal(res["best_E"].cpu().numpy(), ref["best_E"])
    np.testing.assert_array_equal(_u64(res["best_seq"]).reshape(ref["best_seq"].shape), ref["best_seq"])
    np.testing.assert_array_equal(res["steps_done"].cpu().numpy(), ref["steps_done"])
    np.testing.assert_array_equal(_u64(res["digest"]), ref["digest"])


@settings(max_examples=30, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow])
@given(L=st.integers(3, 192), n=st.integers(1, 300), walk_len=st.integers(0, 400),
       seed=st.integers(0, 2**64 - 1))
def test_full_walks_random_shapes(L, n, walk_len, seed):
    per_walk = max(walk_len, 1) * L * L * L / 2
    n = max(1, min(n, int(BUDGET / per_walk)))
    print(f"[fuzz full] L={L} n={n} walk_len={walk_len} seed={seed}", flush=True)
    labs = _labs()
    res = labs.full_walks(L, n, walk_len, seed=seed)
    torch.cuda.synchronize()
    ref = O.full_walks(L, O.full_starts(L, n, seed), walk_len)
    np.testing.assert_array_equal(res["best_E"].cpu().numpy(), ref["best_E"])
    np.testing.assert_array_equal(_u64(res["best_seq"]).reshape(ref["best_seq"].shape), ref["best_seq"])
    np.testing.assert_array_equal(res["steps_done"].cpu().numpy(), ref["steps_done"])
    np.testing.assert_array_equal(_u64(res["digest"]), ref["digest"])
