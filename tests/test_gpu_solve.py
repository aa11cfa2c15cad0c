"""Alg. 1 solver driver on the GPU: the global best over rounds equals the
oracle's best over the same seeded walks, and the stopping conditions
(rounds, target energy, time) end the run as declared."""
import numpy as np
import pytest

from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[case] {request.node.name}", flush=True)
    yield
    torch.cuda.empty_cache()


def _labs():
    from paper_2210_15962_amd import labs
    return labs


def test_rounds_equal_oracle_walks():
    labs = _labs()
    L, n, rounds, seed = 61, 128, 3, 77
    D = (L + 1) // 2
    r = labs.solve(L, n, max_rounds=rounds, seed=seed)
    wl = 8 * D
    starts = O.starts(L, n * rounds, seed)           # round k = walks k*n .. k*n+n-1
    ref = O.walks(L, starts, wl)
    E = ref["best_E"]
    first = int(np.argmin(E))                         # round-major: first walk reaching the minimum
    assert r["rounds"] == rounds
    assert r["best_E"] == int(E.min())
    np.testing.assert_array_equal(r["best_seq"], ref["best_seq"][first])
    assert r["nfes"] == rounds * n * wl * (D - 1)
    assert r["walk_steps"] == int(ref["steps_done"].sum())
    assert not r["reached_target"] and r["target_seconds"] == -1.0


def test_target_energy_stops_the_run():
    labs = _labs()
    L = 27
    E_min = int(O.bruteforce(L)[0])
    r = labs.solve(L, 256, target_E=E_min, max_rounds=50, seed=1)
    assert r["reached_target"] and r["best_E"] == E_min
    assert 0 < r["target_nfes"] <= r["nfes"] and 0 <= r["target_seconds"] <= r["seconds"]
    assert O.energy_packed(r["best_seq"], L) == E_min


def test_time_limit_stops_the_run():
    labs = _labs()
    r = labs.solve(101, 1024, time_limit_s=0.5, seed=3)
    assert r["rounds"] >= 1 and r["seconds"] >= 0.5
    assert r["seconds"] < 5.0


def test_resumed_run_equals_uninterrupted_run():
    """Rounds are deterministic in (seed, round): two rounds, then two more
    from first_round = 2, give the best of four uninterrupted rounds."""
    labs = _labs()
    L, n, seed = 71, 256, 5
    full = labs.solve(L, n, max_rounds=4, seed=seed)
    a = labs.solve(L, n, max_rounds=2, seed=seed)
    b = labs.solve(L, n, max_rounds=2, seed=seed, first_round=2)
    best = a if a["best_E"] <= b["best_E"] else b
    assert full["best_E"] == best["best_E"]
    np.testing.assert_array_equal(full["best_seq"], best["best_seq"])
    assert full["nfes"] == a["nfes"] + b["nfes"]
    assert full["walk_steps"] == a["walk_steps"] + b["walk_steps"]
    # and the resumed rounds are the oracle's walks 2n .. 4n - 1
    D = (L + 1) // 2
    ref = O.walks(L, O.starts(L, 4 * n, seed)[2 * n:], 8 * D)
    assert b["best_E"] == int(ref["best_E"].min())
