"""Whole-space walks (labs_full_walks) against the whole-space oracle: every
walk's best energy, best sequence, move count and digest, and the traces of
the first walks, bit-exact, over lengths that cross every lag-word, key-word
and table-entry boundary, with ragged block tails, trapped walks, explicit
and seeded starts, and chunked launches."""
import numpy as np
import pytest

from oracle import oracle as O
import labs_inputs as I

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


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _compare(L, keys, res, walk_len, n_trace=0):
    ref = O.full_walks(L, keys, walk_len)
    np.testing.assert_array_equal(res["best_E"].cpu().numpy(), ref["best_E"])
    np.testing.assert_array_equal(_u64(res["best_seq"]).reshape(ref["best_seq"].shape), ref["best_seq"])
    np.testing.assert_array_equal(res["steps_done"].cpu().numpy(), ref["steps_done"])
    np.testing.assert_array_equal(_u64(res["digest"]), ref["digest"])
    for i in range(n_trace):
        r = O.full_walk(L, keys[i], walk_len)
        np.testing.assert_array_equal(res["trace_j"][i].cpu().numpy()[: r.steps], r.trace_j)
        np.testing.assert_array_equal(res["trace_E"][i].cpu().numpy()[: r.steps], r.trace_E)


LENGTHS = [3, 4, 5, 8, 13, 16, 27, 32, 33, 34, 50, 63, 64, 65, 66, 95, 96, 97, 98, 127, 128, 129,
           150, 160, 161, 162, 191, 192, 193, 194, 200, 224, 225, 226, 247, 255]


@pytest.mark.parametrize("L", LENGTHS)
def test_seeded_walks_match_oracle(L):
    labs = _labs()
    n = 70                                          # two workgroups, the second ragged
    walk_len = 400 if L <= 64 else (150 if L <= 128 else (60 if L <= 192 else 30))
    print(f"[full] L={L} n={n} walk_len={walk_len}", flush=True)
    res = labs.full_walks(L, n, walk_len, seed=L, n_trace=2)
    torch.cuda.synchronize()
    _compare(L, O.full_starts(L, n, L), res, walk_len, n_trace=2)


@pytest.mark.parametrize("L", [3, 4, 5, 6, 7])
def test_trapped_walks(L):
    labs = _labs()
    n, walk_len = 64, 300                          # more moves than states
    res = labs.full_walks(L, n, walk_len, seed=7, n_trace=4)
    torch.cuda.synchronize()
    sd = res["steps_done"].cpu().numpy()
    assert (sd < (1 << L)).all()
    _compare(L, O.full_starts(L, n, 7), res, walk_len, n_trace=4)


@pytest.mark.parametrize("L", [20, 71, 130, 192, 247])
def test_explicit_starts_and_chunks(L):
    labs = _labs()
    n, walk_len = 200, (120 if L <= 192 else 40)
    keys = I.random_full_keys(L, n, seed=L + 3)
    st = torch.from_numpy(I.as_int64_keys(keys)).cuda()
    res = labs.full_walks(L, n, walk_len, starts_t=st, n_trace=1)
    # four chunks of at most 64 resident walks give identical results
    plan = labs.make_plan(max_concurrent=64)
    ws = labs.alloc_workspace(labs.full_workspace_bytes(L, 64, walk_len))
    res2 = labs.full_walks(L, n, walk_len, starts_t=st, plan=plan, workspace=ws)
    torch.cuda.synchronize()
    _compare(L, keys, res, walk_len, n_trace=1)
    np.testing.assert_array_equal(_u64(res2["digest"]), _u64(res["digest"]))
    np.testing.assert_array_equal(res2["best_E"].cpu().numpy(), res["best_E"].cpu().numpy())


def test_seeded_starts_equal_explicit_oracle_starts_and_walk_len_zero():
    labs = _labs()
    L, n = 100, 96
    keys = O.full_starts(L, n, 11)
    res = labs.full_walks(L, n, 0, seed=11)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_u64(res["best_seq"]), keys)
    assert (res["steps_done"].cpu().numpy() == 0).all()
    np.testing.assert_array_equal(res["best_E"].cpu().numpy(),
                                  [O.full_energy_packed(k, L) for k in keys])


def test_cap_counts_cover_every_scan():
    labs = _labs()
    L, n, walk_len = 128, 256, 500
    res = labs.full_walks(L, n, walk_len, seed=1, cap_steps=True)
    torch.cuda.synchronize()
    caps = res["cap_steps"].cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(caps.sum(axis=1), res["steps_done"].cpu().numpy()
                                  + (res["steps_done"].cpu().numpy() < walk_len))


def _unpack_full(keys, L):
    """int8 +-1 sequences [n, L] from packed whole-space keys (bit i-1 = s_i)."""
    bits = np.unpackbits(np.ascontiguousarray(keys).view(np.uint8).reshape(len(keys), -1),
                         axis=1, bitorder="little")[:, :L]
    return (1 - 2 * bits.astype(np.int8)).astype(np.int8)


@pytest.mark.parametrize("L,steps,prefix", [(128, 32768, 1500), (64, 32768, 3000), (192, 16384, 600)])
def test_bench_workload_65536_walks(L, steps, prefix):
    """The whole-space bench configurations (bench.py --full L): E of every
    best sequence recomputed by the energy kernel, E = floor(L/2) (mod 4), and
    trace prefixes plus prefix-length runs of sampled walks against the oracle."""
    labs = _labs()
    n = 65536
    print(f"[full] L={L} n={n} steps={steps}", flush=True)
    plan = labs.make_plan()
    ws = labs.alloc_workspace(labs.full_workspace_bytes(L, n, steps, plan))
    res = labs.full_walks(L, n, steps, seed=0, plan=plan, workspace=ws, n_trace=2)
    torch.cuda.synchronize()
    del ws
    torch.cuda.empty_cache()
    best = _u64(res["best_seq"]).reshape(n, -1)
    E_best = res["best_E"].cpu().numpy()
    s = _unpack_full(best, L)
    E = np.concatenate([labs.energy(torch.from_numpy(s[i:i + 16384]).cuda()).cpu().numpy()
                        for i in range(0, n, 16384)])
    np.testing.assert_array_equal(E, E_best)
    assert ((E_best - L // 2) % 4 == 0).all() and (E_best >= L // 2).all()
    assert (res["steps_done"].cpu().numpy() <= steps).all()
    keys = O.full_starts(L, n, 0)
    for i in range(2):
        r = O.full_walk(L, keys[i], prefix)
        np.testing.assert_array_equal(res["trace_j"][i].cpu().numpy()[: r.steps], r.trace_j)
        np.testing.assert_array_equal(res["trace_E"][i].cpu().numpy()[: r.steps], r.trace_E)
    idx = I.sample_indices(n, 4, 4, seed=5)
    st = torch.from_numpy(I.as_int64_keys(keys[idx])).cuda()
    short = labs.full_walks(L, len(idx), prefix, starts_t=st, plan=plan)
    torch.cuda.synchronize()
    _compare(L, keys[idx], short, prefix)


def _first(res, k):
    return {key: (v[:k] if v is not None else None) for key, v in res.items()}


def test_batch_of_mixed_lengths_matches_standalone_and_oracle():
    """labs_full_walks_batch: instances across the three kernel groups
    (classes 1-4, 5-7, 8), ragged walk counts, an empty walk, explicit starts
    and traces; every instance equals its standalone labs_full_walks run bit
    for bit, and the oracle on its first walks."""
    labs = _labs()
    Ls = [3, 16, 33, 64, 97, 128, 129, 130, 161, 200, 225, 226, 255]
    specs = []
    for i, L in enumerate(Ls):
        n = [70, 64, 1, 130][i % 4]
        wl = 300 if L <= 64 else (120 if L <= 128 else 40)
        specs.append(dict(L=L, n_walks=n, walk_len=wl, seed=100 + i, n_trace=min(n, 2)))
    specs.append(dict(L=50, n_walks=5, walk_len=0, seed=7))
    keys140 = I.random_full_keys(140, 20, seed=5)
    specs.append(dict(L=140, n_walks=20, walk_len=60,
                      starts_t=torch.from_numpy(I.as_int64_keys(keys140)).cuda()))
    print(f"[full batch] {len(specs)} instances", flush=True)
    res = labs.full_walks_batch(specs)
    torch.cuda.synchronize()
    for sp, r in zip(specs, res):
        alone = labs.full_walks(sp["L"], sp["n_walks"], sp["walk_len"], seed=sp.get("seed", 0),
                                starts_t=sp.get("starts_t"), n_trace=sp.get("n_trace", 0))
        torch.cuda.synchronize()
        for key in ("best_seq", "best_E", "steps_done", "digest", "trace_j", "trace_E"):
            if key in alone and alone[key] is not None:
                np.testing.assert_array_equal(r[key].cpu().numpy(), alone[key].cpu().numpy())
    for idx in (0, 3, 6, 9, 12):
        sp = specs[idx]
        k = min(sp["n_walks"], 2)
        _compare(sp["L"], O.full_starts(sp["L"], k, sp["seed"]), _first(res[idx], k), sp["walk_len"],
                 n_trace=min(k, sp["n_trace"]))
    _compare(140, keys140[:3], _first(res[-1], 3), 60)
    assert (res[-2]["steps_done"].cpu().numpy() == 0).all()


def test_batch_rejects_invalid_instances():
    labs = _labs()
    for bad in (dict(L=256, n_walks=4, walk_len=10), dict(L=2, n_walks=4, walk_len=10),
                dict(L=64, n_walks=4, walk_len=10, lanes_per_walk=2),
                dict(L=64, n_walks=4, walk_len=-1)):
        with pytest.raises(labs.LabsError) as e:
            labs.full_walks_batch([dict(L=20, n_walks=8, walk_len=5), bad])
        assert e.value.code == labs.LABS_EINVAL
