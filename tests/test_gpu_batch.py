"""Mixed-length batches in one persistent launch, their hipGraph form and the
tuning table: every instance must equal its standalone labs_walks run (and the
oracle on sampled walks), whatever the lanes per walk and load factor."""
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


def _specs(n_inst, lo, hi, n_walks, walk_len, seed, lanes=(0, 2, 4, 8), n_trace=0):
    Ls = I.odd_lengths(n_inst, lo, hi, seed=seed)
    return [dict(L=int(L), n_walks=int(n_walks[i % len(n_walks)]), walk_len=walk_len,
                 seed=1000 + i, lanes_per_walk=lanes[i % len(lanes)], n_trace=n_trace)
            for i, L in enumerate(Ls)]


def _standalone(sp):
    labs = _labs()
    plan = labs.make_plan(lanes_per_walk=sp["lanes_per_walk"] or 4,
                          load_factor=sp.get("load_factor", 0.0))
    st = sp.get("starts_t")
    return labs.walks(sp["L"], sp["n_walks"], sp["walk_len"], seed=sp["seed"], starts_t=st, plan=plan)


def _assert_same(a, b):
    np.testing.assert_array_equal(_u64(a["digest"]), _u64(b["digest"]))
    np.testing.assert_array_equal(a["best_E"].cpu().numpy(), b["best_E"].cpu().numpy())
    np.testing.assert_array_equal(_u64(a["best_seq"]), _u64(b["best_seq"]))
    np.testing.assert_array_equal(a["steps_done"].cpu().numpy(), b["steps_done"].cpu().numpy())


def test_mixed_batch_equals_standalone_and_oracle():
    labs = _labs()
    specs = _specs(14, 61, 223, n_walks=[64, 100, 257, 31], walk_len=700, seed=5, n_trace=2)
    specs += [dict(L=7, n_walks=40, walk_len=100, seed=7, lanes_per_walk=2, n_trace=2),   # traps
              dict(L=27, n_walks=64, walk_len=4096, seed=0, lanes_per_walk=8, n_trace=2),
              dict(L=301, n_walks=20, walk_len=60, seed=9, lanes_per_walk=4, n_trace=2),
              dict(L=101, n_walks=0, walk_len=10, seed=1, lanes_per_walk=4)]
    keys = I.random_start_keys(151, 70, seed=3)
    specs.append(dict(L=151, n_walks=70, walk_len=500, seed=0, lanes_per_walk=2, n_trace=2,
                      starts_t=torch.from_numpy(I.as_int64_keys(keys)).cuda()))
    res = labs.walks_batch(specs)
    torch.cuda.synchronize()
    for sp, r in zip(specs, res):
        if sp["n_walks"] == 0:
            continue
        _assert_same(r, _standalone(sp))
        L = sp["L"]
        st = keys if "starts_t" in sp else O.starts(L, sp["n_walks"], sp["seed"])
        for i in range(2):
            o = O.walk(L, st[i], sp["walk_len"])
            assert r["best_E"][i].item() == o.best_E
            assert _u64(r["digest"])[i] == o.digest
            np.testing.assert_array_equal(r["trace_j"][i].cpu().numpy()[: o.steps], o.trace_j)
            np.testing.assert_array_equal(r["trace_E"][i].cpu().numpy()[: o.steps], o.trace_E)


def test_batch_graph_replays_match_eager():
    labs = _labs()
    specs = _specs(8, 61, 223, n_walks=[128, 64], walk_len=600, seed=11)
    eager = labs.walks_batch(specs)
    torch.cuda.synchronize()
    g = labs.BatchGraph(specs)
    x = torch.randn(512, 512, device="cuda")
    for rep in range(3):
        for r in g.results:
            for t in r.values():
                t.zero_()
        torch.cuda.synchronize()
        g.launch()
        y = (x @ x).sum()            # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        for a, b in zip(g.results, eager):
            _assert_same(a, b)
    g.close()


def test_config4_256_instances_one_launch():
    """256 instances, L uniform odd in [61, 223], 1024 walks x 32,768 moves.
    Two whole walks of every instance, read from the batch output, against
    the oracle (results stored by tests/golden/make_golden.py)."""
    import json
    import os
    labs = _labs()
    Ls = I.odd_lengths(256, 61, 223, seed=0)
    specs = [dict(L=int(L), n_walks=1024, walk_len=32768, seed=i) for i, L in enumerate(Ls)]
    g = labs.BatchGraph(specs)
    res = g.launch()
    torch.cuda.synchronize()
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "batch_mixedL_61_223_32768moves.json")) as f:
        doc = json.load(f)
    assert len(doc["walks"]) == 512
    for w in doc["walks"]:
        r = res[w["inst"]]
        assert specs[w["inst"]]["L"] == w["L"]
        k = w["walk"]
        assert r["best_E"][k].item() == w["best_E"], (w["inst"], k)
        assert _u64(r["digest"])[k] == w["digest"], (w["inst"], k)
        assert r["steps_done"][k].item() == w["steps_done"], (w["inst"], k)
        np.testing.assert_array_equal(_u64(r["best_seq"])[k], np.array(w["best_seq"], dtype=np.uint64))
    for idx in I.sample_indices(256, 2, 3, seed=4):
        sp = dict(specs[idx])
        sp["lanes_per_walk"] = labs.tune_get(sp["L"])[0]
        _assert_same(res[idx], _standalone(sp))
        E = res[idx]["best_E"].cpu().numpy()
        m = (sp["L"] - 1) // 2
        assert ((E - m) % 8 == 0).all() and (E >= m).all()
    # oracle on the first moves of two walks of two instances
    for idx in (0, 255):
        L = specs[idx]["L"]
        st = O.starts(L, 2, idx)
        short = labs.walks(L, 2, 1500, seed=idx)
        ref = O.walks(L, st, 1500)
        np.testing.assert_array_equal(_u64(short["digest"]), ref["digest"])
    g.close()


def test_autotune_sets_table_and_keeps_results():
    labs = _labs()
    L = 121
    base = labs.walks(L, 512, 400, seed=3, plan=labs.make_plan(lanes_per_walk=2))
    lanes, lf = labs.autotune(L, n_walks=2048, walk_len=512)
    assert lanes in (2, 4, 8) and lf in (0.5, 0.67)
    assert labs.tune_get(L)[:2] == (lanes, lf) and labs.tune_get(L)[2]
    tuned = labs.walks_batch([dict(L=L, n_walks=512, walk_len=400, seed=3)])[0]
    _assert_same(tuned, base)


def test_class_groups_sequential_and_concurrent_agree():
    """A batch spanning kernels of different occupancy runs as several
    launches; with a workspace holding every group's grid at once the groups
    run concurrently.  Both equal the standalone runs, eagerly and as graphs."""
    import ctypes
    labs = _labs()
    specs = [dict(L=L, n_walks=n, walk_len=900, seed=s, lanes_per_walk=4)
             for L, n, s in [(301, 300, 1), (261, 128, 2), (201, 200, 3), (131, 256, 4), (67, 129, 5)]]
    alone = [_standalone(sp) for sp in specs]
    outs = [labs._alloc_outputs(sp["L"], sp["n_walks"], sp["walk_len"], 0) for sp in specs]
    nb = labs.U64(0)
    labs._check(labs.lib().labs_batch_workspace_bytes(labs.make_instances(specs, outs), len(specs),
                                                      ctypes.byref(nb)))
    seq = labs.walks_batch(specs, workspace=labs.alloc_workspace(nb.value))
    conc_ws = labs.alloc_workspace(nb.value * 3)          # room for every group's grid at once
    conc = labs.walks_batch(specs, workspace=conc_ws)
    torch.cuda.synchronize()
    for a, b, c in zip(seq, conc, alone):
        _assert_same(a, c)
        _assert_same(b, c)
    g = labs.BatchGraph(specs, workspace=conc_ws)
    for _ in range(2):
        for r in g.results:
            for t in r.values():
                t.zero_()
        torch.cuda.synchronize()
        res = g.launch()
        torch.cuda.synchronize()
        for a, c in zip(res, alone):
            _assert_same(a, c)
    g.close()


def test_batch_reports_one_scan_per_move():
    """Batches report each walk's neighbourhood scans by plane cap: one scan per
    move, plus the last scan of a trapped walk."""
    labs = _labs()
    specs = _specs(6, 61, 301, n_walks=[100, 257], walk_len=900, seed=13)
    specs.append(dict(L=7, n_walks=40, walk_len=100, seed=7, lanes_per_walk=2))   # traps
    for sp in specs:
        sp["cap_steps"] = True
    res = labs.walks_batch(specs)
    torch.cuda.synchronize()
    for sp, r in zip(specs, res):
        caps = r["cap_steps"].cpu().numpy().astype(np.int64).sum(1)
        sd = r["steps_done"].cpu().numpy()
        trapped = sd < sp["walk_len"]
        np.testing.assert_array_equal(caps, sd + trapped.astype(np.int64))
        _assert_same(r, _standalone(sp))
    assert (res[-1]["steps_done"].cpu().numpy() < 100).any()       # some L = 7 walk trapped
