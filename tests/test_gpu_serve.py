"""Continuous-batching server: every request's results equal its standalone
labs_walks run (and the oracle on sampled walks) whether it ran alone or in a
mix, requests that arrive while others run are admitted before those finish,
and admission, queue limits, time-outs and counters behave as declared."""
import time

import numpy as np
import pytest

from oracle import oracle as O
import labs_inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

POOL = 4 << 30      # 4 GiB pool: ample for the requests below


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[case] {request.node.name}", flush=True)
    yield
    torch.cuda.empty_cache()


def _labs():
    from paper_2210_15962_amd import labs
    return labs


def _standalone(L, n, walk_len, seed, starts=None):
    labs = _labs()
    st = None if starts is None else torch.from_numpy(I.as_int64_keys(starts)).cuda()
    r = labs.walks(L, n, walk_len, seed=seed, starts_t=st)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items() if k in ("best_seq", "best_E", "steps_done", "digest")}


def _assert_same(served, alone):
    np.testing.assert_array_equal(served["digest"], alone["digest"].view(np.uint64))
    np.testing.assert_array_equal(served["best_E"], alone["best_E"])
    np.testing.assert_array_equal(served["best_seq"].reshape(-1), alone["best_seq"].view(np.uint64).reshape(-1))
    np.testing.assert_array_equal(served["steps_done"], alone["steps_done"])


@pytest.mark.parametrize("chunk", [700, 0])
def test_mix_equals_alone_and_oracle(chunk):
    """chunk 700: every launch advances each request by at most 700 moves;
    chunk 0: launches run until a request can be admitted or has finished."""
    labs = _labs()
    Ls = [int(x) for x in I.odd_lengths(6, 121, 301, seed=21)] + [7, 27]
    reqs = [dict(L=L, n=[128, 300, 64, 257][i % 4], walk_len=[3000, 2500, 1800][i % 3], seed=50 + i)
            for i, L in enumerate(Ls)]
    reqs.append(dict(L=27, n=16, walk_len=0, seed=3))                  # nothing to walk
    keys = I.random_start_keys(151, 40, seed=8)
    reqs.append(dict(L=151, n=40, walk_len=2222, seed=0, starts=keys))
    with labs.Server(pool_bytes=POOL, chunk_steps=chunk) as srv:
        ids = []
        for i, q in enumerate(reqs):
            ids.append(srv.submit(q["L"], q["n"], q["walk_len"], q["seed"], q.get("starts")))
            if i % 3 == 2:
                time.sleep(0.02)                                       # arrivals spread out
        out = [srv.wait(rid, timeout_s=120) for rid in ids]
        st = srv.stats()
    for q, r in zip(reqs, out):
        assert r is not None
        alone = _standalone(q["L"], q["n"], q["walk_len"], q["seed"], q.get("starts"))
        _assert_same(r, alone)
        assert r["total_steps"] == int(alone["steps_done"].sum())
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]
    # oracle on two walks of three requests
    for q, r in [(reqs[0], out[0]), (reqs[6], out[6]), (reqs[-1], out[-1])]:
        starts = q["starts"] if "starts" in q else O.starts(q["L"], 2, q["seed"])
        for i in range(2):
            o = O.walk(q["L"], starts[i], q["walk_len"])
            assert r["best_E"][i] == o.best_E and r["digest"][i] == o.digest
            assert r["steps_done"][i] == o.steps
    assert st["submitted"] == st["admitted"] == st["completed"] == len(reqs)
    assert st["pending"] == 0 and st["active"] == 0 and st["pool_used"] == 0
    if chunk:
        assert st["launches"] >= 5                                     # 3000 moves / 700 per launch
    else:
        assert st["launches"] >= 2                                     # spread arrivals stop launches
    assert st["walk_steps"] == sum(r["total_steps"] for r in out)
    assert 0 < st["pool_peak"] <= st["pool_bytes"]


@pytest.mark.parametrize("chunk", [1024, 0])
def test_late_arrival_joins_running_request(chunk):
    """A short request submitted while a long one runs finishes first (with
    chunk 0 its arrival stops the running launch, and so does its completion)."""
    labs = _labs()
    with labs.Server(pool_bytes=POOL, chunk_steps=chunk) as srv:
        a = srv.submit(201, 256, 40000, seed=1)
        while srv.stats()["admitted"] < 1:
            time.sleep(0.001)
        time.sleep(0.05)
        b = srv.submit(161, 64, 2048, seed=2)
        rb = srv.wait(b, timeout_s=120)
        ra = srv.wait(a, timeout_s=120)
        st = srv.stats()
    if not chunk:
        assert st["launches"] >= 3          # a alone, a + b until b finishes, the rest of a
    assert rb["t_done_ns"] < ra["t_done_ns"]
    assert rb["t_admit_ns"] < ra["t_done_ns"]
    _assert_same(rb, _standalone(161, 64, 2048, 2))
    sample = _standalone(201, 256, 40000, 1)
    _assert_same(ra, sample)


def test_admission_waits_for_memory_and_queue_limit():
    labs = _labs()
    L, n, wl = 301, 64, 20000
    with labs.Server(pool_bytes=POOL) as probe:
        r = probe.wait(probe.submit(L, n, wl, seed=5), timeout_s=120)
        st = probe.stats()
        fp = st["pool_peak"]
        ctl = POOL - st["pool_bytes"]
    alone = _standalone(L, n, wl, 5)
    _assert_same(r, alone)
    # a pool that holds one such request at a time, and a queue of one
    with labs.Server(pool_bytes=ctl + fp + fp // 2, max_pending=1) as srv:
        a = srv.submit(L, n, wl, seed=5)
        while srv.stats()["admitted"] < 1:
            time.sleep(0.001)
        b = srv.submit(L, n, wl, seed=6)                  # waits for memory
        with pytest.raises(labs.LabsError) as e:
            srv.submit(L, n, wl, seed=7)                  # queue full
        assert e.value.code == labs.LABS_EBUSY
        s = srv.stats()
        assert s["pending"] == 1 and s["active"] == 1
        with pytest.raises(labs.LabsError) as e:
            srv.submit(L, 1 << 22, 1 << 20, seed=7)       # can never fit the pool
        assert e.value.code == labs.LABS_EINVAL
        ra = srv.wait(a, timeout_s=120)
        rb = srv.wait(b, timeout_s=120)
        assert rb["t_admit_ns"] >= ra["t_done_ns"]        # admitted only after a freed memory
        assert srv.stats()["pool_peak"] == fp
    _assert_same(ra, alone)
    _assert_same(rb, _standalone(L, n, wl, 6))


def test_finished_request_frees_memory_for_the_queue():
    """Default launches: a pool that holds two of these requests (equal
    footprints: same walk_len, key words and entry size) and a queue of two.
    The short-L request finishes first; its completion stops the launch, so
    the third request is admitted while the first still runs.  Every result
    equals its standalone run."""
    labs = _labs()
    Ls, n, wl = [189, 131, 187, 133], 64, 6000
    with labs.Server(pool_bytes=POOL, load_factor=0.5) as probe:
        probe.wait(probe.submit(Ls[0], n, wl, seed=0), timeout_s=120)
        st = probe.stats()
        fp, ctl = st["pool_peak"], POOL - st["pool_bytes"]
    with labs.Server(pool_bytes=ctl + 2 * fp + fp // 2, load_factor=0.5) as srv:
        ids = [srv.submit(L, n, wl, seed=30 + i) for i, L in enumerate(Ls)]
        out = [srv.wait(rid, timeout_s=120) for rid in ids]
        st = srv.stats()
    for i, (L, r) in enumerate(zip(Ls, out)):
        _assert_same(r, _standalone(L, n, wl, 30 + i))
    assert st["completed"] == len(Ls) and st["pool_used"] == 0
    assert st["pool_peak"] == 2 * fp
    assert out[1]["t_done_ns"] < out[0]["t_done_ns"]
    assert out[1]["t_done_ns"] <= out[2]["t_admit_ns"] < out[0]["t_done_ns"]


def test_poll_wait_timeout_and_unknown_ids():
    labs = _labs()
    with labs.Server(pool_bytes=POOL, chunk_steps=2048) as srv:
        rid = srv.submit(251, 512, 30000, seed=9)
        assert srv.poll(rid) is None
        assert srv.wait(rid, timeout_s=0.001) is None
        r = srv.wait(rid)
        assert r is not None and r["total_steps"] > 0
        with pytest.raises(labs.LabsError) as e:
            srv.poll(rid)                                 # already collected
        assert e.value.code == labs.LABS_ENOTFOUND
        with pytest.raises(labs.LabsError) as e:
            srv.poll(12345)
        assert e.value.code == labs.LABS_ENOTFOUND
        for bad in [(28, 4, 10), (385, 4, 10), (27, 0, 10), (27, 4, -1)]:
            with pytest.raises(labs.LabsError) as e:
                srv.submit(*bad)
            assert e.value.code == labs.LABS_EINVAL
        bad_start = np.array([[1 << 20]], dtype=np.uint64)     # bit above D = 14
        with pytest.raises(labs.LabsError):
            srv.submit(27, 1, 10, starts=bad_start)


def test_destroy_with_work_in_flight():
    labs = _labs()
    srv = labs.Server(pool_bytes=POOL, chunk_steps=512)
    for i in range(4):
        srv.submit(221, 256, 20000, seed=i)
    time.sleep(0.05)
    srv.close()                                           # returns after the current launch
    srv.close()


@pytest.mark.parametrize("chunk", [0, 700])
def test_whole_space_server_matches_standalone_and_oracle(chunk):
    """A whole-space server (whole_space=True): requests of odd and even L
    across the three kernel groups, with spread arrivals, explicit starts and
    an empty walk; every request equals its standalone labs_full_walks run,
    and the oracle on its first walks."""
    labs = _labs()
    reqs = [dict(L=L, n=n, walk_len=wl, seed=70 + i)
            for i, (L, n, wl) in enumerate([(20, 96, 2500), (64, 130, 1800), (128, 64, 1500),
                                            (150, 70, 900), (200, 40, 700), (255, 33, 500)])]
    reqs.append(dict(L=50, n=8, walk_len=0, seed=3))
    keys = I.random_full_keys(97, 24, seed=9)
    reqs.append(dict(L=97, n=24, walk_len=1200, seed=0, starts=keys))
    with labs.Server(pool_bytes=POOL, chunk_steps=chunk, whole_space=True) as srv:
        ids = []
        for i, q in enumerate(reqs):
            ids.append(srv.submit(q["L"], q["n"], q["walk_len"], q["seed"], q.get("starts")))
            if i % 2 == 1:
                time.sleep(0.02)
        out = [srv.wait(rid, timeout_s=120) for rid in ids]
        st = srv.stats()
        with pytest.raises(labs.LabsError) as e:
            srv.submit(256, 4, 10)                        # whole space: L <= 255
        assert e.value.code == labs.LABS_EINVAL
    for q, r in zip(reqs, out):
        assert r is not None
        st_t = None if "starts" not in q else torch.from_numpy(I.as_int64_keys(q["starts"])).cuda()
        alone = labs.full_walks(q["L"], q["n"], q["walk_len"], seed=q["seed"], starts_t=st_t)
        torch.cuda.synchronize()
        alone = {k: v.cpu().numpy() for k, v in alone.items() if v is not None}
        _assert_same(r, alone)
    for q, r in [(reqs[0], out[0]), (reqs[4], out[4]), (reqs[-1], out[-1])]:
        starts = q["starts"] if "starts" in q else O.full_starts(q["L"], 2, q["seed"])
        for i in range(2):
            o = O.full_walk(q["L"], starts[i], q["walk_len"])
            assert r["best_E"][i] == o.best_E and r["digest"][i] == o.digest
            assert r["steps_done"][i] == o.steps
    assert st["completed"] == len(reqs) and st["pool_used"] == 0
