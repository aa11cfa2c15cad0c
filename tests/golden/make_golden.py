"""Writes the full-length walk results the GPU parity tests compare against.

Every value here comes from the CPU oracle (``oracle/``): walks follow Eq. 3
and Alg. 2 (walk length counts moves, ties to the lowest free-bit index, best
kept with a strict "<" from the first pivot, a trapped walk stops), every
neighbour energy recomputed from Eq. 1 on the Eq. 2 expansion.  Starts are the
SplitMix64 starts of the seeded workloads; sampled walk indices come from
``labs_inputs.sample_indices`` (random numbers only).

Workloads (all full length, as the benchmark runs them):

* ``walks_L151_seed0_131072moves.json`` -- L = 151, 65,536 walks from seed 0,
  131,072 moves: walks 0..15 plus 16 seeded-random indices.
* ``walks_L101_seed0_65536moves.json`` -- L = 101, 16,384 walks from seed 0,
  65,536 moves: walks 0..63 plus 64 seeded-random indices.
* ``batch_mixedL_61_223_32768moves.json`` -- 256 instances, L_i uniform odd in
  [61, 223] (``labs_inputs.odd_lengths(256, 61, 223, seed=0)``), instance i
  seeded with i, 1,024 walks x 32,768 moves: walk 0 and one seeded-random walk
  of every instance.

Usage (repo root): ``python tests/golden/make_golden.py [--threads N] [--only NAME]``.
The oracle needs about 3.5 CPU-hours in all (O(D L^2) per move; 35 minutes
on 6 threads of a 2.7 GHz Xeon); it runs the walks on N host threads.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import labs_inputs as I  # noqa: E402
from oracle import oracle as O  # noqa: E402


def _oracle_tag() -> str:
    with open(os.path.join(ROOT, "oracle", "labs_oracle.cpp"), "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def headline_jobs():
    L, n, wl = 151, 65536, 131072
    idx = I.sample_indices(n, 16, 16, seed=31)
    st = O.starts(L, n, 0)
    return "walks_L151_seed0_131072moves.json", dict(L=L, n_walks=n, walk_len=wl, seed=0), \
        [dict(L=L, walk=int(w), start=st[w], walk_len=wl) for w in idx]


def config2_jobs():
    L, n, wl = 101, 16384, 65536
    idx = I.sample_indices(n, 64, 64, seed=21)
    st = O.starts(L, n, 0)
    return "walks_L101_seed0_65536moves.json", dict(L=L, n_walks=n, walk_len=wl, seed=0), \
        [dict(L=L, walk=int(w), start=st[w], walk_len=wl) for w in idx]


def batch_jobs():
    Ls = [int(L) for L in I.odd_lengths(256, 61, 223, seed=0)]
    wl, n = 32768, 1024
    jobs = []
    for i, L in enumerate(Ls):
        st = O.starts(L, n, i)
        for w in I.sample_indices(n, 1, 1, seed=1000 + i):
            jobs.append(dict(L=L, inst=i, walk=int(w), start=st[w], walk_len=wl))
    return "batch_mixedL_61_223_32768moves.json", \
        dict(n_instances=256, L_range=[61, 223], n_walks=n, walk_len=wl, seed="instance index"), jobs


def run_jobs(jobs, threads):
    def one(job):
        r = O.walk(job["L"], job["start"], job["walk_len"], trace=False)
        out = {k: v for k, v in job.items() if k not in ("start", "walk_len")}
        out.update(best_E=r.best_E, best_seq=[int(x) for x in r.best_seq],
                   steps_done=r.steps, digest=int(r.digest))
        return out
    # longest walks first, so the pool ends on short ones
    order = sorted(range(len(jobs)), key=lambda k: -jobs[k]["L"])
    res = [None] * len(jobs)
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        futs = {ex.submit(one, jobs[k]): k for k in order}
        for f in cf.as_completed(futs):
            res[futs[f]] = f.result()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", type=str, default="")
    args = ap.parse_args()
    for make in (headline_jobs, config2_jobs, batch_jobs):
        name, workload, jobs = make()
        if args.only and args.only not in name:
            continue
        t0 = time.time()
        res = run_jobs(jobs, args.threads)
        doc = {
            "source": "oracle/labs_oracle.cpp (Eq. 1 direct energies, Eq. 2 expansion, "
                      "Eq. 3 / Alg. 2 walk rules); written by tests/golden/make_golden.py",
            "oracle_sha1_12": _oracle_tag(),
            "workload": workload,
            "walks": res,
        }
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(doc, f, indent=0)
            f.write("\n")
        print(f"{name}: {len(res)} walks in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
