"""Benchmark of the skew-symmetric LABS walk engine on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
labs_walks over the headline workload (L = 151, 65,536 walks of 131,072 moves
from seeded uniform starts).  Prints one JSON line with walk steps/s (Sum of
steps_done over the timed steps / time), neighbour evaluations/s, the INT32
VALU roofline of the walk kernel, the served stream (p50/p99 latency and
served vs plain-batch steps/s at 10, 25 and 200 req/s) and the CPU oracle baseline.
Other workloads run alone under their flags (--full, --full-batch, --paper-regime,
--mixed-batch, --serve-sweep, --serve-full-sweep, --solve-target).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Headline workload: walks at L = 151.  At load factor 0.55 the 65,536 visited
# tables (131,073 keys each, 12-byte entries, 10 per 128-byte bucket) take
# 186 GiB, so every walk stays resident in one launch.
WORKLOAD = dict(L=151, n_walks=65536, walk_len=131072)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit lane-op per cycle.
INT32_VALU_PEAK = 256 * 4 * 16 * 2.4e9


def lag_words(L: int) -> int:
    return ((L - 1) // 2 + 31) // 32


def planes_of(nw: int, w: int) -> int:
    lmax = min(64 * nw + 1, 383)
    mx = (lmax - 64 * w - 1) // 2
    b = 0
    while (1 << b) < mx:
        b += 1
    return 1 + b


# Plane caps reported per scan by the walk kernel, in the order of cap_steps.
CAPS = (4, 5, 6, 0)


def ops_per_scan(L: int, cap: int = 0) -> int:
    """Algorithmic 32-bit lane-ops of one neighbourhood scan (all D candidates)
    in the bit-sliced form: one 3-input bitwise op and one popcount per C
    plane word whose lag word holds at least one lag of the candidate's
    forward range, the same for its backward range, and one pair per word of
    the squared term.  Words outside a candidate's lag range are not counted
    (the kernel skips them).  cap > 0: every lag word is evaluated on `cap`
    planes (exact while every c_t fits in cap bits); cap = 0: on the stored
    per-word plane counts."""
    D, m = (L + 1) // 2, (L - 1) // 2
    nw = lag_words(L)
    pl = [planes_of(nw, w) if cap == 0 else min(cap, planes_of(nw, w)) for w in range(nw)]
    tot = 0
    for j in range(1, D + 1):
        nc = D if j & 1 else m
        r = (j - 1) >> 1
        nF = nc - 1 - r if j < D else 0
        nB = r
        fw, bw, q = (nF + 31) // 32, (nB + 31) // 32, (min(nF, nB) + 31) // 32
        tot += 2 * (sum(pl[:fw]) + sum(pl[:bw]) + q)
    return tot


def ops_per_candidate(L: int) -> float:
    """Uncapped algorithmic lane-ops per neighbour evaluation (average over j)."""
    return ops_per_scan(L, 0) / ((L + 1) // 2)


def full_planes_of(nw: int, w: int) -> int:
    mx = (32 * nw + 1 - 1 - 32 * w) // 2 + 1
    b = 0
    while (1 << b) < mx:
        b += 1
    return 1 + b


def full_ops_per_scan(L: int, cap: int = 0) -> int:
    """Algorithmic 32-bit lane-ops of one whole-space neighbourhood scan (all L
    positions): per lag word of a candidate's forward range one 3-input
    bitwise op and one popcount per c plane plus one pair for the even-C
    correction, the same for its backward range, and one pair per word of the
    squared term; cap as in ops_per_scan."""
    nw = (L - 1 + 31) // 32
    pl = [full_planes_of(nw, w) if cap == 0 else min(cap, full_planes_of(nw, w)) for w in range(nw)]
    tot = 0
    for i in range(1, L + 1):
        nF, nB = L - i, i - 1
        fw, bw, q = (nF + 31) // 32, (nB + 31) // 32, (min(nF, nB) + 31) // 32
        tot += 2 * (sum(pl[:fw]) + fw + sum(pl[:bw]) + bw + q)
    return tot


def kernel_source_tag(name: str = "labs_kernels.hip") -> str:
    """sha1 prefix of a kernel source together with the device headers it
    includes (a change to any of them changes the kernel)."""
    import hashlib
    h = hashlib.sha1()
    for part in (name, "labs_device.h", "labs_internal.h"):
        with open(os.path.join(ROOT, "paper_2210_15962_amd", "csrc", part), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def load_counter_traffic(kernel_tag: str, name: str = "walk_kernel_L151_traffic.json"):
    """HBM bytes per launch measured by rocprofv3 --pmc, if recorded for this
    kernel build (profiles/<name>.json written from the counter runs)."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            d = json.load(f)
        if d.get("kernel_tag") == kernel_tag:
            return d.get("bytes_per_launch")
    except (OSError, ValueError):
        pass
    return None


def cpu_model() -> str:
    """The host CPU's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _cpu_rates(total_steps: int, dt: float, cores: int, evals_per_step: int) -> dict:
    return {"per_core_steps_per_s": total_steps / dt / cores,
            "evals_per_s": total_steps * evals_per_step / dt,
            "per_core_evals_per_s": total_steps * evals_per_step / dt / cores,
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def cpu_baseline(L: int, seconds_target: float = 15.0):
    """The CPU oracle (untuned) on a bounded sample of the same workload."""
    import numpy as np
    from oracle import oracle as O
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(cores, 64))
    # calibrate: one walk of 256 moves on one core
    st = O.starts(L, cores, seed=0)
    t0 = time.time()
    O.walk(L, st[0], 256, trace=False)
    per_step = (time.time() - t0) / 256
    steps = int(max(256, min(131072, seconds_target / max(per_step, 1e-9))))
    t0 = time.time()
    res = O.walks(L, st, steps, n_threads=cores)
    dt = time.time() - t0
    total = int(res["steps_done"].sum())
    return {"value": total / dt, "unit": "walk steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} walks x {steps} moves at L={L} (seed 0 starts), "
                      f"one walk per host thread, {dt:.1f} s wall",
            **_cpu_rates(total, dt, cores, (L + 1) // 2)}


def cpu_baseline_full(L: int, seconds_target: float = 15.0):
    """The whole-space CPU oracle (untuned) on a bounded sample of the workload."""
    from oracle import oracle as O
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(cores, 64))
    st = O.full_starts(L, cores, seed=0)
    t0 = time.time()
    O.full_walk(L, st[0], 64, trace=False)
    per_step = (time.time() - t0) / 64
    steps = int(max(64, min(32768, seconds_target / max(per_step, 1e-9))))
    t0 = time.time()
    res = O.full_walks(L, st, steps, n_threads=cores)
    dt = time.time() - t0
    total = int(res["steps_done"].sum())
    return {"value": total / dt, "unit": "walk steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} whole-space walks x {steps} moves at L={L} (seed 0 starts), "
                      f"one walk per host thread, {dt:.1f} s wall",
            **_cpu_rates(total, dt, cores, L)}


FULL_WORKLOAD = dict(L=128, n_walks=65536, walk_len=32768)


def calibration_copy(mib: int):
    """A plain device copy of known size, run for the HBM-counter scale."""
    import torch
    if mib:
        src_t = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t


def run_full(L: int, n: int, walk_len: int, steps: int, warmup: int, cpu: bool, calib_mib: int = 0):
    """Whole-space walks (labs_full_walks): walk steps/s, neighbour evals/s
    (L per move) and the INT32 VALU roofline of the whole-space kernel."""
    import torch
    from paper_2210_15962_amd import labs
    plan = labs.make_plan()
    ws = labs.alloc_workspace(labs.full_workspace_bytes(L, n, walk_len, plan))
    calibration_copy(calib_mib)
    for w in range(warmup):
        labs.full_walks(L, n, walk_len, seed=1000 + w, plan=plan, workspace=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    kernel_ms, results = 0.0, []
    t0 = time.perf_counter()
    for s in range(steps):
        ev0.record(stream)
        res = labs.full_walks(L, n, walk_len, seed=s, plan=plan, workspace=ws, cap_steps=True)
        ev1.record(stream)
        ev1.synchronize()
        kernel_ms += ev0.elapsed_time(ev1)
        results.append((res["steps_done"], res["cap_steps"]))
    wall = time.perf_counter() - t0
    del ws
    torch.cuda.empty_cache()
    total = int(sum(int(r[0].sum().item()) for r in results))
    cap_scans = [int(sum(int(r[1][:, k].sum().item()) for r in results)) for k in range(4)]
    alg_ops = sum(c * full_ops_per_scan(L, cap) for c, cap in zip(cap_scans, CAPS))
    avg_launch_s = kernel_ms / 1e3 / steps
    achieved = alg_ops / steps / avg_launch_s
    nw = (L - 1 + 31) // 32
    tag = f"full_walk_kernel<NW={nw}>@{kernel_source_tag('labs_full.hip')}"
    sps = total / wall
    out = {"metric": "whole-space walk steps/s", "value": sps, "unit": "walk steps/s",
           "steps": steps, "warmup": warmup, "ms_per_step": wall * 1e3 / steps, "dtype": "int32",
           "data": "synthetic",
           "config": {"workload": f"whole-space LABS self-avoiding walks, L={L}, {n} walks x "
                                  f"{walk_len} moves, seeded uniform starts",
                      "L": L, "n_walks": n, "walk_len": walk_len, "lanes_per_walk": 4},
           "neighbour_evals_per_s": sps * L,
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_VALU_PEAK / 1e12,
                        "unit": "TOP/s", "frac": achieved / INT32_VALU_PEAK,
                        "traffic": load_counter_traffic(tag, f"full_walk_kernel_L{L}_traffic.json"),
                        "kernel": tag, "avg_launch_ms": avg_launch_s * 1e3,
                        "alg_ops_per_launch": alg_ops / steps,
                        "ops_per_neighbour_eval": alg_ops / max(sum(cap_scans) * L, 1),
                        "scans_by_plane_cap": {str(c or "all"): v for c, v in zip(CAPS, cap_scans)}}}
    if cpu:
        out["cpu_baseline"] = cpu_baseline_full(L)
    return out


# Served streams: skew-symmetric requests (L odd in [121, 301], 4,096 walks x
# 65,536 moves) or whole-space requests (L in [64, 255], 4,096 walks x 16,384
# moves), both from seeded starts.
SERVE_SKEW = dict(lo=121, hi=301, n_walks=4096, walk_len=65536, seed_base=10_000)
SERVE_FULL = dict(lo=64, hi=255, n_walks=4096, walk_len=16384, seed_base=20_000)


def serve_workload(n_req: int, rate: float, seed: int = 0, full: bool = False):
    """Served stream: Poisson arrivals at `rate`, L uniform over the stream's
    range (odd lengths for skew-symmetric requests, every length for
    whole-space ones)."""
    import labs_inputs as I
    w = SERVE_FULL if full else SERVE_SKEW
    Ls = (I.lengths if full else I.odd_lengths)(n_req, w["lo"], w["hi"], seed=seed)
    t = I.poisson_arrivals(rate, n_req, seed=seed + 1)
    return [dict(L=int(L), n_walks=w["n_walks"], walk_len=w["walk_len"], seed=w["seed_base"] + i,
                 t_arrive=float(t[i])) for i, L in enumerate(Ls)]


def run_plain_batch(n_req: int, load_factor: float, full: bool = False):
    """The served stream's requests as one plain mixed-L batch (persistent
    launches); the workspace is allocated before the timed region."""
    import torch
    from paper_2210_15962_amd import labs
    reqs = serve_workload(n_req, 1.0, full=full)
    specs = [dict(L=q["L"], n_walks=q["n_walks"], walk_len=q["walk_len"], seed=q["seed"],
                  load_factor=load_factor) for q in reqs]
    if full:
        ws = labs.alloc_workspace(labs.full_batch_workspace_bytes(specs))
    else:
        ws = labs.alloc_workspace(labs.batch_workspace_bytes(specs))
    torch.cuda.synchronize()
    tb = time.perf_counter()
    out = (labs.full_walks_batch if full else labs.walks_batch)(specs, workspace=ws)
    torch.cuda.synchronize()
    tb = time.perf_counter() - tb
    bsteps = int(sum(int(o["steps_done"].sum().item()) for o in out))
    bdig = [o["digest"].cpu().numpy() for o in out]
    del out, ws
    torch.cuda.empty_cache()
    return bsteps / tb, bsteps, bdig


def run_serving(n_req: int, rate: float, load_factor: float, chunk: int, batch=None,
                pool_frac: float = 0.85, full: bool = False):
    """Serve the stream through labs_serve_* (Poisson arrivals at `rate`; a
    whole-space server when `full`) and compare with the same requests as one
    plain batch; returns latency percentiles and both throughputs."""
    import numpy as np
    import torch
    from paper_2210_15962_amd import labs
    w = SERVE_FULL if full else SERVE_SKEW
    reqs = serve_workload(n_req, rate, full=full)
    batch_rate, bsteps, bdig = batch if batch is not None else run_plain_batch(n_req, load_factor, full)
    free, _ = torch.cuda.mem_get_info()
    pool = int(free * pool_frac)
    with labs.Server(pool_bytes=pool, load_factor=load_factor, chunk_steps=chunk, whole_space=full) as srv:
        ids = []
        t0 = time.perf_counter()
        for q in reqs:
            dt = q["t_arrive"] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            ids.append(srv.submit(q["L"], q["n_walks"], q["walk_len"], q["seed"]))
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    lat = np.array([(r["t_done_ns"] - r["t_submit_ns"]) / 1e6 for r in res])
    steps = sum(r["total_steps"] for r in res)
    span = (max(r["t_done_ns"] for r in res) - min(r["t_submit_ns"] for r in res)) / 1e9
    served = steps / span
    same = all(np.array_equal(r["digest"], d.view(np.uint64)) for r, d in zip(res, bdig))
    return {"rate_req_per_s": rate, "requests": n_req, "whole_space": full,
            "walks_per_request": w["n_walks"], "moves_per_walk": w["walk_len"], "L_range": [w["lo"], w["hi"]],
            "chunk_steps": chunk,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "served_steps_per_s": served, "served_busy_steps_per_s": steps / (st["busy_ns"] / 1e9),
            "batch_steps_per_s": batch_rate, "served_over_batch": served / batch_rate,
            "launches": st["launches"], "pool_gib": st["pool_bytes"] / 2**30,
            "pool_peak_gib": st["pool_peak"] / 2**30,
            "offered_over_capacity": rate * w["n_walks"] * w["walk_len"] / batch_rate,
            "served_equals_batch": bool(same and steps == bsteps)}


def run_mixed_batch(steps: int, warmup: int, autotune: bool):
    """256 instances, L uniform odd in [61, 223], 1,024 walks x 32,768 moves
    each, in one persistent launch captured in a hipGraph; replays timed with
    HIP events.  With autotune, every distinct L is tuned first."""
    import torch
    import labs_inputs as I
    from paper_2210_15962_amd import labs
    Ls = [int(L) for L in I.odd_lengths(256, 61, 223, seed=0)]
    specs = [dict(L=L, n_walks=1024, walk_len=32768, seed=i, cap_steps=True) for i, L in enumerate(Ls)]
    tuned = {}
    t_tune = 0.0
    if autotune:
        t0 = time.perf_counter()
        for L in sorted(set(Ls)):
            tuned[L] = labs.autotune(L)
        t_tune = time.perf_counter() - t0
    g = labs.BatchGraph(specs)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        g.launch()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        ev0.record(stream)
        res = g.launch()
        ev1.record(stream)
        ev1.synchronize()
        ms += ev0.elapsed_time(ev1)
    wall = time.perf_counter() - t0
    # every replay recomputes the same outputs: read them once
    per_replay = int(sum(int(r["steps_done"].sum().item()) for r in res))
    total = per_replay * steps
    alg = 0
    caps_all = [0, 0, 0, 0]
    for L, r in zip(Ls, res):
        c = r["cap_steps"].sum(0).cpu().numpy()
        alg += sum(int(c[k]) * ops_per_scan(L, cap) for k, cap in enumerate(CAPS))
        caps_all = [caps_all[k] + int(c[k]) for k in range(4)]
    g.close()
    achieved = alg / (ms / steps / 1e3)
    tag = f"batch_kernel@{kernel_source_tag()}"
    lanes = {}
    for L in Ls:
        k = labs.tune_get(L)[0]
        lanes[k] = lanes.get(k, 0) + 1
    return {"workload": "256 instances, L uniform odd in [61, 223], 1024 walks x 32768 moves, "
                        "one persistent launch per replay (hipGraph)",
            "steps_per_s": total / wall, "steps_per_s_events": per_replay / (ms / steps / 1e3),
            "ms_per_launch": ms / steps, "replays": steps,
            "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_VALU_PEAK / 1e12,
                         "unit": "TOP/s", "frac": achieved / INT32_VALU_PEAK,
                         "traffic": load_counter_traffic(tag, "batch_kernel_mixedL_61_223_traffic.json"),
                         "kernel": tag, "alg_ops_per_launch": alg,
                         "scans_by_plane_cap": {str(c or "all"): v for c, v in zip(CAPS, caps_all)}},
            "autotuned": autotune, "tune_seconds": t_tune,
            "instances_by_lanes_per_walk": {str(k): v for k, v in sorted(lanes.items())},
            "distinct_L": len(set(Ls))}


def run_full_batch(steps: int, warmup: int):
    """Whole-space mixed-length batch: 128 instances, L uniform over [64, 255]
    (every length, odd or even), 1,024 walks x 8,192 moves each, instance i
    seeded with i; one labs_full_walks_batch call per step, timed with HIP
    events on the launch stream, the workspace allocated beforehand."""
    import torch
    import labs_inputs as I
    from paper_2210_15962_amd import labs
    Ls = [int(L) for L in I.lengths(128, 64, 255, seed=0)]
    specs = [dict(L=L, n_walks=1024, walk_len=8192, seed=i, cap_steps=True) for i, L in enumerate(Ls)]
    ws = labs.alloc_workspace(labs.full_batch_workspace_bytes(specs))
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        labs.full_walks_batch(specs, workspace=ws)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms, total, alg = 0.0, 0, 0
    caps_all = [0, 0, 0, 0]
    t0 = time.perf_counter()
    results = []
    for _ in range(steps):
        ev0.record(stream)
        res = labs.full_walks_batch(specs, workspace=ws)
        ev1.record(stream)
        ev1.synchronize()
        ms += ev0.elapsed_time(ev1)
        results.append(res)
    wall = time.perf_counter() - t0
    for res in results:
        for L, r in zip(Ls, res):
            total += int(r["steps_done"].sum().item())
            c = r["cap_steps"].sum(0).cpu().numpy()
            alg += sum(int(c[k]) * full_ops_per_scan(L, cap) for k, cap in enumerate(CAPS))
            caps_all = [caps_all[k] + int(c[k]) for k in range(4)]
    del ws
    torch.cuda.empty_cache()
    achieved = alg / (ms / 1e3)
    return {"workload": "whole space, 128 instances, L uniform in [64, 255], 1024 walks x 8192 moves, "
                        "persistent launches per class group",
            "steps_per_s": total / wall, "steps_per_s_events": total / (ms / 1e3),
            "ms_per_step": ms / steps, "steps": steps,
            "neighbour_evals_per_s": sum(int(r["steps_done"].sum().item()) * L for L, r in zip(Ls, results[-1]))
                                     / (ms / steps / 1e3),
            "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_VALU_PEAK / 1e12,
                         "unit": "TOP/s", "frac": achieved / INT32_VALU_PEAK, "traffic": None,
                         "kernel": f"full_batch_kernel@{kernel_source_tag('labs_full.hip')}",
                         "alg_ops_per_step": alg / steps,
                         "scans_by_plane_cap": {str(c or "all"): v for c, v in zip(CAPS, caps_all)}}}


def run_solve_target(L: int, target: int, time_limit: float, walks: int, seed: int):
    """Alg. 1 driver until E <= target (a Table 1 energy) or the time limit:
    time-to-target and NFEs-to-target against the lambda model's mean 1/lambda."""
    from paper_2210_15962_amd import labs
    r = labs.solve(L, walks, target_E=target, time_limit_s=time_limit, seed=seed)
    D = (L + 1) // 2
    return {"workload": f"Alg. 1 rounds of {walks} walks x 8D={8 * D} moves at L={L}, target E <= {target}",
            "seed": seed, "reached": r["reached_target"], "best_E": r["best_E"],
            "best_key_hex": "".join("%016x" % int(w) for w in r["best_seq"][::-1]),
            "time_to_target_s": r["target_seconds"], "nfes_to_target": r["target_nfes"],
            "model_mean_nfes": 1.0 / labs.lambda_model(L), "rounds": r["rounds"],
            "nfes_per_s": r["nfes"] / r["seconds"], "walk_steps_per_s": r["walk_steps"] / r["seconds"],
            "seconds": r["seconds"]}


A100_DERIVED_EVALS_PER_S = 5.5e9    # sokol on an A100, L = 225..247 (from Eq. 7, the lambda model and Table 1)


def run_paper_regime(Ls, walks: int, rounds: int, warmup: int):
    """The paper's own regime (Sec. 4): rounds of fresh walks of 8 D moves each,
    timed per round including the visited-table clears and the initial energies,
    reported in the paper's evaluation count (D - 1 per move, Alg. 1)."""
    import torch
    from paper_2210_15962_amd import labs
    out = []
    for L in Ls:
        D = (L + 1) // 2
        wl = 8 * D
        plan = labs.make_plan()
        ws = labs.alloc_workspace(labs.workspace_bytes(L, walks, wl, plan))
        for w in range(warmup):
            labs.walks(L, walks, wl, seed=10_000 + w, plan=plan, workspace=ws)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        steps, ms = 0, 0.0
        for r in range(rounds):
            ev0.record(stream)
            res = labs.walks(L, walks, wl, seed=r * walks, plan=plan, workspace=ws)
            ev1.record(stream)
            ev1.synchronize()
            ms += ev0.elapsed_time(ev1)
            steps += int(res["steps_done"].sum().item())
        del ws
        torch.cuda.empty_cache()
        sps = steps / (ms / 1e3)
        out.append({"workload": f"paper regime: L={L}, rounds of {walks} walks x 8D={wl} moves",
                    "L": L, "walks_per_round": walks, "walk_len": wl, "rounds": rounds,
                    "ms_per_round": ms / rounds, "walk_steps_per_s": sps,
                    "paper_evals_per_s": sps * (D - 1), "neighbour_evals_per_s": sps * D,
                    "vs_a100_derived": sps * (D - 1) / A100_DERIVED_EVALS_PER_S})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lanes", type=int, default=4, help="lanes per walk")
    ap.add_argument("--concurrent", type=int, default=65536, help="walks resident at once")
    ap.add_argument("--load-factor", type=float, default=0.55)
    ap.add_argument("--walk-len", type=int, default=WORKLOAD["walk_len"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-rates", type=str, default="10,25,200",
                    help="arrival rates (req/s) of the serving legs in the default run")
    ap.add_argument("--serve-chunk", type=int, default=0,
                    help="moves per launch per request (0: launches end when a request can be "
                         "admitted or has finished)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-sweep", type=str, default="",
                    help="comma-separated arrival rates: serve only, one JSON line per rate")
    ap.add_argument("--serve-full-sweep", type=str, default="",
                    help="as --serve-sweep for a whole-space server (L in [64, 255], 4096 walks x "
                         "16384 moves per request)")
    ap.add_argument("--solve-target", type=str, default="",
                    help="L:E -- Alg. 1 driver until E or --solve-time-limit (time-to-target)")
    ap.add_argument("--solve-time-limit", type=float, default=600.0)
    ap.add_argument("--solve-walks", type=int, default=262144)
    ap.add_argument("--solve-seeds", type=str, default="0")
    ap.add_argument("--full", type=int, default=0,
                    help="whole-space walks at this L only (65,536 walks x 32,768 moves by default)")
    ap.add_argument("--full-walks", type=int, default=FULL_WORKLOAD["n_walks"])
    ap.add_argument("--full-walk-len", type=int, default=FULL_WORKLOAD["walk_len"])
    ap.add_argument("--paper-regime", type=str, default="",
                    help="comma-separated L: rounds of fresh 8D-move walks (Sec. 4) only")
    ap.add_argument("--paper-walks", type=int, default=262144)
    ap.add_argument("--full-batch", action="store_true",
                    help="whole-space mixed-length batch (128 instances, L in [64, 255]) only")
    ap.add_argument("--mixed-batch", action="store_true",
                    help="256-instance mixed-L batch (hipGraph replays) only, default then autotuned")
    ap.add_argument("--no-autotune", action="store_true",
                    help="with --mixed-batch: the default plan only (no autotuned leg)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(walks are independent: N GPUs would each run their own batch).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2210_15962_amd import labs

    if args.solve_target:
        Ls, Es = args.solve_target.split(":")
        for sd in [int(x) for x in args.solve_seeds.split(",")]:
            print(json.dumps(run_solve_target(int(Ls), int(Es), args.solve_time_limit, args.solve_walks, sd)),
                  flush=True)
        return

    if args.full:
        print(json.dumps(run_full(args.full, args.full_walks, args.full_walk_len, args.steps,
                                  args.warmup, not args.no_cpu_baseline, args.calibration_copy_mib)),
              flush=True)
        return

    if args.paper_regime:
        for r in run_paper_regime([int(x) for x in args.paper_regime.split(",")], args.paper_walks,
                                  args.steps, args.warmup):
            print(json.dumps(r), flush=True)
        return

    if args.full_batch:
        print(json.dumps(run_full_batch(args.steps, args.warmup)), flush=True)
        return

    if args.mixed_batch:
        calibration_copy(args.calibration_copy_mib)
        for tune in ((False,) if args.no_autotune else (False, True)):
            print(json.dumps(run_mixed_batch(args.steps, args.warmup, tune)), flush=True)
        return

    if args.serve_sweep or args.serve_full_sweep:
        full = bool(args.serve_full_sweep)
        batch = run_plain_batch(args.serve_requests, args.load_factor, full)
        for rate in [float(x) for x in (args.serve_full_sweep or args.serve_sweep).split(",")]:
            print(json.dumps(run_serving(args.serve_requests, rate, args.load_factor, args.serve_chunk,
                                         batch=batch, full=full)), flush=True)
        return

    L, n = WORKLOAD["L"], WORKLOAD["n_walks"]
    walk_len = args.walk_len
    D = (L + 1) // 2
    plan = labs.make_plan(lanes_per_walk=args.lanes, load_factor=args.load_factor,
                          max_concurrent=args.concurrent)
    conc = min(n, args.concurrent)
    launches = (n + conc - 1) // conc
    ws = labs.alloc_workspace(labs.workspace_bytes(L, n, walk_len, plan))
    stream = torch.cuda.current_stream()
    calibration_copy(args.calibration_copy_mib)

    def one_step(seed):
        return labs.walks(L, n, walk_len, seed=seed, plan=plan, workspace=ws, cap_steps=True)

    for w in range(args.warmup):
        one_step(1000 + w)
    torch.cuda.synchronize()

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    total_steps = 0
    kernel_ms = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for s in range(args.steps):
        ev0.record(stream)
        res = one_step(s)
        ev1.record(stream)
        results.append((res["steps_done"], res["cap_steps"]))
        ev1.synchronize()
        kernel_ms += ev0.elapsed_time(ev1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_steps = int(sum(int(r[0].sum().item()) for r in results))
    cap_scans = [int(sum(int(r[1][:, k].sum().item()) for r in results)) for k in range(4)]
    scans = sum(cap_scans)

    steps_per_s = total_steps / wall
    avg_launch_s = kernel_ms / 1e3 / (args.steps * launches)
    # algorithmic work: every scan priced at the plane count it needed
    alg_ops = sum(c * ops_per_scan(L, cap) for c, cap in zip(cap_scans, CAPS))
    alg_ops_per_launch = alg_ops / (args.steps * launches)
    achieved = alg_ops_per_launch / avg_launch_s
    tag = f"walk_kernel<NW={lag_words(L)},G={args.lanes}>@{kernel_source_tag()}"
    traffic = load_counter_traffic(tag)

    out = {
        "metric": "walk steps/s & neighbour evals/s at L=151 (% INT32 peak); served p50/p99 latency",
        "value": steps_per_s,
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"skew-symmetric LABS self-avoiding walks, L={L}, {n} walks x "
                               f"{walk_len} moves, seeded uniform starts",
                   "L": L, "n_walks": n, "walk_len": walk_len, "lanes_per_walk": args.lanes,
                   "walks_resident": conc, "launches_per_step": launches,
                   "load_factor": args.load_factor},
        "neighbour_evals_per_s": steps_per_s * D,
        "paper_evals_per_s": steps_per_s * (D - 1),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_VALU_PEAK / 1e12,
                     "unit": "TOP/s", "frac": achieved / INT32_VALU_PEAK, "traffic": traffic,
                     "kernel": tag, "avg_launch_ms": avg_launch_s * 1e3,
                     "alg_ops_per_launch": alg_ops_per_launch,
                     "ops_per_neighbour_eval": alg_ops / max(scans * D, 1),
                     "ops_per_neighbour_eval_uncapped": ops_per_candidate(L),
                     "scans_by_plane_cap": {str(c or "all"): v for c, v in zip(CAPS, cap_scans)}},
    }
    del ws
    torch.cuda.empty_cache()
    if not args.no_serve:
        # near capacity (10 req/s), just saturated (25) and far past it (200)
        batch = run_plain_batch(args.serve_requests, args.load_factor)
        out["serving"] = [run_serving(args.serve_requests, rate, args.load_factor, args.serve_chunk,
                                      batch=batch)
                          for rate in [float(x) for x in args.serve_rates.split(",")]]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(L)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
