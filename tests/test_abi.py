"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/labs.h, validates arguments, and its host helpers agree
with the oracle's packing conventions."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
import labs_inputs as I
from paper_2210_15962_amd import labs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "labs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(labs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["labs_energy", "labs_walks", "labs_walks_workspace_bytes", "labs_pack_skew",
              "labs_unpack_skew", "labs_expand_skew", "labs_starts", "labs_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(labs.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in labs.h but not exported"


def test_l_max_and_key_words():
    assert labs.l_max() == 383 == O.l_max()
    for L in [3, 5, 127, 129, 255, 257, 383]:
        assert labs.key_words(L) == O.key_words(L)
    for bad in [-1, 0, 1, 2, 4, 384, 385, 1001]:
        assert labs.key_words(bad) == 0


@pytest.mark.parametrize("L", [3, 27, 101, 127, 129, 151, 255, 301, 383])
def test_pack_unpack_expand_match_oracle(L):
    keys = I.random_start_keys(L, 16, seed=L)
    x = labs.unpack_skew(keys, L)
    for i in range(16):
        assert np.array_equal(x[i], O.unpack(keys[i], L))
    assert np.array_equal(labs.pack_skew(x, L), keys)
    s = labs.expand_skew(x, L)
    for i in range(16):
        assert np.array_equal(s[i], O.expand_skew(x[i], L))


def test_host_helpers_reject_bad_input():
    with pytest.raises(labs.LabsError):
        labs.pack_skew(np.array([[1, 0]], dtype=np.int8), 3)
    with pytest.raises(labs.LabsError):
        labs.expand_skew(np.array([[1, 2]], dtype=np.int8), 3)
    with pytest.raises(labs.LabsError):
        labs.unpack_skew(np.array([[0b100]], dtype=np.uint64), 3)   # bit above D=2
    lib = labs.lib()
    buf = np.zeros(8, dtype=np.uint64)
    for bad_L in [2, 4, 1, 0, -3, 385]:
        assert lib.labs_pack_skew(buf.ctypes.data, bad_L, 1, buf.ctypes.data) == labs.LABS_EINVAL
    assert lib.labs_pack_skew(buf.ctypes.data, 27, -1, buf.ctypes.data) == labs.LABS_EINVAL
    assert lib.labs_pack_skew(None, 27, 1, buf.ctypes.data) == labs.LABS_EINVAL
    assert b"L=" in lib.labs_last_error() or len(lib.labs_last_error()) > 0


def test_workspace_sizing():
    # one bucket of 128 bytes holds 10 entries of 12 bytes (D <= 95), 8 of 16
    # (D <= 127) or 4 of 32
    b = labs.workspace_bytes(27, 64, 4096)
    per_walk = b // 64
    assert per_walk % 128 == 0
    assert per_walk // 128 * 10 * 0.5 >= 4097           # load factor 0.5 by default
    assert (per_walk // 128 - 1) * 10 * 0.5 < 4097
    assert labs.min_workspace_bytes(27, 4096) == per_walk
    p = labs.make_plan(load_factor=0.25)
    assert labs.min_workspace_bytes(27, 4096, p) >= 2 * per_walk - 128
    assert labs.workspace_bytes(27, 64, 4096, labs.make_plan(max_concurrent=8)) == 8 * per_walk
    # 16-byte entries from D = 96 on, 32-byte entries from D = 128 on
    ratio16 = labs.min_workspace_bytes(191, 100_000) / labs.min_workspace_bytes(189, 100_000)
    assert abs(ratio16 - 10 / 8) < 1e-3
    assert labs.min_workspace_bytes(255, 1000) >= labs.min_workspace_bytes(253, 1000) * 2 - 128
    assert labs.workspace_bytes(27, 0, 10) == 0


def test_walks_argument_errors_before_any_launch():
    lib = labs.lib()
    out = labs.WalkOut(1, 1, 1, None, None, None, 0)
    ws = ctypes.c_void_p(1)
    ref = ctypes.byref
    # invalid L, negative sizes, missing workspace / outputs, bad plans
    assert lib.labs_walks(None, 28, 4, 10, 0, ref(out), ws, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_walks(None, 27, -1, 10, 0, ref(out), ws, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_walks(None, 27, 4, -1, 0, ref(out), ws, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_walks(None, 27, 4, 10, 0, None, ws, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_walks(None, 27, 4, 10, 0, ref(out), None, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_walks(None, 27, 4, 10, 0, ref(out), ws, 8, None, None) == labs.LABS_EINVAL
    bad = labs.make_plan(lanes_per_walk=3)
    assert lib.labs_walks(None, 27, 4, 10, 0, ref(out), ws, 1 << 30, ref(bad), None) == labs.LABS_EINVAL
    bad = labs.make_plan(load_factor=0.95)
    assert lib.labs_walks(None, 27, 4, 10, 0, ref(out), ws, 1 << 30, ref(bad), None) == labs.LABS_EINVAL
    missing = labs.WalkOut(1, None, 1, None, None, None, 0)
    assert lib.labs_walks(None, 27, 4, 10, 0, ref(missing), ws, 1 << 30, None, None) == labs.LABS_EINVAL
    tr = labs.WalkOut(1, 1, 1, None, None, None, 2)
    assert lib.labs_walks(None, 27, 4, 10, 0, ref(tr), ws, 1 << 30, None, None) == labs.LABS_EINVAL
    # zero walks is a no-op
    assert lib.labs_walks(None, 27, 0, 10, 0, ref(out), ws, 0, None, None) == labs.LABS_OK


def test_energy_argument_errors_before_any_launch():
    lib = labs.lib()
    assert lib.labs_energy(None, 0, 1, None, None) == labs.LABS_EINVAL
    assert lib.labs_energy(None, 1025, 1, None, None) == labs.LABS_EINVAL
    assert lib.labs_energy(None, 10, -1, None, None) == labs.LABS_EINVAL
    assert lib.labs_energy(None, 10, 1, None, None) == labs.LABS_EINVAL
    assert lib.labs_energy(None, 10, 0, None, None) == labs.LABS_OK
    assert lib.labs_starts(28, 1, 0, ctypes.c_void_p(1), None) == labs.LABS_EINVAL


def test_tune_table_roundtrip():
    lib = labs.lib()
    assert lib.labs_tune_set(28, 4, 0.5) == labs.LABS_EINVAL
    assert lib.labs_tune_set(29, 3, 0.5) == labs.LABS_EINVAL
    assert lib.labs_tune_set(29, 4, 0.95) == labs.LABS_EINVAL
    g, lf, found = labs.tune_get(31)
    assert (g, lf, found) == (4, 0.5, False)          # built-in default
    labs.tune_set(31, 8, 0.67)
    assert labs.tune_get(31) == (8, 0.67, True)
    labs.tune_set(31, 4, 0.5)


def test_batch_validation_before_any_launch():
    lib = labs.lib()
    empty = {"best_seq": None, "best_E": None, "steps_done": None, "digest": None}
    arr = labs.make_instances([dict(L=28, n_walks=4, walk_len=10)], [empty])
    ws = ctypes.c_void_p(1)
    assert lib.labs_walks_batch(arr, 1, ws, 1 << 30, None) == labs.LABS_EINVAL
    b = labs.U64(0)
    assert lib.labs_batch_workspace_bytes(arr, 1, ctypes.byref(b)) == labs.LABS_EINVAL
    arr = labs.make_instances([dict(L=27, n_walks=4, walk_len=10, lanes_per_walk=1)], [empty])
    assert lib.labs_walks_batch(arr, 1, ws, 1 << 30, None) == labs.LABS_EINVAL   # batches: 2/4/8
    arr = labs.make_instances([dict(L=27, n_walks=4, walk_len=10)], [empty])
    assert lib.labs_walks_batch(arr, 1, ws, 1 << 30, None) == labs.LABS_EINVAL   # no outputs
    assert lib.labs_walks_batch(arr, -1, ws, 1 << 30, None) == labs.LABS_EINVAL
    assert lib.labs_walks_batch(arr, 0, ws, 0, None) == labs.LABS_OK            # nothing to run


def test_full_batch_validation_before_any_launch():
    lib = labs.lib()
    empty = {"best_seq": None, "best_E": None, "steps_done": None, "digest": None}
    ws = ctypes.c_void_p(1)
    b = labs.U64(0)
    for bad in (dict(L=256, n_walks=4, walk_len=10), dict(L=2, n_walks=4, walk_len=10),
                dict(L=64, n_walks=4, walk_len=10, lanes_per_walk=2),   # whole space: 4 lanes
                dict(L=64, n_walks=4, walk_len=-1), dict(L=64, n_walks=4, walk_len=10)):  # no outputs
        arr = labs.make_instances([bad], [empty])
        assert lib.labs_full_walks_batch(arr, 1, ws, 1 << 30, None) == labs.LABS_EINVAL
        assert lib.labs_full_batch_workspace_bytes(arr, 1, ctypes.byref(b)) in (
            labs.LABS_EINVAL, labs.LABS_EDEVICE)           # outputs are checked before the device
    arr = labs.make_instances([dict(L=256, n_walks=4, walk_len=10)], [empty])
    assert lib.labs_full_batch_workspace_bytes(arr, 1, ctypes.byref(b)) == labs.LABS_EINVAL
    assert lib.labs_full_walks_batch(arr, -1, ws, 1 << 30, None) == labs.LABS_EINVAL
    assert lib.labs_full_walks_batch(arr, 0, ws, 0, None) == labs.LABS_OK       # nothing to run


def test_serve_validation_before_any_device_call():
    lib = labs.lib()
    h = ctypes.c_void_p()
    assert lib.labs_serve_create(None, None) == labs.LABS_EINVAL
    for cfg in [labs.ServeCfg(0, 0, 3, 0, 0.0), labs.ServeCfg(0, -1, 0, 0, 0.0),
                labs.ServeCfg(0, 0, 0, -5, 0.0), labs.ServeCfg(0, 0, 0, 0, 0.95)]:
        assert lib.labs_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == labs.LABS_EINVAL
        assert not h.value
    for cfg in [labs.ServeCfg(0, 0, 0, 0, 0.0, 2), labs.ServeCfg(0, 0, 8, 0, 0.0, 1)]:
        assert lib.labs_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == labs.LABS_EINVAL   # whole space: 0/1, 4 lanes
        assert not h.value
    rid = labs.U64(0)
    assert lib.labs_serve_submit(None, 27, 1, 1, 0, None, ctypes.byref(rid)) == labs.LABS_EINVAL
    assert lib.labs_serve_poll(None, 1, None) == labs.LABS_EINVAL
    assert lib.labs_serve_wait(None, 1, 0, None) == labs.LABS_EINVAL
    assert lib.labs_serve_stats(None, None) == labs.LABS_EINVAL
    assert lib.labs_serve_destroy(None) == labs.LABS_OK


def test_stopping_model_matches_oracle():
    import math
    for L in [71, 101, 121, 171, 223, 247]:
        assert labs.lambda_model(L) == pytest.approx(O.lambda_model(L), rel=1e-14)
        assert labs.nses_limit(L) == pytest.approx(O.nses_limit(L), rel=1e-14)
        n = labs.nses_limit(L, 0.99, 100)
        assert labs.optimality_probability(L, 100 * n) == pytest.approx(0.99, abs=1e-12)
        assert labs.optimality_probability(L, 1e9) == pytest.approx(O.optimality_probability(L, 1e9), rel=1e-14)
    for bad in [(0, 0.99, 100), (101, 0.0, 100), (101, 1.0, 100), (101, 0.5, 0)]:
        assert math.isnan(labs.nses_limit(*bad))
    assert math.isnan(labs.optimality_probability(101, -1.0))
    assert math.isnan(labs.lambda_model(0))


def test_solve_validation_before_any_launch():
    lib = labs.lib()
    nb = labs.U64(0)
    cfg = labs.SolveCfg(64, 0, 0, 0.0, 0.0, 0, 0, 0, labs.Plan(0, 0.0, 0))
    assert lib.labs_solve_workspace_bytes(27, ctypes.byref(cfg), ctypes.byref(nb)) == labs.LABS_EINVAL
    assert b"stopping" in lib.labs_last_error()
    cfg.max_rounds = 2
    assert lib.labs_solve_workspace_bytes(28, ctypes.byref(cfg), ctypes.byref(nb)) == labs.LABS_EINVAL
    assert lib.labs_solve_workspace_bytes(27, ctypes.byref(cfg), ctypes.byref(nb)) == labs.LABS_OK
    # tables for 64 walks of 8 D = 112 moves, plus per-walk energies, steps and sequences
    assert nb.value >= labs.workspace_bytes(27, 64, 112) + 64 * (4 + 8 + 8)
    res = labs.SolveResult()
    assert lib.labs_solve(27, ctypes.byref(cfg), None, nb.value, None, ctypes.byref(res)) == labs.LABS_EINVAL
    assert lib.labs_solve(27, ctypes.byref(cfg), ctypes.c_void_p(1), 16, None, ctypes.byref(res)) == labs.LABS_EINVAL
    cfg.first_round = -1
    assert lib.labs_solve_workspace_bytes(27, ctypes.byref(cfg), ctypes.byref(nb)) == labs.LABS_EINVAL
    cfg.first_round = 5
    assert lib.labs_solve_workspace_bytes(27, ctypes.byref(cfg), ctypes.byref(nb)) == labs.LABS_OK
    cfg.walks_per_round = 0
    assert lib.labs_solve(27, ctypes.byref(cfg), ctypes.c_void_p(1), 1 << 40, None, ctypes.byref(res)) == labs.LABS_EINVAL


def test_tuning_table_json_roundtrip(tmp_path):
    labs.tune_set(201, 2, 0.6)
    labs.tune_set(203, 8, 0.4)
    path = str(tmp_path / "tune.json")
    table = labs.save_tuning(path)
    assert table["201"] == {"lanes_per_walk": 2, "load_factor": 0.6}
    labs.tune_set(201, 4, 0.5)
    labs.tune_set(203, 4, 0.5)
    assert labs.load_tuning(path) == len(table)
    assert labs.tune_get(201) == (2, 0.6, True) and labs.tune_get(203) == (8, 0.4, True)


def test_full_space_sizes_and_validation_before_any_launch():
    assert labs.full_l_max() == 255 == O.full_l_max()
    for L in [3, 4, 63, 64, 65, 128, 129, 192, 193, 247, 255]:
        assert labs.full_key_words(L) == O.full_key_words(L)
    for bad in [-1, 0, 1, 2, 256, 383]:
        assert labs.full_key_words(bad) == 0
    # 12-byte entries up to L = 95, 16-byte entries up to L = 127, then 32-byte entries
    b95 = labs.full_workspace_bytes(95, 1, 100_000)
    b96 = labs.full_workspace_bytes(96, 1, 100_000)
    assert abs(b96 / b95 - 10 / 8) < 1e-3
    b127 = labs.full_workspace_bytes(127, 1, 1000)
    b128 = labs.full_workspace_bytes(128, 1, 1000)
    assert b128 >= 2 * b127 - 128 and b127 // 128 * 8 * 0.5 >= 1001
    assert labs.full_workspace_bytes(64, 10, 100, labs.make_plan(max_concurrent=4)) == \
        4 * labs.full_workspace_bytes(64, 1, 100)
    lib = labs.lib()
    out = labs.WalkOut(1, 1, 1, None, None, None, 0)
    ws = ctypes.c_void_p(1)
    ref = ctypes.byref
    for bad_L in (2, 256, -5):
        assert lib.labs_full_walks(None, bad_L, 4, 10, 0, ref(out), ws, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_full_walks(None, 64, -1, 10, 0, ref(out), ws, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_full_walks(None, 64, 4, -1, 0, ref(out), ws, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_full_walks(None, 64, 4, 10, 0, None, ws, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_full_walks(None, 64, 4, 10, 0, ref(out), None, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_full_walks(None, 64, 4, 10, 0, ref(out), ws, 8, None, None) == labs.LABS_EINVAL
    for G in (1, 2, 8, 3):
        bad = labs.make_plan(lanes_per_walk=G)
        assert lib.labs_full_walks(None, 64, 4, 10, 0, ref(out), ws, 1 << 30, ref(bad), None) == labs.LABS_EINVAL
    tr = labs.WalkOut(1, 1, 1, None, None, None, 5)
    assert lib.labs_full_walks(None, 64, 4, 10, 0, ref(tr), ws, 1 << 30, None, None) == labs.LABS_EINVAL
    assert lib.labs_full_walks(None, 64, 0, 10, 0, ref(out), ws, 0, None, None) == labs.LABS_OK


def test_tables_over_4_gib_are_sized_in_64_bits():
    """Visited tables of 2^25 buckets and more (over 4 GiB per walk) are valid
    sizes: the per-walk size is computed in 64 bits and only a bucket count of
    2^32 or more is refused (the kernels index buckets in 32 bits and bytes in 64)."""
    lf = labs.make_plan(load_factor=0.00008)
    keys = 30_001                                   # walk_len + 1 pivots
    per_walk = labs.min_workspace_bytes(101, 30_000, lf)
    n_buckets = per_walk // 128
    assert n_buckets >= keys / (10 * 0.00008) and n_buckets >= 1 << 25
    assert per_walk > 1 << 32
    assert labs.workspace_bytes(101, 3, 30_000, lf) == 3 * per_walk
    assert labs.full_workspace_bytes(100, 2, 30_000, lf) == 2 * labs.full_workspace_bytes(100, 1, 30_000, lf)
    assert labs.full_workspace_bytes(100, 1, 30_000, lf) > 1 << 32
    # 2^31 moves at load 0.04 would need more than 2^32 buckets
    lib = labs.lib()
    nb = labs.U64(0)
    huge = labs.make_plan(load_factor=0.04)
    assert lib.labs_walks_workspace_bytes(101, 1, 1 << 31, ctypes.byref(huge), ctypes.byref(nb)) == labs.LABS_EINVAL
    assert b"too large" in lib.labs_last_error()
    assert lib.labs_full_walks_workspace_bytes(100, 1, 1 << 31, ctypes.byref(huge), ctypes.byref(nb)) == labs.LABS_EINVAL


def test_noalloc_rejects_tables_beyond_its_scratch_before_any_device_call():
    lib = labs.lib()
    out = labs.WalkOut(1, 1, 1, None, None, None, 0)
    ref = ctypes.byref
    # one walk of 2^22 moves at load 0.5 needs 128 MiB of table: over 64 MiB
    assert labs.min_workspace_bytes(151, 1 << 22) > labs.NOALLOC_SCRATCH_BYTES
    assert lib.labs_walks_noalloc(None, 151, 4, 1 << 22, 0, ref(out), None, None) == labs.LABS_EINVAL
    assert b"fixed scratch" in lib.labs_last_error()
    assert lib.labs_walks_noalloc(None, 28, 4, 10, 0, ref(out), None, None) == labs.LABS_EINVAL
    assert lib.labs_walks_noalloc(None, 27, -1, 10, 0, ref(out), None, None) == labs.LABS_EINVAL
    assert lib.labs_walks_noalloc(None, 27, 4, 10, 0, None, None, None) == labs.LABS_EINVAL
    assert lib.labs_walks_noalloc(None, 27, 0, 10, 0, ref(out), None, None) == labs.LABS_OK
