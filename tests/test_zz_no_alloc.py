"""labs_walks_noalloc (visited tables in the library's fixed device array)
against labs_walks with a caller workspace: bit-exact results on two calls in
a row, the second smaller than the first, so the second runs on a scratch
array still holding the first call's tables."""
import ctypes

import numpy as np
import pytest

import labs_inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _same(a, b):
    for k in ("best_seq", "best_E", "steps_done", "digest", "trace_j", "trace_E"):
        np.testing.assert_array_equal(a[k].cpu().numpy(), b[k].cpu().numpy(), err_msg=k)


def test_noalloc_equals_workspace_walks_on_two_calls():
    from paper_2210_15962_amd import labs
    print("\n[case] noalloc L=151 3000x2000 then L=61 200x500", flush=True)
    # 1: 3000 walks of L = 151, tables of 64 KiB: three chunks of the 64 MiB array
    L, n, wl = 151, 3000, 2000
    assert labs.NOALLOC_SCRATCH_BYTES // labs.min_workspace_bytes(L, wl) < n
    a = labs.walks_noalloc(L, n, wl, seed=5, n_trace=2)
    b = labs.walks(L, n, wl, seed=5, n_trace=2)
    torch.cuda.synchronize()
    _same(a, b)
    # 2: a smaller call with explicit starts
    L2, n2, wl2 = 61, 200, 500
    keys = I.random_start_keys(L2, n2, seed=61)
    st = torch.from_numpy(I.as_int64_keys(keys)).cuda()
    a2 = labs.walks_noalloc(L2, n2, wl2, starts_t=st, n_trace=2,
                            plan=labs.make_plan(lanes_per_walk=2, load_factor=0.67))
    b2 = labs.walks(L2, n2, wl2, starts_t=st, n_trace=2)
    torch.cuda.synchronize()
    _same(a2, b2)
    # the library's error for a table over the array's size
    with pytest.raises(labs.LabsError):
        labs.walks_noalloc(151, 2, 1 << 22, seed=0)
