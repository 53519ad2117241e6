"""rrt_get_hits_rows_noalloc, the entry point for callers that cannot
allocate: through the C ABI, its output equals rrt_get_hits_rows' on two calls
in a row, the second with fewer sources, and it rejects requests beyond its
fixed staging array with RRT_E_CAPACITY."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _call(L, name, s, src, cap, n_ray):
    off = np.zeros(src.size * n_ray + 1, np.int64)
    hj = np.zeros(max(cap, 1), np.int32)
    hi = np.zeros(max(cap, 1), np.int32)
    hf = np.zeros(max(cap, 1), np.float32)
    arrays = (hj.ctypes.data, hi.ctypes.data, hf.ctypes.data) if cap > 0 else (None, None, None)
    rc = getattr(L, name)(s._h, src.size, src.ctypes.data, cap, off.ctypes.data, *arrays)
    return rc, off, hj[: off[-1]], hi[: off[-1]], hf[: off[-1]]


def test_no_alloc_hit_rows_match_the_workspace_form():
    from paper_1304_4235_amd import Solver, lib
    L = lib()
    wl = W.isothermal_halo(n=20000, seed=31)
    s = Solver.from_workload(wl)
    rng = np.random.default_rng(3)
    for m in (96, 17):                                  # a smaller second call
        src = np.ascontiguousarray(rng.choice(wl.n, m, replace=False).astype(np.int64))
        rc, off, *_ = _call(L, "rrt_get_hits_rows", s, src, 0, wl.n_ray)
        assert rc == 0
        cap = int(off[-1])
        assert cap > m * wl.n_ray
        want = _call(L, "rrt_get_hits_rows", s, src, cap, wl.n_ray)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        got = _call(L, "rrt_get_hits_rows_noalloc", s, src, cap, wl.n_ray)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        assert want[0] == 0 and got[0] == 0
        for a, b in zip(want[1:], got[1:]):
            np.testing.assert_array_equal(a, b)
    # beyond the fixed array: an error, and the context still works
    big = np.ascontiguousarray(np.arange(1025, dtype=np.int64))
    rc, *_ = _call(L, "rrt_get_hits_rows_noalloc", s, big, 1, wl.n_ray)
    assert rc == -6
    rc, *_ = _call(L, "rrt_get_hits_rows_noalloc", s, big[:10], 0, wl.n_ray)
    assert rc == 0
    s.close()
