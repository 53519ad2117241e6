"""Trees and ray-particle hit sets bit for bit at the benchmarked sizes, and the
device-memory, flag and statistics contracts of the boundary.

Hit lists of sampled sources come from the library's wave-cooperative walk
(the walk that evaluates columns and records paths) and from the recorded
paths themselves (what the streaming product sums); both are compared with
the oracle's brute force over every particle (Sec. 4.1.1, eq. colden: which
particles a ray intersects).  Trees are compared with the oracle's reference
tree, including the tree of independent halos."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

LEAF = 16              # the library's default leaf size


def _say(*a):
    print(*a, flush=True)


def _solver(wl, **kw):
    from paper_1304_4235_amd import Solver
    return Solver.from_workload(wl, **kw)


def _tree_equal(g, o):
    np.testing.assert_array_equal(g["codes"], o["codes"])
    np.testing.assert_array_equal(g["perm"], o["perm"])
    assert g["n_nodes"] == o["n_nodes"]
    for k in ("lo", "hi", "skip", "count"):
        np.testing.assert_array_equal(g[k], o[k], err_msg=k)
    leaf = o["count"] > 0
    np.testing.assert_array_equal(g["first"][leaf], o["first"][leaf])
    if "seg_root" in o:
        np.testing.assert_array_equal(g["seg_root"], o["seg_root"])
        np.testing.assert_array_equal(g["seg_end"], o["seg_end"])


def test_full_halo_tree_bit_exact():
    wl = W.make_config(1)
    s = _solver(wl)
    _say("halo tree: oracle")
    _tree_equal(s.tree(), oracle.lbvh(wl.pos, wl.h, LEAF))


def _batch6():
    sizes, peaks = [300, 2000, 9, 5000, 1, 700], [0.5, 3.0, 1.0, 10.0, 1.0, 0.05]
    parts = [W.isothermal_halo(n=n, n_peak=p, n_bins=16, seed=700 + i)
             for i, (n, p) in enumerate(zip(sizes, peaks))]
    off = np.zeros(len(parts) + 1, np.int64)
    off[1:] = np.cumsum([p.n for p in parts])
    cat = lambda f: np.concatenate([getattr(p, f) for p in parts])
    p0 = parts[0]
    return W.Workload(name="batch6", pos=cat("pos"), h=cat("h"), mu=cat("mu"), n_H=cat("n_H"),
                      T=cat("T"), dirs=p0.dirs, sigma=p0.sigma, w=p0.w, l_ray=p0.l_ray, box=0.0,
                      tol=p0.tol, max_iter=p0.max_iter, halo_offsets=off)


@pytest.mark.parametrize("which", ["batch6", "full"])
def test_batch_tree_bit_exact(which):
    """The tree of independent halos (halo index above the Morton key, leaves
    within one halo, one subtree per halo) equals the oracle's."""
    wl = _batch6() if which == "batch6" else W.make_config(3)
    s = _solver(wl)
    g = s.tree()
    _say("batch tree", which, wl.n, "particles,", g["n_nodes"], "nodes: oracle")
    _tree_equal(g, oracle.lbvh(wl.pos, wl.h, LEAF, halo_offsets=wl.halo_offsets))


@pytest.mark.parametrize("which", ["halo", "field", "batch"])
def test_repeated_builds_give_the_same_tree(which):
    """The bottom-up refit orders its threads with the arrival flags alone
    (agent-scope atomics, no fence): every rebuild of the full-size trees gives
    the same arrays, equal to the oracle's."""
    wl = W.make_config({"halo": 1, "field": 2, "batch": 3}[which])
    s = _solver(wl)
    first = s.tree()
    for _ in range(4):
        s.build_tree()
        _tree_equal(s.tree(), first)
    _say(which, "tree: 5 builds agree,", first["n_nodes"], "nodes: oracle")
    if which == "field":
        _tree_equal(first, oracle.lbvh(wl.pos, wl.h, LEAF))


def _rows(off, a, b, r):
    return a[off[r]:off[r + 1]], b[off[r]:off[r + 1]]


def _check_hit_rows(s, wl, src, base=0, part=None, paths=True):
    """The walk's hit lists (particle, image) equal the oracle's exactly; the
    recorded paths (when there are any) hold the same particles; per-hit
    factors agree."""
    ref_wl = wl if part is None else part
    x = np.ones(ref_wl.n)
    _, o_off, o_j, o_img, o_fac = oracle.columns(ref_wl, x, sources=src, hits=True,
                                                 factors=True)
    g_off, g_j, g_img, g_fac = s.hits_rows(base + np.asarray(src))
    if paths:
        p_off, p_j, p_fac = s.path_rows(base + np.asarray(src))
    mu = ref_wl.mu.astype(np.float64)
    nr = wl.n_ray
    tot = 0
    for i in range(len(src)):
        for k in range(nr):
            r = i * nr + k
            oj, oi = _rows(o_off, o_j, o_img, r)
            gj, gi = _rows(g_off, g_j, g_img, r)
            want = sorted(zip(oj.tolist(), oi.tolist()))
            got = sorted(zip((gj - base).tolist(), gi.tolist()))
            assert got == want, f"source {src[i]} ray {k}: hit sets differ"
            if paths:
                pj, _ = _rows(p_off, p_j, p_fac, r)
                assert sorted((pj - base).tolist()) == sorted(oj.tolist()), \
                    f"source {src[i]} ray {k}: recorded path differs"
            # factors: mu_j K/h^2 (FP32 K/h^2) against the oracle's quadrature
            of, _ = _rows(o_off, o_fac, o_img, r)
            gf, _ = _rows(g_off, g_fac, g_img, r)
            order_o = np.lexsort((oi, oj))
            order_g = np.lexsort((gi, gj))
            fo = of[order_o]
            fg = gf[order_g].astype(np.float64) * mu[(gj - base)[order_g]]
            assert np.sum(np.abs(fg - fo)) <= 1e-6 * max(np.sum(fo), 1e-300)
            tot += len(oj)
    return tot


def test_full_halo_hit_sets_exact():
    """24 sources x 12 rays of the 262144-particle halo."""
    wl = W.make_config(1)
    s = _solver(wl)
    s.compute_columns(want_N=False, count=False)            # records the paths
    src = np.sort(np.random.default_rng(21).choice(wl.n, 24, replace=False))
    tot = _check_hit_rows(s, wl, src)
    _say("halo hits compared:", tot)
    assert tot > 24 * 12 * 100


def test_full_field_hit_sets_exact():
    """8 sources x 48 rays of the 2.1M-particle periodic field."""
    wl = W.make_config(2)
    s = _solver(wl)
    s.compute_columns(want_N=False, count=False)
    src = np.sort(np.random.default_rng(22).choice(wl.n, 8, replace=False))
    tot = _check_hit_rows(s, wl, src)
    _say("field hits compared:", tot)
    assert tot > 8 * 48 * 20


def test_full_batch_hit_sets_exact():
    """4 sources in each of the smallest, the largest and two other halos of
    the 64-halo batch (7.1M particles, one context)."""
    wl = W.make_config(3)
    s = _solver(wl)
    s.compute_columns(want_N=False, count=False)
    paths = s.timing()["path_hits"] >= 0             # the whole batch's may not fit
    _say("batch paths recorded:", paths)
    sizes = np.diff(wl.halo_offsets)
    rng = np.random.default_rng(23)
    tot = 0
    for h in sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 40}):
        a, b = int(wl.halo_offsets[h]), int(wl.halo_offsets[h + 1])
        part = W.Workload(name=f"halo{h}", pos=wl.pos[a:b], h=wl.h[a:b], mu=wl.mu[a:b],
                          n_H=wl.n_H[a:b], T=wl.T[a:b], dirs=wl.dirs, sigma=wl.sigma, w=wl.w,
                          l_ray=wl.l_ray, box=wl.box, tol=wl.tol, max_iter=wl.max_iter)
        src = np.sort(rng.choice(part.n, 4, replace=False))
        _say("batch halo", h, "of", part.n, "particles")
        tot += _check_hit_rows(s, wl, src, base=a, part=part, paths=paths)
    assert tot > 0


def test_trace_stats_count_the_walk():
    """The walk's tallies: its intersections are the recorded ones, every hit
    took a pair test, and a packet visits no more leaves than nodes."""
    wl = W.isothermal_halo(n=16384, seed=3)
    s = _solver(wl)
    _, hits = s.compute_columns(want_N=False)
    st = s.trace_stats()
    _say(st)
    assert st["hits"] == hits and st["rays"] == wl.n * wl.n_ray
    assert st["pair_tests"] >= st["hits"] > 0
    assert st["packet_leaf_visits"] <= st["packet_node_visits"]
    assert st["ray_node_visits"] >= st["rays"]            # every ray enters the root


# ---------------------------------------------------------------------------
# device memory: the caller's workspace and path buffer only
# ---------------------------------------------------------------------------
def test_no_device_allocation_after_the_workspace_is_set():
    """With the workspace and path buffer given, a full solve, a K-step forward
    and a backward leave the device's free memory unchanged: the library
    allocates nothing of its own."""
    from paper_1304_4235_amd import lib
    L = lib()
    wl = W.isothermal_halo(n=20000, n_bins=16, seed=5)
    K = 6
    s = _solver(wl)
    s._K = K
    s._ensure_ws()
    x = torch.empty(wl.n, dtype=torch.float64, device="cuda")
    lnG = torch.empty_like(x)
    dn = torch.empty_like(x)
    gl = torch.ones_like(x)
    dw = np.zeros(wl.n_bins)
    it, md = C.c_int32(0), C.c_double(0)

    def rounds(m):
        for _ in range(m):
            assert L.rrt_set_state(s._h, None) == 0
            assert L.rrt_iterate_equilibrium(s._h, 200, 1e-3, x.data_ptr(), C.byref(it),
                                             C.byref(md)) == 0
            assert L.rrt_forward(s._h, K, lnG.data_ptr(), x.data_ptr()) == 0
            assert L.rrt_backward(s._h, gl.data_ptr(), None, dw.ctypes.data,
                                  dn.data_ptr()) == 0
            assert L.rrt_build_tree(s._h) == 0

    rounds(2)                  # every kernel has run once (code objects are loaded)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    info0 = s.workspace_info()
    rec0 = s.recording_stats()
    rounds(2)
    torch.cuda.synchronize()
    assert s.recording_stats()[0] - rec0[0] == 2       # one walk each, into the path buffer
    free1 = torch.cuda.mem_get_info()[0]
    info1 = s.workspace_info()
    _say("free", free0, free1, "workspace", info0, info1)
    assert free1 == free0
    assert info1["ws_size"] == info0["ws_size"] and info1["path_size"] == info0["path_size"]
    assert info1["ws_used"] <= info1["ws_size"] and info1["path_used"] <= info1["path_size"]
    assert np.all(np.isfinite(dw)) and bool(torch.isfinite(dn).all())


def test_workspace_grows_by_moving_the_context():
    """A solver whose workspace is replaced by a larger one mid-way (the library
    copies its buffers over) gives the same iterates as one that never moved."""
    from paper_1304_4235_amd import lib
    wl = W.isothermal_halo(n=8192, seed=6)
    a, b = _solver(wl), _solver(wl)
    ra = a.iterate(3, 0.0)
    rb = b.iterate(3, 0.0)
    bigger = torch.empty(b._ws.numel() * 2, dtype=torch.uint8, device="cuda")
    assert lib().rrt_set_workspace(b._h, C.c_void_p(bigger.data_ptr()), bigger.numel()) == 0
    b._ws = bigger
    ra = a.iterate(4, 0.0)
    rb = b.iterate(4, 0.0)
    np.testing.assert_array_equal(ra["x"].cpu().numpy(), rb["x"].cpu().numpy())


def test_large_exports_grow_a_fragmented_workspace():
    """Exporting the recorded paths and the hit lists of 4096 sources of the
    full halo stages tens of MB in one piece: the binding grows the workspace
    past its end when a request finds no piece large enough (the used blocks
    are spread), and both exports agree on every ray's count."""
    wl = W.make_config(1)
    s = _solver(wl)
    s.compute_columns()
    src = s.tree()["perm"][:4096].astype(np.int64)
    before = s.workspace_info()["ws_size"]
    off_p, hj_p, hf_p = s.path_rows(src)
    off_h, hj_h, hi_h, hf_h = s.hits_rows(src)
    assert s.workspace_info()["ws_size"] > before
    assert off_p.size == off_h.size == 4096 * wl.n_ray + 1
    np.testing.assert_array_equal(off_p, off_h)
    assert hj_p.size == off_p[-1] > 0
    s.close()


def test_too_small_workspace_is_an_error_not_a_fault():
    from paper_1304_4235_amd import RRTError, Solver, lib
    s = Solver(10.0)
    need = s.workspace_size(n=200000, n_ray=12, n_bins=1)
    assert need > s._ws.numel()
    wl = W.isothermal_halo(n=200000, n_bins=1, seed=7)
    rc = lib().rrt_set_particles(s._h, wl.n, None, None, None, None, None, None)
    assert rc == -1                                  # null arrays: RRT_E_ARG
    pos = torch.tensor(wl.pos, device="cuda")
    f = torch.ones(wl.n, dtype=torch.float32, device="cuda")
    rc = lib().rrt_set_particles(s._h, wl.n, pos.data_ptr(), f.data_ptr(), f.data_ptr(),
                                 f.data_ptr(), f.data_ptr(), None)
    assert rc == -5                                  # RRT_E_WORKSPACE, nothing changed
    before = s.workspace_info()["ws_size"]
    s.set_particles(wl.pos, wl.h, wl.mu, wl.n_H, wl.T)  # the binding grows it
    assert s.workspace_info()["ws_size"] > before
    with pytest.raises(RRTError, match="RRT_E_STATE"):
        s.compute_columns()


# ---------------------------------------------------------------------------
# device flags and statistics
# ---------------------------------------------------------------------------
def test_bad_state_and_density_are_reported_at_the_next_sync():
    from paper_1304_4235_amd import RRTError
    wl = W.isothermal_halo(n=4096, seed=8)
    s = _solver(wl)
    x = np.full(wl.n, 0.01)
    x[123] = np.nan
    s.set_state(torch.tensor(x))                       # flagged on the device
    with pytest.raises(RRTError, match="RRT_E_INPUT"):
        s.iterate(3, 0.0)
    s.set_state(None)                                  # the flag was reported and cleared
    assert s.iterate(2, 0.0)["iters"] == 2
    nH = wl.n_H.astype(np.float32).copy()
    nH[7] = -1.0
    s.set_density(torch.tensor(nH))
    with pytest.raises(RRTError, match="RRT_E_INPUT"):
        s.compute_columns()
    s.set_density(torch.tensor(wl.n_H))
    s.set_state(None)
    assert np.isfinite(s.iterate(2, 0.0)["x"].cpu().numpy()).all()


def test_convergence_counts_per_sweep():
    """The paper's convergence statistic (Sec. 4): per sweep, the particles
    whose change is below tol, absolutely and relative to x, recomputed from
    the iterates themselves."""
    wl = W.make_config(0)
    s = _solver(wl)
    tol = 1e-3
    prev = s.get_state()["x"].cpu().numpy()
    sweeps = 0
    while True:
        r = s.iterate(1, tol)
        cur = r["x"].cpu().numpy()
        cv = s.convergence()
        assert cv["max_dx"].size == 1
        d = np.abs(cur - prev)
        assert cv["n_abs"][0] == int(np.sum(d < tol))
        assert cv["n_rel"][0] == int(np.sum(d < tol * prev))
        assert cv["max_dx"][0] == d.max()
        prev, sweeps = cur, sweeps + 1
        if r["converged"] or sweeps >= 20:
            break
    assert r["converged"] and cv["n_abs"][0] == wl.n
    full = _solver(wl).iterate(20, tol)
    assert full["iters"] == sweeps
