"""Independent halos in one context: the segmented tree, per-halo convergence
on the device and the graph-replayed iterations, against one solve per halo."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _batch(sizes, peaks, seed=7, n_bins=16):
    parts = [W.isothermal_halo(n=n, n_peak=p, n_bins=n_bins, seed=seed * 100 + i)
             for i, (n, p) in enumerate(zip(sizes, peaks))]
    off = np.zeros(len(parts) + 1, np.int64)
    off[1:] = np.cumsum([p.n for p in parts])
    cat = lambda f: np.concatenate([getattr(p, f) for p in parts])
    p0 = parts[0]
    wl = W.Workload(name="batch", pos=cat("pos"), h=cat("h"), mu=cat("mu"), n_H=cat("n_H"),
                    T=cat("T"), dirs=p0.dirs, sigma=p0.sigma, w=p0.w, l_ray=p0.l_ray, box=0.0,
                    tol=p0.tol, max_iter=p0.max_iter, halo_offsets=off)
    return wl, parts


def _solver(wl, **kw):
    from paper_1304_4235_amd import Solver
    return Solver.from_workload(wl, **kw)


SIZES = [300, 2000, 9, 5000, 1, 700]
PEAKS = [0.5, 3.0, 1.0, 10.0, 1.0, 0.05]


@pytest.mark.parametrize("paths", [-1, 0])
def test_batched_equals_one_solve_per_halo(paths):
    wl, parts = _batch(SIZES, PEAKS)
    sb = _solver(wl, record_paths=paths)
    rb = sb.iterate_halos(200, 1e-3, per_launch=8)
    assert rb["converged"]
    xb = rb["x"].cpu().numpy()
    for h, p in enumerate(parts):
        s = _solver(p, record_paths=paths)
        r = s.iterate(200, 1e-3)
        a, b = wl.halo_offsets[h], wl.halo_offsets[h + 1]
        assert rb["halo_iters"][h] == r["iters"], h
        np.testing.assert_allclose(xb[a:b], r["x"].cpu().numpy(), rtol=1e-9)


def test_batched_hits_stay_in_their_halo():
    wl, parts = _batch(SIZES, PEAKS)
    sb = _solver(wl)
    off, hj, hi = sb.hits()
    for h, p in enumerate(parts):
        a, b = wl.halo_offsets[h], wl.halo_offsets[h + 1]
        s = _solver(p)
        o2, j2, i2 = s.hits()
        for src in range(0, p.n, max(1, p.n // 17)):
            for k in range(12):
                r = (a + src) * 12 + k
                got = sorted(hj[off[r]:off[r + 1]].tolist())
                assert all(a <= j < b for j in got)
                want = sorted((j2[o2[src * 12 + k]:o2[src * 12 + k + 1]] + a).tolist())
                assert got == want


def test_batch_parity_with_oracle_small():
    """Two small halos of the batch against the FP64 oracle, end to end."""
    wl, parts = _batch([400, 900], [2.0, 0.3], seed=9)
    sb = _solver(wl)
    rb = sb.iterate_halos(200, 1e-3, per_launch=4)
    xb = rb["x"].cpu().numpy()
    for h, p in enumerate(parts):
        ref = oracle.solve(p)
        a, b = wl.halo_offsets[h], wl.halo_offsets[h + 1]
        assert rb["halo_iters"][h] == ref["iters"]
        rel = np.abs(xb[a:b] - ref["x_hist"][-1]) / ref["x_hist"][-1]
        assert rel.max() <= 1e-4


def test_one_halo_graph_equals_host_loop():
    wl = W.isothermal_halo(n=6000, n_bins=16, seed=3)
    a = _solver(wl).iterate(200, 1e-3)
    r = _solver(wl).iterate_halos(200, 1e-3, per_launch=8)
    assert r["halo_iters"][0] == a["iters"]
    np.testing.assert_array_equal(r["x"].cpu().numpy(), a["x"].cpu().numpy())


def test_replay_length_does_not_change_results():
    wl, _ = _batch(SIZES, PEAKS, seed=8)
    outs = []
    for per in (1, 5, 64):
        r = _solver(wl).iterate_halos(200, 1e-3, per_launch=per)
        outs.append((r["halo_iters"].copy(), r["x"].cpu().numpy()))
    for its, x in outs[1:]:
        np.testing.assert_array_equal(its, outs[0][0])
        np.testing.assert_array_equal(x, outs[0][1])
    # a second call on the same solver, from the same (thin) state, replays the
    # cached graph
    s = _solver(wl)
    r1 = s.iterate_halos(200, 1e-3, per_launch=5)
    s.set_state(None)
    r2 = s.iterate_halos(200, 1e-3, per_launch=5)
    np.testing.assert_array_equal(r1["x"].cpu().numpy(), r2["x"].cpu().numpy())


@pytest.mark.parametrize("frac", [0.45, 0.2])
def test_grouped_recording_under_a_small_budget(frac):
    """With paths larger than the budget, halos run in groups whose paths fit
    (and a halo too large for the budget traverses): same results per halo."""
    wl, parts = _batch(SIZES, PEAKS, seed=12)
    probe = _solver(wl, record_paths=0)
    _, hits = probe.compute_columns(want_N=False)
    budget = int(8 * hits * frac)
    sb = _solver(wl, record_paths=-1, path_budget=budget)
    rb = sb.iterate_halos(200, 1e-3, per_launch=4)
    xb = rb["x"].cpu().numpy()
    for h, p in enumerate(parts):
        r = _solver(p).iterate(200, 1e-3)
        a, b = wl.halo_offsets[h], wl.halo_offsets[h + 1]
        assert rb["halo_iters"][h] == r["iters"], h
        np.testing.assert_allclose(xb[a:b], r["x"].cpu().numpy(), rtol=1e-9)
    # afterwards the batch still gives whole-batch columns
    N1, h1 = sb.compute_columns()
    N2, h2 = _solver(wl, record_paths=0).compute_columns()
    assert h1 == h2


def test_batched_solve_over_row_tiles_matches_plain():
    """Row tiles in the batched solve: built before the graph is captured, and
    the tile product skips the rows of halos that have stopped, as the plain
    product does.  Same iteration counts, same states to summation order."""
    wl, parts = _batch(SIZES, PEAKS)
    out = []
    for tiles in (0, 1):
        sb = _solver(wl)
        sb.set_tuning(tiles=tiles)
        sb.enable_timing(True)
        rb = sb.iterate_halos(200, 1e-3, per_launch=8)
        assert rb["converged"]
        if tiles:
            assert sb.timing()["tile_set_total"] > 0, "row tiles were not built"
        out.append(rb)
    np.testing.assert_array_equal(out[0]["halo_iters"], out[1]["halo_iters"])
    np.testing.assert_allclose(out[1]["x"].cpu().numpy(), out[0]["x"].cpu().numpy(), rtol=1e-9)


def test_autotuner_picks_change_no_result(tmp_path):
    """The autotuner times its knobs on a batch and caches the picks, keeping
    the library's defaults instead when one solve of the whole batch is faster
    with them; the picks change the launch shapes only: the same iterations per
    halo and the same states (to summation order) as the defaults."""
    import json
    from paper_1304_4235_amd import autotune
    wl, parts = _batch(SIZES, PEAKS)
    cache = str(tmp_path / "tune.json")
    space = dict(leaf=[4, 8], trace_block=[64, 256], packet=[64, 1], path_group=[16, 32],
                 per_launch=[4, 16])
    res = autotune.tune(wl, space=space, reps=1, cache_path=cache, use_cache=False)
    best = res["best"]
    assert set(best) == {"leaf", "trace_block", "packet", "path_group", "per_launch"}
    whole = res["whole"]
    if whole["defaults_ms"] < whole["picks_ms"]:
        assert best == autotune.DEFAULTS
    else:
        assert best["leaf"] in space["leaf"] and best["per_launch"] in space["per_launch"]
    again = autotune.tune(wl, space=space, cache_path=cache, use_cache=True)
    assert again == json.loads(json.dumps(res))                # served from the cache
    ref = _solver(wl).iterate_halos(200, 1e-3, per_launch=8)
    s = _solver(wl)
    autotune.apply(s, best)
    s.build_tree()
    r = s.iterate_halos(200, 1e-3, per_launch=best["per_launch"])
    np.testing.assert_array_equal(r["halo_iters"], ref["halo_iters"])
    np.testing.assert_allclose(r["x"].cpu().numpy(), ref["x"].cpu().numpy(), rtol=1e-9)


@pytest.mark.parametrize("paths", [-1, 0])
def test_packet_queue_gives_the_grid_results(paths):
    """The persistent walk (a resident grid whose waves take 64-ray packets of
    every halo from one counter) against one wave per packet: the same hit
    lists, recorded paths, columns and iterates bit for bit, on the batch with
    a one-particle halo and halos smaller than a packet."""
    wl, _ = _batch(SIZES, PEAKS)
    out = []
    for q in (0, 1):
        s = _solver(wl, record_paths=paths)
        s.set_tuning(packet_queue=q)
        off, hj, hi = s.hits()
        N, h = s.compute_columns()
        r = s.iterate_halos(200, 1e-3, per_launch=8)
        src = np.arange(0, wl.n, 37)
        ro, pj, pf = s.path_rows(src) if paths != 0 else (None, None, None)
        out.append((off, hj, hi, N.cpu().numpy(), h, r["x"].cpu().numpy(), r["halo_iters"],
                    ro, pj, pf))
    for a, b in zip(out[0], out[1]):
        if a is None:
            continue
        if isinstance(a, np.ndarray):
            np.testing.assert_array_equal(a, b)
        else:
            assert a == b
