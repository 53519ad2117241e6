"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Bars (written in each test):
  * tree arrays and ray-particle hit sets: bit-exact;
  * columns: relative 1e-6;
  * ln Gamma: absolute 1e-4 (= 1e-4 relative Gamma) where tau_eff <= 100;
    beyond, |d tau_eff| <= 1e-6 tau_eff (Gamma underflows there);
  * x: relative 1e-4.
Columns are compared for the same state x on both sides, so each iteration of
the order-independent update can be checked on a sample of source particles.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

COL_RTOL = 1e-6
LNG_ATOL = 1e-4
TAU_RTOL = 1e-6
X_RTOL = 1e-4


def _solver(wl, **kw):
    from paper_1304_4235_amd import Solver
    return Solver.from_workload(wl, **kw)


def _say(*a):
    print(*a, flush=True)


def _check_columns(Ng, No):
    Ng = np.asarray(Ng)
    err = np.abs(Ng - No)
    bad = err > COL_RTOL * np.abs(No) + 1e-300
    assert not bad.any(), f"columns differ: max rel {np.max(err / np.maximum(No, 1e-300)):.3e}"


def _check_rates(lnG_g, lnG_o, tau_o):
    lnG_g, lnG_o, tau_o = map(np.asarray, (lnG_g, lnG_o, tau_o))
    thin = tau_o <= 100
    d = np.abs(lnG_g - lnG_o)
    assert np.all(d[thin] <= LNG_ATOL), f"ln Gamma differs by {d[thin].max():.3e}"
    if (~thin).any():
        assert np.all(d[~thin] <= TAU_RTOL * tau_o[~thin]), "tau_eff differs"


def _check_x(xg, xo):
    xg, xo = np.asarray(xg), np.asarray(xo)
    rel = np.abs(xg - xo) / np.abs(xo)
    assert np.all(rel <= X_RTOL), f"x differs: max rel {rel.max():.3e}"


def _hitsets(off, hj, hi, rows):
    return [sorted(zip(hj[off[r]:off[r + 1]].tolist(), hi[off[r]:off[r + 1]].tolist()))
            for r in rows]


# ---------------------------------------------------------------------------
# tree
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,leaf,dup", [(1, 4, False), (2, 1, False), (3, 4, False),
                                        (5, 4, False), (1000, 1, False), (4099, 4, False),
                                        (10007, 8, False), (3000, 4, True), (17, 16, False),
                                        (10007, 16, False), (4099, 12, False), (3000, 16, True)])
def test_tree_bit_exact(n, leaf, dup):
    rng = np.random.default_rng(n + leaf)
    pos = rng.uniform(-30, 30, (n, 3)).astype(np.float32)
    if dup:
        pos[n // 2:] = pos[: n - n // 2]
    h = rng.uniform(0.5, 3, n).astype(np.float32)
    wl = W.Workload(name="tree", pos=pos, h=h, mu=np.ones(n, np.float32),
                    n_H=np.ones(n, np.float32), T=np.full(n, 1e4, np.float32),
                    dirs=W.healpix_dirs(1), sigma=np.array([W.SIGMA_TH]),
                    w=np.array([1e-12 / W.SIGMA_TH]), l_ray=10.0, box=0.0, tol=1e-3, max_iter=5)
    _say("tree", n, leaf, dup)
    s = _solver(wl, leaf_size=leaf)
    g = s.tree()
    o = oracle.lbvh(pos, h, leaf)
    np.testing.assert_array_equal(g["codes"], o["codes"])
    np.testing.assert_array_equal(g["perm"], o["perm"])
    assert g["n_nodes"] == o["n_nodes"]
    np.testing.assert_array_equal(g["lo"], o["lo"])
    np.testing.assert_array_equal(g["hi"], o["hi"])
    np.testing.assert_array_equal(g["skip"], o["skip"])
    np.testing.assert_array_equal(g["count"], o["count"])
    leaf_nodes = o["count"] > 0
    np.testing.assert_array_equal(g["first"][leaf_nodes], o["first"][leaf_nodes])


# ---------------------------------------------------------------------------
# lattice (periodic, single bin): hit sets, columns, one step, full solve
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def lattice():
    return W.make_config(0)


@pytest.fixture(scope="module")
def lattice_oracle(lattice):
    _say("oracle solve: uniform lattice 16^3")
    return oracle.solve(lattice)


def test_lattice_hit_sets_exact(lattice):
    wl = lattice
    s = _solver(wl)
    _say("lattice hit sets")
    off, hj, hi = s.hits()
    src = np.arange(0, wl.n, 61)
    N, o_off, o_hj, o_hi = oracle.columns(wl, oracle.x_thin(wl), sources=src, hits=True)
    for i, p in enumerate(src):
        rows = [p * wl.n_ray + k for k in range(wl.n_ray)]
        got = _hitsets(off, hj, hi, rows)
        want = _hitsets(o_off, o_hj, o_hi, [i * wl.n_ray + k for k in range(wl.n_ray)])
        assert got == want, f"source {p}"
    assert off[-1] > 300 * wl.n * wl.n_ray      # ~320 hits per ray


@pytest.mark.parametrize("paths", [-1, 0])
def test_lattice_columns_and_step(lattice, paths):
    wl = lattice
    s = _solver(wl, record_paths=paths)
    rng = np.random.default_rng(0)
    x = oracle.x_thin(wl) * rng.uniform(1, 50, wl.n)
    s.set_state(torch.tensor(x))
    _say("lattice columns for a given state")
    N, nh = s.compute_columns()
    lnG, G, tau = s.compute_gamma()
    xn, mdx = s.update_equilibrium()
    src = np.arange(0, wl.n, 37)
    ref = oracle.step(wl, x, sources=src)
    _check_columns(N.cpu().numpy()[src], ref["N"])
    _check_rates(lnG.cpu().numpy()[src], ref["lnG"], ref["tau"])
    _check_x(xn.cpu().numpy()[src], ref["x_new"])
    assert mdx == pytest.approx(np.max(np.abs(xn.cpu().numpy() - x)), rel=1e-12)


def test_lattice_solve_every_iteration(lattice, lattice_oracle):
    """Each GPU iterate against the oracle's step from the oracle's previous iterate."""
    wl, ref = lattice, lattice_oracle
    s = _solver(wl)
    assert ref["iters"] >= 2
    src = np.arange(0, wl.n, 53)
    for k in range(ref["iters"]):
        _say("lattice iteration", k)
        s.set_state(torch.tensor(ref["x_hist"][k]))
        s.compute_columns(want_N=False, count=False)
        lnG, G, tau = s.compute_gamma()
        xn, _ = s.update_equilibrium()
        lnG_o = ref["lnG_hist"][k]
        tau_o = math.log(oracle.gamma_thin(wl)) - lnG_o
        _check_rates(lnG.cpu().numpy(), lnG_o, tau_o)
        _check_x(xn.cpu().numpy(), ref["x_hist"][k + 1])


def test_lattice_end_to_end(lattice, lattice_oracle):
    wl, ref = lattice, lattice_oracle
    s = _solver(wl)
    _say("lattice end to end")
    r = s.iterate(wl.max_iter, wl.tol)
    assert r["converged"]
    assert r["iters"] == ref["iters"]
    _check_x(r["x"].cpu().numpy(), ref["x_hist"][-1])


# ---------------------------------------------------------------------------
# isolated halos with a 128-bin power-law spectrum
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("paths", [-1, 0])
def test_small_halo_step_all_sources(paths):
    wl = W.isothermal_halo(n=8192, seed=11)
    s = _solver(wl, record_paths=paths)
    x = oracle.x_thin(wl) * np.linspace(1.0, 1e3, wl.n)
    x = np.minimum(x, 0.99)
    s.set_state(torch.tensor(x))
    _say("small halo step")
    N, nh = s.compute_columns()
    lnG, _, _ = s.compute_gamma()
    xn, _ = s.update_equilibrium()
    ref = oracle.step(wl, x)
    _check_columns(N.cpu().numpy(), ref["N"])
    _check_rates(lnG.cpu().numpy(), ref["lnG"], ref["tau"])
    _check_x(xn.cpu().numpy(), ref["x_new"])


def test_small_halo_hits_exact():
    wl = W.isothermal_halo(n=8192, seed=12)
    s = _solver(wl)
    _say("small halo hits")
    off, hj, hi = s.hits()
    src = np.arange(0, wl.n, 97)
    _, o_off, o_hj, o_hi = oracle.columns(wl, np.ones(wl.n), sources=src, hits=True)
    for i, p in enumerate(src):
        got = _hitsets(off, hj, hi, [p * 12 + k for k in range(12)])
        want = _hitsets(o_off, o_hj, o_hi, [i * 12 + k for k in range(12)])
        assert got == want


def test_full_halo_sampled_sources():
    """The 262144-particle halo: the GPU solve's iterates, checked one step at a
    time on sampled sources against the oracle fed the same state."""
    wl = W.make_config(1)
    s = _solver(wl)
    rng = np.random.default_rng(1)
    src = np.sort(rng.choice(wl.n, 24, replace=False))
    x = oracle.x_thin(wl)
    for k in range(3):
        _say("full halo iteration", k)
        s.set_state(torch.tensor(x))
        N, _ = s.compute_columns()
        lnG, _, _ = s.compute_gamma()
        xn, _ = s.update_equilibrium()
        ref = oracle.step(wl, x, sources=src)
        _check_columns(N.cpu().numpy()[src], ref["N"])
        _check_rates(lnG.cpu().numpy()[src], ref["lnG"], ref["tau"])
        _check_x(xn.cpu().numpy()[src], ref["x_new"])
        x = xn.cpu().numpy()


def test_full_halo_late_iterates():
    """The benchmarked solve of the 262144-particle halo runs 120 sweeps from
    the optically thin state: the GPU's own iterates at sweep 60 and at the
    last sweep, checked one step at a time on 24 sources against the oracle
    fed the same state (the deep-shielding regime of the converged solve)."""
    wl = W.make_config(1)
    s = _solver(wl)
    r = s.iterate(wl.max_iter, wl.tol, want_x=False)
    assert r["converged"]
    K = r["iters"]
    _say("halo: converged in", K, "sweeps")
    rng = np.random.default_rng(2)
    src = np.sort(rng.choice(wl.n, 24, replace=False))
    s.set_state(None)
    done = 0
    for k in (K // 2, K - 1):
        x = s.iterate(k - done, 0.0)["x"].cpu().numpy()     # x^k, the GPU's own iterate
        done = k
        _say("halo: step from sweep", k)
        s.set_state(torch.tensor(x))
        N, _ = s.compute_columns()
        lnG, _, tau = s.compute_gamma()
        xn, _ = s.update_equilibrium()
        ref = oracle.step(wl, x, sources=src)
        _check_columns(N.cpu().numpy()[src], ref["N"])
        _check_rates(lnG.cpu().numpy()[src], ref["lnG"], ref["tau"])
        _check_x(xn.cpu().numpy()[src], ref["x_new"])
        s.set_state(torch.tensor(x))


def _halo_of(wl, h):
    a, b = int(wl.halo_offsets[h]), int(wl.halo_offsets[h + 1])
    part = W.Workload(name=f"{wl.name}_halo{h}", pos=wl.pos[a:b], h=wl.h[a:b], mu=wl.mu[a:b],
                      n_H=wl.n_H[a:b], T=wl.T[a:b], dirs=wl.dirs, sigma=wl.sigma, w=wl.w,
                      l_ray=wl.l_ray, box=wl.box, tol=wl.tol, max_iter=wl.max_iter)
    return part, a


def test_full_batch_sampled_sources(tmp_path):
    """The 64-halo batch at full size (7.1M particles), solved in one context
    with the launch knobs the autotuner picks for it (over a reduced space):
    the final state's columns, rates and next update, on sampled sources of
    the smallest, the largest and two other halos, against the oracle fed that
    halo's state."""
    from paper_1304_4235_amd import autotune
    wl = W.make_config(3)
    space = dict(leaf=[8], trace_block=[128, 256], packet=[64], path_group=[16, 32],
                 per_launch=[16])
    best = autotune.tune(wl, space=space, reps=1, cache_path=str(tmp_path / "tune.json"),
                         use_cache=False)["best"]
    _say("full batch: tuned knobs", best)
    s = _solver(wl)
    autotune.apply(s, best)
    s.build_tree()                         # the leaf size applies from the next build
    r = s.iterate_halos(wl.max_iter, wl.tol, per_launch=best["per_launch"])
    assert r["converged"]
    _say("full batch: iterations per halo", r["halo_iters"].min(), "to", r["halo_iters"].max())
    x = r["x"].cpu().numpy()
    N, _ = s.compute_columns()
    lnG, _, _ = s.compute_gamma()
    xn, _ = s.update_equilibrium()
    N, lnG, xn = N.cpu().numpy(), lnG.cpu().numpy(), xn.cpu().numpy()
    sizes = np.diff(wl.halo_offsets)
    rng = np.random.default_rng(4)
    for h in sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 40}):
        part, a = _halo_of(wl, h)
        src = np.sort(rng.choice(part.n, 4, replace=False))
        _say("full batch: halo", h, "of", part.n, "particles, sources", src)
        ref = oracle.step(part, x[a:a + part.n], sources=src)
        _check_columns(N[a + src], ref["N"])
        _check_rates(lnG[a + src], ref["lnG"], ref["tau"])
        _check_x(xn[a + src], ref["x_new"])


# ---------------------------------------------------------------------------
# periodic lognormal field: 48 rays, many bins, fixed iteration count
# ---------------------------------------------------------------------------
def test_lognormal_small_every_particle():
    """12^3 particles at the 128^3 field's mean spacing (78 kpc), so that h
    spans several times l_ray and many kernels cross the periodic boundary;
    48 rays, 32 bins, 3 fixed iterations, every particle."""
    wl = W.lognormal_field(n_grid=12, box=937.5, n_bins=32, max_iter=3)
    _say("oracle solve: lognormal 12^3")
    ref = oracle.solve(wl)
    assert ref["iters"] == 3
    s = _solver(wl)
    off, hj, hi = s.hits()
    src = np.arange(0, wl.n, 23)
    _, o_off, o_hj, o_hi = oracle.columns(wl, np.ones(wl.n), sources=src, hits=True)
    nr = wl.n_ray
    for i, p in enumerate(src):
        got = _hitsets(off, hj, hi, [p * nr + k for k in range(nr)])
        want = _hitsets(o_off, o_hj, o_hi, [i * nr + k for k in range(nr)])
        assert got == want, f"source {p}"
    assert np.any(o_hi != (8 | 8 << 4 | 8 << 8)), "no periodic image was hit"
    for k in range(3):
        _say("lognormal iteration", k)
        s.set_state(torch.tensor(ref["x_hist"][k]))
        s.compute_columns(want_N=False, count=False)
        lnG, _, _ = s.compute_gamma()
        xn, _ = s.update_equilibrium()
        lnG_o = ref["lnG_hist"][k]
        _check_rates(lnG.cpu().numpy(), lnG_o, math.log(oracle.gamma_thin(wl)) - lnG_o)
        _check_x(xn.cpu().numpy(), ref["x_hist"][k + 1])
    s.set_state(None)
    r = s.iterate(wl.max_iter, wl.tol)
    assert r["iters"] == 3 and not r["converged"]
    _check_x(r["x"].cpu().numpy(), ref["x_hist"][3])


def test_lognormal_full_sampled_sources():
    """The 128^3 field (2097152 particles, 10 Mpc periodic box, 48 rays, 256
    bins): every one of its 10 GPU iterates checked one step at a time on 8
    sampled sources against the oracle fed the same state."""
    wl = W.make_config(2)
    s = _solver(wl)
    rng = np.random.default_rng(3)
    src = np.sort(rng.choice(wl.n, 8, replace=False))
    x = oracle.x_thin(wl)
    assert wl.max_iter == 10
    for k in range(wl.max_iter):
        _say("lognormal field iteration", k)
        s.set_state(torch.tensor(x))
        N, nh = s.compute_columns()
        lnG, _, _ = s.compute_gamma()
        xn, _ = s.update_equilibrium()
        ref = oracle.step(wl, x, sources=src)
        _check_columns(N.cpu().numpy()[src], ref["N"])
        _check_rates(lnG.cpu().numpy()[src], ref["lnG"], ref["tau"])
        _check_x(xn.cpu().numpy()[src], ref["x_new"])
        x = xn.cpu().numpy()
    assert nh > 5e9                      # ~72 intersections per ray


# ---------------------------------------------------------------------------
# edge cases and invariances
# ---------------------------------------------------------------------------
def _tiny(pos, h, L=10.0, box=0.0, dirs=None):
    pos = np.asarray(pos, np.float32).reshape(-1, 3)
    n = pos.shape[0]
    return W.Workload(name="tiny", pos=pos, h=np.asarray(h, np.float32).reshape(n),
                      mu=np.full(n, 1e18, np.float32), n_H=np.full(n, 1e-2, np.float32),
                      T=np.full(n, 1e4, np.float32),
                      dirs=W.healpix_dirs(1) if dirs is None else dirs,
                      sigma=np.array([W.SIGMA_TH]), w=np.array([1e-12 / W.SIGMA_TH]),
                      l_ray=L, box=box, tol=1e-6, max_iter=20)


def test_single_particle_self_column():
    wl = _tiny([(1.0, 2.0, 3.0)], [2.0])
    s = _solver(wl)
    x = np.array([0.5])
    s.set_state(torch.tensor(x))
    N, nh = s.compute_columns()
    assert nh == 12
    _check_columns(N.cpu().numpy(), oracle.columns(wl, x))


def test_zero_length_rays_give_thin_rate():
    wl = _tiny(np.random.default_rng(2).uniform(0, 5, (50, 3)), np.full(50, 1.5), L=0.0)
    s = _solver(wl)
    N, nh = s.compute_columns()
    assert float(N.abs().max()) == 0.0
    lnG, G, tau = s.compute_gamma()
    np.testing.assert_allclose(G.cpu().numpy(), 1e-12, rtol=1e-12)


def test_periodic_images_small_box():
    """Rays longer than the box: images up to two boxes away."""
    rng = np.random.default_rng(3)
    wl = _tiny(rng.uniform(0, 10, (200, 3)), rng.uniform(0.8, 2.0, 200), L=21.0, box=10.0)
    s = _solver(wl)
    off, hj, hi = s.hits()
    src = np.arange(0, 200, 9)
    x = np.full(200, 0.3)
    N_o, o_off, o_hj, o_hi = oracle.columns(wl, x, sources=src, hits=True)
    for i, p in enumerate(src):
        assert _hitsets(off, hj, hi, [p * 12 + k for k in range(12)]) == \
            _hitsets(o_off, o_hj, o_hi, [i * 12 + k for k in range(12)])
    s.set_state(torch.tensor(x))
    N, _ = s.compute_columns()
    _check_columns(N.cpu().numpy()[src], N_o)


def test_permutation_invariance_and_determinism():
    wl = W.isothermal_halo(n=4096, seed=5)
    perm = np.random.default_rng(9).permutation(wl.n)
    wl2 = W.Workload(**{**wl.__dict__, "pos": wl.pos[perm], "h": wl.h[perm], "mu": wl.mu[perm],
                        "n_H": wl.n_H[perm], "T": wl.T[perm]})
    a = _solver(wl).iterate(10, 0.0)
    b = _solver(wl2).iterate(10, 0.0)
    c = _solver(wl).iterate(10, 0.0)
    np.testing.assert_array_equal(a["x"].cpu().numpy(), c["x"].cpu().numpy())  # run to run
    np.testing.assert_allclose(a["x"].cpu().numpy()[perm], b["x"].cpu().numpy(), rtol=1e-6)


def test_resume_from_state():
    wl = W.isothermal_halo(n=4096, seed=6)
    full = _solver(wl).iterate(4, 0.0)
    s = _solver(wl)
    half = s.iterate(2, 0.0)
    s2 = _solver(wl)
    s2.set_state(half["x"])
    rest = s2.iterate(2, 0.0)
    np.testing.assert_array_equal(full["x"].cpu().numpy(), rest["x"].cpu().numpy())


def test_bad_input_is_rejected():
    from paper_1304_4235_amd import RRTError, Solver
    wl = _tiny([(0, 0, 0), (1, 1, 1)], [1.0, -1.0])
    with pytest.raises(RRTError, match="RRT_E_INPUT"):
        Solver.from_workload(wl)
    wl = _tiny([(0, 0, np.nan), (1, 1, 1)], [1.0, 1.0])
    with pytest.raises(RRTError, match="RRT_E_INPUT"):
        Solver.from_workload(wl)
    s = Solver(10.0)
    with pytest.raises(RRTError, match="RRT_E_STATE"):
        s.compute_columns()


def test_empty_and_degenerate_arguments_are_rejected():
    """Empty inputs are errors at the boundary, not silent no-ops: no particles,
    no rays, no bins; so are a non-unit direction, a non-positive cross-section,
    a negative weight and a spectrum whose optically thin rate is zero."""
    from paper_1304_4235_amd import RRTError, Solver
    s = Solver(10.0)
    e = np.zeros(0, np.float32)
    with pytest.raises(RRTError, match="RRT_E_ARG"):
        s.set_particles(np.zeros((0, 3), np.float32), e, e, e, e)
    for dirs in (np.zeros((0, 3)), np.array([[1.0, 1.0, 0.0]])):
        with pytest.raises(RRTError, match="RRT_E_ARG"):
            s.set_rays(dirs)
    for sigma, w in [([], []), ([-6e-18], [1.0]), ([6e-18], [-1.0]), ([6e-18, 1e-18], [0.0, 0.0]),
                     ([6e-18], [np.nan])]:
        with pytest.raises(RRTError, match="RRT_E_ARG"):
            s.set_spectrum(np.array(sigma, float), np.array(w, float))
    # the context still works after the rejected calls
    wl = _tiny([(1.0, 2.0, 3.0), (1.5, 2.0, 3.0)], [2.0, 2.0])
    t = Solver.from_workload(wl)
    N, hits = t.compute_columns()
    assert hits > 0 and np.all(np.isfinite(N.cpu().numpy()))
    t.close()
    s.close()


# ---------------------------------------------------------------------------
# recorded paths vs traversal
# ---------------------------------------------------------------------------
def test_recorded_paths_match_traversal():
    """Recorded paths hold the same intersections and factors as a traversal:
    the columns agree to summation-order rounding, and the counts exactly."""
    wl = W.isothermal_halo(n=16384, seed=21)
    a = _solver(wl, record_paths=1)
    b = _solver(wl, record_paths=0)
    x = np.minimum(oracle.x_thin(wl) * np.geomspace(1, 1e4, wl.n), 0.999)
    for s in (a, b):
        s.set_state(torch.tensor(x))
    Na, ha = a.compute_columns()
    Nb, hb = b.compute_columns()
    assert ha == hb and ha > 0
    assert a.timing()["path_hits"] == ha
    np.testing.assert_allclose(Na.cpu().numpy(), Nb.cpu().numpy(), rtol=1e-12, atol=0)
    # a second state reuses the recorded paths
    x2 = np.minimum(x * 3, 0.999)
    a.set_state(torch.tensor(x2))
    b.set_state(torch.tensor(x2))
    np.testing.assert_allclose(a.compute_columns()[0].cpu().numpy(),
                               b.compute_columns()[0].cpu().numpy(), rtol=1e-12, atol=0)


def _tile_workload(which):
    if which == "halo_small":
        return W.isothermal_halo(n=20000, seed=23)
    if which == "halo_full":
        return W.make_config(1)
    if which == "field_small":
        return W.lognormal_field(n_grid=24, box=1875.0, n_bins=16, max_iter=3)
    return W.make_config(0)                                   # periodic lattice


@pytest.mark.parametrize("which", ["halo_small", "halo_full", "field_small", "lattice"])
def test_row_tiles_give_identical_columns(which):
    """After a few evaluations over the same recorded paths the columns come
    from row tiles (each tile's particle values staged in LDS, 16-bit local
    indices): the same products as the plain product over the recorded paths,
    so the columns agree to FP64 summation order, for any state."""
    wl = _tile_workload(which)
    s = _solver(wl)
    rng = np.random.default_rng(9)
    xs = [np.minimum(oracle.x_thin(wl) * rng.uniform(1, 1e3, wl.n), 0.99) for _ in range(2)]
    s.set_tuning(tiles=0)
    ref = []
    for x in xs:
        s.set_state(torch.tensor(x))
        N, _ = s.compute_columns()
        ref.append(N.clone())
    s.set_tuning(tiles=1)
    s.enable_timing(True)
    for _ in range(10):
        s.compute_columns(want_N=False, count=False)
    tm = s.timing()
    assert tm["tile_set_total"] > 0 and tm["n_tile"] >= 1, "row tiles were not built"
    _say(which, "tiles: distinct particles staged", tm["tile_set_total"],
         "of", tm["path_hits"], "intersections")
    for x, r in zip(xs, ref):
        s.set_state(torch.tensor(x))
        N, _ = s.compute_columns()
        np.testing.assert_allclose(N.cpu().numpy(), r.cpu().numpy(), rtol=1e-13, atol=0)
    if which == "halo_small":
        src = np.arange(0, wl.n, 401)
        x = xs[1]
        ref_o = oracle.step(wl, x, sources=src)
        _check_columns(N.cpu().numpy()[src], ref_o["N"])
    # a new geometry drops the tiles with the recorded paths
    s.build_tree()
    assert s.timing()["tile_set_total"] == -1


def test_path_budget_fallback_and_error():
    from paper_1304_4235_amd import RRTError
    wl = W.isothermal_halo(n=4096, seed=22)
    small = _solver(wl, record_paths=-1, path_budget=1024)
    full = _solver(wl, record_paths=1)
    r1 = small.iterate(6, 0.0)
    r2 = full.iterate(6, 0.0)
    assert small.timing()["path_hits"] == -1          # fell back to traversal
    np.testing.assert_allclose(r1["x"].cpu().numpy(), r2["x"].cpu().numpy(), rtol=1e-10)
    need = _solver(wl, record_paths=1, path_budget=1024)
    with pytest.raises(RRTError, match="RRT_E_WORKSPACE"):
        need.compute_columns()
    assert small.recording_stats()[4] >= 1               # recorded as not fitting


@pytest.mark.parametrize("which", ["lattice", "halo"])
def test_wave_and_lane_traversals_agree(which):
    """The wave-cooperative walk gives every lane exactly its own walk's hits in
    the same order, so hit lists match and columns match bit for bit."""
    wl = W.make_config(0) if which == "lattice" else W.isothermal_halo(n=20000, seed=31)
    a = _solver(wl, traversal=0, record_paths=0)
    b = _solver(wl, traversal=1, record_paths=0)
    x = np.minimum(oracle.x_thin(wl) * np.geomspace(1, 1e3, wl.n), 0.999)
    for s in (a, b):
        s.set_state(torch.tensor(x))
    Na, ha = a.compute_columns()
    Nb, hb = b.compute_columns()
    assert ha == hb
    np.testing.assert_array_equal(Na.cpu().numpy(), Nb.cpu().numpy())
    oa, ja, ia = a.hits()
    ob, jb, ib = b.hits()
    np.testing.assert_array_equal(oa, ob)
    np.testing.assert_array_equal(ja, jb)
    np.testing.assert_array_equal(ia, ib)


@pytest.mark.parametrize("rank", [0, 5])
def test_field_shard_owned_columns_equal_the_whole_field(rank):
    """One GPU's share of a periodic field: block `rank` of 8 plus every
    particle within l_ray + max(h) of it, in the same periodic box.  The rays
    of owned sources reach only particles of the shard, so their columns equal
    those of the whole field (summation order aside)."""
    wl = W.lognormal_field(n_grid=40, box=3125.0, n_bins=16)
    rng = np.random.default_rng(31)
    x = np.minimum(oracle.x_thin(wl) * rng.uniform(1, 1e3, wl.n), 0.99)
    full = _solver(wl)
    full.set_state(torch.tensor(x))
    N_full, _ = full.compute_columns()
    N_full = N_full.cpu().numpy()
    full.close()
    sh = W.field_shard(wl, rank, 8)
    idx, n_own = sh.meta["index"], sh.meta["n_owned"]
    _say("shard", rank, "owned", n_own, "ghosts", sh.n - n_own)
    assert 0 < n_own < sh.n < wl.n
    s = _solver(sh)
    s.set_state(torch.tensor(x[idx]))
    N_sh, _ = s.compute_columns()
    np.testing.assert_allclose(N_sh.cpu().numpy()[:n_own], N_full[idx[:n_own]], rtol=1e-12,
                               atol=0)
    s.close()


@pytest.mark.parametrize("room", ["ample", "short"])
def test_one_pass_recording_equals_two_passes(room):
    """One-pass recording (hits appended to pool chunks, then compacted) gives
    the same recorded paths as a counting walk followed by a recording walk:
    bit-identical columns over them and the same counts.  The pool is capped
    from the first recording's count so that the second recording takes one
    pass whatever the intersections per ray; a pool of about 2000 chunks runs
    short at once (two chunks per slice, so every block of chunks a wave takes
    is a slice's partial last one), and the recording falls back to the second
    walk with the counts it has.  The recording statistics say which walks
    ran: the first
    recording follows the count the Solver makes to size its path buffer."""
    wl = W.isothermal_halo(n=16384, seed=21)
    x = np.minimum(oracle.x_thin(wl) * np.geomspace(1, 1e4, wl.n), 0.999)
    out = []
    for one_pass in (False, True):
        s = _solver(wl, record_paths=1)
        s.set_tuning(one_pass=0)
        _, first = s.compute_columns(want_N=False)       # one walk after the count
        np.testing.assert_array_equal(s.recording_stats(), [0, 0, 1, 0, 0])
        if one_pass:
            cap = first * 3 // 64 + 4096 if room == "ample" else 2000
            s.set_tuning(one_pass=int(cap))
        s.build_tree()                                     # drops the paths
        s.set_state(torch.tensor(x))
        N, hits = s.compute_columns()
        assert s.timing()["path_hits"] == hits == first
        st = s.recording_stats()
        if not one_pass:
            np.testing.assert_array_equal(st, [0, 0, 1, 1, 0])   # count + record walks
        elif room == "ample":
            np.testing.assert_array_equal(st, [1, 0, 1, 0, 0])   # one walk
        else:
            np.testing.assert_array_equal(st, [0, 1, 1, 0, 0])   # ran short: second walk
        out.append(N.cpu().numpy())
    np.testing.assert_array_equal(out[0], out[1])


def test_full_halo_one_walk_recording():
    """The 262144-particle halo with the default knobs, as the solve of a
    whole step runs it: a context's second recording (one walk into the pool
    sized from the first, chunks taken from 1024 slices) records the same
    paths as its first (a counting walk, then a recording walk): the same
    count, bit-identical columns, and sampled sources equal to the oracle."""
    wl = W.make_config(1)
    s = _solver(wl)
    x = oracle.x_thin(wl)
    cols = []
    for k in range(2):
        _say("full halo recording", k)
        if k:
            s.build_tree()                                 # drops the paths
        s.set_state(torch.tensor(x))
        N, hits = s.compute_columns()
        assert hits == s.timing()["path_hits"]
        cols.append((N.cpu().numpy(), hits))
    assert cols[1][1] == cols[0][1]
    np.testing.assert_array_equal(cols[1][0], cols[0][0])
    # the first recording followed the Solver's count, the second took one walk
    np.testing.assert_array_equal(s.recording_stats(), [1, 0, 1, 0, 0])
    src = np.sort(np.random.default_rng(5).choice(wl.n, 16, replace=False))
    ref = oracle.step(wl, x, sources=src)
    _check_columns(cols[1][0][src], ref["N"])
    s.close()


@pytest.mark.parametrize("which", ["lattice", "field_small", "halo_full"])
def test_streamed_product_equals_its_definition(which):
    """The streamed product (blocks of consecutive rows read through LDS
    windows of 2048 entries) against the product with 32 lanes per row, and on
    sampled rays against its definition written out on the host: N = the FP64
    sum over the ray's recorded hits of fl32(mux_j * factor), mux_j =
    fl32(mu_j x_j).  The full halo has blocks of more than one window, so rows
    that straddle windows are covered."""
    wl = _tile_workload(which)
    s = _solver(wl)
    rng = np.random.default_rng(17)
    x = np.minimum(oracle.x_thin(wl) * rng.uniform(1, 1e3, wl.n), 0.99)
    s.set_state(torch.tensor(x))
    s.set_tuning(path_group=32)
    Ng, hg = s.compute_columns()
    s.set_tuning(path_group=0)
    Ns, hs = s.compute_columns()
    assert hg == hs
    Ng, Ns = Ng.cpu().numpy(), Ns.cpu().numpy()
    np.testing.assert_allclose(Ns, Ng, rtol=1e-13, atol=0)
    # blocks of the stream in tree order: R rows, R from the mean row length
    cnt = np.zeros(s.n * s.n_ray + 1, np.int64)
    s._call("rrt_get_hits", 0, cnt.ctypes.data, None, None)
    per_ray = np.diff(cnt).reshape(s.n, s.n_ray)
    perm = s.tree()["perm"]
    rows = per_ray[perm].T.reshape(-1)                # row k * n + ps
    mean = rows.sum() / rows.size
    R = 64
    while R > 4 and R * mean > 2048:
        R //= 2
    pad = (-rows.size) % R
    blocks = np.concatenate([rows, np.zeros(pad, np.int64)]).reshape(-1, R).sum(axis=1)
    _say(which, "rows per block", R, "largest block", int(blocks.max()), "entries")
    if which == "halo_full":
        assert blocks.max() > 2048, "no block spans two windows"
    src = rng.choice(wl.n, 48, replace=False)
    ro, hj, fac = s.path_rows(src)
    mux = (np.asarray(wl.mu, np.float64) * x).astype(np.float32)
    for i, p in enumerate(src):
        for k in range(s.n_ray):
            a, b = ro[i * s.n_ray + k], ro[i * s.n_ray + k + 1]
            terms = (mux[hj[a:b]] * fac[a:b]).astype(np.float32).astype(np.float64)
            exact = math.fsum(terms)
            bound = 1e-15 * max(b - a, 1) * np.abs(terms).sum()
            assert abs(Ns[p, k] - exact) <= bound, (p, k, Ns[p, k], exact)


def test_rates_of_thin_and_thick_rays_on_the_same_columns():
    """The rate of a particle from its rays' columns (Sec. 3.3, eq. gamma_shld):
    the kernel sums a ray's bins with hardware exponentials, or, for a ray
    thin in every bin ((sigma_b - sigma_min) N <= 0.15), as the degree-5
    Taylor form of the same sum.  Both against the FP64 rate of the oracle on
    the GPU's own columns, on a state with rays on both sides of the switch."""
    wl = W.isothermal_halo(n=20000, seed=29)
    s = _solver(wl)
    x = np.minimum(oracle.x_thin(wl) * np.geomspace(1.0, 100.0, wl.n), 0.99)
    s.set_state(torch.tensor(x))
    N, _ = s.compute_columns()
    lnG, _, _ = s.compute_gamma()
    N = N.cpu().numpy()
    sig = np.asarray(wl.sigma, np.float64)
    y = (sig.max() - sig.min()) * N
    thin = float(np.mean(y <= 0.15))
    _say("rays thin in every bin:", thin)
    assert 0.1 < thin < 0.9, "the state should put rays on both sides of the switch"
    ref, _, _ = oracle.gamma(N, sig, np.asarray(wl.w, np.float64))
    err = np.abs(lnG.cpu().numpy() - ref)
    _say("max |ln Gamma - oracle| on the same columns:", float(err.max()))
    assert err.max() < 5e-6
