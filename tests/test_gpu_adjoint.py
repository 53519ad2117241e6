"""Reverse mode through K unrolled iterations: gradients of ln Gamma and x with
respect to the bin weights and the particle densities.

Checked against central finite differences of the GPU forward itself and of
the FP64 oracle's K-step solve, and coordinate by coordinate against the
oracle's own reverse mode (itself pinned to central differences of its solve)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _setup(wl, K, paths=-1):
    from paper_1304_4235_amd import Solver
    s = Solver.from_workload(wl, record_paths=paths)
    return s


def _loss_parts(wl, seed=0):
    rng = np.random.default_rng(seed)
    c_x = torch.tensor(rng.uniform(-1, 1, wl.n), dtype=torch.float64, device="cuda")
    return c_x


def _gpu_loss(s, w, nH, K, lnG_t, c_x):
    s.set_spectrum(s.sigma, w)
    s.set_density(torch.tensor(nH, dtype=torch.float32))
    lnG, x = s.forward(K)
    return float((((lnG - lnG_t) / np.log(10)) ** 2).sum() + (c_x * x).sum())


def _adjoint(s, w, nH, K, lnG_t, c_x):
    s.set_spectrum(s.sigma, w)
    s.set_density(torch.tensor(nH, dtype=torch.float32))
    lnG, x = s.forward(K)
    g_lnG = 2 * (lnG - lnG_t) / np.log(10) ** 2
    dw, dn = s.backward(g_lnG, c_x)
    return dw, dn.cpu().numpy()


@pytest.mark.parametrize("paths", [-1, 0])
def test_adjoint_vs_gpu_central_differences(paths):
    wl = W.isothermal_halo(n=4096, n_bins=16, seed=41, n_peak=3.0)
    K = 6
    s = _setup(wl, K, paths)
    w0 = wl.w.copy()
    nH0 = wl.n_H.astype(np.float32).copy()
    # target from 1.2x the weights
    s.set_spectrum(s.sigma, 1.2 * w0)
    lnG_t, _ = s.forward(K)
    c_x = _loss_parts(wl)
    dw, dn = _adjoint(s, w0, nH0, K, lnG_t, c_x)
    rng = np.random.default_rng(3)
    # weights: relative step 1e-3
    for b in rng.choice(wl.n_bins, 6, replace=False):
        h = 1e-3 * w0[b]
        wp, wm = w0.copy(), w0.copy()
        wp[b] += h
        wm[b] -= h
        fd = (_gpu_loss(s, wp, nH0, K, lnG_t, c_x) - _gpu_loss(s, wm, nH0, K, lnG_t, c_x)) / (2 * h)
        _say("w", b, dw[b], fd)
        assert abs(dw[b] - fd) <= 2e-3 * abs(fd) + 1e-4 * np.max(np.abs(dw)) 
    # densities: relative step 1e-2 (in FP32).  The forward rounds mu x and
    # the chord factors to FP32, so the loss moves by a few of its ulps whenever
    # any rounding flips; for a low-density particle a 1e-3 step leaves that
    # noise at several percent of the difference (measured: 948 / 967 / 977.6
    # at steps 1e-3 / 3e-3 / 1e-2 against an adjoint of 976.3), while the
    # central difference's own error at 1e-2 is far below the tolerance.
    scale = np.max(np.abs(dn))
    big = np.argsort(-np.abs(dn))[:4]
    for j in list(rng.choice(wl.n, 6, replace=False)) + list(big):
        up = np.float32(nH0[j] * (1 + 1e-2))
        dn_ = np.float32(nH0[j] * (1 - 1e-2))
        npl, nmi = nH0.copy(), nH0.copy()
        npl[j], nmi[j] = up, dn_
        fd = (_gpu_loss(s, w0, npl, K, lnG_t, c_x) - _gpu_loss(s, w0, nmi, K, lnG_t, c_x)) / \
            (float(up) - float(dn_))
        _say("n", j, dn[j], fd)
        assert abs(dn[j] - fd) <= 5e-3 * abs(fd) + 1e-4 * scale


def test_adjoint_vs_oracle_central_differences():
    """Tiny periodic lattice: GPU adjoint against central differences of the FP64
    oracle's K-step solve."""
    wl = W.make_config(0, n_side_lattice=6, box=37.5, max_iter=3)
    wl.sigma, wl.w = W.power_law_spectrum(6, 1.5, 1e-12)
    wl.n_H = np.full(wl.n, 5e-3, np.float32)
    K = 3
    s = _setup(wl, K)
    w0 = wl.w.copy()
    nH0 = wl.n_H.copy()
    mu0 = wl.mu.copy()
    s.set_spectrum(s.sigma, 1.2 * w0)
    lnG_t = s.forward(K)[0].cpu().numpy()
    rng = np.random.default_rng(5)
    c_x = rng.uniform(-1, 1, wl.n)
    dw, dn = _adjoint(s, w0, nH0, K, torch.tensor(lnG_t, device="cuda"),
                      torch.tensor(c_x, device="cuda"))

    def oloss(w, nH, mu):
        wl2 = W.Workload(**{**wl.__dict__, "w": w, "n_H": nH, "mu": mu})
        r = oracle.solve(wl2, max_iter=K, tol=0.0)
        lnG, x = r["lnG_hist"][-1], r["x_hist"][-1]
        return np.sum(((lnG - lnG_t) / np.log(10)) ** 2) + np.sum(c_x * x)

    for b in range(wl.n_bins):
        h = 1e-4 * w0[b]
        wp, wm = w0.copy(), w0.copy()
        wp[b] += h
        wm[b] -= h
        fd = (oloss(wp, nH0, mu0) - oloss(wm, nH0, mu0)) / (2 * h)
        _say("oracle w", b, dw[b], fd)
        assert abs(dw[b] - fd) <= 2e-3 * abs(fd) + 1e-4 * np.max(np.abs(dw))
    scale = np.max(np.abs(dn))
    for j in rng.choice(wl.n, 5, replace=False):
        up, lo = np.float32(nH0[j] * (1 + 1e-3)), np.float32(nH0[j] * (1 - 1e-3))
        npl, nmi = nH0.copy(), nH0.copy()
        mpl, mmi = mu0.copy(), mu0.copy()
        npl[j], nmi[j] = up, lo
        mpl[j] = np.float32(np.float64(mu0[j]) * np.float64(up) / np.float64(nH0[j]))
        mmi[j] = np.float32(np.float64(mu0[j]) * np.float64(lo) / np.float64(nH0[j]))
        fd = (oloss(w0, npl, mpl) - oloss(w0, nmi, mmi)) / (float(up) - float(lo))
        _say("oracle n", j, dn[j], fd)
        assert abs(dn[j] - fd) <= 5e-3 * abs(fd) + 1e-4 * scale


def test_autograd_function_matches_solver():
    """RRTFunction's gradients are Solver.backward's on the same loss, bit for
    bit, and within the oracle-gradient bar of the FP64 oracle's reverse mode
    on the lattice; a backward whose forward is no longer the solver's latest
    raises instead of returning the gradient at other parameters."""
    from paper_1304_4235_amd.autograd import RRTFunction, log10_rate_loss
    wl = W.isothermal_halo(n=2048, n_bins=8, seed=43)
    K = 4
    s = _setup(wl, K)
    w = torch.tensor(wl.w, dtype=torch.float64, requires_grad=True)
    nH = torch.tensor(wl.n_H, dtype=torch.float32, device="cuda", requires_grad=True)
    with torch.no_grad():
        lnG_t, _ = RRTFunction.apply(w * 1.2, nH, s, K)
    lnG, x = RRTFunction.apply(w, nH, s, K)
    loss = log10_rate_loss(lnG, lnG_t) + x.sum()
    loss.backward()
    # the same loss through the solver's own entry points
    s.set_spectrum(s.sigma, wl.w)
    s.set_density(torch.tensor(wl.n_H, dtype=torch.float32))
    lnG2, x2 = s.forward(K)
    assert torch.equal(lnG2, lnG.detach()) and torch.equal(x2, x.detach())
    # the output derivatives by the same operations as above
    l2, x2r = lnG2.clone().requires_grad_(True), x2.clone().requires_grad_(True)
    (log10_rate_loss(l2, lnG_t) + x2r.sum()).backward()
    dw, dn = s.backward(l2.grad, x2r.grad)
    np.testing.assert_array_equal(w.grad.numpy(), dw)
    np.testing.assert_array_equal(nH.grad.cpu().numpy(), dn.to(torch.float32).cpu().numpy())
    assert float(w.grad.abs().sum()) > 0 and float(nH.grad.abs().sum()) > 0
    # a second forward in between: the first graph's backward refuses
    lnG3, x3 = RRTFunction.apply(w, nH, s, K)
    with torch.no_grad():
        RRTFunction.apply(w * 1.1, nH, s, K)
    with pytest.raises(RuntimeError, match="another forward"):
        (lnG3.sum() + x3.sum()).backward()


def test_autograd_function_against_the_oracle_adjoint():
    """On the periodic lattice, RRTFunction's gradients of a loss of ln Gamma
    and x equal the FP64 oracle's reverse mode of the same K-step map, every
    coordinate, at the oracle-gradient bar."""
    from paper_1304_4235_amd.autograd import RRTFunction
    wl = W.make_config(0)
    K = 3
    s = _setup(wl, K)
    rng = np.random.default_rng(44)
    c_l = rng.uniform(-1, 1, wl.n)
    c_x = rng.uniform(-1, 1, wl.n)
    w = torch.tensor(wl.w, dtype=torch.float64, requires_grad=True)
    nH = torch.tensor(wl.n_H, dtype=torch.float32, device="cuda", requires_grad=True)
    lnG, x = RRTFunction.apply(w, nH, s, K)
    loss = (torch.tensor(c_l, device="cuda") * lnG).sum() + \
        (torch.tensor(c_x, device="cuda") * x).sum()
    loss.backward()
    ref = oracle.adjoint(wl, K, dL_dlnG=c_l, dL_dx=c_x)
    gw, gn = w.grad.numpy(), nH.grad.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(gw, ref["dw"], rtol=1e-5, atol=1e-5 * np.max(np.abs(ref["dw"])))
    np.testing.assert_allclose(gn, ref["dnH"], rtol=1e-5,
                               atol=1e-5 * np.max(np.abs(ref["dnH"])))


def test_full_halo_gradient_central_differences():
    """The 262144-particle halo, 128 bins: K frozen from a converged base run,
    loss sum (log10 Gamma - log10 Gamma_target)^2 with the target from 1.2x the
    weights; 32 coordinates by central differences of the GPU forward.

    Weights and the 12 largest density gradients at relative step 1e-3
    (measured: 4.2e-5 and 1.3e-4 relative; bars 5e-4 and 1e-3).  12 random
    densities at relative step 1e-2: most sit in the outskirts with gradients
    near 5e-5 of the largest, where the difference quotient of the FP32
    forward through 120 iterations carries an absolute floor (measured 4e-5 of
    the largest gradient at step 1e-2, 1.9e-4 at 1e-3; up to 10% of such a
    coordinate), so they take an absolute bar of 2e-4 of the largest.  The
    small coordinates' relative accuracy is checked against the oracle's
    reverse mode instead, where no difference quotient is involved."""
    wl = W.make_config(4)
    from paper_1304_4235_amd import Solver
    s = Solver.from_workload(wl)
    K = s.iterate(wl.max_iter, wl.tol, want_x=False)["iters"]
    _say("frozen K", K)
    w0 = wl.w.copy()
    nH0 = wl.n_H.astype(np.float32).copy()
    s.set_spectrum(s.sigma, 1.2 * w0)
    lnG_t, _ = s.forward(K)
    c_x = torch.zeros(wl.n, dtype=torch.float64, device="cuda")
    dw, dn = _adjoint(s, w0, nH0, K, lnG_t, c_x)
    assert np.all(np.isfinite(dw)) and np.all(np.isfinite(dn))
    rng = np.random.default_rng(11)
    scale_n = np.max(np.abs(dn))
    checked = 0
    for b in rng.choice(wl.n_bins, 8, replace=False):
        h = 1e-3 * w0[b]
        wp, wm = w0.copy(), w0.copy()
        wp[b] += h
        wm[b] -= h
        fd = (_gpu_loss(s, wp, nH0, K, lnG_t, c_x) - _gpu_loss(s, wm, nH0, K, lnG_t, c_x)) / (2 * h)
        _say("w", b, dw[b], fd)
        assert abs(dw[b] - fd) <= 5e-4 * abs(fd)
        checked += 1
    # densities: the largest-gradient particles and random ones
    top = list(np.argsort(-np.abs(dn))[:12])
    for j in top + list(rng.choice(wl.n, 12, replace=False)):
        rel = 1e-3 if j in top else 1e-2
        up, lo = np.float32(nH0[j] * (1 + rel)), np.float32(nH0[j] * (1 - rel))
        npl, nmi = nH0.copy(), nH0.copy()
        npl[j], nmi[j] = up, lo
        fd = (_gpu_loss(s, w0, npl, K, lnG_t, c_x) - _gpu_loss(s, w0, nmi, K, lnG_t, c_x)) / \
            (float(up) - float(lo))
        _say("n", j, dn[j], fd)
        if j in top:
            assert abs(dn[j] - fd) <= 1e-3 * abs(fd)
        else:
            assert abs(dn[j] - fd) <= 1e-3 * abs(fd) + 2e-4 * scale_n
        checked += 1
    assert checked == 32


def test_full_field_gradient_central_differences():
    """The differentiation workload at the sizes it names: 256 per-bin weights
    and the 2.1M densities of the lognormal field (48 rays), K = 10 (the
    field's fixed iteration count); the same loss and 32-coordinate
    central-difference check as the halo's, at relative step 1e-2: a bin
    carries about 1/256 of each rate and the field's densities are near
    1e-5 cm^-3, so a 1e-3 step moves the loss by about as much as the FP32
    rounding of the forward does (measured at 1e-3: a hard bin -0.0189
    against -0.0208, a low-density particle 0.446 against 0.512, while the
    largest components agreed to 2e-4).  Measured at 1e-2: weights 3.7e-6
    relative, densities 1.9e-4 relative at most (bars 1e-4 and 1e-3)."""
    wl = W.make_config(2)
    from paper_1304_4235_amd import Solver
    s = Solver.from_workload(wl)
    K = wl.max_iter
    w0 = wl.w.copy()
    nH0 = wl.n_H.astype(np.float32).copy()
    s.set_spectrum(s.sigma, 1.2 * w0)
    lnG_t, _ = s.forward(K)
    c_x = torch.zeros(wl.n, dtype=torch.float64, device="cuda")
    dw, dn = _adjoint(s, w0, nH0, K, lnG_t, c_x)
    assert dw.size == 256 and dn.size == wl.n
    assert np.all(np.isfinite(dw)) and np.all(np.isfinite(dn))
    rng = np.random.default_rng(12)
    scale_n = np.max(np.abs(dn))
    checked = 0
    for b in rng.choice(wl.n_bins, 8, replace=False):
        h = 1e-2 * w0[b]
        wp, wm = w0.copy(), w0.copy()
        wp[b] += h
        wm[b] -= h
        fd = (_gpu_loss(s, wp, nH0, K, lnG_t, c_x) - _gpu_loss(s, wm, nH0, K, lnG_t, c_x)) / (2 * h)
        _say("w", b, dw[b], fd)
        assert abs(dw[b] - fd) <= 1e-4 * abs(fd)
        checked += 1
    cand = list(np.argsort(-np.abs(dn))[:12]) + list(rng.choice(wl.n, 12, replace=False))
    for j in cand:
        up, lo = np.float32(nH0[j] * (1 + 1e-2)), np.float32(nH0[j] * (1 - 1e-2))
        npl, nmi = nH0.copy(), nH0.copy()
        npl[j], nmi[j] = up, lo
        fd = (_gpu_loss(s, w0, npl, K, lnG_t, c_x) - _gpu_loss(s, w0, nmi, K, lnG_t, c_x)) / \
            (float(up) - float(lo))
        _say("n", j, dn[j], fd)
        assert abs(dn[j] - fd) <= 1e-3 * abs(fd)
        checked += 1
    assert checked == 32


def test_transposed_paths_deterministic_and_match_scatter():
    """The gather over transposed paths is deterministic and equals the
    atomic scatter of a re-traversal to summation-order rounding."""
    wl = W.isothermal_halo(n=8192, n_bins=16, seed=45)
    K = 5
    sa = _setup(wl, K, paths=-1)
    sb = _setup(wl, K, paths=0)
    out = []
    for s in (sa, sa, sb):
        lnG, x = s.forward(K)
        g = torch.ones_like(lnG)
        dw, dn = s.backward(g, None)
        out.append((dw, dn.cpu().numpy()))
    np.testing.assert_array_equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_allclose(out[0][1], out[2][1], rtol=1e-9, atol=1e-12 * np.abs(out[2][1]).max())
    np.testing.assert_allclose(out[0][0], out[2][0], rtol=1e-9)


def _many_rays(m=32, n_side=16):
    """m^3 jittered lattice (unit spacing, isolated) with h = 0.6 and l_ray =
    0.5: one or two intersections per ray, but 12 n_side^2 = 3072 rays per
    particle, so 64 lanes per ray exceed 2^32 work-items (100663296 rays)."""
    rng = np.random.default_rng(77)
    g = np.stack(np.meshgrid(*[np.arange(m)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pos = (g + 0.5 + rng.uniform(-0.1, 0.1, g.shape)).astype(np.float32)
    n = m ** 3
    sigma, w = W.power_law_spectrum(16, 1.5, 1e-12)
    return W.Workload(name="many_rays", pos=pos, h=np.full(n, 0.6, np.float32),
                      mu=np.full(n, 1e18, np.float32), n_H=np.full(n, 1e-2, np.float32),
                      T=np.full(n, 1e4, np.float32), dirs=W.healpix_dirs(n_side), sigma=sigma,
                      w=w, l_ray=0.5, box=0.0, tol=1e-6, max_iter=3)


def test_many_rays_products_cover_every_ray():
    """1e8 rays: every lane grouping of the path product, and the three
    transposed products of the reverse mode (gather over transposed paths,
    atomic scatter over paths, scatter by re-traversal), cover every ray; the
    columns of sampled sources match the oracle."""
    wl = _many_rays()
    assert wl.n * wl.n_ray * 64 > 2 ** 32
    K = 2
    s = _setup(wl, K)
    _say("many rays: columns by lane grouping")
    rng = np.random.default_rng(5)
    x = np.minimum(oracle.x_thin(wl) * rng.uniform(1, 100, wl.n), 0.9)
    x2 = np.minimum(x * 2.0, 0.95)
    s.set_tuning(path_group=8)
    s.set_state(torch.tensor(x))
    Na, _ = s.compute_columns()
    Na = Na.clone()
    for g in (16, 32, 64):
        s.set_tuning(path_group=g)
        s.set_state(torch.tensor(x2))            # different columns in the buffer first
        s.compute_columns(want_N=False, count=False)
        s.set_state(torch.tensor(x))
        Nb, _ = s.compute_columns()
        assert torch.equal(Nb, Na), f"lane group {g}"
    src = np.array([0, wl.n // 2, wl.n - 1])
    ref = oracle.step(wl, x, sources=src)
    got = Na.cpu().numpy()[src]
    np.testing.assert_allclose(got, ref["N"], rtol=1e-6, atol=0)
    _say("many rays: reverse-mode products")
    s.set_tuning(path_group=0)
    out = []
    for mode in (0, 1, 2):
        s.set_tuning(adjoint_scatter=mode)
        lnG, xk = s.forward(K)
        dw, dn = s.backward(torch.ones_like(lnG), None)
        out.append((dw, dn.cpu().numpy()))
    sb = _setup(wl, K, paths=0)
    lnG, xk = sb.forward(K)
    dw, dn = sb.backward(torch.ones_like(lnG), None)
    out.append((dw, dn.cpu().numpy()))
    for i in (1, 2, 3):
        np.testing.assert_allclose(out[i][1], out[0][1], rtol=1e-9,
                                   atol=1e-12 * np.abs(out[0][1]).max())
        np.testing.assert_allclose(out[i][0], out[0][0], rtol=1e-9)
    s.close()
    sb.close()


def test_tile_scatter_matches_transposed_gather():
    """Reverse mode accumulating per row tile in LDS (one global atomic per
    distinct particle of a tile) against the deterministic gather over the
    transposed paths: the same products, summed in another order."""
    wl = W.isothermal_halo(n=8192, n_bins=16, seed=46)
    K = 4
    s = _setup(wl, K)
    s.enable_timing(True)
    out = []
    for mode in (0, 2):
        s.set_tuning(adjoint_scatter=mode)
        lnG, x = s.forward(K)
        dw, dn = s.backward(torch.ones_like(lnG), None)
        out.append((dw, dn.cpu().numpy()))
    assert s.timing()["tile_set_total"] > 0          # the row tiles were built
    np.testing.assert_allclose(out[1][1], out[0][1], rtol=1e-9,
                               atol=1e-12 * np.abs(out[0][1]).max())
    np.testing.assert_allclose(out[1][0], out[0][0], rtol=1e-9)


def _adjoint_cases():
    lat = W.make_config(0, n_side_lattice=6, box=37.5, max_iter=3)
    lat.sigma, lat.w = W.power_law_spectrum(6, 1.5, 1e-12)
    rng = np.random.default_rng(1)
    lat.n_H = (np.full(lat.n, 5e-3) * rng.uniform(0.5, 2.0, lat.n)).astype(np.float32)
    halo = W.isothermal_halo(n=3000, n_bins=16, seed=47, n_peak=3.0)
    return {"lattice": (lat, 3), "halo": (halo, 4)}


# The device path takes per-hit factors and bin terms in FP32 (~1e-7 relative
# each) and sums in FP64; measured agreement is ~3e-7 (weights) and ~8e-7 of
# the largest density gradient.
GRAD_RTOL = 1e-5     # per coordinate, relative
GRAD_ATOL = 1e-5     # times the largest gradient of the vector
# Every density gradient at or above 1e-4 of the largest, on its own scale:
# measured at most 1.3e-4 relative (median 1e-7, no signed bias) on this halo
# and on a 20000-particle, 64-bin halo at K = 6.  Below 1e-4 of the largest a
# coordinate is a cancellation of terms of the largest's size and FP32
# products limit it to the absolute bar above.
SMALL_FROM = 1e-4
SMALL_RTOL = 1e-3


@pytest.mark.parametrize("case", ["lattice", "halo"])
def test_adjoint_matches_oracle_adjoint_everywhere(case):
    """Every bin-weight and every density gradient against the FP64 oracle's
    reverse mode of the same K iterations, for each transposed product:
    gather over transposed paths, atomic scatter over paths, row-tile scatter,
    and scatter by re-traversal."""
    wl, K = _adjoint_cases()[case]
    rng = np.random.default_rng(11)
    gl, gx = rng.uniform(-1, 1, wl.n), rng.uniform(-1, 1, wl.n)
    _say(case, "oracle adjoint, n", wl.n, "K", K)
    ref = oracle.adjoint(wl, K, gl, gx)
    runs = [("transposed", -1, 0), ("atomic", -1, 1), ("tiles", -1, 2), ("traversal", 0, 0)]
    for name, paths, mode in runs:
        _say(case, name)
        s = _setup(wl, K, paths)
        s.set_tuning(adjoint_scatter=mode)
        lnG, x = s.forward(K)
        np.testing.assert_allclose(x.cpu().numpy(), ref["x"], rtol=1e-4)
        dw, dn = s.backward(torch.tensor(gl, device="cuda"), torch.tensor(gx, device="cuda"))
        dn = dn.cpu().numpy()
        ew = np.abs(dw - ref["dw"])
        en = np.abs(dn - ref["dnH"])
        _say(f"  dw max rel {np.max(ew / np.abs(ref['dw'])):.2e}  dn max err/scale "
             f"{en.max() / np.abs(ref['dnH']).max():.2e}")
        assert np.all(ew <= GRAD_RTOL * np.abs(ref["dw"]) + GRAD_ATOL * np.abs(ref["dw"]).max())
        assert np.all(en <= GRAD_RTOL * np.abs(ref["dnH"]) + GRAD_ATOL * np.abs(ref["dnH"]).max())
        big = np.abs(ref["dnH"]) >= SMALL_FROM * np.abs(ref["dnH"]).max()
        _say(f"  dn max rel over |g| >= {SMALL_FROM:g} max: "
             f"{np.max(en[big] / np.abs(ref['dnH'][big])):.2e} ({big.sum()} of {wl.n})")
        assert np.all(en[big] <= SMALL_RTOL * np.abs(ref["dnH"][big]))
        s.close()


def test_kept_and_recomputed_columns_give_the_same_gradients():
    """The reverse mode reads each iteration's columns as kept by the forward,
    or recomputes them from the kept states: the same columns, so the same
    gradients (bit for bit with the deterministic gather)."""
    wl = W.isothermal_halo(n=4096, n_bins=16, seed=48, n_peak=3.0)
    K = 5
    s = _setup(wl, K)
    rng = np.random.default_rng(12)
    gl = torch.tensor(rng.uniform(-1, 1, wl.n), device="cuda")
    gx = torch.tensor(rng.uniform(-1, 1, wl.n), device="cuda")
    out = []
    for keep in (1, 0, 1):
        s.set_tuning(keep_columns=keep)
        lnG, x = s.forward(K)
        dw, dn = s.backward(gl, gx)
        out.append((dw, dn.cpu().numpy()))
    for dw, dn in out[1:]:
        np.testing.assert_array_equal(dw, out[0][0])
        np.testing.assert_array_equal(dn, out[0][1])
    s.close()


def test_backward_needs_a_forward_with_the_current_parameters():
    from paper_1304_4235_amd import RRTError
    wl = W.isothermal_halo(n=1024, n_bins=4, seed=49)
    s = _setup(wl, 2)
    for change in ("spectrum", "density", "tree"):
        lnG, x = s.forward(2)
        if change == "spectrum":
            s.set_spectrum(s.sigma, 1.1 * wl.w)
        elif change == "density":
            s.set_density(torch.tensor(wl.n_H * 1.1, dtype=torch.float32))
        else:
            s.build_tree()
        with pytest.raises(RRTError):
            s.backward(torch.ones_like(lnG), None)
    lnG, x = s.forward(2)
    dw, dn = s.backward(torch.ones_like(lnG), None)
    assert np.all(np.isfinite(dw))
    s.close()
