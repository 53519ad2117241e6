"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: a value or
bound the paper states, a closed form from the paper, an invariant of the
method, a special case with a textbook answer, or brute force done another way.
"""
import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import integrate, special

import oracle
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_statements.json")))


# ---------------------------------------------------------------------------
# kernel (Sec. 4.1.1, Appendix B)
# ---------------------------------------------------------------------------
def test_kernel_constants_from_defining_conditions():
    """sigma is fixed by G(0, sigma^2) = M4(0, h); N by unit volume integral."""
    kc = oracle.kernel_constants()
    h = 1.0
    sigma2 = kc["sigma_over_h"] ** 2
    # untruncated normalised Gaussian at the origin equals M4's central value
    g0 = 1.0 / (2 * math.pi * sigma2) ** 1.5
    assert abs(g0 - 8 / (math.pi * h ** 3)) < 1e-13 * g0
    assert abs(kc["A2h2"] - 1 / (2 * sigma2)) < 1e-13
    assert abs(kc["t"] ** 2 - kc["A2h2"]) < 1e-13
    assert abs(kc["t"] - 2 * math.pi ** (1 / 6)) < 1e-14
    # volume normalisation of the truncated kernel, evaluated independently by scipy
    v, _ = integrate.quad(lambda r: 4 * math.pi * r * r * oracle.Gt(r, h), 0, h,
                          epsabs=1e-13, epsrel=1e-13, limit=200)
    assert abs(v - GOLD["kernel_norm"]["value"]) < 1e-12


@pytest.mark.parametrize("h", [0.37, 1.0, 14.2, 480.0])
def test_kernel_normalisation_both_kernels(h):
    assert abs(oracle.kernel_norm(h, "Gt") - 1.0) < 1e-12
    assert abs(oracle.kernel_norm(h, "M4") - 1.0) < 1e-12


def test_appendix_b_kernel_comparison():
    h = 1.0
    m4max = oracle.M4(0.0, h)
    assert oracle.Gt(h, h) / m4max < GOLD["gt_at_h_over_m4_max_below"]["value"]
    r = np.linspace(0, h, 20001)
    diff = max(abs(oracle.Gt(x, h) - oracle.M4(x, h)) for x in r) / m4max
    # the paper says "smaller than 3%"; exactly it is 3.03%, so allow the rounding
    assert 0.025 < diff < GOLD["gt_minus_m4_over_m4_max_below"]["value"] + 0.0015
    assert oracle.Gt(1.0000001, h) == 0.0 and oracle.M4(1.0000001, h) == 0.0


@pytest.mark.parametrize("p", range(0, 23))
def test_gk15_exact_on_polynomials(p):
    """K15 integrates degree <= 22 exactly; its 7-point Gauss part degree <= 13."""
    k, err = oracle.gk15_poly(p, -0.7, 1.3)
    exact = (1.3 ** (p + 1) - (-0.7) ** (p + 1)) / (p + 1)
    assert abs(k - exact) < 1e-14 * max(1.0, abs(exact))
    if p <= 13:
        assert err < 1e-14 * max(1.0, abs(exact))


def test_chord_quadrature_matches_closed_form():
    """Adaptive quadrature of G_t vs the paper's closed form I(h,b,z1,z2)."""
    rng = np.random.default_rng(1)
    for _ in range(300):
        h = float(np.exp(rng.uniform(-1, 6)))
        b = h * float(rng.uniform(0, 0.999))
        l = math.sqrt(h * h - b * b)
        z1, z2 = np.sort(rng.uniform(-l, l, 2))
        q = oracle.chord_quad(h, b, z1, z2)
        c = oracle.chord_closed(h, b, z1, z2)
        assert abs(q - c) <= 1e-12 * abs(oracle.chord_closed(h, 0, -h, h))


def test_full_chord_values():
    """F(q) = (N h^3 sqrt(pi)/t) e^{-t^2 q^2} erf(t sqrt(1-q^2)) / h^2 from the closed form."""
    kc = oracle.kernel_constants()
    t, Nh3 = kc["t"], kc["Nh3"]
    for q in [0.0, 0.25, 0.5, 0.9, 0.999]:
        l = math.sqrt(1 - q * q)
        F = Nh3 * math.sqrt(math.pi) / t * math.exp(-t * t * q * q) * math.erf(t * l)
        assert abs(oracle.chord_quad(1.0, q, -l, l) - F) < 1e-13 * F + 1e-16
    assert abs(oracle.chord_quad(1.0, 0.0, -1.0, 1.0) - 1.8794448) < 1e-7


def test_uniform_medium_column_normalisation():
    """Integrated over the impact plane, one particle's column is its content:
    2 pi int_0^h b F(b) db = 1.  So a ray through a uniform medium sees n L."""
    def F(b):
        l = math.sqrt(max(0.0, 1 - b * b))
        return oracle.chord_quad(1.0, b, -l, l)
    v, _ = integrate.quad(lambda b: 2 * math.pi * b * F(b), 0, 1, epsabs=1e-13, epsrel=1e-13,
                          limit=200)
    assert abs(v - 1.0) < 1e-10


# ---------------------------------------------------------------------------
# columns: geometry of single hits, brute-force predicate, images
# ---------------------------------------------------------------------------
def _one(pos, h, mu=1.0, x=1.0, dirs=((1.0, 0.0, 0.0),), L=10.0, box=0.0):
    """Workload-like object with explicit particles; source is particle 0."""
    pos = np.asarray(pos, np.float32).reshape(-1, 3)
    n = pos.shape[0]
    wl = W.Workload(name="t", pos=pos, h=np.asarray(h, np.float32).reshape(n),
                    mu=np.full(n, mu, np.float32), n_H=np.ones(n, np.float32),
                    T=np.full(n, 1e4, np.float32), dirs=np.asarray(dirs, np.float64),
                    sigma=np.array([W.SIGMA_TH]), w=np.array([1e-12 / W.SIGMA_TH]),
                    l_ray=float(L), box=float(box), tol=1e-3, max_iter=10)
    return wl, np.full(n, x, np.float64)


def _closed_clip(h, b, sp, L):
    l = math.sqrt(h * h - b * b)
    z1, z2 = max(-sp, -l), min(L - sp, l)
    return oracle.chord_closed(h, b, z1, z2) if z2 > z1 else 0.0


@pytest.mark.parametrize("case", [
    # (position of the target relative to the source at the origin, h, L)
    ((5.0, 0.5, 0.0), 1.0, 10.0),      # full chord
    ((0.5, 0.3, 0.0), 1.0, 10.0),      # ray starts inside the kernel
    ((9.8, 0.0, 0.4), 1.0, 10.0),      # ray ends inside the kernel
    ((-0.5, 0.2, 0.1), 1.0, 10.0),     # target behind the origin, origin inside
    ((3.0, 0.0, 0.0), 5.0, 2.0),       # segment entirely inside the kernel
])
def test_single_particle_column_closed_form(case):
    d, h, L = case
    hs = 1.0 / 1024                      # exactly representable in FP32
    wl, x = _one([(0, 0, 0), d], [hs, h], mu=2.5, x=0.4, L=L)
    N = oracle.columns(wl, x, sources=[0])
    sp = d[0]
    b = math.hypot(d[1], d[2])
    # the source itself contributes half its central chord
    self_term = 2.5 * 0.4 * _closed_clip(hs, 0.0, 0.0, L)
    expect = 2.5 * 0.4 * _closed_clip(h, b, sp, L) + self_term
    assert abs(N[0, 0] - expect) < 1e-12 * expect


def test_self_term_is_half_central_chord():
    wl, x = _one([(0, 0, 0)], [2.0], mu=1.0, x=1.0, L=10.0)
    N = oracle.columns(wl, x)
    assert abs(N[0, 0] - 0.5 * oracle.chord_quad(2.0, 0.0, -2.0, 2.0)) < 1e-14
    wl0, _ = _one([(0, 0, 0)], [2.0], L=0.0)
    assert oracle.columns(wl0, x)[0, 0] == 0.0


def _brute_hits_other_way(pos, h, src, u, L):
    """Distance from each point to the segment by minimising over the segment's
    parameter in closed form, in long double, written independently."""
    p = np.asarray(pos, np.longdouble)
    o = p[src]
    uu = np.asarray(u, np.longdouble)
    d = p - o
    tt = np.clip(d @ uu, 0, L)
    dist2 = ((d - tt[:, None] * uu[None, :]) ** 2).sum(1)
    return dist2, np.asarray(h, np.longdouble) ** 2


def test_hit_predicate_against_independent_distance():
    rng = np.random.default_rng(3)
    n = 600
    pos = rng.uniform(0, 20, size=(n, 3)).astype(np.float32)
    h = rng.uniform(0.5, 2.0, size=n).astype(np.float32)
    dirs = W.healpix_dirs(1)
    wl, x = _one(pos, h, dirs=dirs, L=8.0)
    srcs = np.arange(0, n, 50)
    N, off, hj, _ = oracle.columns(wl, x, sources=srcs, hits=True)
    checked = 0
    for i, s in enumerate(srcs):
        for k in range(12):
            got = set(hj[off[i * 12 + k]: off[i * 12 + k + 1]].tolist())
            d2, h2 = _brute_hits_other_way(pos, h, s, dirs[k], 8.0)
            clear = np.abs(d2 - h2) > 1e-9 * h2          # away from exact tangency
            want = set(np.nonzero((d2 < h2) & clear)[0].tolist())
            assert want <= got
            assert not (got - want - set(np.nonzero(~clear)[0].tolist()))
            checked += len(want)
    assert checked > 100


def test_periodic_image_hit():
    """A ray leaving the box meets the periodic image of a particle near the far wall."""
    wl, x = _one([(9.5, 5.0, 5.0), (0.5, 5.0, 5.25)], [1 / 64, 0.5], L=2.0, box=10.0)
    N, off, hj, hi = oracle.columns(wl, x, sources=[0], hits=True)
    pairs = set(zip(hj.tolist(), hi.tolist()))
    code = lambda sx, sy, sz: (sx + 8) | ((sy + 8) << 4) | ((sz + 8) << 8)
    assert (1, code(1, 0, 0)) in pairs and (0, code(0, 0, 0)) in pairs
    expect = _closed_clip(0.5, 0.25, 1.0, 2.0) + _closed_clip(1 / 64, 0.0, 0.0, 2.0)
    assert abs(N[0, 0] - expect) < 1e-12 * expect


def test_image_shift_can_exceed_one_box():
    """When L + h exceeds the box, images two boxes away are reached too."""
    wl, x = _one([(0.2, 5.0, 5.0), (0.1, 5.0, 5.0)], [0.3, 0.3], L=20.05, box=10.0)
    N, off, hj, hi = oracle.columns(wl, x, sources=[0], hits=True)
    code = lambda sx: (sx + 8) | (8 << 4) | (8 << 8)
    assert (1, code(2)) in set(zip(hj.tolist(), hi.tolist()))


def test_permutation_invariance():
    wl = W.make_config(0, n_side_lattice=6, box=37.5)
    x = oracle.x_thin(wl) * np.linspace(1, 3, wl.n)
    perm = np.random.default_rng(2).permutation(wl.n)
    wl2 = W.Workload(**{**wl.__dict__, "pos": wl.pos[perm], "h": wl.h[perm], "mu": wl.mu[perm],
                        "n_H": wl.n_H[perm], "T": wl.T[perm]})
    src = np.arange(0, wl.n, 7)
    N1, o1, j1, i1 = oracle.columns(wl, x, sources=src, hits=True)
    inv = np.argsort(perm)
    N2, o2, j2, i2 = oracle.columns(wl2, x[perm], sources=inv[src], hits=True)
    np.testing.assert_array_equal(o1, o2)
    for r in range(len(o1) - 1):
        a = sorted(zip(j1[o1[r]:o1[r + 1]].tolist(), i1[o1[r]:o1[r + 1]].tolist()))
        b = sorted(zip(perm[j2[o2[r]:o2[r + 1]]].tolist(), i2[o2[r]:o2[r + 1]].tolist()))
        assert a == b
    np.testing.assert_allclose(N1, N2, rtol=1e-13)


def test_galilean_invariance_isolated():
    """Shifting every particle by an exactly representable offset leaves each
    ray's hits and column unchanged (Sec. 3.4.1)."""
    rng = np.random.default_rng(4)
    pos = np.round(rng.uniform(-20, 20, (300, 3)) * 64) / 64      # few mantissa bits
    h = np.round(rng.uniform(1, 4, 300) * 64) / 64
    wl, x = _one(pos, h, dirs=W.healpix_dirs(1), L=15.0)
    wl2, _ = _one(pos + 256.0, h, dirs=W.healpix_dirs(1), L=15.0)
    assert np.all(wl2.pos.astype(np.float64) == pos + 256.0)
    src = np.arange(0, 300, 11)
    a = oracle.columns(wl, x, sources=src, hits=True)
    b = oracle.columns(wl2, x, sources=src, hits=True)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[2], b[2])


def test_uniform_lattice_mean_column():
    """Rays through the uniform periodic lattice see close to n_HI L on average."""
    wl = W.make_config(0)
    x = np.full(wl.n, 1e-3)
    src = np.arange(0, wl.n, 97)
    N = oracle.columns(wl, x, sources=src)
    expect = 1.5e-3 * 1e-3 * 100.0 * W.KPC_CM
    assert abs(N.mean() / expect - 1) < 2e-3


# ---------------------------------------------------------------------------
# Gamma (Sec. 3.3, eq. gamma_shld)
# ---------------------------------------------------------------------------
def test_gamma_thin_exact_when_transparent():
    sig, w = W.power_law_spectrum(64, 1.5, 1e-12)
    N = np.zeros((5, 12))
    lnG, G, tau = oracle.gamma(N, sig, w)
    # exact in real arithmetic; the log-sum-exp over 768 terms rounds a few ulp
    np.testing.assert_allclose(G, np.sum(w * sig), rtol=1e-13)
    assert np.all(np.abs(tau) < 1e-13)


def test_gamma_single_bin_closed_form():
    N = np.array([[1e17, 3e17, 0.0, 5e18], [1e20, 1e21, 2e21, 1e22]])
    s, w = W.SIGMA_TH, 1e-12 / W.SIGMA_TH
    lnG, G, tau = oracle.gamma(N, np.array([s]), np.array([w]))
    for p in range(2):
        m = np.min(s * N[p])
        ref = math.log(w * s) - m + math.log(np.mean(np.exp(-(s * N[p] - m))))
        assert abs(lnG[p] - ref) < 1e-12 * max(1, abs(ref))
    assert abs(tau[1] - (s * 1e20 - math.log(np.mean(np.exp(-s * (N[1] - 1e20)))))) < 1e-9


def test_gamma_matches_direct_sum_where_representable():
    rng = np.random.default_rng(8)
    sig, w = W.power_law_spectrum(32, 1.5, 1e-12)
    N = rng.uniform(0, 3e18, (20, 12))
    lnG, G, _ = oracle.gamma(N, sig, w)
    direct = np.mean((w * sig * np.exp(-sig[None, None, :] * N[:, :, None])).sum(-1), axis=1)
    np.testing.assert_allclose(G, direct, rtol=1e-13)


# ---------------------------------------------------------------------------
# rates and the equilibrium root (Appendix C.3)
# ---------------------------------------------------------------------------
def test_rates_at_1e4K_against_literature():
    # case A 4.18e-13, case B 2.59e-13 (standard tabulations at 10^4 K); the fits
    # reproduce them to a few percent.  Collisional ionisation ~ 6e-16 at 10^4 K.
    assert abs(oracle.alpha_A(1e4)[0] / 4.18e-13 - 1) < 0.04
    assert abs(oracle.alpha_B(1e4)[0] / 2.59e-13 - 1) < 0.02
    assert 5e-16 < oracle.gamma_coll(1e4)[0] < 7.5e-16
    # collisional ionisation rises steeply with temperature, recombination falls
    T = np.array([5e3, 1e4, 3e4, 1e5, 1e6])
    assert np.all(np.diff(oracle.gamma_coll(T)) > 0)
    assert np.all(np.diff(oracle.alpha_A(T)) < 0)


def test_xeq_collisional_limit_and_upper_root():
    a, g = oracle.alpha_A(1e4)[0], oracle.gamma_coll(1e4)[0]
    x = oracle.xeq(0.0, 1e-3, a, g)
    # eq. xphys; Q^2 - 4PR cancels to (R - P)^2 here, leaving ~1e-13 rounding
    assert abs(x - a / (a + g)) < 1e-12
    # x+ = 1 at zero rate: the other root of R x^2 + Q x + P
    R, P = (g + a) * 1e-3, a * 1e-3
    assert abs(P / (R * x) - 1.0) < 1e-13


def test_xeq_thin_limit():
    a, g = oracle.alpha_A(1e4)[0], oracle.gamma_coll(1e4)[0]
    for nH in [1e-6, 1e-5, 1e-4]:
        G = 1e-12
        x = oracle.xeq(G, nH, a, g)
        assert abs(x / (a * nH / G) - 1) < 2e-3     # x ~ alpha n_H / Gamma


def test_xeq_against_high_precision_literal_root():
    """The stable root equals the printed (-Q - sqrt(Q^2-4PR))/(2R) in 60 digits."""
    getcontext().prec = 60
    rng = np.random.default_rng(9)
    for _ in range(200):
        T = float(10 ** rng.uniform(3.5, 6))
        nH = float(10 ** rng.uniform(-7, 2))
        G = float(10 ** rng.uniform(-20, -10)) if rng.uniform() < 0.9 else 0.0
        a, g = oracle.alpha_A(T)[0], oracle.gamma_coll(T)[0]
        x = oracle.xeq(G, nH, a, g)
        Da, Dg, Dn, DG = Decimal(a), Decimal(g), Decimal(nH), Decimal(G)
        R = (Dg + Da) * Dn
        Q = -(DG + Da * Dn + R)
        P = Da * Dn
        D = Q * Q - 4 * P * R
        xl = (-Q - D.sqrt()) / (2 * R)
        # FP64 rounding of Q^2 - 4PR is amplified by |Q|/sqrt(D) (large when both
        # Gamma and gamma_coll are tiny next to alpha n_H)
        cond = abs(Q) / max(D.sqrt(), Decimal(1e-300))
        tol = Decimal(1e-13) + Decimal(4e-16) * cond
        assert abs(Decimal(float(x)) - xl) <= tol * xl


def test_slab_solver_matches_analytic_slab():
    """The slice-by-slice slab solver built on the oracle's root and rates
    reproduces the analytic depth z(x) of Appendix C.4 (eq. analytic_slab_eqn)."""
    nH, T, sig = 1.5e-3, 1e4, W.SIGMA_TH
    G0 = 1e-12
    depth = 200.0 * W.KPC_CM
    # slices thin in optical depth: N_H sigma per slice well below unity
    n_sl = 40000
    z, xs = oracle.slab_numerical(G0, nH, T, sig, depth, n_sl)
    a, g = oracle.alpha_A(T)[0], oracle.gamma_coll(T)[0]
    x_ce = a / (a + g)
    x0 = oracle.xeq(G0, nH, a, g)
    sel = (xs > 2 * x0) & (xs < 0.99 * x_ce)
    assert sel.sum() > 100
    za = oracle.slab_depth_analytic(xs[sel], x0, x_ce, nH, sig)
    # compare depths in units of the slice width
    dz = depth / n_sl
    assert np.max(np.abs(za - z[sel])) < 3 * dz
    assert xs[-1] > 0.99 * x_ce                     # fully neutral far side


# ---------------------------------------------------------------------------
# fixed point (Sec. 3.3, Sec. 4)
# ---------------------------------------------------------------------------
def _small_lattice():
    return W.make_config(0, n_side_lattice=8, box=50.0, max_iter=8)


def test_fixed_point_monotone_case_a():
    """From x_thin, each x_p^(k) is non-decreasing (columns grow with x, Gamma
    falls with columns, the root falls with Gamma) and bounded by x_ce."""
    wl = _small_lattice()
    r = oracle.solve(wl, max_iter=6, tol=0.0)
    xh = r["x_hist"]
    assert np.all(np.diff(xh, axis=0) >= -1e-15 * xh[1:])
    a, g = oracle.alpha_A(1e4)[0], oracle.gamma_coll(1e4)[0]
    assert np.all(xh <= a / (a + g) * (1 + 1e-12))      # Gamma = 0 root rounds ~1e-13


def test_fixed_point_thin_limit_l0():
    """With l_ray = 0 the result is the optically thin state (Appendix A)."""
    wl = _small_lattice()
    wl.l_ray = 0.0
    r = oracle.solve(wl, max_iter=3, tol=1e-30)
    np.testing.assert_allclose(r["x_hist"][-1], oracle.x_thin(wl), rtol=1e-13)
    np.testing.assert_allclose(r["lnG_hist"][-1], math.log(oracle.gamma_thin(wl)), rtol=1e-14)


def test_solve_equals_repeated_steps():
    wl = _small_lattice()
    r = oracle.solve(wl, max_iter=3, tol=0.0)
    x = r["x_hist"][0]
    for k in range(3):
        s = oracle.step(wl, x)
        np.testing.assert_allclose(s["x_new"], r["x_hist"][k + 1], rtol=1e-14)
        x = s["x_new"]


def test_resume_from_state_is_exact():
    wl = _small_lattice()
    full = oracle.solve(wl, max_iter=4, tol=0.0)
    half = oracle.solve(wl, max_iter=2, tol=0.0)
    rest = oracle.solve(wl, max_iter=2, tol=0.0, x_init=half["x_hist"][-1])
    np.testing.assert_array_equal(full["x_hist"][-1], rest["x_hist"][-1])


# ---------------------------------------------------------------------------
# the paper's own update rule (Sec. 4): tau_skip, case B where tau_eff >= 1,
# relative convergence, density-ordered updates
# ---------------------------------------------------------------------------
def _rule_halo():
    return W.isothermal_halo(n=240, seed=61, n_bins=6, n_peak=30.0)


def test_rule_defaults_are_the_order_independent_update():
    wl = _small_lattice()
    a = oracle.solve(wl, max_iter=4, tol=0.0)
    b = oracle.solve_rule(wl, max_iter=4, tol=0.0)
    np.testing.assert_array_equal(a["x_hist"], b["x_hist"])
    np.testing.assert_array_equal(a["lnG_hist"], b["lnG_hist"])
    assert not b["skipped"].any()


@pytest.mark.parametrize("n_blocks", [1, 5, 240])
def test_rule_density_order_against_single_source_steps(n_blocks):
    """Blocked Gauss-Seidel in density-descending order, redone by hand: each
    block's particles take one order-independent step (oracle.step restricted
    to them) from the state that already holds the earlier blocks' updates."""
    wl = _rule_halo()
    r = oracle.solve_rule(wl, n_blocks=n_blocks, max_iter=3, tol=0.0)
    order = sorted(range(wl.n), key=lambda i: (-float(wl.n_H[i]), i))
    size = -(-wl.n // n_blocks)
    x = oracle.x_thin(wl)
    for k in range(3):
        for b0 in range(0, wl.n, size):
            blk = np.array(order[b0:b0 + size])
            x[blk] = oracle.step(wl, x, sources=blk)["x_new"]
        np.testing.assert_allclose(r["x_hist"][k + 1], x, rtol=1e-13)


def test_rule_density_order_converges_to_the_same_fixed_point():
    """Gauss-Seidel needs fewer sweeps here and reaches the fixed point of the
    order-independent update; from x_thin its iterates are monotone too."""
    wl = _rule_halo()
    j = oracle.solve_rule(wl, max_iter=200, tol=1e-9)
    g = oracle.solve_rule(wl, n_blocks=wl.n, max_iter=200, tol=1e-9)
    assert g["iters"] < j["iters"]
    np.testing.assert_allclose(g["x_hist"][-1], j["x_hist"][-1], rtol=1e-6)
    assert np.all(np.diff(g["x_hist"], axis=0) >= -1e-15 * g["x_hist"][1:])


def test_rule_case_b_in_thick_gas_and_case_a_in_thin_gas():
    """Deep in the lattice Gamma underflows, so the converged x is the
    collisional root x_ce = alpha / (alpha + gamma) with case B rates where
    tau_eff >= 1 (eq. xroots at Gamma = 0); optically thin gas is untouched."""
    wl = W.make_config(0, n_side_lattice=8, box=50.0, max_iter=30)
    wl.mu = wl.mu * np.float32(8.0)                  # thicker: tau_eff ~ 1e3
    rb = oracle.solve_rule(wl, tau_case_b=1.0, max_iter=30, tol=1e-12)
    aB, g = oracle.alpha_B(1e4)[0], oracle.gamma_coll(1e4)[0]
    np.testing.assert_allclose(rb["x_hist"][-1], aB / (aB + g), rtol=1e-9)
    ra = oracle.solve_rule(wl, max_iter=30, tol=1e-12)
    aA = oracle.alpha_A(1e4)[0]
    np.testing.assert_allclose(ra["x_hist"][-1], aA / (aA + g), rtol=1e-9)
    thin = W.make_config(0, n_side_lattice=6, box=37.5, max_iter=4)
    thin.mu = thin.mu * np.float32(1e-6)             # tau_eff ~ 1e-6
    t_a = oracle.solve_rule(thin, max_iter=4, tol=0.0)
    t_b = oracle.solve_rule(thin, tau_case_b=1.0, max_iter=4, tol=0.0)
    np.testing.assert_array_equal(t_a["x_hist"], t_b["x_hist"])


def test_rule_tau_skip_freezes_thin_particles():
    """The skipped set is the particles whose first rate (an order-independent
    step from x_thin) gives tau_eff < tau_skip; they keep x_thin exactly."""
    wl = _rule_halo()
    x0 = oracle.x_thin(wl)
    first = oracle.step(wl, x0)
    tau_skip = float(np.median(first["tau"]))
    r = oracle.solve_rule(wl, tau_skip=tau_skip, max_iter=6, tol=0.0)
    np.testing.assert_array_equal(r["skipped"], first["tau"] < tau_skip)
    np.testing.assert_array_equal(r["x_hist"][-1][r["skipped"]], x0[r["skipped"]])
    moved = ~r["skipped"]
    assert np.all(r["x_hist"][-1][moved] > x0[moved])


def test_rule_relative_convergence():
    """The stop test max |dx| / x < tol, recomputed from the iterates."""
    wl = _rule_halo()
    tol = 2e-2
    r = oracle.solve_rule(wl, relative=True, max_iter=100, tol=tol)
    xh = r["x_hist"]
    rel = np.max(np.abs(np.diff(xh, axis=0)) / xh[:-1], axis=1)
    np.testing.assert_allclose(r["maxdx"], rel, rtol=1e-12)
    assert rel[-1] < tol and np.all(rel[:-1] >= tol)


# ---------------------------------------------------------------------------
# non-equilibrium evolution (Appendix C.3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("G,nH,x0", [(1e-12, 1e-3, 1e-5), (1e-13, 1e-1, 0.9), (0.0, 1e-2, 0.3),
                                     (1e-11, 1e-4, 0.5)])
def test_x_evolve_against_numerical_integration(G, nH, x0):
    """The closed form against a high-accuracy integration of eq. dxdt."""
    from scipy.integrate import solve_ivp
    a, g = oracle.alpha_A(1e4)[0], oracle.gamma_coll(1e4)[0]
    trc = 1.0 / ((a + g) * nH)
    ts = np.array([0.0, 0.01, 0.3, 2.0, 10.0]) * trc
    rhs = lambda t, x: [-(G + g * (1 - x[0]) * nH) * x[0] + a * (1 - x[0]) * nH * (1 - x[0])]
    sol = solve_ivp(rhs, (0, ts[-1]), [x0], t_eval=ts, rtol=1e-12, atol=1e-16, method="Radau")
    got = oracle.x_evolve(x0, G, nH, a, g, ts)
    np.testing.assert_allclose(got, sol.y[0], rtol=1e-8, atol=1e-14)


def test_x_evolve_limits():
    a, g = oracle.alpha_A(1e4)[0], oracle.gamma_coll(1e4)[0]
    for G, nH, x0 in [(1e-12, 1e-3, 1e-5), (1e-15, 1.0, 0.2)]:
        assert oracle.x_evolve(x0, G, nH, a, g, 0.0) == pytest.approx(x0, rel=1e-15)
        assert oracle.x_evolve(x0, G, nH, a, g, 1e30) == pytest.approx(
            oracle.xeq(G, nH, a, g), rel=1e-12)


# ---------------------------------------------------------------------------
# near/far scheme (Sec. 4.1.2) and the slab solution of Appendix C.4
# ---------------------------------------------------------------------------
_A, _G = oracle.alpha_A(1e4)[0], oracle.gamma_coll(1e4)[0]


def test_slab_rate_at_the_surface_is_the_incident_rate():
    for lg0 in (-25.0, -27.6, -35.0):
        assert abs(oracle.slab_lnG(lg0, 1e-2, _A, _G, W.SIGMA_TH, 0.0) - lg0) < 1e-14


@pytest.mark.parametrize("N", [1e16, 3e17, 1e18, 4e18])
def test_slab_rate_against_the_slice_by_slice_solver(N):
    """The inverse solution against an independent numerical slab (pinned to
    the analytic depth above): rate at depth = Gamma0 exp(-HI optical depth)."""
    nH, G0 = 1e-2, 1e-12
    _, xs = oracle.slab_numerical(G0, nH, 1e4, W.SIGMA_TH, N / nH, 40000)
    tau = float(np.sum(xs) * W.SIGMA_TH * N / 40000)
    got = oracle.slab_lnG(math.log(G0), nH, _A, _G, W.SIGMA_TH, N)
    assert abs(got - (math.log(G0) - tau)) < 1e-7 * max(1.0, tau)


def test_slab_rate_limits():
    """Highly ionised gas is attenuated by its surface neutral fraction
    (ln Gamma = ln Gamma0 - sigma x0 N to first order); deep in a thick slab each
    extra column adds x_ce of neutral gas, so d ln Gamma / dN -> -sigma x_ce."""
    nH, G0 = 1e-6, 1e-12
    x0 = oracle.xeq(G0, nH, _A, _G)
    N = 1e15                                      # sigma x0 N ~ 4e-5
    got = oracle.slab_lnG(math.log(G0), nH, _A, _G, W.SIGMA_TH, N)
    assert abs((math.log(G0) - got) / (W.SIGMA_TH * x0 * N) - 1) < 1e-3
    N1, N2 = 5e20, 6e20
    l1 = oracle.slab_lnG(math.log(G0), 1e-2, _A, _G, W.SIGMA_TH, N1)
    l2 = oracle.slab_lnG(math.log(G0), 1e-2, _A, _G, W.SIGMA_TH, N2)
    slope = (l2 - l1) / (N2 - N1)
    assert abs(slope / (-W.SIGMA_TH * _A / (_A + _G)) - 1) < 1e-9
    assert l2 < l1 < math.log(G0)


_SLAB_CASES = [(Nf, Nn, nH) for Nf in (0.0, 3e17, 1e19) for Nn in (1e16, 1e18, 1e20, 3e21)
               for nH in (1e-3, 0.3)]


def test_poly_slab_with_one_bin_is_the_analytic_slab():
    """The polychromatic slab (quadrature of 1/x over the HI column, bisection
    for the bottom) with one bin against the closed form of App. C.4, from
    optically thin to 1e4 e-folds deep."""
    a, g = oracle.alpha_A(1e4)[0], oracle.gamma_coll(1e4)[0]
    sig, w = W.grey_spectrum(1e-12)
    for Nf, Nn, nH in _SLAB_CASES:
        lp = oracle.slab_lnG_poly(sig, w, Nf, nH, a, g, Nn)[()]
        la = oracle.slab_lnG(math.log(w[0] * sig[0]) - sig[0] * Nf, nH, a, g, sig[0], Nn)[()]
        assert abs(lp - la) <= 1e-12 * abs(la) + 1e-10, (Nf, Nn, nH, lp, la)


@pytest.mark.parametrize("Nf,Nn,nH", [(0.0, 1e20, 0.3), (3e17, 3e21, 1e-3), (0.0, 3e21, 0.3),
                                      (1e19, 3e21, 0.3), (3e17, 1e18, 0.3)])
def test_poly_slab_against_rk4_in_the_hydrogen_column(Nf, Nn, nH):
    """Eight bins: the same slab as the ODE dy/dt = x_-(Gamma(N_far + y)) in the
    total hydrogen column t, by RK4 at n and 2n steps; the quadrature form
    agrees within twice RK4's own change between them."""
    a, g = oracle.alpha_A(1e4)[0], oracle.gamma_coll(1e4)[0]
    sig, w = W.power_law_spectrum(8, 1.5, 1e-12)
    lp = oracle.slab_lnG_poly(sig, w, Nf, nH, a, g, Nn)[()]
    r1 = oracle.slab_rk4_poly(sig, w, Nf, nH, a, g, Nn, 3000)
    r2 = oracle.slab_rk4_poly(sig, w, Nf, nH, a, g, Nn, 6000)
    assert abs(lp - r2) <= 2.0 * abs(r1 - r2) + 1e-10 * abs(lp), (lp, r1, r2)


def test_poly_slab_limits():
    a, g = oracle.alpha_A(1e4)[0], oracle.gamma_coll(1e4)[0]
    sig, w = W.power_law_spectrum(8, 1.5, 1e-12)
    lnws = np.log(w * sig)
    for Nf in (0.0, 1e18):
        # a slab of zero thickness passes the far-attenuated rate unchanged
        lf = oracle.slab_lnG_poly(sig, w, Nf, 0.1, a, g, 0.0)[()]
        v = lnws - sig * Nf
        assert lf == pytest.approx(v.max() + math.log(np.exp(v - v.max()).sum()), abs=1e-13)
        # thicker slabs let less through; denser gas too (more recombination)
        Ns = [1e17, 1e18, 1e19, 1e20, 1e21]
        ls = [oracle.slab_lnG_poly(sig, w, Nf, 0.1, a, g, Nn)[()] for Nn in Ns]
        assert all(l2 < l1 for l1, l2 in zip(ls, ls[1:]))
        assert oracle.slab_lnG_poly(sig, w, Nf, 1.0, a, g, 1e20)[()] < \
            oracle.slab_lnG_poly(sig, w, Nf, 0.01, a, g, 1e20)[()]


def test_near_far_rate_poly_with_one_bin_equals_mono():
    """The near/far step for one bin through both code paths of the oracle: the
    analytic slab and the polychromatic one."""
    wl = W.make_config(0, n_side_lattice=6, box=37.5)
    rng = np.random.default_rng(6)
    x = np.minimum(oracle.x_thin(wl) * rng.uniform(1, 300, wl.n), 0.99)
    src = np.array([0, 9, 100, 215])
    mono = oracle.step_near_far(wl, x, src)
    wl2 = W.Workload(**{**wl.__dict__, "sigma": np.repeat(wl.sigma, 2), "w": np.repeat(wl.w, 2) / 2})
    poly = oracle.step_near_far(wl2, x, src)
    np.testing.assert_allclose(poly["lnG"], mono["lnG"], rtol=1e-11, atol=1e-11)


def test_near_far_columns_split_the_plain_column():
    """With every x = 1 the far and near columns add up to the plain column;
    each ray from a source hits every near particle, and the near set is the
    particles whose kernel contains the source (brute force, periodic images)."""
    wl = W.make_config(0, n_side_lattice=6, box=37.5)
    src = np.array([0, 7, 100, 215])
    ones = np.ones(wl.n)
    Nf, Nn, cnt = oracle.columns_near_far(wl, ones, src)
    Np = oracle.columns(wl, ones, src)
    np.testing.assert_allclose(Nf + Nn, Np, rtol=1e-12)
    pos = wl.pos.astype(np.float64)
    for i, p in enumerate(src):
        d = pos - pos[p]
        d -= wl.box * np.round(d / wl.box)           # minimum image: h < box / 2 here
        inside = np.sum(np.sum(d * d, axis=1) < wl.h.astype(np.float64) ** 2)
        assert np.all(cnt[i] == inside), (cnt[i], inside)
    assert np.all(Nn > 0) and np.all(Nf > 0)


# ---------------------------------------------------------------------------
# reverse mode
# ---------------------------------------------------------------------------
def test_hit_factors_rebuild_the_columns():
    """Per-hit factors (column per unit neutral fraction) summed with any x give
    the columns at that x: the column is linear in x (eq. colden)."""
    wl = W.make_config(0, n_side_lattice=6, box=37.5)
    rng = np.random.default_rng(3)
    x = rng.uniform(0.01, 1.0, wl.n)
    src = np.array([0, 5, 77, 215])
    N, off, hj, _, hf = oracle.columns(wl, np.ones(wl.n), src, hits=True, factors=True)
    assert np.all(hf > 0)
    np.testing.assert_allclose(np.add.reduceat(hf, off[:-1]).reshape(N.shape), N, rtol=1e-12)
    Nx = oracle.columns(wl, x, src)
    rebuilt = np.add.reduceat(hf * x[hj], off[:-1]).reshape(N.shape)
    np.testing.assert_allclose(rebuilt, Nx, rtol=1e-12)


@pytest.mark.parametrize("G,nH,T", [(1e-12, 1e-3, 1e4), (3e-14, 0.3, 1e4), (1e-12, 2.0, 3e4),
                                    (1e-15, 1e-5, 8e3)])
def test_xeq_partials_against_central_differences(G, nH, T):
    a, g = oracle.alpha_A(T)[0], oracle.gamma_coll(T)[0]
    x = oracle.xeq(G, nH, a, g)[()]
    dG, dn = oracle.xeq_partials(x, G, nH, a, g)
    eG, en = 1e-5 * G, 1e-5 * nH
    fG = (oracle.xeq(G + eG, nH, a, g) - oracle.xeq(G - eG, nH, a, g))[()] / (2 * eG)
    fn = (oracle.xeq(G, nH + en, a, g) - oracle.xeq(G, nH - en, a, g))[()] / (2 * en)
    assert abs(dG / fG - 1) < 1e-7 and abs(dn / fn - 1) < 1e-7


def _adjoint_case():
    wl = W.make_config(0, n_side_lattice=6, box=37.5, max_iter=3)
    wl.sigma, wl.w = W.power_law_spectrum(6, 1.5, 1e-12)
    rng = np.random.default_rng(1)
    wl.n_H = (np.full(wl.n, 5e-3) * rng.uniform(0.5, 2.0, wl.n)).astype(np.float32)
    return wl


def test_adjoint_against_central_differences_of_the_solve():
    """The oracle's reverse mode against central differences of its own K-step
    solve (an independent computation): every bin weight, and densities with
    mu scaled alongside n_H in FP32 (the rounding of mu limits those to ~2e-5).
    A dropped term (x^0's dependence, mu's scaling, the x_- partials, the chain
    through the columns) moves some gradient by more than 5 percent here."""
    wl = _adjoint_case()
    K = 3
    rng = np.random.default_rng(5)
    gl, gx = rng.uniform(-1, 1, wl.n), rng.uniform(-1, 1, wl.n)
    r = oracle.adjoint(wl, K, gl, gx)
    ref = oracle.solve(wl, max_iter=K, tol=0.0)
    np.testing.assert_array_equal(r["x"], ref["x_hist"][-1])

    def loss(w, nH, mu):
        wl2 = W.Workload(**{**wl.__dict__, "w": w, "n_H": nH, "mu": mu})
        f = oracle.solve(wl2, max_iter=K, tol=0.0)
        return np.sum(gl * f["lnG_hist"][-1]) + np.sum(gx * f["x_hist"][-1])

    w0, n0, m0 = wl.w.copy(), wl.n_H.copy(), wl.mu.copy()
    for b in range(wl.n_bins):
        e = 1e-4 * w0[b]
        wp, wm = w0.copy(), w0.copy()
        wp[b] += e
        wm[b] -= e
        fd = (loss(wp, n0, m0) - loss(wm, n0, m0)) / (2 * e)
        assert abs(r["dw"][b] - fd) <= 1e-6 * abs(fd), (b, r["dw"][b], fd)
    scale = np.abs(r["dnH"]).max()
    for j in list(rng.choice(wl.n, 10, replace=False)) + [int(np.argmax(np.abs(r["dnH"])))]:
        up, lo = np.float32(n0[j] * (1 + 1e-3)), np.float32(n0[j] * (1 - 1e-3))
        npl, nmi, mpl, mmi = n0.copy(), n0.copy(), m0.copy(), m0.copy()
        npl[j], nmi[j] = up, lo
        mpl[j] = np.float32(np.float64(m0[j]) * np.float64(up) / np.float64(n0[j]))
        mmi[j] = np.float32(np.float64(m0[j]) * np.float64(lo) / np.float64(n0[j]))
        fd = (loss(w0, npl, mpl) - loss(w0, nmi, mmi)) / (float(up) - float(lo))
        assert abs(r["dnH"][j] - fd) <= 2e-4 * abs(fd) + 1e-6 * scale, (j, r["dnH"][j], fd)


def test_adjoint_is_linear_in_the_output_derivatives():
    wl = _adjoint_case()
    rng = np.random.default_rng(9)
    a, b = rng.uniform(-1, 1, wl.n), rng.uniform(-1, 1, wl.n)
    ra, rb = oracle.adjoint(wl, 2, a, None), oracle.adjoint(wl, 2, None, b)
    rab = oracle.adjoint(wl, 2, a, b)
    np.testing.assert_allclose(rab["dw"], ra["dw"] + rb["dw"], rtol=1e-12)
    np.testing.assert_allclose(rab["dnH"], ra["dnH"] + rb["dnH"], rtol=1e-10,
                               atol=1e-13 * np.abs(rab["dnH"]).max())
    z = oracle.adjoint(wl, 2, None, None)
    assert not np.any(z["dw"]) and not np.any(z["dnH"])


# ---------------------------------------------------------------------------
# reference tree
# ---------------------------------------------------------------------------
def _tree_case(n, seed=0, dup=False):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-30, 30, (n, 3)).astype(np.float32)
    if dup:
        pos[n // 2:] = pos[: n - n // 2]
    h = rng.uniform(0.5, 3, n).astype(np.float32)
    return pos, h


def test_morton_definition():
    pos = np.array([[0, 0, 0], [1, 1, 1], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float32)
    c = oracle.morton(pos)
    top = 2097151
    def spread(v):
        return sum(((v >> i) & 1) << (3 * i) for i in range(21))
    assert c[0] == 0
    assert c[1] == (spread(top) << 2) | (spread(top) << 1) | spread(top)
    assert c[2] == spread(top) << 2 and c[3] == spread(top) << 1 and c[4] == spread(top)


@pytest.mark.parametrize("n,leaf,dup", [(1, 4, False), (2, 1, False), (7, 4, False),
                                        (1000, 1, False), (1000, 4, False), (777, 8, True)])
def test_reference_tree_structure(n, leaf, dup):
    pos, h = _tree_case(n, dup=dup)
    t = oracle.lbvh(pos, h, leaf)
    perm = t["perm"]
    assert sorted(perm.tolist()) == list(range(n))
    codes = t["codes"]
    assert np.all(codes[:-1] <= codes[1:])
    m = t["n_nodes"]
    sp, sh = pos[perm], h[perm]
    leaves = []
    for i in range(m):
        f, c, s = t["first"][i], t["count"][i], t["skip"][i]
        assert i < s <= m
        if c > 0:                                    # leaf: its range, nothing below
            assert c <= leaf and s == i + 1
            leaves.append((f, c))
            lo = (sp[f:f + c] - sh[f:f + c, None]).min(0)
            hi = (sp[f:f + c] + sh[f:f + c, None]).max(0)
            np.testing.assert_array_equal(t["lo"][i], lo)
            np.testing.assert_array_equal(t["hi"][i], hi)
        else:                                        # internal: two children tile it
            l, r = i + 1, t["skip"][i + 1]
            assert t["skip"][r] == s
            np.testing.assert_array_equal(t["lo"][i], np.minimum(t["lo"][l], t["lo"][r]))
            np.testing.assert_array_equal(t["hi"][i], np.maximum(t["hi"][l], t["hi"][r]))
    # leaves partition the sorted order in sequence
    assert [f for f, _ in leaves] == list(np.cumsum([0] + [c for _, c in leaves])[:-1])
    assert sum(c for _, c in leaves) == n


def test_reference_tree_query_finds_brute_force_hits():
    """Walking the tree with its skip links and boxes reaches every particle the
    brute-force predicate hits."""
    pos, h = _tree_case(500, seed=3)
    t = oracle.lbvh(pos, h, 4)
    dirs = W.healpix_dirs(1)
    wl, x = _one(pos, h, dirs=dirs, L=12.0)
    src = np.arange(0, 500, 25)
    _, off, hj, _ = oracle.columns(wl, x, sources=src, hits=True)
    inv = np.empty(500, np.int64)
    inv[t["perm"]] = np.arange(500)
    for i, s in enumerate(src):
        for k in range(12):
            o = pos[s].astype(np.float64)
            e = o + 12.0 * dirs[k]
            reached = set()
            node = 0
            while node < t["n_nodes"]:
                lo, hi = t["lo"][node], t["hi"][node]
                # segment-box overlap by clipping the parameter interval
                t0, t1 = 0.0, 1.0
                ok = True
                for a in range(3):
                    dd = e[a] - o[a]
                    if abs(dd) < 1e-300:
                        ok = ok and lo[a] <= o[a] <= hi[a]
                    else:
                        u0, u1 = (lo[a] - o[a]) / dd, (hi[a] - o[a]) / dd
                        t0, t1 = max(t0, min(u0, u1)), min(t1, max(u0, u1))
                ok = ok and t0 <= t1
                if ok and t["count"][node] > 0:
                    f = t["first"][node]
                    reached.update(range(f, f + t["count"][node]))
                node = node + 1 if (ok and t["count"][node] == 0) else t["skip"][node]
            want = set(inv[hj[off[i * 12 + k]: off[i * 12 + k + 1]]].tolist())
            assert want <= reached


def _halo_case(sizes, seed=0):
    """Halos of the given sizes at different places, overlapping in space."""
    rng = np.random.default_rng(seed)
    pos, h = [], []
    for g, m in enumerate(sizes):
        c = rng.uniform(-20, 20, 3)
        pos.append(c + rng.normal(0, 4 + g, (m, 3)))
        h.append(rng.uniform(0.3, 2.5, m))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return np.concatenate(pos).astype(np.float32), np.concatenate(h).astype(np.float32), off


def test_halo_keys_definition():
    """With H halos the key is the halo index above a Morton code of
    floor((63 - ceil(log2 H)) / 3) bits per axis over the common scene cube."""
    pos = np.array([[0, 0, 0], [1, 1, 1], [1, 0, 0], [0, 0, 1], [0.5, 0.25, 0.75]], np.float32)
    for H, bits in [(2, 20), (3, 20), (4, 20), (5, 20), (8, 20), (9, 19), (64, 19), (65, 18),
                    (513, 17)]:
        # the last particles one per halo; halos past the fifth are empty
        off = np.array([0] + list(range(max(1, 6 - H), 5)) + [5] * max(1, H - 4), np.int64)
        assert off.size == H + 1
        c = oracle.morton(pos, halo_offsets=off)
        top = (1 << bits) - 1

        def spread(v):
            return sum(((v >> i) & 1) << (3 * i) for i in range(bits))

        q = np.minimum(np.floor(pos.astype(np.float64) * (1 << bits)), top).astype(np.int64)
        for j in range(5):
            g = int(np.searchsorted(off, j, side="right") - 1)
            want = (g << (3 * bits)) | (spread(int(q[j, 0])) << 2) | \
                (spread(int(q[j, 1])) << 1) | spread(int(q[j, 2]))
            assert int(c[j]) == want, (H, j)
    # one halo: the plain 21-bit code
    np.testing.assert_array_equal(oracle.morton(pos, halo_offsets=[0, 5]), oracle.morton(pos))


def test_halo_tree_with_one_halo_is_the_plain_tree():
    pos, h = _tree_case(1000, seed=7)
    a = oracle.lbvh(pos, h, 4)
    b = oracle.lbvh(pos, h, 4, halo_offsets=[0, 1000])
    for k in ("perm", "codes", "lo", "hi", "skip", "first", "count"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("sizes,leaf", [((300, 1, 2, 57, 640), 8), ((5, 5, 5, 5), 4),
                                        ((1, 1), 8), ((2000, 33), 1)])
def test_halo_tree_structure(sizes, leaf):
    """Every halo's particles are one contiguous run of the sorted order, and
    one subtree [seg_root, seg_end) holds exactly them; no leaf mixes halos;
    boxes, skip links and leaf ranges as in the plain tree."""
    pos, h, off = _halo_case(sizes)
    t = oracle.lbvh(pos, h, leaf, halo_offsets=off)
    n, m = pos.shape[0], t["n_nodes"]
    perm = t["perm"]
    assert sorted(perm.tolist()) == list(range(n))
    halo = np.searchsorted(off, np.arange(n), side="right") - 1     # input index -> halo
    hs = halo[perm]
    np.testing.assert_array_equal(hs, np.sort(hs))                  # contiguous runs
    np.testing.assert_array_equal(np.searchsorted(hs, np.arange(len(sizes))), off[:-1])
    sp, sh = pos[perm], h[perm]
    covered = np.zeros(n, bool)
    for i in range(m):
        f, c, s = t["first"][i], t["count"][i], t["skip"][i]
        assert i < s <= m
        if c > 0:
            assert c <= leaf and s == i + 1
            assert np.all(hs[f:f + c] == hs[f]), "a leaf mixes halos"
            assert not covered[f:f + c].any()
            covered[f:f + c] = True
            np.testing.assert_array_equal(t["lo"][i], (sp[f:f + c] - sh[f:f + c, None]).min(0))
            np.testing.assert_array_equal(t["hi"][i], (sp[f:f + c] + sh[f:f + c, None]).max(0))
        else:
            l, r = i + 1, t["skip"][i + 1]
            assert t["skip"][r] == s
    assert covered.all()
    for g in range(len(sizes)):
        a, b = t["seg_root"][g], t["seg_end"][g]
        assert 0 <= a < b <= m and t["skip"][a] == b
        got = []
        for i in range(a, b):
            if t["count"][i] > 0:
                got.extend(range(t["first"][i], t["first"][i] + t["count"][i]))
        assert got == list(range(off[g], off[g + 1])), f"halo {g} subtree"
        # the root is the topmost such node: its parent's range is wider
        if a > 0:
            parents = [i for i in range(a) if t["count"][i] == 0 and i < a < t["skip"][i]]
            p = max(parents)
            assert t["skip"][p] - p > b - a


def test_halo_tree_query_finds_each_halos_brute_force_hits():
    """Walking halo g's subtree reaches every particle of halo g that the
    brute-force predicate hits on a ray from a particle of halo g."""
    sizes = (120, 7, 260)
    pos, h, off = _halo_case(sizes, seed=5)
    t = oracle.lbvh(pos, h, 4, halo_offsets=off)
    dirs = W.healpix_dirs(1)
    inv = np.empty(pos.shape[0], np.int64)
    inv[t["perm"]] = np.arange(pos.shape[0])
    for g in range(len(sizes)):
        a, b = int(off[g]), int(off[g + 1])
        wl, x = _one(pos[a:b], h[a:b], dirs=dirs, L=9.0)
        src = np.arange(0, b - a, max(1, (b - a) // 6))
        _, o, hj, _ = oracle.columns(wl, x, sources=src, hits=True)
        for i, s in enumerate(src):
            for k in range(12):
                org = pos[a + s].astype(np.float64)
                e = org + 9.0 * dirs[k]
                reached, node = set(), int(t["seg_root"][g])
                while node < t["seg_end"][g]:
                    lo, hi = t["lo"][node], t["hi"][node]
                    t0, t1, ok = 0.0, 1.0, True
                    for ax in range(3):
                        dd = e[ax] - org[ax]
                        if abs(dd) < 1e-300:
                            ok = ok and lo[ax] <= org[ax] <= hi[ax]
                        else:
                            u0, u1 = (lo[ax] - org[ax]) / dd, (hi[ax] - org[ax]) / dd
                            t0, t1 = max(t0, min(u0, u1)), min(t1, max(u0, u1))
                    ok = ok and t0 <= t1
                    if ok and t["count"][node] > 0:
                        f = t["first"][node]
                        reached.update(range(f, f + t["count"][node]))
                    node = node + 1 if (ok and t["count"][node] == 0) else t["skip"][node]
                want = set(inv[a + hj[o[i * 12 + k]: o[i * 12 + k + 1]]].tolist())
                assert want <= reached


# ---------------------------------------------------------------------------
# plane-slab reference profile (the reference of the slab tests, Sec. 5.1)
# ---------------------------------------------------------------------------
def test_plane_slab_profile_one_bin_is_the_analytic_slab():
    """For one bin the profile's x(z) is Appendix C.4's analytic slab: the
    analytic depth of each profile x equals its z; the surface takes the thin
    rate's root and the far side is neutral."""
    nH, T = 1.5e-3, 1e4
    sig, w = W.grey_spectrum(1e-12)
    depth = 200.0
    z, x, NHI = oracle.plane_slab_profile(sig, w, nH, T, depth, n_points=600)
    a, g = oracle.alpha_A(np.array([T]))[0], oracle.gamma_coll(np.array([T]))[0]
    x_ce = a / (a + g)
    x0 = oracle.xeq(1e-12, nH, a, g)
    assert abs(x[0] - x0) <= 1e-12 * x0
    sel = (x > 2 * x0) & (x < 0.99 * x_ce)
    assert sel.sum() > 20
    za = oracle.slab_depth_analytic(x[sel], x0, x_ce, nH, sig[0]) / oracle.KPC_CM
    assert np.max(np.abs(za - z[sel])) < 1e-6 * depth
    assert x[-1] > 0.99 * x_ce
    # the HI column is the integral of x over the hydrogen column
    assert np.all(np.diff(NHI) > 0)
    t = z * nH * oracle.KPC_CM
    assert abs(NHI[-1] - np.trapezoid(x, t)) <= 1e-12 * NHI[-1]


def test_plane_slab_profile_power_law_is_monotone_and_harder():
    """Eight power-law bins: x rises monotonically with depth from the thin
    rate's root, and the front lies deeper than for one bin at 13.6 eV with the
    same thin rate (harder photons penetrate further)."""
    nH, T, depth = 1.5e-3, 1e4, 200.0
    sig, w = W.power_law_spectrum(8, 1.5, 1e-12)
    z, x, _ = oracle.plane_slab_profile(sig, w, nH, T, depth, n_points=400)
    a, g = oracle.alpha_A(np.array([T]))[0], oracle.gamma_coll(np.array([T]))[0]
    assert abs(x[0] - oracle.xeq(1e-12, nH, a, g)) <= 1e-12 * x[0]
    assert np.all(np.diff(x) > 0)
    sg, wg = W.grey_spectrum(1e-12)
    zg, xg, _ = oracle.plane_slab_profile(sg, wg, nH, T, depth, n_points=400)
    half = 0.5 * a / (a + g)
    assert np.interp(half, x, z) > np.interp(half, xg, zg) + 20.0


# ---------------------------------------------------------------------------
# spherical reference (the halo test, Sec. 5.4)
# ---------------------------------------------------------------------------
def test_sphere_columns_uniform_sphere_chords():
    """Columns through a uniform sphere with x = 1 are n_H times the chord from
    the start point to the surface, -r mu + sqrt(R^2 - r^2 (1 - mu^2)), capped by
    the ray length (midpoint rule: within one step of the edge)."""
    R, L, nH, n_s = 50.0, 80.0, 2e-3, 4000
    r = np.array([0.0, 10.0, 30.0, 49.0])
    mu = np.array([-1.0, -0.6, -0.1, 0.0, 0.4, 1.0])
    N = oracle.sphere_columns(r, mu, lambda q: np.full_like(q, nH), lambda q: np.ones_like(q),
                              R, L, n_s)
    chord = -r[:, None] * mu[None, :] + np.sqrt(R ** 2 - r[:, None] ** 2 * (1 - mu[None, :] ** 2))
    want = nH * np.minimum(chord, L) * oracle.KPC_CM
    assert np.all(np.abs(N - want) <= nH * (L / n_s) * oracle.KPC_CM * 1.0001)


def test_spherical_profile_thin_limit_and_neutral_core():
    """A near-empty sphere takes the thin rate's root at every radius; the
    workload's halo is neutral in its core, ionised at its edge, and x falls
    monotonically with radius."""
    sig, w = W.power_law_spectrum(8, 1.5, 1e-12)
    T = 1e4
    a, g = oracle.alpha_A(np.array([T]))[0], oracle.gamma_coll(np.array([T]))[0]
    r, x, _ = oracle.spherical_profile(1e-9, 1.0, 150.0, T, sig, w, 100.0, n_sh=24, n_mu=8,
                                       n_s=200)
    nH = 1e-9 / (1 + r ** 2)
    want = oracle.xeq(np.full_like(r, 1e-12), nH, np.full_like(r, a), np.full_like(r, g))
    assert np.max(np.abs(x - want) / want) < 1e-8
    r, x, its = oracle.spherical_profile(1.0, 1.0, 150.0, T, sig, w, 100.0, n_sh=60, n_mu=16,
                                         n_s=600)
    assert its < 1000
    assert x[0] > 0.99 * a / (a + g) and x[-1] < 1e-3
    assert np.all(np.diff(x) <= 1e-12)


def test_two_sided_slab_profile_thick_faces_are_one_sided_at_half_intensity():
    """A slab lit on both faces and thick enough that neither face's radiation
    crosses it: near each face the profile is the one-sided analytic slab
    (App. C.4) lit by half the spectrum, and it is symmetric about the midplane."""
    sig, w = W.grey_spectrum(1e-12)
    D = 400.0
    z, x, below, above, its = oracle.two_sided_slab_profile(sig, w, 1.5e-3, 1e4, D,
                                                            n_points=8000)
    assert its < 10000
    assert np.max(np.abs(x - x[::-1]) / x) < 1e-8
    assert np.allclose(below + above, below[-1], rtol=1e-12)
    zs, xs, _ = oracle.plane_slab_profile(sig, 0.5 * w, 1.5e-3, 1e4, 150.0, n_points=300)
    for xf in (np.interp(D - zs, z, x), np.interp(zs, z, x)):
        assert np.max(np.abs(np.log10(xf) - np.log10(xs))) < 0.01


def _near_far_lnG(n_ray, N_far, N_near, nH=1.5e-3, T=1e4, bins=1, share=1):
    a, g = oracle.alpha_A(np.array([T]))[0], oracle.gamma_coll(np.array([T]))[0]
    Nf = np.ascontiguousarray(N_far, np.float64)
    Nn = np.ascontiguousarray(N_near, np.float64)
    one = lambda v: np.array([v], np.float64)
    out = np.zeros(1)
    if bins == 1:
        sig, w = W.grey_spectrum(1e-12)
        oracle.lib().orc_gamma_near_far(1, n_ray, oracle._p(Nf), oracle._p(Nn), float(w[0]),
                                        float(sig[0]), oracle._p(one(nH)), oracle._p(one(a)),
                                        oracle._p(one(g)), oracle._p(out), share)
    else:
        sig, w = W.power_law_spectrum(bins, 1.5, 1e-12)
        oracle.lib().orc_gamma_near_far_poly(1, n_ray, oracle._p(Nf), oracle._p(Nn), bins,
                                             oracle._p(sig), oracle._p(w), oracle._p(one(nH)),
                                             oracle._p(one(a)), oracle._p(one(g)),
                                             oracle._p(out), 1, share)
    return out[0], sig, w, a, g


@pytest.mark.parametrize("bins", [1, 8])
def test_near_far_rays_light_their_slabs_with_their_share(bins):
    """eq. gammashld sums 4 pi / N_ray times each ray's slab rate: with 4 pi
    inside w, each near slab is lit by 1/N_ray of the far-attenuated spectrum
    and the rays' bottom rates add up.  So: the thin limit returns Gamma_thin
    exactly; a ray that is blocked contributes nothing, and the other ray's
    slab is the one-sided slab lit by half the spectrum (the error the paper
    reads off its two-sided slab vanishes once one ray meets a high optical
    depth, Sec. 5.3)."""
    N = 3e20
    thin, *_ = _near_far_lnG(4, [0.0] * 4, [0.0] * 4, bins=bins)
    assert abs(thin - math.log(1e-12)) < 1e-12
    two, sig, w, a, g = _near_far_lnG(2, [0.0, 1e30], [N, N], bins=bins)
    if bins == 1:
        want = oracle.slab_lnG(math.log(0.5 * w[0] * sig[0]), 1.5e-3, a, g, sig[0], N)
    else:
        want = oracle.slab_lnG_poly(sig, 0.5 * w, 0.0, 1.5e-3, a, g, N)
    assert abs(two - float(want)) < 1e-9


@pytest.mark.parametrize("bins", [1, 8])
def test_near_far_variant_lights_each_slab_with_the_whole_spectrum(bins):
    """The variant weighting lights every ray's near slab with the whole
    far-attenuated spectrum and averages the rays: when every ray sees the same
    columns (light from all directions alike) it is the one-sided slab lit by
    the whole spectrum, where the paper's weighting gives N_ray slabs lit by
    1/N_ray each; the thin limit is Gamma_thin in both."""
    N = 3e20
    thin, *_ = _near_far_lnG(4, [0.0] * 4, [0.0] * 4, bins=bins, share=0)
    assert abs(thin - math.log(1e-12)) < 1e-12
    iso, sig, w, a, g = _near_far_lnG(4, [1e17] * 4, [N] * 4, bins=bins, share=0)
    paper, *_ = _near_far_lnG(4, [1e17] * 4, [N] * 4, bins=bins, share=1)
    if bins == 1:
        want = oracle.slab_lnG(math.log(w[0] * sig[0]) - sig[0] * 1e17, 1.5e-3, a, g, sig[0], N)
        quarter = oracle.slab_lnG(math.log(0.25 * w[0] * sig[0]) - sig[0] * 1e17, 1.5e-3, a, g,
                                  sig[0], N)
    else:
        want = oracle.slab_lnG_poly(sig, w, 1e17, 1.5e-3, a, g, N)
        quarter = oracle.slab_lnG_poly(sig, 0.25 * w, 1e17, 1.5e-3, a, g, N)
    assert abs(iso - float(want)) < 1e-9
    assert abs(paper - (float(quarter) + math.log(4.0))) < 1e-9
    assert paper < iso
