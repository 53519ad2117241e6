"""Host checks of the seeded input generators (no GPU, no oracle arithmetic)."""
import math

import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("ns", [1, 2, 3])
def test_healpix_count_norm_and_balance(ns):
    d = W.healpix_dirs(ns)
    assert d.shape == (12 * ns * ns, 3)                      # N_pix = 12 N_side^2
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(d.sum(0), 0.0, atol=1e-13)    # pixel centres balance


@pytest.mark.parametrize("ns", [1, 2, 4])
def test_healpix_ring_heights(ns):
    """Cap rings at z = 1 - i^2/(3 ns^2), belt rings at z = 4/3 - 2i/(3 ns)."""
    d = W.healpix_dirs(ns)
    z = np.unique(np.round(d[:, 2], 12))[::-1]
    expect = []
    for i in range(1, 4 * ns):
        if i < ns:
            expect.append(1 - i * i / (3 * ns * ns))
        elif i <= 3 * ns:
            expect.append(4 / 3 - 2 * i / (3 * ns))
        else:
            ii = 4 * ns - i
            expect.append(-(1 - ii * ii / (3 * ns * ns)))
    np.testing.assert_allclose(z, np.round(expect, 12), atol=1e-12)
    # equal-area pixels: each ring's pixel count times (4 pi / N_pix) equals the ring's
    # band area, so the counts sum to N_pix
    counts = [np.sum(np.isclose(d[:, 2], e, atol=1e-12)) for e in expect]
    assert sum(counts) == 12 * ns * ns


def test_healpix_nside1_vectors():
    d = W.healpix_dirs(1)
    s = math.sqrt(5.0 / 9.0) / math.sqrt(2.0)
    np.testing.assert_allclose(d[0], [s, s, 2 / 3], atol=1e-15)
    np.testing.assert_allclose(d[4], [0, 1, 0], atol=1e-15)
    np.testing.assert_allclose(d[7], [1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(d[11], [s, -s, -2 / 3], atol=1e-15)
    # symmetric under z -> -z
    np.testing.assert_allclose(np.sort(d[:, 2]), np.sort(-d[:, 2]), atol=1e-15)


def test_sigma_th_value():
    # hydrogenic threshold cross-section, 6.30e-18 cm^2 (Appendix C.1)
    assert abs(W.SIGMA_TH - 6.304e-18) / 6.304e-18 < 1e-3


def test_power_law_spectrum():
    sig, w = W.power_law_spectrum(128, 1.5, 1e-12)
    assert sig.shape == w.shape == (128,)
    assert abs(np.sum(sig * w) - 1e-12) < 1e-24
    e = 4.0 ** (np.arange(129) / 128)
    nu = np.sqrt(e[:-1] * e[1:])
    np.testing.assert_allclose(sig, W.SIGMA_TH * nu ** -3, rtol=1e-14)
    # w_b ~ J_b dnu_b / nu_b with J ~ nu^-1.5
    r = w / (nu ** -1.5 * np.diff(e) / nu)
    np.testing.assert_allclose(r / r[0], 1.0, rtol=1e-12)
    assert np.all(np.diff(sig) < 0)


def test_uniform_lattice_recipe():
    a = W.make_config(0)
    b = W.make_config(0)
    assert a.n == 4096 and a.n_ray == 12 and a.n_bins == 1
    np.testing.assert_array_equal(a.pos, b.pos)              # seeded
    assert a.pos.dtype == np.float32 and a.h.dtype == np.float32
    assert np.all(a.pos >= 0) and np.all(a.pos < 100.0)
    assert 13.0 < a.h.min() and a.h.max() < 15.5
    # sum of hydrogen = n_H V_box  (mu in atoms per kpc_cm^2)
    tot = a.mu.astype(np.float64).sum() * W.KPC_CM ** 2
    assert abs(tot / (1.5e-3 * 1e6 * W.KPC_CM ** 3) - 1) < 1e-6
    assert abs(a.w[0] * a.sigma[0] - 1e-12) < 1e-27


def _minimage_dist(p, q, box):
    d = np.abs(p - q)
    if box > 0:
        d = np.minimum(d, box - d)
    return np.sqrt((d * d).sum(-1))


@pytest.mark.parametrize("box", [0.0, 50.0])
def test_smoothing_length_rule(box):
    """Exactly 48 other particles lie within h, none on the boundary."""
    rng = np.random.default_rng(5)
    pos = rng.uniform(0, 50.0, size=(700, 3))
    h = W.smoothing_lengths(pos, box=box)
    for i in range(0, 700, 37):
        d = _minimage_dist(pos, pos[i], box)
        d[i] = np.inf
        assert np.sum(d < h[i]) == 48
        assert np.min(np.abs(d - h[i])) > 0


def test_halo_recipe_small():
    wl = W.isothermal_halo(n=4096, seed=7)
    r = np.linalg.norm(wl.pos.astype(np.float64), axis=1)
    assert r.max() <= 150.0 + 1e-4
    # cored r^-2 profile: median radius of the mass distribution
    x = np.median(r)
    assert 60 < x < 90                                      # (x - atan x) has median ~74
    np.testing.assert_allclose(wl.n_H, 1.0 / (1.0 + r ** 2), rtol=1e-5)
    assert wl.n_bins == 128 and wl.box == 0.0


def test_lognormal_recipe_small():
    wl = W.lognormal_field(n_grid=16, box=1000.0, n_side=1, n_bins=8)
    assert wl.n == 16 ** 3
    assert np.all(wl.pos >= 0) and np.all(wl.pos < 1000.0)
    rho = wl.n_H / 1e-5
    np.testing.assert_allclose(wl.T, 1e4 * rho ** 0.6, rtol=1e-5)


def test_halo_batch_offsets():
    wl = W.halo_batch(n_halo=3, n_lo=512, n_hi=2048, n_bins=4)
    off = wl.halo_offsets
    assert off[0] == 0 and off[-1] == wl.n and np.all(np.diff(off) >= 512)
    sub = wl.subset_halo(1)
    assert sub.n == off[2] - off[1]


def test_field_shard_holds_everything_owned_rays_can_reach():
    """Blocks of a periodic field: owned particles partition the field; every
    particle within l_ray + h_j (periodic distance) of an owned source is in
    that source's shard."""
    wl = W.lognormal_field(n_grid=16, box=1250.0, n_bins=4)
    owned_total = 0
    rng = np.random.default_rng(2)
    for r in range(8):
        sh = W.field_shard(wl, r, 8)
        idx, n_own = sh.meta["index"], sh.meta["n_owned"]
        assert len(np.unique(idx)) == len(idx)
        owned_total += n_own
        inside = set(idx.tolist())
        p = wl.pos.astype(np.float64)
        for s in rng.choice(idx[:n_own], 20, replace=False):
            d = p - p[s]
            d -= wl.box * np.round(d / wl.box)
            reach = np.sqrt((d * d).sum(1)) <= wl.l_ray + wl.h.astype(np.float64)
            assert set(np.nonzero(reach)[0].tolist()) <= inside
    assert owned_total == wl.n


def test_one_sided_slab_recipe():
    """The slab of the physics checks: a jittered lattice filling 0..depth in z
    with the stated spacing and density, one ray to the lit face (two for
    faces = 2), rays long enough to cross the slab, and the stated thin rate."""
    wl = W.one_sided_slab(n_xy=6, n_z=8, depth=50.0)
    a = wl.meta["spacing"]
    assert wl.n == 6 * 6 * 8 and a == 50.0 / 8
    assert wl.pos[:, 2].min() > 0 and wl.pos[:, 2].max() < 50.0
    assert np.all(np.abs(wl.pos / a - np.round(wl.pos / a - 0.5) - 0.5) <= 0.1 + 1e-5)
    np.testing.assert_allclose(wl.mu, 1.5e-3 * a ** 3 * W.KPC_CM, rtol=1e-6)
    np.testing.assert_array_equal(wl.dirs, [[0.0, 0.0, 1.0]])
    assert wl.l_ray >= 50.0 and wl.box == 0.0
    assert abs(np.sum(wl.w * wl.sigma) - 1e-12) < 1e-24
    two = W.one_sided_slab(n_xy=6, n_z=8, depth=50.0, faces=2, n_bins=8)
    np.testing.assert_array_equal(two.dirs, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    assert two.n_bins == 8 and abs(np.sum(two.w * two.sigma) - 1e-12) < 1e-24
