"""Seeded synthetic inputs for the reverse-ray-tracing hot path.

This module only *generates inputs*: particle positions, smoothing lengths,
hydrogen contents, densities, temperatures, HEALPix ray directions and the
binned UV-background spectrum.  It holds none of the method's arithmetic (no
kernel integrals, columns, photoionisation rates or equilibrium roots); both
the FP64 oracle and the HIP library consume exactly the arrays built here.

Units
-----
* positions and smoothing lengths: kpc (FP32)
* ``mu``: hydrogen atoms in the particle divided by (1 kpc in cm)^2, so that
  ``mu * x * (line integral of the kernel in kpc^-2)`` is a column in cm^-2
  (FP32; raw atom counts ~1e64 would overflow FP32)
* ``n_H``: cm^-3, ``T``: K
* ``dirs``: FP64 unit vectors [n_ray, 3]
* ``sigma``: cm^2 per frequency bin, ``w``: bin weight 4*pi*J*dnu/(h*nu) in
  photons cm^-2 s^-1, so that sum(w*sigma) is the optically thin rate in s^-1.

The recipes follow the paper's workloads in shape: a uniform periodic medium
(Section 5 slabs use n_H = 1.5e-3 cm^-3, T = 1e4 K), roughly r^-2 gaseous halos
(Section 5.4, Test 4) and a cosmological field, lit by a power-law background
between 1 and 4 Rydberg (Section 4 defaults; Appendix C.2 power laws).  The
OWLS halo stacks and the HM01 spectrum the paper uses are not available, so
these seeded synthetic inputs stand in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

KPC_CM = 3.0856775814913673e21          # 1 kpc in cm
# Hydrogen threshold cross-section sigma_th = 2^9 pi / (3 e^4) * alpha_fs * pi a0^2
# (Appendix C.1); evaluated from CODATA alpha_fs and a0.
ALPHA_FS = 7.2973525693e-3
BOHR_CM = 5.29177210903e-9
SIGMA_TH = (2.0 ** 9 * math.pi / (3.0 * math.e ** 4)) * ALPHA_FS * math.pi * BOHR_CM ** 2

BASE_SEED = 13044235


@dataclasses.dataclass
class Workload:
    name: str
    pos: np.ndarray          # float32 [n, 3]
    h: np.ndarray            # float32 [n]
    mu: np.ndarray           # float32 [n]
    n_H: np.ndarray          # float32 [n]
    T: np.ndarray            # float32 [n]
    dirs: np.ndarray         # float64 [n_ray, 3]
    sigma: np.ndarray        # float64 [n_bins]
    w: np.ndarray            # float64 [n_bins]
    l_ray: float             # kpc
    box: float               # kpc, 0 = isolated
    tol: float               # max |dx| stopping tolerance
    max_iter: int
    halo_offsets: Optional[np.ndarray] = None   # int64 [n_halo + 1] for batches
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_ray(self) -> int:
        return int(self.dirs.shape[0])

    @property
    def n_bins(self) -> int:
        return int(self.sigma.shape[0])

    def subset_halo(self, i: int) -> "Workload":
        """One halo of a batched workload as a stand-alone workload."""
        a, b = int(self.halo_offsets[i]), int(self.halo_offsets[i + 1])
        return dataclasses.replace(
            self, name=f"{self.name}[{i}]", pos=self.pos[a:b].copy(), h=self.h[a:b].copy(),
            mu=self.mu[a:b].copy(), n_H=self.n_H[a:b].copy(), T=self.T[a:b].copy(),
            halo_offsets=None, meta=dict(self.meta))


# ----------------------------------------------------------------------------
# HEALPix ray directions (Gorski et al. 2005, RING scheme pixel centres)
# ----------------------------------------------------------------------------
def healpix_dirs(n_side: int) -> np.ndarray:
    """Unit vectors of the 12*n_side^2 HEALPix pixel centres in RING order.

    Rings run from the north pole (i = 1) to the south pole (i = 4 n_side - 1);
    within a ring pixels are ordered by increasing azimuth.  Polar-cap rings hold
    4i pixels at z = 1 - i^2/(3 n_side^2) with phi = pi/(2i) (j - 1/2); belt rings
    hold 4 n_side pixels at z = 4/3 - 2i/(3 n_side) with
    phi = pi/(2 n_side) (j - s/2), s = (i - n_side + 1) mod 2.
    """
    if n_side < 1:
        raise ValueError("n_side must be a positive integer")
    ns = n_side
    out = []
    for i in range(1, 4 * ns):
        if i < ns:                                   # north cap
            z = 1.0 - i * i / (3.0 * ns * ns)
            phis = [math.pi / (2.0 * i) * (j - 0.5) for j in range(1, 4 * i + 1)]
        elif i <= 3 * ns:                            # equatorial belt
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns)
            s = (i - ns + 1) % 2
            phis = [math.pi / (2.0 * ns) * (j - 0.5 * s) for j in range(1, 4 * ns + 1)]
        else:                                        # south cap
            ii = 4 * ns - i
            z = -(1.0 - ii * ii / (3.0 * ns * ns))
            phis = [math.pi / (2.0 * ii) * (j - 0.5) for j in range(1, 4 * ii + 1)]
        st = math.sqrt(max(0.0, (1.0 - z) * (1.0 + z)))
        for phi in phis:
            out.append((st * math.cos(phi), st * math.sin(phi), z))
    d = np.asarray(out, dtype=np.float64)
    assert d.shape[0] == 12 * ns * ns
    return d


# ----------------------------------------------------------------------------
# Spectrum (discrete bins between 1 and q Rydberg)
# ----------------------------------------------------------------------------
def power_law_spectrum(n_bins: int, alpha_J: float, gamma_thin: float, q: float = 4.0,
                       sigma_slope: float = 3.0):
    """Log-spaced bins over [nu_th, q nu_th]; J ~ nu^-alpha_J, sigma ~ nu^-sigma_slope.

    Bin b has edges nu_th q^(b/n) and nu_th q^((b+1)/n) and its centre at their
    geometric mean.  w_b = 4 pi J_b dnu_b / (h nu_b) up to one overall factor that
    is fixed so that sum_b w_b sigma_b equals ``gamma_thin`` (Eq. gamma with the
    frequency integral done bin by bin).
    """
    e = np.arange(n_bins + 1, dtype=np.float64)
    edges = q ** (e / n_bins)                         # in units of nu_th
    centre = np.sqrt(edges[:-1] * edges[1:])
    dnu = edges[1:] - edges[:-1]
    sigma = SIGMA_TH * centre ** (-sigma_slope)
    shape = centre ** (-alpha_J) * dnu / centre       # J dnu / nu, constants dropped
    w = shape * (gamma_thin / float(np.sum(shape * sigma)))
    return sigma.astype(np.float64), w.astype(np.float64)


def grey_spectrum(gamma_thin: float, sigma: float = SIGMA_TH):
    """A single bin of photons at 13.6 eV carrying the given thin rate."""
    return np.array([sigma], dtype=np.float64), np.array([gamma_thin / sigma], dtype=np.float64)


# ----------------------------------------------------------------------------
# Smoothing lengths
# ----------------------------------------------------------------------------
def smoothing_lengths(pos: np.ndarray, n_ngb: int = 48, box: float = 0.0) -> np.ndarray:
    """h_j = (d_48 + d_49)/2: mean distance to the 48th and 49th nearest others.

    Distances use the minimum image in a periodic box.  Taking the midpoint keeps
    the 48th neighbour strictly inside the kernel and the 49th strictly outside,
    so no neighbour sits exactly on a kernel boundary.
    """
    from scipy.spatial import cKDTree
    p = np.asarray(pos, dtype=np.float64)
    if p.shape[0] < n_ngb + 2:
        # too few particles for the neighbour rule: the largest separation, or
        # 1 kpc for a lone particle
        if p.shape[0] < 2:
            return np.ones(p.shape[0])
        d = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(-1))
        return np.maximum(d.max(1), 1e-3)
    if box > 0:
        tree = cKDTree(np.mod(p, box), boxsize=box)
        d, _ = tree.query(np.mod(p, box), k=n_ngb + 2, workers=-1)
    else:
        tree = cKDTree(p)
        d, _ = tree.query(p, k=n_ngb + 2, workers=-1)
    # column 0 is the particle itself
    return (0.5 * (d[:, n_ngb] + d[:, n_ngb + 1])).astype(np.float64)


def _to_box_f32(p: np.ndarray, box: float) -> np.ndarray:
    """Cast to FP32 and wrap into [0, box) after rounding."""
    q = np.asarray(p, dtype=np.float64) % box
    f = q.astype(np.float32)
    f[f >= np.float32(box)] -= np.float32(box)
    f[f < 0] += np.float32(box)
    f[f >= np.float32(box)] = np.float32(0.0)
    return f


# ----------------------------------------------------------------------------
# Config recipes
# ----------------------------------------------------------------------------
def uniform_lattice(n_side_lattice: int = 16, box: float = 100.0, n_H: float = 1.5e-3,
                    T: float = 1e4, jitter: float = 0.1, n_side: int = 1,
                    l_ray: float = 100.0, gamma_thin: float = 1e-12,
                    seed: int = BASE_SEED + 0, tol: float = 1e-3, max_iter: int = 200,
                    name: str = "uniform_lattice") -> Workload:
    """Jittered cubic lattice in a periodic box with uniform n_H and T.

    Each coordinate is displaced uniformly by up to +-``jitter`` lattice spacings.
    Every particle carries the same hydrogen content n_H * V_box / N.
    """
    rng = np.random.default_rng(seed)
    m = n_side_lattice
    a = box / m
    idx = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1)
    idx = idx.reshape(-1, 3).astype(np.float64)
    pos64 = (idx + 0.5 + rng.uniform(-jitter, jitter, size=idx.shape)) * a
    pos = _to_box_f32(pos64, box)
    n = pos.shape[0]
    h = smoothing_lengths(pos, box=box).astype(np.float32)
    n_atoms_per_kpc2 = n_H * box ** 3 * KPC_CM / n      # atoms / (kpc_cm)^2
    mu = np.full(n, n_atoms_per_kpc2, dtype=np.float32)
    sigma, w = grey_spectrum(gamma_thin)
    return Workload(name=name, pos=pos, h=h, mu=mu,
                    n_H=np.full(n, n_H, dtype=np.float32), T=np.full(n, T, dtype=np.float32),
                    dirs=healpix_dirs(n_side), sigma=sigma, w=w, l_ray=float(l_ray),
                    box=float(box), tol=tol, max_iter=max_iter,
                    meta=dict(recipe="uniform_lattice", lattice=m, seed=seed))


def _halo_particles(rng, n: int, n_peak: float, r_core: float, r_max: float):
    """Radii and directions for equal-mass particles of n_H = n0 / (1 + (r/rc)^2)."""
    def mass(r):  # enclosed mass in units of 4 pi n0 rc^3
        x = r / r_core
        return x - np.arctan(x)
    u = rng.uniform(0.0, 1.0, size=n) * mass(r_max)
    lo = np.zeros(n)
    hi = np.full(n, r_max)
    for _ in range(64):                       # bisection on the enclosed mass
        mid = 0.5 * (lo + hi)
        below = mass(mid) < u
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    r = 0.5 * (lo + hi)
    cz = rng.uniform(-1.0, 1.0, size=n)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=n)
    st = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    pos = np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * cz], -1)
    nH = n_peak / (1.0 + (r / r_core) ** 2)
    total = 4.0 * math.pi * n_peak * r_core ** 3 * mass(r_max)   # n_H * kpc^3
    mu = total * KPC_CM / n
    return pos, nH, mu


def isothermal_halo(n: int = 262144, n_peak: float = 1.0, r_core: float = 1.0,
                    r_max: float = 150.0, T: float = 1e4, n_side: int = 1, n_bins: int = 128,
                    alpha_J: float = 1.5, gamma_thin: float = 1e-12, l_ray: float = 100.0,
                    seed: int = BASE_SEED + 1, tol: float = 1e-3, max_iter: int = 200,
                    name: str = "isothermal_halo") -> Workload:
    """An isolated cored r^-2 halo, n_H = n_peak / (1 + (r/r_core)^2), r <= r_max."""
    rng = np.random.default_rng(seed)
    pos64, nH, mu = _halo_particles(rng, n, n_peak, r_core, r_max)
    pos = pos64.astype(np.float32)
    h = smoothing_lengths(pos).astype(np.float32)
    sigma, w = power_law_spectrum(n_bins, alpha_J, gamma_thin)
    return Workload(name=name, pos=pos, h=h, mu=np.full(n, mu, dtype=np.float32),
                    n_H=nH.astype(np.float32), T=np.full(n, T, dtype=np.float32),
                    dirs=healpix_dirs(n_side), sigma=sigma, w=w, l_ray=float(l_ray), box=0.0,
                    tol=tol, max_iter=max_iter,
                    meta=dict(recipe="isothermal_halo", n_peak=n_peak, r_core=r_core,
                              r_max=r_max, seed=seed))


def one_sided_slab(n_xy: int = 24, n_z: int = 32, depth: float = 200.0, n_H: float = 1.5e-3,
                   T: float = 1e4, gamma_thin: float = 1e-12, n_bins: int = 1,
                   jitter: float = 0.1, seed: int = BASE_SEED + 5, tol: float = 1e-5,
                   max_iter: int = 400, name: str = "one_sided_slab",
                   faces: int = 1) -> Workload:
    """A slab of uniform n_H and T lit on one face: the setting of the paper's
    slab tests (Sec. 5.2, 5.3), with a jittered lattice standing in for its
    glass and a grey or power-law spectrum for its UV background.

    n_xy x n_xy x n_z particles with spacing depth / n_z fill 0 <= z <= depth
    (isolated: no periodic images).  Every particle casts one ray, along +z
    towards the lit face at z = depth, of length 2 depth; with faces = 2 a
    second one along -z, so that both faces are lit (Sec. 5.3's two-sided
    slab).  One bin at 13.6 eV (n_bins = 1), else n_bins power-law bins
    (J ~ nu^-1.5), each spectrum carrying the optically thin rate gamma_thin.
    """
    rng = np.random.default_rng(seed)
    a = depth / n_z
    idx = np.stack(np.meshgrid(np.arange(n_xy), np.arange(n_xy), np.arange(n_z), indexing="ij"),
                   -1).reshape(-1, 3).astype(np.float64)
    pos = ((idx + 0.5 + rng.uniform(-jitter, jitter, size=idx.shape)) * a).astype(np.float32)
    n = pos.shape[0]
    h = smoothing_lengths(pos).astype(np.float32)
    mu = np.full(n, n_H * a ** 3 * KPC_CM, dtype=np.float32)    # atoms / (kpc_cm)^2
    if n_bins == 1:
        sigma, w = grey_spectrum(gamma_thin)
    else:
        sigma, w = power_law_spectrum(n_bins, 1.5, gamma_thin)
    return Workload(name=name, pos=pos, h=h, mu=mu,
                    n_H=np.full(n, n_H, dtype=np.float32), T=np.full(n, T, dtype=np.float32),
                    dirs=np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]][:faces]), sigma=sigma,
                    w=w, l_ray=float(2 * depth), box=0.0, tol=tol, max_iter=max_iter,
                    meta=dict(recipe="one_sided_slab", spacing=a, depth=depth, n_xy=n_xy,
                              seed=seed, faces=faces))


def lognormal_field(n_grid: int = 128, box: float = 10000.0, sigma_ln: float = 1.5,
                    slope: float = -2.5, n_mean: float = 1e-5, T0: float = 1e4,
                    T_slope: float = 0.6, n_side: int = 2, n_bins: int = 256,
                    alpha_J: float = 1.5, gamma_thin: float = 1e-12, l_ray: float = 100.0,
                    seed: int = BASE_SEED + 2, max_iter: int = 10,
                    name: str = "lognormal_field") -> Workload:
    """Periodic lognormal density field sampled by n_grid^3 equal-mass particles.

    A Gaussian random field with P(k) ~ k^slope on an n_grid^3 mesh is scaled to a
    standard deviation ``sigma_ln``; rho = exp(field) normalised to mean one.
    Particles fall into cells multinomially with probability ~ rho and uniformly
    within a cell.  n_H = n_mean * rho_cell, T = T0 * rho_cell^T_slope.
    """
    rng = np.random.default_rng(seed)
    m = n_grid
    white = rng.standard_normal((m, m, m))
    k = np.fft.fftfreq(m) * m
    kz = np.fft.rfftfreq(m) * m
    kk = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2)
    amp = np.zeros_like(kk)
    amp[kk > 0] = kk[kk > 0] ** (slope / 2.0)
    g = np.fft.irfftn(np.fft.rfftn(white) * amp, s=(m, m, m), axes=(0, 1, 2))
    g = (g - g.mean()) * (sigma_ln / g.std())
    rho = np.exp(g)
    rho /= rho.mean()
    n = m ** 3
    counts = rng.multinomial(n, (rho / rho.sum()).ravel())
    cell = np.repeat(np.arange(m ** 3), counts)
    ci = np.stack(np.unravel_index(cell, (m, m, m)), -1).astype(np.float64)
    a = box / m
    pos = _to_box_f32((ci + rng.uniform(0.0, 1.0, size=ci.shape)) * a, box)
    rho_p = rho.ravel()[cell]
    h = smoothing_lengths(pos, box=box).astype(np.float32)
    mu = n_mean * box ** 3 * KPC_CM / n
    sigma, w = power_law_spectrum(n_bins, alpha_J, gamma_thin)
    return Workload(name=name, pos=pos, h=h, mu=np.full(n, mu, dtype=np.float32),
                    n_H=(n_mean * rho_p).astype(np.float32),
                    T=(T0 * rho_p ** T_slope).astype(np.float32), dirs=healpix_dirs(n_side),
                    sigma=sigma, w=w, l_ray=float(l_ray), box=float(box), tol=0.0,
                    max_iter=max_iter, meta=dict(recipe="lognormal_field", n_grid=m, seed=seed))


def halo_batch(n_halo: int = 64, n_lo: int = 8192, n_hi: int = 524288, peak_lo: float = 0.01,
               peak_hi: float = 10.0, n_bins: int = 128, seed: int = BASE_SEED + 3,
               name: str = "halo_batch", **kw) -> Workload:
    """Independent isolated halos of log-uniform size and peak density, concatenated."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_halo)).astype(np.int64)
    peaks = np.exp(rng.uniform(math.log(peak_lo), math.log(peak_hi), size=n_halo))
    parts = [isothermal_halo(n=int(ni), n_peak=float(pk), n_bins=n_bins,
                             seed=seed * 1000 + i, **kw)
             for i, (ni, pk) in enumerate(zip(ns, peaks))]
    off = np.zeros(n_halo + 1, dtype=np.int64)
    off[1:] = np.cumsum([p.n for p in parts])
    cat = lambda f: np.concatenate([getattr(p, f) for p in parts])
    p0 = parts[0]
    return Workload(name=name, pos=cat("pos"), h=cat("h"), mu=cat("mu"), n_H=cat("n_H"),
                    T=cat("T"), dirs=p0.dirs, sigma=p0.sigma, w=p0.w, l_ray=p0.l_ray, box=0.0,
                    tol=p0.tol, max_iter=p0.max_iter, halo_offsets=off,
                    meta=dict(recipe="halo_batch", n=ns.tolist(), n_peak=peaks.tolist(),
                              seed=seed))


def field_shard(wl: Workload, rank: int, n_ranks: int = 8) -> Workload:
    """One GPU's share of a periodic field split into n_ranks = m^3 cubic blocks:
    the particles of block ``rank`` (owned, first) and every other particle whose
    periodic distance to the block is at most l_ray + max(h) on each axis
    (ghosts), kept in the same periodic box.  Every particle a ray from an owned
    source can reach is in the shard, so owned sources see the same
    intersections as in the whole field.  meta["n_owned"] counts the owned
    particles and meta["index"] maps shard particles to the field's."""
    assert wl.box > 0.0, "shards of a periodic field"
    m = round(n_ranks ** (1.0 / 3.0))
    assert m ** 3 == n_ranks and 0 <= rank < n_ranks
    side = wl.box / m
    cell = np.array([rank // (m * m), (rank // m) % m, rank % m], dtype=np.float64)
    lo = cell * side
    p = wl.pos.astype(np.float64)
    owned = np.all((p >= lo) & (p < lo + side), axis=1)
    reach = wl.l_ray + float(wl.h.max())
    # periodic distance of each coordinate to the block's interval
    c = lo + 0.5 * side
    d = np.abs(p - c)
    d = np.minimum(d, wl.box - d) - 0.5 * side
    near = np.all(d <= reach, axis=1) & ~owned
    idx = np.concatenate([np.nonzero(owned)[0], np.nonzero(near)[0]])
    meta = dict(wl.meta, shard=rank, n_ranks=n_ranks, n_owned=int(owned.sum()), index=idx)
    return dataclasses.replace(wl, name=f"{wl.name}_shard{rank}of{n_ranks}", pos=wl.pos[idx],
                               h=wl.h[idx], mu=wl.mu[idx], n_H=wl.n_H[idx], T=wl.T[idx],
                               meta=meta)


def make_config(i: int, **kw) -> Workload:
    """The five configurations by index (0-based); keyword overrides shrink them."""
    if i == 0:
        return uniform_lattice(**kw)
    if i == 1 or i == 4:
        return isothermal_halo(**kw)
    if i == 2:
        return lognormal_field(**kw)
    if i == 3:
        return halo_batch(**kw)
    raise ValueError(f"no configuration {i}")
