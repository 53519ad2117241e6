"""Python access to the FP64 reference of the reverse ray tracer.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this package; the product library never does.  All
arithmetic lives in ``oracle.c`` (plain C, FP64, serial per source particle)
plus the short plain-Python slab solvers below; nothing here is shared with the
HIP path, which it checks.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
GCC_FLAGS = ["-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-mfma",
             "-fopenmp", "-Wall"]
KPC_CM = 3.0856775814913673e21          # 1 kpc in cm (IAU 2012 au, parsec by definition)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so beside it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        d, i32, i64, vp = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        L.orc_kernel_constants.argtypes = [vp]
        L.orc_Gt.argtypes = [d, d]; L.orc_Gt.restype = d
        L.orc_M4.argtypes = [d, d]; L.orc_M4.restype = d
        L.orc_chord_closed.argtypes = [d, d, d, d]; L.orc_chord_closed.restype = d
        L.orc_chord_quad.argtypes = [d, d, d, d, d]; L.orc_chord_quad.restype = d
        L.orc_gk15_poly.argtypes = [d, d, d, vp, vp]
        L.orc_kernel_norm.argtypes = [d, i32]; L.orc_kernel_norm.restype = d
        L.orc_columns.argtypes = [i64, vp, vp, vp, vp, i32, vp, d, d, i64, vp, d, i32,
                                  vp, vp, vp, vp, vp, vp, i32]
        L.orc_columns.restype = C.c_int
        L.orc_gamma.argtypes = [i64, i32, vp, i32, vp, vp, vp, vp, vp]
        for f in ("orc_alpha_A", "orc_alpha_B", "orc_gamma_coll"):
            getattr(L, f).argtypes = [d]; getattr(L, f).restype = d
        L.orc_xeq.argtypes = [d, d, d, d, d]; L.orc_xeq.restype = d
        L.orc_solve.argtypes = [i64, vp, vp, vp, vp, vp, i32, vp, i32, vp, vp, d, d, d, i32,
                                vp, d, i32, vp, vp, vp, vp, vp]
        L.orc_solve.restype = C.c_int
        L.orc_solve_rule.argtypes = [i64, vp, vp, vp, vp, vp, i32, vp, i32, vp, vp, d, d, d,
                                     i32, d, d, i32, i32, d, i32, vp, vp, vp, vp, vp]
        L.orc_solve_rule.restype = C.c_int
        L.orc_columns_near_far.argtypes = [i64, vp, vp, vp, vp, i32, vp, d, d, i64, vp, d, vp, vp,
                                           vp, i32]
        L.orc_columns_near_far.restype = C.c_int
        L.orc_x_evolve.argtypes = [d, d, d, d, d, d]
        L.orc_x_evolve.restype = d
        L.orc_slab_lnG.argtypes = [d, d, d, d, d, d]
        L.orc_slab_lnG.restype = d
        L.orc_gamma_near_far.argtypes = [i64, i32, vp, vp, d, d, vp, vp, vp, vp, i32]
        L.orc_slab_lnG_poly.argtypes = [i32, vp, vp, d, d, d, d, d]
        L.orc_slab_lnG_poly.restype = d
        L.orc_gamma_near_far_poly.argtypes = [i64, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, i32, i32]
        L.orc_morton.argtypes = [i64, vp, vp]
        L.orc_lbvh.argtypes = [i64, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.orc_lbvh.restype = i64
        L.orc_morton_seg.argtypes = [i64, vp, i32, vp, vp]
        L.orc_lbvh_seg.argtypes = [i64, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_lbvh_seg.restype = i64
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


DEFAULT_RTOL = 1e-13
# threads the oracle may spread independent source particles over (0 = OpenMP default)
N_THREADS = int(os.environ.get("RRT_ORACLE_THREADS", "0"))


# ----------------------------------------------------------------------------
# kernel (Sec. 4.1.1)
# ----------------------------------------------------------------------------
def kernel_constants() -> dict:
    out = np.zeros(4)
    lib().orc_kernel_constants(_p(out))
    return dict(t=out[0], A2h2=out[1], sigma_over_h=out[2], Nh3=out[3])


def Gt(r: float, h: float) -> float:
    return lib().orc_Gt(float(r), float(h))


def M4(r: float, h: float) -> float:
    return lib().orc_M4(float(r), float(h))


def chord_closed(h, b, z1, z2) -> float:
    return lib().orc_chord_closed(float(h), float(b), float(z1), float(z2))


def chord_quad(h, b, z1, z2, rtol=DEFAULT_RTOL) -> float:
    return lib().orc_chord_quad(float(h), float(b) ** 2, float(z1), float(z2), float(rtol))


def gk15_poly(p, a, b):
    k, e = np.zeros(1), np.zeros(1)
    lib().orc_gk15_poly(float(p), float(a), float(b), _p(k), _p(e))
    return float(k[0]), float(e[0])


def kernel_norm(h: float, which: str = "Gt") -> float:
    return lib().orc_kernel_norm(float(h), 0 if which == "Gt" else 1)


# ----------------------------------------------------------------------------
# columns, rates, equilibrium (Sec. 3.3, 4.1.1, Appendix C.3)
# ----------------------------------------------------------------------------
def columns(wl, x: np.ndarray, sources=None, hits: bool = False, rtol=DEFAULT_RTOL,
            n_threads: int = None, factors: bool = False):
    """Columns N[src, k] in cm^-2 for the given source particles (all by default).

    With ``hits=True`` also returns (row_off, hit_j, hit_img): the hit list of
    ray (src_i, k) is hit_j[row_off[i*n_ray+k] : row_off[i*n_ray+k+1]] with the
    periodic image code (sx+8) | (sy+8)<<4 | (sz+8)<<8 in hit_img.  With
    ``factors=True`` as well, hit_fac: each hit's column per unit neutral
    fraction (mu_j times its clipped chord integral, cm^-2), so that
    N[i, k] = sum over the ray's hits of hit_fac * x[hit_j].
    """
    L = lib()
    n = wl.n
    src = _c(np.arange(n) if sources is None else sources, np.int64)
    pos, h, mu = _c(wl.pos, np.float32), _c(wl.h, np.float32), _c(wl.mu, np.float32)
    xx, dirs = _c(x, np.float64), _c(wl.dirs, np.float64)
    nt = N_THREADS if n_threads is None else n_threads
    N = np.zeros((src.size, wl.n_ray), np.float64)
    if not hits:
        rc = L.orc_columns(n, _p(pos), _p(h), _p(mu), _p(xx), wl.n_ray, _p(dirs), wl.l_ray,
                           wl.box, src.size, _p(src), rtol, 1, _p(N), None, None, None, None, None,
                           nt)
        assert rc == 0
        return N
    cnt = np.zeros(src.size * wl.n_ray, np.int64)
    rc = L.orc_columns(n, _p(pos), _p(h), _p(mu), _p(xx), wl.n_ray, _p(dirs), wl.l_ray, wl.box,
                       src.size, _p(src), rtol, 0, None, _p(cnt), None, None, None, None, nt)
    assert rc == 0
    off = np.zeros(cnt.size + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    hj = np.zeros(max(1, int(off[-1])), np.int32)
    hi = np.zeros(max(1, int(off[-1])), np.int32)
    hf = np.zeros(max(1, int(off[-1])), np.float64) if factors else None
    rc = L.orc_columns(n, _p(pos), _p(h), _p(mu), _p(xx), wl.n_ray, _p(dirs), wl.l_ray, wl.box,
                       src.size, _p(src), rtol, 1, _p(N), None, _p(off[:-1].copy()), _p(hj),
                       _p(hi), _p(hf), nt)
    assert rc == 0
    if factors:
        return N, off, hj[: off[-1]], hi[: off[-1]], hf[: off[-1]]
    return N, off, hj[: off[-1]], hi[: off[-1]]


def columns_and_counts(wl, x: np.ndarray, sources, rtol=DEFAULT_RTOL, n_threads: int = None):
    """Columns and per-ray intersection counts in one brute-force pass."""
    L = lib()
    src = _c(sources, np.int64)
    nt = N_THREADS if n_threads is None else n_threads
    N = np.zeros((src.size, wl.n_ray), np.float64)
    cnt = np.zeros(src.size * wl.n_ray, np.int64)
    rc = L.orc_columns(wl.n, _p(_c(wl.pos, np.float32)), _p(_c(wl.h, np.float32)),
                       _p(_c(wl.mu, np.float32)), _p(_c(x, np.float64)), wl.n_ray,
                       _p(_c(wl.dirs, np.float64)), wl.l_ray, wl.box, src.size, _p(src), rtol, 1,
                       _p(N), _p(cnt), None, None, None, None, nt)
    assert rc == 0
    return N, cnt.reshape(src.size, wl.n_ray)


def gamma(N: np.ndarray, sigma: np.ndarray, w: np.ndarray):
    """(ln Gamma, Gamma, tau_eff) per source from columns N[src, k]."""
    N = _c(N, np.float64)
    ns, nr = N.shape
    lnG, G, tau = np.zeros(ns), np.zeros(ns), np.zeros(ns)
    lib().orc_gamma(ns, nr, _p(N), sigma.size, _p(_c(sigma, np.float64)), _p(_c(w, np.float64)),
                    _p(lnG), _p(G), _p(tau))
    return lnG, G, tau


def alpha_A(T):
    return np.array([lib().orc_alpha_A(float(t)) for t in np.atleast_1d(T)])


def alpha_B(T):
    return np.array([lib().orc_alpha_B(float(t)) for t in np.atleast_1d(T)])


def gamma_coll(T):
    return np.array([lib().orc_gamma_coll(float(t)) for t in np.atleast_1d(T)])


def xeq(Gamma, nH, alpha, gcoll, y=0.0):
    f = lib().orc_xeq
    G, n, a, g = np.broadcast_arrays(np.asarray(Gamma, float), np.asarray(nH, float),
                                     np.asarray(alpha, float), np.asarray(gcoll, float))
    return np.array([f(float(G.flat[i]), float(n.flat[i]), float(a.flat[i]), float(g.flat[i]),
                       float(y)) for i in range(G.size)]).reshape(G.shape)


def gamma_thin(wl) -> float:
    return float(np.sum(wl.w * wl.sigma))


def x_thin(wl) -> np.ndarray:
    T = wl.T.astype(np.float64)
    return xeq(gamma_thin(wl), wl.n_H.astype(np.float64), alpha_A(T), gamma_coll(T))


def step(wl, x: np.ndarray, sources=None, rtol=DEFAULT_RTOL):
    """One order-independent update for the given sources from the state x.

    Returns dict with N, lnG, G, tau, x_new for those sources."""
    src = np.arange(wl.n) if sources is None else np.asarray(sources)
    N = columns(wl, x, src, rtol=rtol)
    lnG, G, tau = gamma(N, wl.sigma, wl.w)
    T = wl.T[src].astype(np.float64)
    xn = xeq(G, wl.n_H[src].astype(np.float64), alpha_A(T), gamma_coll(T))
    return dict(N=N, lnG=lnG, G=G, tau=tau, x_new=xn)


def solve(wl, max_iter: int = None, tol: float = None, x_init=None, rtol=DEFAULT_RTOL,
          n_threads: int = None):
    """The full fixed point.  Returns dict(x_hist, lnG_hist, N_last, iters, maxdx)."""
    n = wl.n
    mi = wl.max_iter if max_iter is None else max_iter
    tl = wl.tol if tol is None else tol
    xh = np.zeros((mi + 1, n))
    lh = np.zeros((mi, n))
    Nl = np.zeros((n, wl.n_ray))
    it = np.zeros(1, np.int32)
    md = np.zeros(max(1, mi))
    xi = None if x_init is None else _c(x_init, np.float64)
    nt = N_THREADS if n_threads is None else n_threads
    rc = lib().orc_solve(n, _p(_c(wl.pos, np.float32)), _p(_c(wl.h, np.float32)),
                         _p(_c(wl.mu, np.float32)), _p(_c(wl.n_H, np.float32)),
                         _p(_c(wl.T, np.float32)), wl.n_ray, _p(_c(wl.dirs, np.float64)),
                         wl.n_bins, _p(_c(wl.sigma, np.float64)), _p(_c(wl.w, np.float64)),
                         wl.l_ray, wl.box, tl, mi, _p(xi), rtol, nt, _p(xh), _p(lh), _p(Nl),
                         _p(it), _p(md))
    assert rc == 0
    k = int(it[0])
    return dict(x_hist=xh[: k + 1], lnG_hist=lh[:k], N_last=Nl, iters=k, maxdx=md[:k])


def xeq_partials(x, Gamma, nH, alpha, gcoll):
    """Partial derivatives of the physical root x_- of R x^2 + Q x + P = 0
    (Appendix C.3, eq. xroots, y = 0; R = (gamma + alpha) n_H,
    Q = -(Gamma + alpha n_H + R), P = alpha n_H) with respect to Gamma and n_H,
    by implicit differentiation of the quadratic:
        (2 R x + Q) dx = -(x dQ + x^2 dR + dP),   2 R x_- + Q = -sqrt(Q^2 - 4 P R).
    Returns (dx/dGamma, dx/dn_H) at the given root x."""
    x, G, n, a, g = (np.asarray(v, np.float64) for v in (x, Gamma, nH, alpha, gcoll))
    R = (g + a) * n
    Q = -(G + a * n + R)
    P = a * n
    sq = np.sqrt(np.maximum(Q * Q - 4.0 * P * R, 0.0))
    dx_dG = -x / sq                                       # dQ/dGamma = -1
    dx_dn = (-(2.0 * a + g) * x + (g + a) * x * x + a) / sq
    return dx_dG, dx_dn


def adjoint(wl, K: int, dL_dlnG=None, dL_dx=None, rtol=DEFAULT_RTOL, n_threads: int = None):
    """Reverse mode of K order-independent iterations from the optically thin
    state (Sec. 3.3, Sec. 4): x^0 = x_-(Gamma_thin), then K times columns
    (eq. colden) -> Gamma (eq. gamma_shld) -> x^k = x_-(Gamma^k).  Parameters:
    the bin weights w and the densities n_H, a particle's hydrogen content
    scaling with its density (mu_j proportional to n_H,j at fixed h).

    Given dL/d ln Gamma^K and dL/dx^K (None = zero), returns dict(dw, dnH,
    lnG, x) with the forward outputs ln Gamma^K and x^K of the oracle's solve.
    The chain rule is written out step by step, last iteration first:
      x^k = x_-(Gamma^k):   lbar = xbar dx/dGamma Gamma,  nbar += xbar dx/dn_H
      ln Gamma^k = ln (1/N_ray) sum_k' sum_b w_b sigma_b exp(-sigma_b N_k'):
          with pi_{k'b} each term's share of the sum,
          wbar_b += lbar sum_k' pi_{k'b} / w_b,  Nbar_k' = -lbar sum_b sigma_b pi_{k'b}
      N_{pk'} = sum over hits of f_h x^{k-1}_j (f_h proportional to mu_j):
          xbar^{k-1}_j = sum over j's hits of Nbar f_h,
          nbar_j += sum over j's hits of Nbar f_h x^{k-1}_j / n_H,j
    and finally x^0's own dependence on Gamma_thin = sum_b w_b sigma_b and n_H.
    """
    n, nr = wl.n, wl.n_ray
    sig = np.asarray(wl.sigma, np.float64)
    w = np.asarray(wl.w, np.float64)
    nH = np.asarray(wl.n_H, np.float32).astype(np.float64)
    T = np.asarray(wl.T, np.float32).astype(np.float64)
    al, ga = alpha_A(T), gamma_coll(T)
    fw = solve(wl, max_iter=K, tol=0.0, rtol=rtol, n_threads=n_threads)
    assert fw["iters"] == K
    xh, lh = fw["x_hist"], fw["lnG_hist"]
    _, off, hj, _, hf = columns(wl, xh[0], hits=True, factors=True, rtol=rtol,
                                n_threads=n_threads)
    ray = np.repeat(np.arange(n * nr), np.diff(off))      # ray row p * n_ray + k' of each hit
    xbar = np.zeros(n) if dL_dx is None else np.asarray(dL_dx, np.float64).copy()
    dw = np.zeros(sig.size)
    dn = np.zeros(n)
    lnws = np.log(w * sig)
    for k in range(K, 0, -1):
        lnG = lh[k - 1]
        G = np.exp(lnG)
        dxdG, dxdn = xeq_partials(xh[k], G, nH, al, ga)
        lbar = xbar * dxdG * G
        if k == K and dL_dlnG is not None:
            lbar = lbar + np.asarray(dL_dlnG, np.float64)
        dn += xbar * dxdn
        N = columns(wl, xh[k - 1], rtol=rtol, n_threads=n_threads)
        pi = np.exp(lnws[None, None, :] - sig[None, None, :] * N[:, :, None]
                    - lnG[:, None, None] - np.log(nr))
        dw += np.einsum("p,pkb->b", lbar, pi) / w
        Nbar = -lbar[:, None] * np.einsum("pkb,b->pk", pi, sig)
        c = Nbar.ravel()[ray] * hf
        xbar = np.bincount(hj, weights=c, minlength=n)
        dn += np.bincount(hj, weights=c * xh[k - 1][hj], minlength=n) / nH
    dxdG0, dxdn0 = xeq_partials(xh[0], np.sum(w * sig), nH, al, ga)
    dn += xbar * dxdn0
    dw += sig * np.sum(xbar * dxdG0)
    return dict(dw=dw, dnH=dn, lnG=lh[K - 1], x=xh[K])


def solve_rule(wl, tau_skip: float = 0.0, tau_case_b: float = float("inf"),
               relative: bool = False, n_blocks: int = 1, max_iter: int = None,
               tol: float = None, rtol=DEFAULT_RTOL, n_threads: int = None):
    """The paper's update rule (Sec. 4): tau_skip, case B where tau_eff >=
    tau_case_b, absolute or relative convergence, and updates in n_blocks
    blocks of the density-descending order (1 = order-independent).
    Returns dict(x_hist, lnG_hist, skipped, iters, maxdx)."""
    n = wl.n
    mi = wl.max_iter if max_iter is None else max_iter
    tl = wl.tol if tol is None else tol
    xh = np.zeros((mi + 1, n))
    lh = np.zeros((mi, n))
    sk = np.zeros(n, np.int32)
    it = np.zeros(1, np.int32)
    md = np.zeros(max(1, mi))
    nt = N_THREADS if n_threads is None else n_threads
    rc = lib().orc_solve_rule(n, _p(_c(wl.pos, np.float32)), _p(_c(wl.h, np.float32)),
                              _p(_c(wl.mu, np.float32)), _p(_c(wl.n_H, np.float32)),
                              _p(_c(wl.T, np.float32)), wl.n_ray, _p(_c(wl.dirs, np.float64)),
                              wl.n_bins, _p(_c(wl.sigma, np.float64)), _p(_c(wl.w, np.float64)),
                              wl.l_ray, wl.box, tl, mi, float(tau_skip), float(tau_case_b),
                              int(bool(relative)), int(n_blocks), rtol, nt, _p(xh), _p(lh),
                              _p(sk), _p(it), _p(md))
    assert rc == 0, rc
    k = int(it[0])
    return dict(x_hist=xh[: k + 1], lnG_hist=lh[:k], skipped=sk.astype(bool), iters=k,
                maxdx=md[:k])


# ----------------------------------------------------------------------------
# non-equilibrium evolution (Appendix C.3, time-dependent solution)
# ----------------------------------------------------------------------------
def x_evolve(x0, Gamma, nH, alpha, gcoll, t):
    """x after time t at constant rates, from x0."""
    f = lib().orc_x_evolve
    b = np.broadcast_arrays(*map(np.asarray, (x0, Gamma, nH, alpha, gcoll, t)))
    out = np.array([f(*map(float, v)) for v in zip(*[a.ravel() for a in b])])
    return out.reshape(b[0].shape)


def evolve(wl, x0: np.ndarray, dt: float, n_steps: int, rtol=DEFAULT_RTOL):
    """n_steps of: columns and Gamma at the current state, then every particle
    advances by dt at that Gamma.  Returns the states after each step."""
    T = wl.T.astype(np.float64)
    nH = wl.n_H.astype(np.float64)
    al, ga = alpha_A(T), gamma_coll(T)
    x = np.asarray(x0, np.float64).copy()
    hist = [x.copy()]
    for _ in range(n_steps):
        N = columns(wl, x, rtol=rtol)
        _, G, _ = gamma(N, wl.sigma, wl.w)
        x = x_evolve(x, G, nH, al, ga, dt)
        hist.append(x.copy())
    return np.array(hist)


# ----------------------------------------------------------------------------
# near/far scheme (Sec. 4.1.2) with the monochromatic slab solution (App. C.4)
# ----------------------------------------------------------------------------
def columns_near_far(wl, x: np.ndarray, sources=None, rtol=DEFAULT_RTOL, n_threads: int = None):
    """Per ray: far HI column, near total-hydrogen column (x = 1) and the number
    of near particles hit.  Arrays [n_src, n_ray]."""
    n = wl.n
    src = _c(np.arange(n) if sources is None else sources, np.int64)
    ns = src.size
    Nf = np.zeros((ns, wl.n_ray))
    Nn = np.zeros((ns, wl.n_ray))
    cnt = np.zeros((ns, wl.n_ray), np.int64)
    nt = N_THREADS if n_threads is None else n_threads
    rc = lib().orc_columns_near_far(n, _p(_c(wl.pos, np.float32)), _p(_c(wl.h, np.float32)),
                                    _p(_c(wl.mu, np.float32)), _p(_c(x, np.float64)), wl.n_ray,
                                    _p(_c(wl.dirs, np.float64)), wl.l_ray, wl.box, ns, _p(src),
                                    rtol, _p(Nf), _p(Nn), _p(cnt), nt)
    assert rc == 0
    return Nf, Nn, cnt


def slab_lnG(lnG0, nH, alpha, gcoll, sigma, N):
    """ln of the rate at total hydrogen column N into a uniform slab (App. C.4)."""
    f = lib().orc_slab_lnG
    b = np.broadcast_arrays(*map(np.asarray, (lnG0, nH, alpha, gcoll, sigma, N)))
    out = np.array([f(*map(float, v)) for v in zip(*[a.ravel() for a in b])])
    return out.reshape(b[0].shape)


def slab_lnG_poly(sigma, w, N_far, nH, alpha, gcoll, N_near):
    """ln of the rate at the bottom of a uniform slab of total hydrogen column
    N_near lit by the binned spectrum (w, sigma) after a far column N_far
    (Sec. 4.1.2, eq. gammashldk; the polychromatic form of App. C.4's slab)."""
    sg, ww = _c(sigma, np.float64), _c(w, np.float64)
    f = lib().orc_slab_lnG_poly
    b = np.broadcast_arrays(*map(np.asarray, (N_far, nH, alpha, gcoll, N_near)))
    out = np.array([f(sg.size, _p(sg), _p(ww), *map(float, v))
                    for v in zip(*[a.ravel() for a in b])])
    return out.reshape(b[0].shape)


def slab_rk4_poly(sigma, w, N_far, nH, alpha, gcoll, N_near, n_steps=4000):
    """The same slab as an ODE in the total hydrogen column t: the HI column y
    below the surface grows as dy/dt = x_-(Gamma(N_far + y)), integrated by
    classical RK4 from t = 0 to N_near.  An independent check of the
    quadrature-and-bisection form.  Returns ln Gamma at the bottom."""
    sg = np.asarray(sigma, np.float64)
    lws = np.log(np.asarray(w, np.float64) * sg)
    f = lib().orc_xeq

    def lnG(N):
        v = lws - sg * N
        m = v.max()
        return m + math.log(np.exp(v - m).sum())

    def rhs(y):
        return f(math.exp(lnG(N_far + y)), nH, alpha, gcoll, 0.0)

    h = N_near / n_steps
    y = 0.0
    for _ in range(n_steps):
        k1 = rhs(y)
        k2 = rhs(y + 0.5 * h * k1)
        k3 = rhs(y + 0.5 * h * k2)
        k4 = rhs(y + h * k3)
        y += h * (k1 + 2 * k2 + 2 * k3 + k4) / 6.0
    return lnG(N_far + y)


def step_near_far(wl, x: np.ndarray, sources=None, rtol=DEFAULT_RTOL, n_threads: int = None,
                  share: bool = True):
    """One order-independent update with the near/far rate: the analytic slab
    for one frequency bin, the polychromatic slab for several.  share: each
    ray's slab lit by the ray's share of the radiation, rates summed (the
    paper's weighting), else lit by all of it, rates averaged (variant)."""
    src = np.arange(wl.n) if sources is None else np.asarray(sources)
    Nf, Nn, cnt = columns_near_far(wl, x, src, rtol=rtol)
    T = wl.T[src].astype(np.float64)
    nH = wl.n_H[src].astype(np.float64)
    al, ga = alpha_A(T), gamma_coll(T)
    lnG = np.zeros(src.size)
    if wl.n_bins == 1:
        lib().orc_gamma_near_far(src.size, wl.n_ray, _p(_c(Nf, np.float64)),
                                 _p(_c(Nn, np.float64)), float(wl.w[0]), float(wl.sigma[0]),
                                 _p(_c(nH, np.float64)), _p(_c(al, np.float64)),
                                 _p(_c(ga, np.float64)), _p(lnG), int(bool(share)))
    else:
        nt = N_THREADS if n_threads is None else n_threads
        lib().orc_gamma_near_far_poly(src.size, wl.n_ray, _p(_c(Nf, np.float64)),
                                      _p(_c(Nn, np.float64)), wl.n_bins,
                                      _p(_c(wl.sigma, np.float64)), _p(_c(wl.w, np.float64)),
                                      _p(_c(nH, np.float64)), _p(_c(al, np.float64)),
                                      _p(_c(ga, np.float64)), _p(lnG), nt, int(bool(share)))
    G = np.exp(lnG)
    xn = xeq(G, nH, al, ga)
    return dict(N_far=Nf, N_near=Nn, near_hits=cnt, lnG=lnG, G=G, x_new=xn,
                tau=math.log(gamma_thin(wl)) - lnG)


def solve_near_far(wl, max_iter: int = None, tol: float = None, rtol=DEFAULT_RTOL,
                   share: bool = True):
    """The order-independent fixed point with the near/far rate, from x_thin."""
    mi = wl.max_iter if max_iter is None else max_iter
    tl = wl.tol if tol is None else tol
    x = x_thin(wl)
    xh, lh, md = [x.copy()], [], []
    for _ in range(mi):
        r = step_near_far(wl, x, rtol=rtol, share=share)
        d = float(np.max(np.abs(r["x_new"] - x)))
        x = r["x_new"]
        xh.append(x.copy())
        lh.append(r["lnG"])
        md.append(d)
        if d < tl:
            break
    return dict(x_hist=np.array(xh), lnG_hist=np.array(lh), iters=len(md), maxdx=np.array(md))


# ----------------------------------------------------------------------------
# reference tree
# ----------------------------------------------------------------------------
def morton(pos: np.ndarray, halo_offsets=None) -> np.ndarray:
    """Tree keys in input order: Morton codes, with the halo index above them
    when halo_offsets (H + 1 input offsets, H > 1) splits the particles into
    independent halos."""
    pos = _c(pos, np.float32)
    out = np.zeros(pos.shape[0], np.uint64)
    if halo_offsets is None:
        lib().orc_morton(pos.shape[0], _p(pos), _p(out))
    else:
        off = _c(halo_offsets, np.int64)
        lib().orc_morton_seg(pos.shape[0], _p(pos), off.size - 1, _p(off), _p(out))
    return out


def lbvh(pos: np.ndarray, h: np.ndarray, leaf_max: int, halo_offsets=None) -> dict:
    """The reference tree (see oracle.c); with halo_offsets, the tree of
    independent halos, each in a subtree of its own: seg_root / seg_end give
    the node range [root, end) of each halo."""
    pos, h = _c(pos, np.float32), _c(h, np.float32)
    n = pos.shape[0]
    m = 2 * n
    perm = np.zeros(n, np.int32)
    codes = np.zeros(n, np.uint64)
    lo = np.zeros((m, 3), np.float32)
    hi = np.zeros((m, 3), np.float32)
    skip = np.zeros(m, np.int32)
    first = np.zeros(m, np.int32)
    count = np.zeros(m, np.int32)
    off = None if halo_offsets is None else _c(halo_offsets, np.int64)
    nh = 1 if off is None else off.size - 1
    root = np.zeros(nh, np.int32)
    end = np.zeros(nh, np.int32)
    nn = lib().orc_lbvh_seg(n, _p(pos), _p(h), leaf_max, nh, _p(off), _p(perm), _p(codes),
                            _p(lo), _p(hi), _p(skip), _p(first), _p(count), _p(root), _p(end))
    assert nn > 0
    out = dict(perm=perm, codes=codes, lo=lo[:nn], hi=hi[:nn], skip=skip[:nn],
               first=first[:nn], count=count[:nn], n_nodes=int(nn))
    if nh > 1:
        out.update(seg_root=root, seg_end=end)
    return out


# ----------------------------------------------------------------------------
# plane-parallel slab (Appendix C.4 and the slab solver of Sec. 5.1)
# ----------------------------------------------------------------------------
def slab_depth_analytic(x, x0, x_ce, nH, sigma):
    """Depth z at which the neutral fraction is x (Appendix C.4, eq. analytic_slab_eqn):
    z n_H sigma = (1/x0 - 1/x) + ln[x(1-x0)/(x0(1-x))] + (1/x_ce) ln[x(x_ce-x0)/(x0(x_ce-x))]."""
    x = np.asarray(x, dtype=np.float64)
    t = (1.0 / x0 - 1.0 / x) + np.log(x * (1.0 - x0) / (x0 * (1.0 - x))) + \
        (1.0 / x_ce) * np.log(x * (x_ce - x0) / (x0 * (x_ce - x)))
    return t / (nH * sigma)


def plane_slab_profile(sigma, w, nH, T, depth, n_points=4000):
    """Neutral fraction and HI column against depth in a uniform plane slab lit
    on one face by the binned spectrum (w, sigma): at every depth the gas is
    in equilibrium with the radiation the HI above it lets through (the
    reference of the paper's slab tests, Sec. 5.1, for any spectrum).  The rate
    at total hydrogen column t below the surface is the bottom rate of
    slab_lnG_poly with no far column; for one bin that is the analytic slab of
    Appendix C.4.  depth in kpc.  Returns (z in kpc at n_points + 1 even steps,
    x, N_HI from the surface in cm^-2 by the trapezoid rule in t)."""
    T = float(T)
    a = float(alpha_A(np.array([T]))[0])
    g = float(gamma_coll(np.array([T]))[0])
    z = np.linspace(0.0, float(depth), n_points + 1)
    t = z * nH * KPC_CM
    lnG = np.array([slab_lnG_poly(sigma, w, 0.0, nH, a, g, tt) for tt in t]).ravel()
    x = xeq(np.exp(lnG), np.full_like(t, nH), np.full_like(t, a), np.full_like(t, g))
    NHI = np.concatenate([[0.0], np.cumsum(0.5 * (x[1:] + x[:-1]) * np.diff(t))])
    return z, x, NHI


def two_sided_slab_profile(sigma, w, nH, T, depth, n_points=4000, tol=1e-12,
                           max_iter=10000):
    """Neutral fraction against height z (kpc) in a uniform plane slab lit
    equally on both faces (the two-sided slab of Sec. 5.3): each height takes
    half the rate the spectrum gives through the HI column below it and half
    through the column above, sum_b w_b sigma_b e^{-sigma_b N}, and x = x_- of
    that rate; iterated from the thin state (Jacobi, columns by the trapezoid
    rule on n_points + 1 heights) until max |dx| < tol.  Returns (z, x,
    N_HI below, N_HI above, iterations)."""
    T = float(T)
    a = float(alpha_A(np.array([T]))[0])
    g = float(gamma_coll(np.array([T]))[0])
    z = np.linspace(0.0, float(depth), n_points + 1)
    dt = np.diff(z) * nH * KPC_CM
    sg, ww = np.asarray(sigma, np.float64), np.asarray(w, np.float64)
    lws = np.log(ww * sg)
    one = np.ones_like(z)
    x = xeq(np.full_like(z, np.sum(ww * sg)), nH * one, a * one, g * one)
    for it in range(max_iter):
        seg = 0.5 * (x[1:] + x[:-1]) * dt
        below = np.concatenate([[0.0], np.cumsum(seg)])
        above = below[-1] - below
        ln_dn = _lse(lws[None, :] - sg[None, :] * below[:, None], axis=1)
        ln_up = _lse(lws[None, :] - sg[None, :] * above[:, None], axis=1)
        lnG = _lse(np.stack([ln_dn, ln_up], 1), axis=1) - math.log(2.0)
        xn = xeq(np.exp(lnG), nH * one, a * one, g * one)
        d = np.max(np.abs(xn - x))
        x = xn
        if d < tol:
            break
    seg = 0.5 * (x[1:] + x[:-1]) * dt
    below = np.concatenate([[0.0], np.cumsum(seg)])
    return z, x, below, below[-1] - below, it + 1


# ---------------------------------------------------------------------------
# spherically symmetric reference (the spherical solver of the halo test, Sec. 5.4)
# ---------------------------------------------------------------------------
def _lse(v, axis, wts=None):
    m = np.max(v, axis=axis, keepdims=True)
    e = np.exp(v - m)
    if wts is not None:
        e = e * wts
    return (m + np.log(np.sum(e, axis=axis, keepdims=True))).squeeze(axis)


def sphere_columns(r, mu, nH_of_r, x_of_r, r_max, l_ray, n_s=1200):
    """HI columns N[i, j] (cm^-2) of rays of length l_ray (kpc) from radius r[i]
    in the direction at cos(angle) mu[j] to the outward radial direction,
    through gas of density nH_of_r(R) and neutral fraction x_of_r(R) out to
    r_max (midpoint rule with n_s steps along the ray)."""
    ds = l_ray / n_s
    s = (np.arange(n_s) + 0.5) * ds
    r3, m3, s3 = r[:, None, None], mu[None, :, None], s[None, None, :]
    R = np.sqrt(np.maximum(r3 ** 2 + s3 ** 2 + 2.0 * r3 * s3 * m3, 0.0))
    f = np.where(R <= r_max, nH_of_r(R) * x_of_r(R), 0.0)
    return np.sum(f, axis=-1) * ds * KPC_CM


def spherical_profile(n_peak, r_core, r_max, T, sigma, w, l_ray, n_sh=120, n_mu=32,
                      n_s=1200, tol=1e-6, max_iter=1000):
    """Equilibrium neutral fraction of the cored isothermal sphere n_H = n_peak
    / (1 + (r/r_core)^2), r <= r_max, in an isotropic binned background (w,
    sigma): shells log-spaced in r from 0.01 kpc, rays of length l_ray from
    each shell over n_mu Gauss-Legendre directions in cos(angle) (the axial
    symmetry does the azimuth), the rate of a shell the direction-weighted
    mean of sum_b w_b sigma_b e^{-sigma_b N} in the log domain, and x = x_- of
    that rate, iterated from the thin state until max |dx| < tol (Jacobi).
    Returns (r in kpc, x, iterations)."""
    r = np.geomspace(0.01, r_max, n_sh)
    mu, wmu = np.polynomial.legendre.leggauss(n_mu)
    wmu = wmu / 2.0
    Tv = np.array([float(T)])
    a, g = float(alpha_A(Tv)[0]), float(gamma_coll(Tv)[0])
    nH_of_r = lambda R: n_peak / (1.0 + (R / r_core) ** 2)
    nH_r = nH_of_r(r)
    sg, ww = np.asarray(sigma, np.float64), np.asarray(w, np.float64)
    lws = np.log(ww * sg)
    lr = np.log(r)
    one = np.ones(n_sh)
    x = xeq(np.full(n_sh, np.sum(ww * sg)), nH_r, a * one, g * one)
    for it in range(max_iter):
        xr = x
        N = sphere_columns(r, mu, nH_of_r,
                           lambda R: np.interp(np.log(np.maximum(R, r[0])), lr, xr),
                           r_max, l_ray, n_s)
        lnS = _lse(lws[None, None, :] - sg[None, None, :] * N[:, :, None], axis=2)
        lnG = _lse(lnS, axis=1, wts=wmu[None, :])
        xn = xeq(np.exp(lnG), nH_r, a * one, g * one)
        d = np.max(np.abs(xn - x))
        x = xn
        if d < tol:
            break
    return r, x, it + 1


def slab_numerical(Gamma0, nH, T, sigma, depth, n_slices):
    """Monochromatic plane-parallel radiation on a uniform slab, solved slice by
    slice from the surface inwards (the slab solver of Sec. 5.1): the HI optical
    depth above a slice attenuates the surface rate, and the slice takes the
    equilibrium root for that rate.  Returns slice-centre depths and x."""
    a = float(alpha_A(T)[0])
    g = float(gamma_coll(T)[0])
    dz = depth / n_slices
    z = (np.arange(n_slices) + 0.5) * dz
    xs = np.zeros(n_slices)
    tau = 0.0
    f = lib().orc_xeq
    for i in range(n_slices):
        # the slice's own half-depth: solve x = x_-(Gamma0 exp(-(tau + x nH sigma dz/2)))
        xi = f(Gamma0 * math.exp(-tau), nH, a, g, 0.0)
        for _ in range(200):
            xn = f(Gamma0 * math.exp(-(tau + 0.5 * xi * nH * sigma * dz)), nH, a, g, 0.0)
            if abs(xn - xi) <= 1e-15 * max(xn, 1e-300):
                xi = xn
                break
            xi = xn
        xs[i] = xi
        tau += xi * nH * sigma * dz
    return z, xs
