"""The paper's near/far scheme for SPH (Sec. 4.1.2) on the GPU against the FP64
oracle: near/far columns per ray, the per-ray slab rate of the near particles
(the monochromatic slab solution of Appendix C.4 for one bin, the
polychromatic slab for several) and the fixed point.

Bars as for the plain scheme: columns 1e-6 relative; ln Gamma 1e-4 absolute
where tau_eff <= 100 (tau_eff 1e-6 relative beyond); x 1e-4 relative.
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


def _say(*a):
    print(*a, flush=True)


def _solver(wl, **kw):
    from paper_1304_4235_amd import Solver
    s = Solver.from_workload(wl, **kw)
    s.set_scheme(True)
    return s


def _check_rates(lnG_g, lnG_o, tau_o):
    thin = tau_o <= 100
    d = np.abs(lnG_g - lnG_o)
    assert np.all(d[thin] <= LNG_ATOL), f"ln Gamma differs by {d[thin].max():.3e}"
    if (~thin).any():
        assert np.all(d[~thin] <= TAU_RTOL * tau_o[~thin]), "tau_eff differs"


def _lattice():
    wl = W.make_config(0, n_side_lattice=8, box=50.0, max_iter=40)
    return wl


def _grey_halo():
    wl = W.isothermal_halo(n=3000, seed=81, n_peak=1.0)
    wl.sigma, wl.w = W.grey_spectrum(1e-12)
    return wl


def _poly(wl, n_bins=8):
    wl.sigma, wl.w = W.power_law_spectrum(n_bins, 1.5, 1e-12)
    return wl


def _case(which):
    return {"lattice": _lattice, "halo": _grey_halo,
            "lattice_poly": lambda: _poly(_lattice()),
            "halo_poly": lambda: _poly(_grey_halo())}[which]()


@pytest.mark.parametrize("which,paths", [("lattice", -1), ("lattice", 0), ("halo", -1),
                                         ("halo", 0), ("lattice_poly", -1), ("halo_poly", -1),
                                         ("halo_poly", 0)])
def test_near_far_columns_rates_and_step(which, paths):
    wl = _case(which)
    s = _solver(wl, record_paths=paths)
    rng = np.random.default_rng(4)
    x = np.minimum(oracle.x_thin(wl) * rng.uniform(1, 300, wl.n), 0.99)
    s.set_state(torch.tensor(x))
    _say(which, "near/far step, paths", paths)
    Nf, _ = s.compute_columns()
    Nn = s.near_columns()
    lnG, _, _ = s.compute_gamma()
    xn, _ = s.update_equilibrium()
    src = np.arange(0, wl.n, max(1, wl.n // 97))
    ref = oracle.step_near_far(wl, x, sources=src)
    np.testing.assert_allclose(Nf.cpu().numpy()[src], ref["N_far"], rtol=COL_RTOL, atol=0)
    np.testing.assert_allclose(Nn.cpu().numpy()[src], ref["N_near"], rtol=COL_RTOL, atol=0)
    assert np.all(ref["N_near"] > 0)
    _check_rates(lnG.cpu().numpy()[src], ref["lnG"], ref["tau"])
    rel = np.abs(xn.cpu().numpy()[src] - ref["x_new"]) / ref["x_new"]
    assert rel.max() <= X_RTOL
    # the near/far rate differs from the plain one (the scheme is in use)
    s2 = _solver(wl, record_paths=paths)
    s2.set_scheme(False)
    s2.set_state(torch.tensor(x))
    s2.compute_columns(want_N=False, count=False)
    lnG_plain, _, _ = s2.compute_gamma()
    assert not np.allclose(lnG_plain.cpu().numpy(), lnG.cpu().numpy(), rtol=1e-3)


@pytest.mark.parametrize("which,mode", [("lattice", 1), ("lattice_poly", 1)])
def test_near_far_fixed_point(which, mode):
    wl = _case(which)
    _say("oracle near/far solve", which, "mode", mode)
    ref = oracle.solve_near_far(wl, max_iter=40, tol=1e-3, share=(mode == 1))
    assert 2 <= ref["iters"] < 40
    s = _solver(wl)
    s.set_scheme(mode)
    r = s.iterate(40, 1e-3)
    assert r["converged"] and r["iters"] == ref["iters"]
    rel = np.abs(r["x"].cpu().numpy() - ref["x_hist"][-1]) / ref["x_hist"][-1]
    assert rel.max() <= X_RTOL
    # every iterate, from the oracle's previous one
    for k in range(ref["iters"]):
        s.set_state(torch.tensor(ref["x_hist"][k]))
        s.compute_columns(want_N=False, count=False)
        s.compute_gamma()
        xn, _ = s.update_equilibrium()
        rel = np.abs(xn.cpu().numpy() - ref["x_hist"][k + 1]) / ref["x_hist"][k + 1]
        assert rel.max() <= X_RTOL, k


def test_near_far_requirements():
    from paper_1304_4235_amd import RRTError
    wl1 = _grey_halo()
    s1 = _solver(wl1)
    with pytest.raises(RRTError):
        s1.forward(2)
    with pytest.raises(RRTError):
        s1.iterate_halos(5, 1e-3)
    s1.set_update_rule(tau_case_b=1.0)
    with pytest.raises(RRTError):
        s1.iterate(5, 1e-3)
    s1.set_update_rule()
    # back to the plain scheme: the plain oracle's step
    s1.set_scheme(False)
    x = oracle.x_thin(wl1)
    s1.set_state(torch.tensor(x))
    s1.compute_columns(want_N=False, count=False)
    lnG, _, tau = s1.compute_gamma()
    src = np.arange(0, wl1.n, 211)
    ref = oracle.step(wl1, x, sources=src)
    _check_rates(lnG.cpu().numpy()[src], ref["lnG"], ref["tau"])
