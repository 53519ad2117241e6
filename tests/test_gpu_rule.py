"""The paper's own update rule (Sec. 4, implementation details) on the GPU,
against the FP64 oracle's solve under the same rule, sweep by sweep:

  * particles whose first rate gives tau_eff < tau_skip are frozen;
  * case B recombination where tau_eff >= 1;
  * convergence on max |dx| / x;
  * updates in blocks of the density-descending order (Gauss-Seidel).

tau_eff decides branches, and the two sides agree on it to ~1e-7, so each
test first checks that no oracle tau_eff lies within 1e-5 of a threshold.
Bar: x within 1e-4 relative after every sweep.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

X_RTOL = 1e-4
MARGIN = 1e-5
SWEEPS = 5


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def halo():
    wl = W.isothermal_halo(n=1500, seed=71, n_bins=8, n_peak=1.0)
    first = oracle.step(wl, oracle.x_thin(wl))
    return wl, float(np.percentile(first["tau"], 30)), first["tau"]


def _gpu_sweeps(wl, rule, sweeps, paths=-1):
    from paper_1304_4235_amd import Solver
    s = Solver.from_workload(wl, record_paths=paths)
    s.set_update_rule(**rule)
    x0 = s.get_state()["x"].cpu().numpy()
    out = []
    for k in range(1, sweeps + 1):
        s.set_state(None)
        r = s.iterate(k, 0.0)
        assert r["iters"] == k
        out.append(r["x"].cpu().numpy())
    s.close()
    return x0, out


def _check_margins(wl, ref, rule, first_tau):
    lg = math.log(oracle.gamma_thin(wl))
    if rule.get("tau_skip", 0.0) > 0.0:
        assert np.min(np.abs(first_tau - rule["tau_skip"])) > MARGIN * rule["tau_skip"]
    if math.isfinite(rule.get("tau_case_b", math.inf)):
        tau = lg - ref["lnG_hist"]
        live = ~ref["skipped"]
        assert np.min(np.abs(tau[:, live] - rule["tau_case_b"])) > MARGIN


def _compare(wl, rule, first_tau, sweeps=SWEEPS, paths=-1):
    ref = oracle.solve_rule(wl, max_iter=sweeps, tol=0.0, **rule)
    _check_margins(wl, ref, rule, first_tau)
    x0, xs = _gpu_sweeps(wl, rule, sweeps, paths)
    for k, xg in enumerate(xs, start=1):
        rel = np.abs(xg - ref["x_hist"][k]) / ref["x_hist"][k]
        assert rel.max() <= X_RTOL, f"sweep {k}: max rel {rel.max():.3e}"
    return ref, x0, xs


@pytest.mark.parametrize("name", ["case_b", "relative", "skip", "blocks", "paper"])
def test_rule_sweeps_match_oracle(halo, name):
    wl, tau_skip, first_tau = halo
    rule = {"case_b": dict(tau_case_b=1.0),
            "relative": dict(relative=True),
            "skip": dict(tau_skip=tau_skip),
            "blocks": dict(n_blocks=7),
            "paper": dict(tau_skip=tau_skip, tau_case_b=1.0, relative=True, n_blocks=16)}[name]
    _say("rule", name, rule)
    ref, x0, xs = _compare(wl, rule, first_tau)
    if "tau_skip" in rule:
        frozen = ref["skipped"]
        assert 0 < frozen.sum() < wl.n
        # frozen particles keep the starting state exactly on the GPU too
        np.testing.assert_array_equal(xs[-1][frozen], x0[frozen])


@pytest.mark.parametrize("paths", [-1, 0])
def test_rule_density_blocks_with_and_without_recorded_paths(halo, paths):
    wl, tau_skip, first_tau = halo
    _compare(wl, dict(n_blocks=5, tau_skip=tau_skip), first_tau, sweeps=3, paths=paths)


def test_rule_one_particle_at_a_time():
    """n_blocks = n: the paper's one-particle-at-a-time update, high to low
    density, on a small halo."""
    wl = W.isothermal_halo(n=300, seed=72, n_bins=6, n_peak=3.0)
    first = oracle.step(wl, oracle.x_thin(wl))
    _compare(wl, dict(n_blocks=wl.n), first["tau"], sweeps=3)


def test_rule_converged_solve_and_counts(halo):
    """Density-ordered blocks converge in fewer sweeps than the
    order-independent update, to the same fixed point, with the oracle's sweep
    count."""
    wl, _, _ = halo
    from paper_1304_4235_amd import Solver
    ref_j = oracle.solve_rule(wl, max_iter=200, tol=1e-3)
    ref_g = oracle.solve_rule(wl, n_blocks=16, max_iter=200, tol=1e-3)
    s = Solver.from_workload(wl)
    rj = s.iterate(200, 1e-3)
    s.set_update_rule(n_blocks=16)
    s.set_state(None)
    rg = s.iterate(200, 1e-3)
    assert rj["converged"] and rg["converged"]
    assert rj["iters"] == ref_j["iters"] and rg["iters"] == ref_g["iters"]
    assert rg["iters"] < rj["iters"]
    for r, ref in ((rj, ref_j), (rg, ref_g)):
        rel = np.abs(r["x"].cpu().numpy() - ref["x_hist"][-1]) / ref["x_hist"][-1]
        assert rel.max() <= X_RTOL


def test_rule_is_rejected_where_it_does_not_apply(halo):
    from paper_1304_4235_amd import RRTError, Solver
    wl, _, _ = halo
    s = Solver.from_workload(wl)
    s.set_update_rule(tau_case_b=1.0)
    with pytest.raises(RRTError):
        s.forward(2)
    with pytest.raises(RRTError):
        s.iterate_halos(10, 1e-3)
    with pytest.raises(RRTError):
        s.set_update_rule(tau_skip=-1.0)
    with pytest.raises(RRTError):
        s.set_update_rule(n_blocks=0)
    s.set_update_rule()
    lnG, x = s.forward(2)
    assert torch.isfinite(lnG).all()
    s.close()


@pytest.mark.parametrize("blocks", [1, 5])
def test_rule_over_row_tiles(halo, blocks):
    """The update rule with row tiles switched on: frozen particles' rows are
    skipped by the tile product as by the plain one; one block of the density
    order walks only its own rows (plain product over its source list)."""
    wl, tau_skip, first_tau = halo
    from paper_1304_4235_amd import Solver
    res = []
    for tiles in (0, 1):
        s = Solver.from_workload(wl)
        s.set_tuning(tiles=tiles)
        s.enable_timing(True)
        s.set_update_rule(n_blocks=blocks, tau_skip=tau_skip)
        r = s.iterate(30, 0.0)
        if tiles:
            tm = s.timing()
            assert tm["tile_set_total"] > 0, "row tiles were not built"
            assert (tm["n_tile"] > 0) == (blocks == 1)
        res.append(r["x"].cpu().numpy())
        s.close()
    np.testing.assert_allclose(res[1], res[0], rtol=1e-9)
