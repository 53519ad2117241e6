"""Autotuner for the launch shapes of librrt on the GPU it runs on.

It times the phases that the knobs affect, on the workload itself, with the
library's HIP-event timers (median of repeats), and keeps the fastest setting
of each knob:

* leaf size, traversal block and ray packet (1 ray per lane, or a packet of 64
  rays walking one node sequence): the count + record traversals of path
  recording (or, without recorded paths, a column traversal);
* lanes per ray of the recorded-path product;
* iterations per graph replay of the batched fixed point.

The phases run on a sample of at most max_n particles, which need not rank
the knobs as the whole workload does, so one solve of the whole workload with
the picks and one with the library's defaults decide between them (on the
64-halo batch: 7.25 s with the picks, 7.22 s with the defaults).

None of the knobs changes a result.  Results are cached in a JSON file keyed
by the device name and a coarse description of the workload.
"""
from __future__ import annotations

import json
import os
import statistics
import time
from typing import Optional

import numpy as np
import torch

DEFAULT_SPACE = dict(leaf=[8, 16], trace_block=[64, 128, 256], packet=[64, 1],
                     path_group=[16, 32, 64], per_launch=[4, 16, 64])
# the library's own settings (and the benchmark's iterations per graph replay)
DEFAULTS = dict(leaf=16, trace_block=128, packet=64, path_group=0, per_launch=8)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rrt_autotune.json")


def workload_key(wl) -> str:
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    n_halo = 1 if getattr(wl, "halo_offsets", None) is None else len(wl.halo_offsets) - 1
    n_bucket = int(round(np.log2(max(wl.n, 1))))
    return (f"{dev}|n~2^{n_bucket}|rays={wl.n_ray}|bins={wl.n_bins}|"
            f"periodic={int(wl.box > 0)}|halos={n_halo}")


def _median(xs):
    return float(statistics.median(xs))


def _sample(wl, max_n: int):
    """A representative part of a large workload: for a batch, whole halos in
    order until max_n particles; a single problem is tuned as it is."""
    off = getattr(wl, "halo_offsets", None)
    if off is None or wl.n <= max_n:
        return wl
    import dataclasses
    k = 1
    while k < len(off) - 1 and off[k + 1] <= max_n:
        k += 1
    b = int(off[k])
    return dataclasses.replace(wl, pos=wl.pos[:b], h=wl.h[:b], mu=wl.mu[:b], n_H=wl.n_H[:b],
                               T=wl.T[:b], halo_offsets=np.asarray(off[:k + 1]).copy())


def tune(wl, space: Optional[dict] = None, reps: int = 3, cache_path: str = DEFAULT_CACHE,
         use_cache: bool = True, verbose: bool = False, max_n: int = 1_000_000) -> dict:
    """Best knob settings for this workload (and the timings behind them)."""
    from . import Solver
    space = dict(DEFAULT_SPACE, **(space or {}))
    key = workload_key(wl)
    cache = {}
    if use_cache and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]
    say = print if verbose else (lambda *a, **k: None)
    full = wl
    wl = _sample(wl, max_n)
    x_probe = None
    table = []
    # do the recorded paths fit?  (otherwise every iteration traverses the tree)
    probe = Solver.from_workload(wl, record_paths=-1)
    probe.compute_columns(want_N=False, count=False)
    paths = probe.timing()["path_hits"] >= 0
    probe.close()
    rec = -1 if paths else 0

    # 1. traversal shape: time path recording (count + record) or a column traversal
    best_tr, best_t = None, float("inf")
    for leaf in space["leaf"]:
        s = Solver.from_workload(wl, record_paths=rec)
        s.set_tuning(leaf=leaf)
        s.build_tree()
        if x_probe is None:
            x_probe = torch.full((wl.n,), 0.01, dtype=torch.float64)
        for block in space["trace_block"]:
            for packet in space["packet"]:
                s.set_tuning(trace_block=block, packet=packet)
                ts = []
                for _ in range(reps):
                    s.build_tree()          # invalidates the recorded paths
                    s.set_state(x_probe)
                    s.enable_timing(True)
                    s.reset_timing()
                    s.compute_columns(want_N=False, count=False)
                    tm = s.timing()
                    ts.append(tm["record_ms"] if paths else tm["trace_ms"])
                t = _median(ts)
                table.append(dict(phase="record", leaf=leaf, trace_block=block, packet=packet,
                                  ms=t))
                say(f"record leaf={leaf} block={block} packet={packet}: {t:.2f} ms")
                if t < best_t:
                    best_t, best_tr = t, dict(leaf=leaf, trace_block=block, packet=packet)
        s.close()

    # 2. lanes per ray of the recorded-path product
    best_g = 0
    if not paths:
        space = dict(space, path_group=[])
    s = Solver.from_workload(wl, record_paths=rec)
    s.set_tuning(**best_tr)
    s.build_tree()
    s.set_state(x_probe)
    s.compute_columns(want_N=False, count=False)           # records the paths
    best_gt = float("inf")
    for group in space["path_group"]:
        s.set_tuning(path_group=group)
        s.enable_timing(True)
        s.reset_timing()
        for _ in range(max(reps, 3)):
            s.compute_columns(want_N=False, count=False)
        t = s.timing()["path_ms"] / max(reps, 3)
        table.append(dict(phase="paths", path_group=group, ms=t))
        say(f"paths group={group}: {t:.3f} ms")
        if t < best_gt:
            best_gt, best_g = t, group
    s.close()

    # 3. iterations per graph replay of the batched fixed point
    best_pl, best_plt = space["per_launch"][0], float("inf")
    s = Solver.from_workload(wl)
    s.set_tuning(path_group=best_g, **best_tr)
    s.build_tree()
    for per in space["per_launch"]:
        ts = []
        for _ in range(reps):
            s.set_state(None)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.iterate_halos(wl.max_iter, wl.tol, per_launch=per, want_x=False)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        t = _median(ts)
        table.append(dict(phase="solve", per_launch=per, ms=t))
        say(f"solve per_launch={per}: {t:.2f} ms")
        if t < best_plt:
            best_plt, best_pl = t, per
    s.close()

    best = dict(best_tr, path_group=best_g, per_launch=best_pl)

    # 4. the phases above time a sample of the workload, which need not rank the
    #    knobs as the whole does: one solve of the whole workload with the picks
    #    and one with the defaults decide (the first solve of each records its
    #    paths and is not timed)
    def whole_solve_ms(knobs):
        sw = Solver.from_workload(full, build=False)
        apply(sw, knobs)
        ts = []
        for _ in range(2):
            sw.build_tree()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sw.iterate_halos(full.max_iter, full.tol, per_launch=knobs["per_launch"],
                             want_x=False)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        sw.close()
        del sw
        torch.cuda.empty_cache()        # the next solver sizes its paths from free memory
        return ts[-1]

    torch.cuda.empty_cache()
    t_picked, t_default = whole_solve_ms(best), whole_solve_ms(DEFAULTS)
    say(f"whole workload: picks {t_picked:.1f} ms, defaults {t_default:.1f} ms")
    if t_default < t_picked:
        best = dict(DEFAULTS)
    result = dict(key=key, best=best, timings=table, recorded_paths=paths,
                  tuned_on=dict(particles=wl.n, of=full.n),
                  whole=dict(picks_ms=t_picked, defaults_ms=t_default))
    if cache_path:
        cache[key] = result
        os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
        tmp = cache_path + ".tmp"
        json.dump(cache, open(tmp, "w"), indent=1)
        os.replace(tmp, cache_path)
    return result


def apply(solver, best: dict) -> None:
    """Set the tuned knobs on a solver (rebuild the tree for a new leaf size)."""
    solver.set_tuning(**{k: v for k, v in best.items() if k != "per_launch"})
