"""Throughput of the reverse-ray-tracing fixed point on one MI355X.

One step = one whole solve of the workload: tree build over particles already
resident in HBM, path recording, then the order-independent fixed point
(columns -> rate -> equilibrium) until max|dx| < tol or the workload's fixed
iteration count.  The default workload is the largest single-problem one, the
2.1M-particle lognormal field (48 rays, 256 bins, 10 iterations).  Reported:

  value   ray-particle intersections per second over the timed steps
          (every iteration's columns sum over all intersections, periodic
          images counted separately);
  particles_per_s_per_iteration  N_p * iterations / time;
  roofline  for the kernel with the most time in the timed steps: algorithmic
          bytes per launch over its average launch duration, timed with HIP
          events on the library's stream, against 8 TB/s HBM.  Per kernel:
            product over recorded paths  8 B per intersection (particle index,
                                         K/h^2) + 16 B per ray (row offset,
                                         FP64 column);
            recording walk (one walk)    20 B per intersection read (x, y, z,
                                         h, mu*x in FP32) + 8 B written (the
                                         entry) + 8 B per ray (its count);
            chunk compaction             16 B per intersection (entry read and
                                         written) + 12 B per ray;
            traversal without recording  20 B per intersection + 8 B per ray;
  sub-objects  the 262144-particle halo (its own steps, update rules, the
          near/far scheme), forward+adjoint against the plain forward on both
          single problems, and the 64-halo batch solved at once against 64
          sequential solves;
  cpu_baseline  the FP64 oracle on one core (primary) and on every host core,
          on a bounded sample of source particles of the same workload (the
          update is order-independent, so a sample of sources at the same
          state is an exact sub-problem), with pair tests per second and the
          extrapolated time of one full column pass.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_HIT = 20.0          # x, y, z, h, mu*x (FP32) of each intersected particle
BYTES_PER_RAY = 8.0           # the FP64 column written per ray
BYTES_PER_PATH_HIT = 8.0      # recorded (particle index, K/h^2) streamed per intersection
BYTES_PER_ROW = 16.0          # row offset read + FP64 column written per ray
BYTES_PER_TILE_HIT = 6.0      # 16-bit local particle index + FP32 K/h^2 per intersection
BYTES_PER_TILE_SET = 8.0      # per distinct particle of a tile: its index + its mu*x
BYTES_PER_WALK_HIT = 28.0     # recording walk: 20 B read + the 8 B entry written
BYTES_PER_WALK_RAY = 8.0      # its per-ray count
BYTES_PER_COMPACT_HIT = 16.0  # compaction: each 8 B entry read and written
BYTES_PER_COMPACT_RAY = 12.0  # row offset and first chunk read per ray
DEFAULT_WORKLOAD = "lognormal_field_2097152"
METRIC = "ray-particle intersections/s + particles/s per iteration; fwd+adjoint vs plain"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str):
    import workloads as W
    if name == "isothermal_halo_262144":
        return W.make_config(1)
    if name == "uniform_lattice_4096":
        return W.make_config(0)
    if name == "lognormal_field_2097152":
        return W.make_config(2)
    if name == "halo_batch_64":
        return W.make_config(3)
    if name == "lognormal_field_shard_0of8":
        return W.field_shard(W.make_config(2), 0, 8)
    if name == "halo_batch_64_small":
        return W.halo_batch(n_lo=2048, n_hi=32768, name="halo_batch_64_small")
    if name.startswith("isothermal_halo_"):
        return W.isothermal_halo(n=int(name.rsplit("_", 1)[1]))
    raise SystemExit(f"unknown workload {name}")


# the kernel behind each timed phase (source file, function, counter-name prefix)
KERNEL_SOURCES = {"recorded_paths": ("paper_1304_4235_amd/csrc/trace.hip", "k_path_stream",
                                     "k_path_stream<"),
                  "row_tiles": ("paper_1304_4235_amd/csrc/tiles.hip", "k_tile_columns",
                                "k_tile_columns<"),
                  "traversal": ("paper_1304_4235_amd/csrc/trace.hip", "k_trace_wave",
                                "k_trace_wave<0,"),
                  "path_recording_walk": ("paper_1304_4235_amd/csrc/trace.hip", "k_trace_wave",
                                          "k_trace_wave<5,"),
                  "chunk_compaction": ("paper_1304_4235_amd/csrc/trace.hip", "k_compact_chunks",
                                       "k_compact_chunks")}


def kernel_source_sha256(path: str, function: str) -> str:
    """Hash of one kernel's definition (signature line to its closing brace)."""
    import hashlib
    txt = open(os.path.join(ROOT, path)).read()
    i = txt.index("\n" + function + "(") + 1
    j = txt.index("\n}\n", i) + 3
    return hashlib.sha256(txt[i:j].encode()).hexdigest()


def measured_traffic(workload: str, kernel_key: str):
    """HBM bytes per launch from the committed counter summary of this workload,
    only while the kernel's source is the one the counters were taken with."""
    f = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if kernel_key not in KERNEL_SOURCES or not os.path.exists(f):
        return None
    path, function, prefix = KERNEL_SOURCES[kernel_key]
    for name, k in json.load(open(f))["kernels"].items():
        if not name.startswith(prefix):
            continue
        if k.get("source_sha256") != kernel_source_sha256(path, function):
            return None
        return k["fetch_bytes"] + k["write_bytes"]
    return None


def measured_cache(workload: str, kernel_key: str):
    """L1 and L2 hit rates and TA busy fraction of the kernel from the committed
    cache-counter summary of this workload, only while the kernel's source is
    the one the counters were taken with (else None)."""
    f = os.path.join(ROOT, "profiles", f"cache_{workload}.json")
    if kernel_key not in KERNEL_SOURCES or not os.path.exists(f):
        return None
    path, function, prefix = KERNEL_SOURCES[kernel_key]
    for name, k in json.load(open(f))["kernels"].items():
        if not name.startswith(prefix):
            continue
        if k.get("source_sha256") != kernel_source_sha256(path, function):
            return None
        return {"l2_hit_rate": k["l2_hit_rate"], "l2_miss_bytes": k["l2_miss_bytes_128"],
                "l1_hit_rate": k["l1_hit_rate"], "ta_busy_frac": k["ta_busy_frac"],
                "source": f"profiles/cache_{workload}.md"}
    return None


def cpu_model() -> str:
    cpu = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return cpu


def _pair_tests(wl, src) -> int:
    """Particle tests the oracle's brute force makes for these sources: every
    particle for every periodic image its per-ray image range spans."""
    if not wl.box:
        return int(src.size * wl.n_ray * wl.n)
    pos = wl.pos.astype(np.float64)
    plo, phi = pos.min(0), pos.max(0)
    hmax = float(np.max(wl.h))
    tot = 0
    for p in src:
        r = pos[p]
        for u in wl.dirs:
            e = r + wl.l_ray * u
            smin, smax = np.minimum(r, e), np.maximum(r, e)
            lo = np.ceil((smin - hmax - phi) / wl.box - 1e-9)
            hi = np.floor((smax + hmax - plo) / wl.box + 1e-9)
            tot += int(np.prod(hi - lo + 1)) * wl.n
    return tot


def _oracle_rate(wl, x, threads, budget_s, seed):
    import oracle
    rng = np.random.default_rng(seed)
    m = 4
    t_used, hits, pairs, done = 0.0, 0, 0, 0
    while True:
        src = np.sort(rng.choice(wl.n, min(m, wl.n), replace=False))
        t0 = time.perf_counter()
        _, cnt = oracle.columns_and_counts(wl, x, src, n_threads=threads)
        dt = time.perf_counter() - t0
        t_used += dt
        hits += int(cnt.sum())
        pairs += _pair_tests(wl, src)
        done += src.size
        if t_used > budget_s / 3 or done >= wl.n:
            break
        m = int(min(wl.n, max(m * 2, m * (budget_s / 2) / max(dt, 1e-3))))
    rays = done * wl.n_ray
    return dict(value=hits / t_used, pair_tests_per_s=pairs / t_used, sources=done,
                intersections=hits, pair_tests=pairs, seconds=t_used,
                extrapolated_full_iteration_s=t_used * (wl.n * wl.n_ray) / rays)


def cpu_baseline(wl, x, budget_s: float = 12.0):
    """The oracle as it stands on the host's cores: one core (the primary
    baseline) and every core, each on a sample of sources at the optically
    thin state, scaled to intersections/s; pair tests/s and the extrapolated
    time of one full column pass (every source and ray) beside it."""
    nproc = os.cpu_count() or 1
    try:
        nproc = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or nproc
    say("cpu baseline: oracle on one core...")
    one = _oracle_rate(wl, x, 1, budget_s, 7)
    say(f"cpu baseline: oracle on {threads} threads...")
    many = _oracle_rate(wl, x, threads, budget_s, 8)
    cpu = cpu_model()
    return {"value": one["value"], "unit": "intersections/s", "cores": 1, "kind": "oracle",
            "sample": f"{one['sources']} random source particles x {wl.n_ray} rays, one column "
                      f"pass (brute force over all {wl.n} particles and their periodic images, "
                      f"adaptive quadrature) at the optically thin state; "
                      f"{one['intersections']} intersections in {one['seconds']:.1f} s on one "
                      f"core of {cpu}",
            "pair_tests_per_s": one["pair_tests_per_s"],
            "extrapolated_full_iteration_s": one["extrapolated_full_iteration_s"],
            "nproc": nproc, "cpu_model": cpu,
            "all_cores": {"value": many["value"], "cores": threads,
                          "pair_tests_per_s": many["pair_tests_per_s"],
                          "extrapolated_full_iteration_s": many["extrapolated_full_iteration_s"],
                          "sample": f"{many['sources']} sources, {many['intersections']} "
                                    f"intersections in {many['seconds']:.1f} s"}}


def kernel_table(tm, steps, hits_per_iter, rays, wl):
    """Every timed kernel with its launches, time, algorithmic bytes per launch
    and achieved GB/s (bytes as in the module docstring)."""
    kernels = {}

    def add(key, name, total_ms, launches, b, **extra):
        if launches <= 0 or total_ms <= 0:
            return
        avg = total_ms / launches
        kernels[key] = dict(kernel=name, launches=launches, total_ms=total_ms,
                            avg_launch_ms=avg, algorithmic_bytes_per_launch=b,
                            achieved=b / (avg * 1e-3) / 1e9, **extra)

    add("traversal", "k_trace_wave<0> (traversal + column, no recorded paths)", tm["trace_ms"],
        tm["n_trace"], BYTES_PER_HIT * hits_per_iter + BYTES_PER_RAY * rays)
    add("recorded_paths", "k_path_stream (columns from recorded paths, streamed by row blocks)",
        tm["path_ms"],
        tm["n_path"], BYTES_PER_PATH_HIT * hits_per_iter + BYTES_PER_ROW * rays)
    add("row_tiles", "k_tile_columns (columns from row tiles)", tm["tile_ms"], tm["n_tile"],
        BYTES_PER_TILE_HIT * hits_per_iter + BYTES_PER_ROW * rays
        + BYTES_PER_TILE_SET * max(tm["tile_set_total"], 0),
        build_ms_per_step=tm["tile_build_ms"] / steps)
    # a recording walk sees every intersection of the geometry once
    add("path_recording_walk", "k_trace_wave<5> (path recording in one walk into pool chunks)",
        tm["chunk_walk_ms"], tm["n_chunk_walk"],
        BYTES_PER_WALK_HIT * hits_per_iter + BYTES_PER_WALK_RAY * rays)
    add("chunk_compaction", "k_compact_chunks (pool chunks into rows)", tm["compact_ms"],
        tm["n_chunk_walk"], BYTES_PER_COMPACT_HIT * hits_per_iter + BYTES_PER_COMPACT_RAY * rays)
    if tm["other_walk_ms"] > 0:
        kernels["counting_and_recording_walks"] = dict(
            kernel="k_trace_wave<1>, <3> (a count walk and a record walk: a context's first "
                   "recording, or a pool that ran short)",
            total_ms=tm["other_walk_ms"])
    kernels["rate_equilibrium"] = dict(kernel="k_gamma (rate and equilibrium, ALU bound)",
                                       total_ms=tm["rate_ms"])
    kernels["tree_build"] = dict(kernel="bounds, Morton keys, radix sort, radix tree, refit, "
                                        "layout", total_ms=tm["build_ms"])
    return kernels


def roofline_of(kernels, workload):
    """The kernel with the most time among those with algorithmic bytes."""
    dom = max((k for k in kernels if "achieved" in kernels[k]),
              key=lambda k: kernels[k]["total_ms"])
    k = kernels[dom]
    return {"bound": "hbm", "kernel": k["kernel"], "achieved": k["achieved"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": k["achieved"] / HBM_PEAK_GBS,
            "traffic": measured_traffic(workload, dom),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated)",
            "cache": measured_cache(workload, dom),
            "avg_launch_ms": k["avg_launch_ms"],
            "algorithmic_bytes_per_launch": k["algorithmic_bytes_per_launch"]}


def forward_adjoint(s, wl, K):
    """Forward+adjoint against the plain forward, K iterations from the thin
    state (the loss of the differentiation workload: log10 rates against those
    under 1.2x the weights)."""
    import torch
    w0 = wl.w.copy()
    s.set_spectrum(wl.sigma, 1.2 * w0)
    lnG_t, _ = s.forward(K)
    s.set_spectrum(wl.sigma, w0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lnG, x = s.forward(K)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t_fb = []
    for rep in range(2):
        # the first backward after a tree build also prepares the transposed
        # product (transposed paths or row tiles, once per geometry)
        say(f"{wl.name}: forward+adjoint {rep + 1}/2 (K={K})")
        t0 = time.perf_counter()
        lnG, x = s.forward(K)
        g = 2.0 * (lnG - lnG_t) / np.log(10.0) ** 2
        s.backward(g, None)
        torch.cuda.synchronize()
        t_fb.append(time.perf_counter() - t0)
    return {"K": K, "plain_forward_ms": t_fwd * 1e3, "forward_plus_adjoint_ms": t_fb[1] * 1e3,
            "ratio": t_fb[1] / t_fwd, "first_after_build_ms": t_fb[0] * 1e3,
            "first_ratio": t_fb[0] / t_fwd,
            "gradients": f"dL/dw over {wl.n_bins} bins and dL/dn_H over {wl.n} particles"}


def run_single(name, steps, warmup, args, rules=False, near_far=False, adjoint=True):
    """Timed whole-solve steps of one workload, its kernels and roofline."""
    import torch
    from paper_1304_4235_amd import Solver
    wl = make_workload(name)
    say(f"workload {wl.name}: n={wl.n} rays={wl.n_ray} bins={wl.n_bins} l_ray={wl.l_ray} "
        f"box={wl.box}")
    s = Solver.from_workload(wl, leaf_size=args.leaf, block_size=args.block,
                             record_paths=args.paths, traversal=args.traversal, build=False)
    if args.tiles:
        s.set_tuning(tiles=1)
    torch.cuda.synchronize()

    def step():
        s.build_tree()
        return s.iterate(wl.max_iter, wl.tol, want_x=False)

    for i in range(warmup):
        step()
        say(f"{wl.name}: warmup {i + 1}/{warmup}")
    torch.cuda.synchronize()
    s.enable_timing(True)
    s.reset_timing()
    rec0 = s.recording_stats()
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = step()
        iters.append(r["iters"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = s.timing()
    rec = (s.recording_stats() - rec0).tolist()
    conv = s.convergence()
    s.enable_timing(False)
    say(f"{wl.name}: timed {steps} steps in {dt:.3f} s; iterations {iters}")
    n_it = int(np.sum(iters))
    hits_per_iter = tm["total_hits"] / max(n_it, 1)
    rays = wl.n * wl.n_ray
    kernels = kernel_table(tm, steps, hits_per_iter, rays, wl)
    res = {
        "value": tm["total_hits"] / dt,
        "ms_per_step": dt / steps * 1e3,
        "config": {"workload": wl.name, "particles": wl.n, "rays_per_particle": wl.n_ray,
                   "frequency_bins": wl.n_bins, "l_ray_kpc": wl.l_ray,
                   "box_kpc": wl.box or None, "tol_abs_dx": wl.tol,
                   "max_iterations": wl.max_iter, "iterations_per_step": iters},
        "particles_per_s_per_iteration": wl.n * n_it / dt,
        "intersections_per_iteration": hits_per_iter,
        "phase_ms_per_step": {"tree_build": tm["build_ms"] / steps,
                              "path_recording": tm["record_ms"] / steps,
                              "path_recording_walk": tm["chunk_walk_ms"] / steps,
                              "chunk_compaction": tm["compact_ms"] / steps,
                              "counting_and_recording_walks": tm["other_walk_ms"] / steps,
                              "columns_from_paths": tm["path_ms"] / steps,
                              "columns_from_row_tiles": tm["tile_ms"] / steps,
                              "row_tile_build": tm["tile_build_ms"] / steps,
                              "traversal": tm["trace_ms"] / steps,
                              "rate_equilibrium": tm["rate_ms"] / steps},
        "roofline": roofline_of(kernels, name),
        "kernels": kernels,
        "recordings": {"one_walk": rec[0], "one_walk_then_second_walk": rec[1],
                       "after_count": rec[2], "count_and_record_walks": rec[3],
                       "did_not_fit": rec[4]},
        "convergence_last_step": {
            "tol": wl.tol if wl.tol > 0 else 1e-3,
            "fraction_converged_abs": (conv["n_abs"] / wl.n).round(6).tolist(),
            "fraction_converged_rel": (conv["n_rel"] / wl.n).round(6).tolist()},
    }
    if "n_owned" in wl.meta:
        # one GPU's share of the field: owned particles plus ghosts within
        # l_ray + max(h); every source is traced, ghosts included
        res["config"]["shard"] = {"rank": wl.meta["shard"], "of": wl.meta["n_ranks"],
                                  "owned_particles": wl.meta["n_owned"],
                                  "ghost_particles": wl.n - wl.meta["n_owned"]}
    if rules and wl.tol > 0:
        # time to solution under the paper's update rules (Sec. 4), same geometry
        # and recorded paths; the order-independent case A solve is the timed step
        rule_set = {"density_blocks_16": dict(n_blocks=16),
                    "paper": dict(tau_skip=1e-4, tau_case_b=1.0, relative=True, n_blocks=16)}
        out = {"order_independent": {"sweeps": int(iters[-1]),
                                     "ms": (dt * 1e3 - tm["build_ms"] - tm["record_ms"])
                                     / steps}}
        for rn, rule in rule_set.items():
            say(f"{wl.name}: update rule {rn}")
            s.set_update_rule(**rule)
            s.set_state(None)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = s.iterate(wl.max_iter, wl.tol, want_x=False)
            torch.cuda.synchronize()
            out[rn] = {"rule": rule, "sweeps": r["iters"], "converged": r["converged"],
                       "ms": (time.perf_counter() - t0) * 1e3}
        s.set_update_rule()
        s.set_state(None)
        res["update_rules"] = out
    if near_far and wl.tol > 0:
        # the paper's near/far scheme against the plain scheme, same geometry:
        # one grey bin carrying the same thin rate (monochromatic slab
        # solution), then the workload's own spectrum (polychromatic slab)
        import workloads as W
        sg, wg = W.grey_spectrum(float(np.sum(wl.sigma * wl.w)))
        out = {"spectrum": "one bin at 13.6 eV, same optically thin rate; "
                           f"near_far_polychromatic: the workload's {wl.n_bins} bins"}
        s.enable_timing(True)
        for sn, nf, spec in (("plain", False, (sg, wg)), ("near_far", True, (sg, wg)),
                             ("near_far_polychromatic", True, (wl.sigma, wl.w))):
            say(f"{wl.name}: scheme {sn}")
            s.set_spectrum(*spec)
            s.set_scheme(nf)
            s.set_state(None)
            s.reset_timing()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = s.iterate(wl.max_iter, wl.tol, want_x=False)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) * 1e3
            tmn = s.timing()
            out[sn] = {"sweeps": r["iters"], "converged": r["converged"], "ms": t,
                       "path_recording_ms": tmn["record_ms"],
                       "ms_per_sweep_after_recording": (t - tmn["record_ms"]) / max(r["iters"], 1)}
        s.enable_timing(False)
        s.set_scheme(False)
        s.set_spectrum(wl.sigma, wl.w)
        s.set_state(None)
        res["near_far_scheme"] = out
    if adjoint:
        res["forward_adjoint"] = forward_adjoint(s, wl, int(iters[-1]))
    s.close()
    del s
    torch.cuda.empty_cache()
    return wl, res


def run_batch(name, args, steps=1, warmup=1):
    """Many independent halos: one batched solve (graph-replayed iterations with
    per-halo convergence) against one solve per halo, each from its own tree,
    with the same launch knobs (autotuned with --tune 1)."""
    import torch
    from paper_1304_4235_amd import Solver, autotune
    wl = make_workload(name)
    n_halo = len(wl.halo_offsets) - 1
    say(f"workload {wl.name}: {n_halo} halos, n={wl.n}")
    tuned = autotune.tune(wl, verbose=True, reps=2) if args.tune else None
    torch.cuda.empty_cache()            # the solver sizes its path buffer from free memory
    best = tuned["best"] if tuned else {}
    s = Solver.from_workload(wl, build=False)
    if best:
        autotune.apply(s, best)
    per = best.get("per_launch", 8)

    def batched():
        s.build_tree()
        return s.iterate_halos(wl.max_iter, wl.tol, per_launch=per, want_x=False)

    for i in range(warmup):
        batched()
        say(f"{wl.name}: warmup {i + 1}/{warmup}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = batched()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    its = r["halo_iters"]
    say(f"{wl.name}: batched {t_batch * 1e3:.1f} ms")
    s.close()
    del s
    torch.cuda.empty_cache()
    # sequential: one solver per halo, data already on the GPU, same knobs
    subs = []
    for h in range(n_halo):
        sh = Solver.from_workload(wl.subset_halo(h), build=False)
        if best:
            autotune.apply(sh, best)
        subs.append(sh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_iters = []
    for i, sh in enumerate(subs):
        sh.build_tree()
        seq_iters.append(sh.iterate(wl.max_iter, wl.tol, want_x=False)["iters"])
        sh.close()
        if i % 8 == 7:
            say(f"{wl.name}: sequential {i + 1}/{n_halo} halos, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    del subs
    torch.cuda.empty_cache()
    return wl, {"workload": wl.name, "halos": n_halo, "particles": wl.n,
                "batched_ms": t_batch * 1e3, "sequential_ms": t_seq * 1e3,
                "speedup": t_seq / t_batch, "iterations_per_halo": its.tolist(),
                "same_iterations_as_sequential": bool(list(its) == seq_iters),
                "tuned": best or None,
                "note": "sequential: one solver per halo, each building its tree, recording "
                        "its paths and iterating; batched: one context, one tree of all "
                        "halos, graph-replayed iterations with per-halo convergence"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle work per CPU baseline line (about)")
    ap.add_argument("--adjoint", type=int, default=1,
                    help="also time forward+adjoint against the plain forward (1 = yes)")
    ap.add_argument("--sub", type=int, default=1,
                    help="with the default workload, also run the halo, the batch and their "
                         "comparisons (1 = yes)")
    ap.add_argument("--sub-steps", type=int, default=5, help="timed steps of the halo sub-run")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a 1 GiB device-to-device copy (traffic counter reference)")
    ap.add_argument("--tune", type=int, default=0, help="autotune launch knobs (batched mode)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--leaf", type=int, default=0)
    ap.add_argument("--traversal", type=int, default=0, help="0 wave-cooperative, 1 per lane")
    ap.add_argument("--rules", type=int, default=1,
                    help="time the halo under the paper's update rules (1 = yes)")
    ap.add_argument("--near-far", type=int, default=1,
                    help="time the near/far scheme on the halo's geometry (1 = yes)")
    ap.add_argument("--tiles", type=int, default=0,
                    help="1: columns from row tiles once the recorded paths have been reused")
    ap.add_argument("--paths", type=int, default=-1,
                    help="-1 record ray paths when they fit (default), 0 traverse every iteration")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    import oracle

    if args.calibrate_copy:
        # a plain device copy of known size: reference for the traffic counters
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload.startswith("halo_batch"):
        wl, res = run_batch(args.workload, args, steps=args.steps, warmup=args.warmup)
        print(json.dumps(dict(metric="batched halo solve time vs sequential solves", unit="ms",
                              **res)), flush=True)
        return

    default = args.workload == DEFAULT_WORKLOAD
    sub_halo = default and args.sub
    wl, res = run_single(args.workload, args.steps, args.warmup, args,
                         rules=not sub_halo and args.rules, near_far=not sub_halo and args.near_far,
                         adjoint=bool(args.adjoint))
    out = {
        "metric": METRIC,
        "value": res.pop("value"),
        "unit": "intersections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 box tests and kernel terms, f64 predicate and sums",
        "data": "synthetic",
        "config": res.pop("config"),
    }
    out.update(res)
    if sub_halo:
        # the single spherical halo: its own whole-solve steps, the paper's update
        # rules and near/far scheme on its geometry, forward+adjoint at its K
        hw, hres = run_single("isothermal_halo_262144", args.sub_steps, 1, args,
                              rules=bool(args.rules), near_far=bool(args.near_far),
                              adjoint=bool(args.adjoint))
        out["isothermal_halo"] = hres
        bw, bres = run_batch("halo_batch_64", args)
        out["halo_batch"] = bres
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, oracle.x_thin(wl), args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
