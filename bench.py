"""Throughput of the reverse-ray-tracing fixed point on one MI355X.

One step = one whole solve of the workload: tree build over particles already
resident in HBM, then the order-independent fixed point (columns -> rate ->
equilibrium) until max|dx| < tol.  Reported:

  value   ray-particle intersections per second over the timed steps
          (every iteration's columns sum over all intersections, periodic
          images counted separately);
  particles_per_s_per_iteration  N_p * iterations / time;
  roofline  for the dominant kernel: algorithmic bytes per launch over the
          average launch duration, timed with HIP events on the library's
          stream, against 8 TB/s HBM.  The product over recorded paths counts
          8 B per intersection (particle index, K/h^2) and 16 B per ray (row
          offset, FP64 column); the traversal without recording counts 20 B
          per intersection (x, y, z, h, mu*x in FP32) and 8 B per ray;
  cpu_baseline  the FP64 oracle on a bounded sample of source particles of
          the same workload (the update is order-independent, so a sample of
          sources at the same state is an exact sub-problem).

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
METRIC = "ray-particle intersections/s + particles/s per iteration; fwd+adjoint vs plain"


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
KERNEL_SOURCES = {"recorded_paths": ("paper_1304_4235_amd/csrc/trace.hip", "k_path_columns",
                                     "k_path_columns<"),
                  "row_tiles": ("paper_1304_4235_amd/csrc/tiles.hip", "k_tile_columns",
                                "k_tile_columns<"),
                  "traversal": ("paper_1304_4235_amd/csrc/trace.hip", "k_trace_wave",
                                "k_trace_wave<0>")}


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


def cpu_baseline(wl, x, budget_s: float = 12.0):
    """The oracle on a bounded sample of sources, scaled to intersections/s."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(7)
    m = 32
    t_used, hits, done = 0.0, 0, 0
    while True:
        src = np.sort(rng.choice(wl.n, min(m, wl.n), replace=False))
        t0 = time.perf_counter()
        _, cnt = oracle.columns_and_counts(wl, x, src, n_threads=threads)
        dt = time.perf_counter() - t0
        t_used += dt
        hits += int(cnt.sum())
        done += src.size
        if t_used > budget_s / 3 or done >= wl.n:
            break
        m = int(min(wl.n, max(m * 2, m * (budget_s / 2) / max(dt, 1e-3))))
    cpu = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": hits / t_used, "unit": "intersections/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{done} random source particles x {wl.n_ray} rays, one column pass "
                      f"(brute force over all {wl.n} particles, adaptive quadrature) at the "
                      f"optically thin state; {hits} intersections in {t_used:.1f} s on {cpu}"}


def bench_batch(args):
    """Many independent halos: one batched solve (graph-replayed iterations with
    per-halo convergence) against one solve per halo, each from its own tree."""
    import torch
    from paper_1304_4235_amd import Solver, autotune
    wl = make_workload(args.workload)
    n_halo = len(wl.halo_offsets) - 1
    print(f"workload {wl.name}: {n_halo} halos, n={wl.n}", file=sys.stderr, flush=True)
    tuned = autotune.tune(wl, verbose=True, reps=2) if args.tune else None
    best = tuned["best"] if tuned else {}
    s = Solver.from_workload(wl, build=False)
    if best:
        autotune.apply(s, best)
    per = best.get("per_launch", 8)

    def batched():
        s.build_tree()
        return s.iterate_halos(wl.max_iter, wl.tol, per_launch=per, want_x=False)

    for _ in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    print(f"tuned {best}; timing the batched solve", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = batched()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    its = r["halo_iters"]
    print(f"batched: {t_batch * 1e3:.1f} ms", file=sys.stderr, flush=True)
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
        if i % 8 == 7:
            print(f"sequential: {i + 1}/{n_halo} halos, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    out = {"metric": "batched halo solve time vs sequential solves", "unit": "ms",
           "workload": wl.name, "halos": n_halo, "particles": wl.n,
           "batched_ms": t_batch * 1e3, "sequential_ms": t_seq * 1e3,
           "speedup": t_seq / t_batch, "iterations_per_halo": its.tolist(),
           "same_iterations_as_sequential": bool(list(its) == seq_iters),
           "tuned": best or None}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="isothermal_halo_262144")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint", type=int, default=1,
                    help="also time forward+adjoint against the plain forward (1 = yes)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a 1 GiB device-to-device copy (traffic counter reference)")
    ap.add_argument("--tune", type=int, default=1, help="autotune launch knobs (batched mode)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--leaf", type=int, default=0)
    ap.add_argument("--traversal", type=int, default=0, help="0 wave-cooperative, 1 per lane")
    ap.add_argument("--rules", type=int, default=1,
                    help="also time the solve under the paper's update rules (1 = yes)")
    ap.add_argument("--near-far", type=int, default=1,
                    help="also time the near/far scheme on the same geometry with a grey "
                         "spectrum (1 = yes)")
    ap.add_argument("--tiles", type=int, default=0,
                    help="1: columns from row tiles once the recorded paths have been reused")
    ap.add_argument("--paths", type=int, default=-1,
                    help="-1 record ray paths when they fit (default), 0 traverse every iteration")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    if args.workload.startswith("halo_batch"):
        return bench_batch(args)

    import torch
    from paper_1304_4235_amd import Solver
    import oracle

    if args.calibrate_copy:
        # a plain device copy of known size: reference for the traffic counters
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    wl = make_workload(args.workload)
    print(f"workload {wl.name}: n={wl.n} rays={wl.n_ray} bins={wl.n_bins} "
          f"l_ray={wl.l_ray} box={wl.box}", file=sys.stderr, flush=True)
    s = Solver.from_workload(wl, leaf_size=args.leaf, block_size=args.block,
                             record_paths=args.paths, traversal=args.traversal, build=False)
    if args.tiles:
        s.set_tuning(tiles=1)
    torch.cuda.synchronize()

    def step():
        s.build_tree()
        return s.iterate(wl.max_iter, wl.tol, want_x=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    s.enable_timing(True)
    s.reset_timing()
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
        iters.append(r["iters"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = s.timing()
    s.enable_timing(False)

    total_hits = tm["total_hits"]
    n_it = int(np.sum(iters))
    hits_per_iter = total_hits / max(n_it, 1)
    rays = wl.n * wl.n_ray
    kernels = {}
    if tm["n_trace"]:
        avg = tm["trace_ms"] / tm["n_trace"]
        b = BYTES_PER_HIT * hits_per_iter + BYTES_PER_RAY * rays
        kernels["traversal"] = dict(kernel="k_trace<0> (traversal + column)", launches=tm["n_trace"],
                                    total_ms=tm["trace_ms"], avg_launch_ms=avg,
                                    algorithmic_bytes_per_launch=b,
                                    achieved=b / (avg * 1e-3) / 1e9)
    if tm["n_path"]:
        avg = tm["path_ms"] / tm["n_path"]
        b = BYTES_PER_PATH_HIT * hits_per_iter + BYTES_PER_ROW * rays
        kernels["recorded_paths"] = dict(kernel="k_path_columns (columns from recorded paths)",
                                         launches=tm["n_path"], total_ms=tm["path_ms"],
                                         avg_launch_ms=avg, algorithmic_bytes_per_launch=b,
                                         achieved=b / (avg * 1e-3) / 1e9)
    if tm["n_tile"]:
        avg = tm["tile_ms"] / tm["n_tile"]
        b = (BYTES_PER_TILE_HIT * hits_per_iter + BYTES_PER_ROW * rays
             + BYTES_PER_TILE_SET * max(tm["tile_set_total"], 0))
        kernels["row_tiles"] = dict(kernel="k_tile_columns (columns from row tiles, particle "
                                           "values staged in LDS)",
                                    launches=tm["n_tile"], total_ms=tm["tile_ms"],
                                    avg_launch_ms=avg, algorithmic_bytes_per_launch=b,
                                    achieved=b / (avg * 1e-3) / 1e9,
                                    build_ms_per_step=tm["tile_build_ms"] / args.steps)
    if tm["record_ms"]:
        kernels["path_recording"] = dict(kernel="k_trace_wave<5> + k_compact_chunks (one walk into pool chunks, then rows; a context's first recording: k_trace_wave<1> + k_trace_wave<3>, count then record)",
                                         total_ms=tm["record_ms"],
                                         per_step_ms=tm["record_ms"] / args.steps)
    dom = max((k for k in kernels if "achieved" in kernels[k]),
              key=lambda k: kernels[k]["total_ms"])
    achieved = kernels[dom]["achieved"]
    alg_bytes = kernels[dom]["algorithmic_bytes_per_launch"]
    avg_trace_ms = kernels[dom]["avg_launch_ms"]
    hits_per_launch = hits_per_iter
    out = {
        "metric": METRIC,
        "value": total_hits / dt,
        "unit": "intersections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 box tests and kernel terms, f64 predicate and sums",
        "data": "synthetic",
        "config": {"workload": wl.name, "particles": wl.n, "rays_per_particle": wl.n_ray,
                   "frequency_bins": wl.n_bins, "l_ray_kpc": wl.l_ray,
                   "box_kpc": wl.box or None, "tol_abs_dx": wl.tol,
                   "iterations_per_step": iters},
        "particles_per_s_per_iteration": wl.n * n_it / dt,
        "intersections_per_iteration": hits_per_launch,
        "phase_ms_per_step": {"traversal": tm["trace_ms"] / args.steps,
                              "path_recording": tm["record_ms"] / args.steps,
                              "columns_from_paths": tm["path_ms"] / args.steps,
                              "columns_from_row_tiles": tm["tile_ms"] / args.steps,
                              "row_tile_build": tm["tile_build_ms"] / args.steps,
                              "rate_equilibrium": tm["rate_ms"] / args.steps,
                              "tree_build": tm["build_ms"] / args.steps},
        "roofline": {"bound": "hbm", "kernel": kernels[dom]["kernel"],
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, dom),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated)",
                     "avg_launch_ms": avg_trace_ms,
                     "algorithmic_bytes_per_launch": alg_bytes},
        "kernels": kernels,
    }
    print(f"timed {args.steps} steps in {dt:.3f} s; iterations {iters}", file=sys.stderr,
          flush=True)
    if "n_owned" in wl.meta:
        # one GPU's share of the field: owned particles plus ghosts within
        # l_ray + max(h); every source is traced, ghosts included
        out["config"]["shard"] = {"rank": wl.meta["shard"], "of": wl.meta["n_ranks"],
                                  "owned_particles": wl.meta["n_owned"],
                                  "ghost_particles": wl.n - wl.meta["n_owned"]}
    if args.rules and wl.tol > 0:
        # time to solution under the paper's update rules (Sec. 4), same geometry
        # and recorded paths; the order-independent case A solve is the timed step
        rules = {"density_blocks_16": dict(n_blocks=16),
                 "paper": dict(tau_skip=1e-4, tau_case_b=1.0, relative=True, n_blocks=16)}
        # the timed solve without its tree build and path recording (the rule
        # solves below reuse both)
        res = {"order_independent": {"sweeps": int(iters[-1]),
                                     "ms": (dt * 1e3 - tm["build_ms"] - tm["record_ms"])
                                     / args.steps}}
        for name, rule in rules.items():
            print(f"update rule {name}", file=sys.stderr, flush=True)
            s.set_update_rule(**rule)
            s.set_state(None)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = s.iterate(wl.max_iter, wl.tol, want_x=False)
            torch.cuda.synchronize()
            res[name] = {"rule": rule, "sweeps": r["iters"], "converged": r["converged"],
                         "ms": (time.perf_counter() - t0) * 1e3}
        s.set_update_rule()
        s.set_state(None)
        out["update_rules"] = res
    if args.near_far and wl.tol > 0:
        # the paper's near/far scheme against the plain scheme, same geometry:
        # one grey bin carrying the same thin rate (monochromatic slab
        # solution), then the workload's own spectrum (polychromatic slab)
        import workloads as W
        sg, wg = W.grey_spectrum(float(np.sum(wl.sigma * wl.w)))
        res = {"spectrum": "one bin at 13.6 eV, same optically thin rate; "
                           f"near_far_polychromatic: the workload's {wl.n_bins} bins"}
        s.enable_timing(True)
        for name, nf, spec in (("plain", False, (sg, wg)), ("near_far", True, (sg, wg)),
                               ("near_far_polychromatic", True, (wl.sigma, wl.w))):
            print(f"scheme {name}", file=sys.stderr, flush=True)
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
            res[name] = {"sweeps": r["iters"], "converged": r["converged"], "ms": t,
                         "path_recording_ms": tmn["record_ms"],
                         "ms_per_sweep_after_recording": (t - tmn["record_ms"]) / max(r["iters"], 1)}
        s.enable_timing(False)
        s.set_scheme(False)
        s.set_spectrum(wl.sigma, wl.w)
        s.set_state(None)
        out["near_far_scheme"] = res
    if args.adjoint:
        # forward+adjoint against the plain forward, K frozen at the solve's iterations
        K = int(iters[-1])
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
            # the first backward after a tree build also transposes the recorded
            # paths (once per geometry); the second reuses them
            print(f"forward+adjoint {rep + 1}/2 (K={K})", file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            lnG, x = s.forward(K)
            g = 2.0 * (lnG - lnG_t) / np.log(10.0) ** 2
            s.backward(g, None)
            torch.cuda.synchronize()
            t_fb.append(time.perf_counter() - t0)
        out["forward_adjoint"] = {"K": K, "plain_forward_ms": t_fwd * 1e3,
                                  "forward_plus_adjoint_ms": t_fb[1] * 1e3,
                                  "ratio": t_fb[1] / t_fwd,
                                  "first_after_build_ms": t_fb[0] * 1e3,
                                  "first_ratio": t_fb[0] / t_fwd,
                                  "gradients": f"dL/dw over {wl.n_bins} bins and dL/dn_H over "
                                               f"{wl.n} particles"}
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle sample)...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, oracle.x_thin(wl))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
