"""ctypes binding of librrt.so (declared in include/rrt.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device memory comes from torch tensors on the current CUDA/HIP device and work
is enqueued on torch's current stream.  If the library is missing this module
raises at import time; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librrt.so")

RRT_OK, RRT_NOT_CONVERGED = 0, 1
TUNE_KEYS = {"trace_block": 1, "packet": 2, "path_group": 3, "leaf": 4, "adjoint_scatter": 5,
             "tiles": 6, "keep_columns": 7, "one_pass": 8}
ERRORS = {-1: "RRT_E_ARG", -2: "RRT_E_HIP", -3: "RRT_E_INPUT", -4: "RRT_E_STATE",
          -5: "RRT_E_NOMEM", -6: "RRT_E_CAPACITY"}


class RRTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("l_ray", C.c_double), ("box", C.c_double), ("path_budget", C.c_int64),
                ("leaf_size", C.c_int32), ("block_size", C.c_int32), ("record_paths", C.c_int32),
                ("traversal", C.c_int32), ("reserved", C.c_int32 * 2)]


# every symbol include/rrt.h declares, with its ctypes signature
_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
SIGNATURES = {
    "rrt_version": ([], C.c_int),
    "rrt_create": ([_vp, _vp, _vp], C.c_int),
    "rrt_destroy": ([_vp], None),
    "rrt_last_error": ([_vp], C.c_char_p),
    "rrt_set_particles": ([_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "rrt_set_rays": ([_vp, _i32, _vp], C.c_int),
    "rrt_healpix_dirs": ([_i32, _vp], C.c_int),
    "rrt_set_spectrum": ([_vp, _i32, _vp, _vp], C.c_int),
    "rrt_build_tree": ([_vp], C.c_int),
    "rrt_compute_columns": ([_vp, _vp, _vp], C.c_int),
    "rrt_compute_gamma": ([_vp, _vp, _vp, _vp], C.c_int),
    "rrt_update_equilibrium": ([_vp, _vp, _vp], C.c_int),
    "rrt_iterate_equilibrium": ([_vp, _i32, _d, _vp, _vp, _vp], C.c_int),
    "rrt_set_state": ([_vp, _vp], C.c_int),
    "rrt_get_state": ([_vp, _vp, _vp, _vp, _vp], C.c_int),
    "rrt_get_tree": ([_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "rrt_get_hits": ([_vp, _i64, _vp, _vp, _vp], C.c_int),
    "rrt_enable_timing": ([_vp, _i32], C.c_int),
    "rrt_get_timing": ([_vp, _vp], C.c_int),
    "rrt_reset_timing": ([_vp], C.c_int),
    "rrt_get_counters": ([_vp, _vp], C.c_int),
    "rrt_set_density": ([_vp, _vp], C.c_int),
    "rrt_set_halos": ([_vp, _i32, _vp], C.c_int),
    "rrt_set_tuning": ([_vp, _i32, _i32], C.c_int),
    "rrt_set_update_rule": ([_vp, _d, _d, _i32, _i32], C.c_int),
    "rrt_set_scheme": ([_vp, _i32], C.c_int),
    "rrt_evolve": ([_vp, _d, _i32, _vp], C.c_int),
    "rrt_get_near_columns": ([_vp, _vp], C.c_int),
    "rrt_iterate_halos": ([_vp, _i32, _d, _i32, _vp, _vp], C.c_int),
    "rrt_forward": ([_vp, _i32, _vp, _vp], C.c_int),
    "rrt_backward": ([_vp, _vp, _vp, _vp, _vp], C.c_int),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"librrt.so not built at {path}; run paper_1304_4235_amd/build.py")
    L = C.CDLL(path)
    for name, (args, res) in SIGNATURES.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


_lib = load()


def lib() -> C.CDLL:
    return _lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return t.data_ptr()
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    raise TypeError(type(t))


def healpix_dirs(n_side: int) -> np.ndarray:
    out = np.zeros((12 * n_side * n_side, 3), np.float64)
    rc = _lib.rrt_healpix_dirs(n_side, out.ctypes.data)
    if rc != RRT_OK:
        raise RRTError(rc, "rrt_healpix_dirs")
    return out


class Solver:
    """One reverse-ray-tracing problem on one GPU (a context of librrt)."""

    def __init__(self, l_ray: float, box: float = 0.0, leaf_size: int = 0, block_size: int = 0,
                 record_paths: int = -1, path_budget: int = 0, traversal: int = 0,
                 device=None):
        dev = torch.device("cuda" if device is None else device)
        if dev.type != "cuda":
            raise ValueError("the solver runs on a GPU device")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        torch.cuda.set_device(self.device)
        self.stream = torch.cuda.current_stream(self.device)
        p = Params(float(l_ray), float(box), int(path_budget), int(leaf_size), int(block_size),
                   int(record_paths), int(traversal), (C.c_int32 * 2)())
        h = C.c_void_p()
        rc = _lib.rrt_create(C.byref(h), C.byref(p), C.c_void_p(self.stream.cuda_stream))
        if rc != RRT_OK:
            raise RRTError(rc, _lib.rrt_last_error(None).decode())
        self._h = h
        self.n = 0
        self.n_ray = 0
        self._keep = []

    # -- plumbing ---------------------------------------------------------
    def _check(self, rc: int, what: str) -> int:
        if rc < 0:
            raise RRTError(rc, f"{what}: {_lib.rrt_last_error(self._h).decode()}")
        return rc

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.rrt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, dtype):
        if isinstance(a, torch.Tensor):
            t = a.to(device=self.device, dtype=dtype)
        else:
            t = torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=self.device)
        return t.contiguous()

    # -- inputs -----------------------------------------------------------
    def set_particles(self, pos, h, mu, n_H, T, x_init=None):
        pos = self._dev(pos, torch.float32).reshape(-1, 3).contiguous()
        n = pos.shape[0]
        h, mu = self._dev(h, torch.float32), self._dev(mu, torch.float32)
        nH, T = self._dev(n_H, torch.float32), self._dev(T, torch.float32)
        xi = None if x_init is None else self._dev(x_init, torch.float64)
        for t in (h, mu, nH, T) + ((xi,) if xi is not None else ()):
            if t.numel() != n:
                raise ValueError("particle arrays must all have n entries")
        self._check(_lib.rrt_set_particles(self._h, n, _ptr(pos), _ptr(h), _ptr(mu), _ptr(nH),
                                           _ptr(T), _ptr(xi)), "rrt_set_particles")
        self._keep = [pos, h, mu, nH, T, xi]      # copied by the library; kept until synced
        self.n = n
        self.n_halo = 1

    def set_tuning(self, **kw):
        """Launch knobs: trace_block, packet (1 or 64), path_group, leaf, adjoint_scatter (0/1),
        tiles (0/1)."""
        for k, v in kw.items():
            self._check(_lib.rrt_set_tuning(self._h, TUNE_KEYS[k], int(v)), f"rrt_set_tuning {k}")

    def set_update_rule(self, tau_skip: float = 0.0, tau_case_b: float = float("inf"),
                        relative: bool = False, n_blocks: int = 1):
        """The paper's update rule for iterate(): frozen thin particles, case B
        above a tau_eff threshold, relative convergence, density-ordered blocks.
        Defaults restore the order-independent case A update."""
        self._check(_lib.rrt_set_update_rule(self._h, float(tau_skip), float(tau_case_b),
                                             int(bool(relative)), int(n_blocks)),
                    "rrt_set_update_rule")

    def evolve(self, dt: float, n_steps: int):
        """Non-equilibrium evolution: n_steps of dt seconds at the rate of each
        step's current state.  Returns x (input order)."""
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._check(_lib.rrt_evolve(self._h, float(dt), int(n_steps), _ptr(x)), "rrt_evolve")
        return x

    def set_scheme(self, near_far):
        """The paper's near/far scheme (True or 1), its variant that lights each
        ray's near slab with the whole far-attenuated spectrum (2), or the plain
        scheme (False or 0)."""
        self._check(_lib.rrt_set_scheme(self._h, int(near_far)), "rrt_set_scheme")

    def near_columns(self):
        """Near total-hydrogen columns [n, n_ray] of the last compute_columns."""
        out = torch.empty(self.n, self.n_ray, dtype=torch.float64, device=self.device)
        self._check(_lib.rrt_get_near_columns(self._h, _ptr(out)), "rrt_get_near_columns")
        return out

    def set_halos(self, offsets):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self._check(_lib.rrt_set_halos(self._h, off.size - 1, off.ctypes.data), "rrt_set_halos")
        self.n_halo = off.size - 1

    def iterate_halos(self, max_iter: int, tol: float, per_launch: int = 8, want_x: bool = True):
        x = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_x else None
        its = np.zeros(getattr(self, "n_halo", 1), np.int32)
        rc = self._check(_lib.rrt_iterate_halos(self._h, int(max_iter), float(tol), int(per_launch),
                                                _ptr(x), its.ctypes.data), "rrt_iterate_halos")
        return dict(x=x, halo_iters=its, converged=(rc == RRT_OK))

    def set_rays(self, dirs):
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        self._check(_lib.rrt_set_rays(self._h, d.shape[0], d.ctypes.data), "rrt_set_rays")
        self.n_ray = d.shape[0]

    def set_spectrum(self, sigma, w):
        s = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64))
        ww = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        if s.shape != ww.shape:
            raise ValueError("sigma and w must have the same length")
        self._check(_lib.rrt_set_spectrum(self._h, s.size, s.ctypes.data, ww.ctypes.data),
                    "rrt_set_spectrum")
        self.n_bins = s.size
        self.sigma = s

    def build_tree(self):
        self._check(_lib.rrt_build_tree(self._h), "rrt_build_tree")
        self._keep = []

    # -- the path ---------------------------------------------------------
    def compute_columns(self, want_N: bool = True, count: bool = True):
        N = torch.empty((self.n, self.n_ray), dtype=torch.float64, device=self.device) \
            if want_N else None
        hits = C.c_int64(0)
        self._check(_lib.rrt_compute_columns(self._h, _ptr(N), C.byref(hits) if count else None),
                    "rrt_compute_columns")
        return N, (hits.value if count else None)

    def compute_gamma(self):
        lnG = torch.empty(self.n, dtype=torch.float64, device=self.device)
        G = torch.empty_like(lnG)
        tau = torch.empty(self.n, dtype=torch.float32, device=self.device)
        self._check(_lib.rrt_compute_gamma(self._h, _ptr(lnG), _ptr(G), _ptr(tau)),
                    "rrt_compute_gamma")
        return lnG, G, tau

    def update_equilibrium(self):
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        md = C.c_double(0)
        self._check(_lib.rrt_update_equilibrium(self._h, _ptr(x), C.byref(md)),
                    "rrt_update_equilibrium")
        return x, md.value

    def iterate(self, max_iter: int, tol: float, want_x: bool = True):
        x = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_x else None
        it = C.c_int32(0)
        md = C.c_double(0)
        rc = self._check(_lib.rrt_iterate_equilibrium(self._h, int(max_iter), float(tol), _ptr(x),
                                                      C.byref(it), C.byref(md)),
                         "rrt_iterate_equilibrium")
        return dict(x=x, iters=it.value, max_dx=md.value, converged=(rc == RRT_OK))

    # -- reverse mode -----------------------------------------------------
    def set_density(self, n_H):
        nH = self._dev(n_H, torch.float32)
        if nH.numel() != self.n:
            raise ValueError("n_H must have n entries")
        self._check(_lib.rrt_set_density(self._h, _ptr(nH)), "rrt_set_density")
        torch.cuda.current_stream(self.device).synchronize()

    def forward(self, K: int):
        """Exactly K iterations from the thin state; keeps the iterates."""
        lnG = torch.empty(self.n, dtype=torch.float64, device=self.device)
        x = torch.empty_like(lnG)
        self._check(_lib.rrt_forward(self._h, int(K), _ptr(lnG), _ptr(x)), "rrt_forward")
        return lnG, x

    def backward(self, dL_dlnG=None, dL_dx=None):
        """Returns (dL/dw as float64 numpy [n_bins], dL/dn_H as a float64 tensor [n])."""
        gl = None if dL_dlnG is None else self._dev(dL_dlnG, torch.float64)
        gx = None if dL_dx is None else self._dev(dL_dx, torch.float64)
        nb = self.n_bins
        dw = np.zeros(nb, np.float64)
        dn = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._check(_lib.rrt_backward(self._h, _ptr(gl), _ptr(gx), dw.ctypes.data, _ptr(dn)),
                    "rrt_backward")
        return dw, dn

    def set_state(self, x=None):
        xs = None if x is None else self._dev(x, torch.float64)
        self._check(_lib.rrt_set_state(self._h, _ptr(xs)), "rrt_set_state")
        if xs is not None:
            torch.cuda.current_stream(self.device).synchronize()

    def get_state(self):
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        lnG, G = torch.empty_like(x), torch.empty_like(x)
        tau = torch.empty(self.n, dtype=torch.float32, device=self.device)
        self._check(_lib.rrt_get_state(self._h, _ptr(x), _ptr(lnG), _ptr(G), _ptr(tau)),
                    "rrt_get_state")
        return dict(x=x, lnG=lnG, G=G, tau=tau)

    # -- inspection -------------------------------------------------------
    def tree(self) -> dict:
        nn = C.c_int64(0)
        self._check(_lib.rrt_get_tree(self._h, 0, C.byref(nn), None, None, None, None, None,
                                      None, None), "rrt_get_tree")
        m = nn.value
        lo = np.zeros((m, 3), np.float32)
        hi = np.zeros((m, 3), np.float32)
        skip = np.zeros(m, np.int32)
        first = np.zeros(m, np.int32)
        count = np.zeros(m, np.int32)
        perm = np.zeros(self.n, np.int32)
        codes = np.zeros(self.n, np.uint64)
        self._check(_lib.rrt_get_tree(self._h, m, C.byref(nn), lo.ctypes.data, hi.ctypes.data,
                                      skip.ctypes.data, first.ctypes.data, count.ctypes.data,
                                      perm.ctypes.data, codes.ctypes.data), "rrt_get_tree")
        return dict(n_nodes=m, lo=lo, hi=hi, skip=skip, first=first, count=count, perm=perm,
                    codes=codes)

    def hits(self):
        off = np.zeros(self.n * self.n_ray + 1, np.int64)
        rc = _lib.rrt_get_hits(self._h, 0, off.ctypes.data, None, None)
        if rc not in (RRT_OK, -6):
            self._check(rc, "rrt_get_hits")
        total = int(off[-1])
        hj = np.zeros(max(total, 1), np.int32)
        hi = np.zeros(max(total, 1), np.int32)
        self._check(_lib.rrt_get_hits(self._h, total, off.ctypes.data, hj.ctypes.data,
                                      hi.ctypes.data), "rrt_get_hits")
        return off, hj[:total], hi[:total]

    def enable_timing(self, on: bool = True):
        self._check(_lib.rrt_enable_timing(self._h, 1 if on else 0), "rrt_enable_timing")

    def reset_timing(self):
        self._check(_lib.rrt_reset_timing(self._h), "rrt_reset_timing")

    def timing(self) -> dict:
        out = np.zeros(12)
        self._check(_lib.rrt_get_timing(self._h, out.ctypes.data), "rrt_get_timing")
        cnt = np.zeros(2, np.int64)
        self._check(_lib.rrt_get_counters(self._h, cnt.ctypes.data), "rrt_get_counters")
        return dict(trace_ms=out[0], rate_ms=out[1], build_ms=out[2], n_trace=int(out[3]),
                    record_ms=out[4], path_ms=out[5], n_path=int(out[6]),
                    path_hits=int(out[7]), tile_ms=out[8], n_tile=int(out[9]),
                    tile_build_ms=out[10], tile_set_total=int(out[11]),
                    last_hits=int(cnt[0]), total_hits=int(cnt[1]))

    # -- convenience ------------------------------------------------------
    @classmethod
    def from_workload(cls, wl, leaf_size: int = 0, block_size: int = 0, record_paths: int = -1,
                      path_budget: int = 0, traversal: int = 0, device=None, x_init=None,
                      build: bool = True) -> "Solver":
        s = cls(wl.l_ray, wl.box, leaf_size=leaf_size, block_size=block_size,
                record_paths=record_paths, path_budget=path_budget, traversal=traversal,
                device=device)
        s.set_particles(wl.pos, wl.h, wl.mu, wl.n_H, wl.T, x_init=x_init)
        if getattr(wl, "halo_offsets", None) is not None:
            s.set_halos(wl.halo_offsets)
        s.set_rays(wl.dirs)
        s.set_spectrum(wl.sigma, wl.w)
        if build:
            s.build_tree()
        return s
