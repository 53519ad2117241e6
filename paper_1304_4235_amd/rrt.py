"""ctypes binding of librrt.so (declared in include/rrt.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device memory comes from torch tensors on the current CUDA/HIP device: the
context's workspace and its path buffer are torch uint8 tensors that the
Solver sizes with the library's own queries (rrt_workspace_size,
rrt_count_paths) and hands over; work is enqueued on torch's current stream.
If the library is missing this module raises at import time; there is no
fallback path.
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
             "tiles": 6, "keep_columns": 7, "one_pass": 8, "packet_queue": 9}
RRT_E_WORKSPACE, RRT_E_CAPACITY = -5, -6
ERRORS = {-1: "RRT_E_ARG", -2: "RRT_E_HIP", -3: "RRT_E_INPUT", -4: "RRT_E_STATE",
          -5: "RRT_E_WORKSPACE", -6: "RRT_E_CAPACITY"}
N_REC_STATS = 5


class RRTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("l_ray", C.c_double), ("box", C.c_double), ("leaf_size", C.c_int32),
                ("block_size", C.c_int32), ("record_paths", C.c_int32),
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
    "rrt_get_timing": ([_vp, _vp, _i32], C.c_int),
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
    "rrt_workspace_size": ([_vp, _i64, _i32, _i32, _i32, _i32, _vp], C.c_int),
    "rrt_set_workspace": ([_vp, _vp, C.c_size_t], C.c_int),
    "rrt_workspace_info": ([_vp, _vp], C.c_int),
    "rrt_count_paths": ([_vp, _vp, _vp, _vp], C.c_int),
    "rrt_set_path_buffer": ([_vp, _vp, C.c_size_t], C.c_int),
    "rrt_get_convergence": ([_vp, _i32, _vp, _vp, _vp, _vp], C.c_int),
    "rrt_get_halo_roots": ([_vp, _vp, _vp], C.c_int),
    "rrt_get_hits_rows": ([_vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp], C.c_int),
    "rrt_get_path_rows": ([_vp, _i32, _vp, _i64, _vp, _vp, _vp], C.c_int),
    "rrt_get_hits_rows_noalloc": ([_vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp], C.c_int),
    "rrt_get_recording_stats": ([_vp, _vp, _i32], C.c_int),
    "rrt_trace_stats": ([_vp, _vp], C.c_int),
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
    """One reverse-ray-tracing problem on one GPU (a context of librrt).

    The Solver owns the context's device memory as torch tensors: a workspace
    (rrt_workspace_size) that grows, by a move inside the library, when the
    problem does, and a path buffer for the recorded ray paths, sized after
    each new geometry from rrt_count_paths within `path_budget` bytes (0: 60%
    of the device memory torch can still hand out).
    """

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
        p = Params(float(l_ray), float(box), int(leaf_size), int(block_size),
                   int(record_paths), int(traversal), (C.c_int32 * 2)())
        h = C.c_void_p()
        rc = _lib.rrt_create(C.byref(h), C.byref(p), C.c_void_p(self.stream.cuda_stream))
        if rc != RRT_OK:
            raise RRTError(rc, _lib.rrt_last_error(None).decode())
        self._h = h
        self.n = 0
        self.n_ray = 0
        self.n_bins = 0
        self.n_halo = 1
        self.record_paths = int(record_paths)
        self.path_budget = int(path_budget)
        self._K = 0
        self._keep = []
        self._ws = None
        self._path = None
        self._unfit_seen = 0
        self._ensure_ws()

    # -- plumbing ---------------------------------------------------------
    def _check(self, rc: int, what: str) -> int:
        if rc < 0:
            raise RRTError(rc, f"{what}: {_lib.rrt_last_error(self._h).decode()}")
        return rc

    def _call(self, name: str, *args) -> int:
        """Call an entry point; when it finds too little room in the workspace
        (RRT_E_WORKSPACE, before it changed any state), grow the workspace by
        what it asked for and call it once more.  The growth is past the
        current end, so the request fits in one piece however the used blocks
        are spread."""
        fn = getattr(_lib, name)
        rc = fn(self._h, *args)
        for _ in range(2):
            if rc != RRT_E_WORKSPACE:
                break
            info = self.workspace_info()
            if info["short_region"] != 0 or info["short_bytes"] == 0:
                break
            self._grow_ws(max(info["ws_used"], info["ws_size"]) + info["short_bytes"])
            rc = fn(self._h, *args)
        return self._check(rc, name)

    def workspace_size(self, n=None, n_ray=None, n_bins=None, n_halo=None, K=None) -> int:
        b = C.c_size_t(0)
        rc = _lib.rrt_workspace_size(
            self._h, int(self.n if n is None else n), int(self.n_ray if n_ray is None else n_ray),
            int(self.n_bins if n_bins is None else n_bins),
            int(self.n_halo if n_halo is None else n_halo), int(self._K if K is None else K),
            C.byref(b))
        self._check(rc, "rrt_workspace_size")
        return int(b.value)

    def workspace_info(self) -> dict:
        out = (C.c_size_t * 6)()
        self._check(_lib.rrt_workspace_info(self._h, out), "rrt_workspace_info")
        return dict(ws_used=int(out[0]), ws_size=int(out[1]), path_used=int(out[2]),
                    path_size=int(out[3]), short_bytes=int(out[4]),
                    short_region=C.c_ssize_t(out[5]).value)

    def _grow_ws(self, need: int):
        """A workspace of at least `need` bytes (with some room to spare); the
        library moves its buffers into it."""
        have = 0 if self._ws is None else self._ws.numel()
        if need <= have:
            return
        size = int(need * 1.05) + (16 << 20)
        size = (size + 4095) // 4096 * 4096
        try:
            ws = torch.empty(size, dtype=torch.uint8, device=self.device)
        except torch.OutOfMemoryError:
            torch.cuda.empty_cache()                 # cached blocks too fragmented
            ws = torch.empty(size, dtype=torch.uint8, device=self.device)
        self._check(_lib.rrt_set_workspace(self._h, C.c_void_p(ws.data_ptr()), size),
                    "rrt_set_workspace")
        self._ws = ws

    def _ensure_ws(self, **sizes):
        self._grow_ws(self.workspace_size(**sizes))

    def _free_bytes(self) -> int:
        free, _ = torch.cuda.mem_get_info(self.device)
        cached = torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
        return int(free + max(cached, 0))

    def set_path_buffer(self, nbytes, fallbacks=()) -> int:
        """Give the context a path buffer of nbytes (0: none).  When the device
        cannot hand out that much, try each smaller size of `fallbacks` in
        turn (then none).  Returns the size given."""
        self._check(_lib.rrt_set_path_buffer(self._h, None, 0), "rrt_set_path_buffer")
        self._path = None                      # the old buffer goes back to torch first
        for size in [int(nbytes), *[int(f) for f in fallbacks]]:
            if size <= 0:
                return 0
            size = (size + 4095) // 4096 * 4096
            try:
                buf = torch.empty(size, dtype=torch.uint8, device=self.device)
            except torch.OutOfMemoryError:
                torch.cuda.empty_cache()
                try:
                    buf = torch.empty(size, dtype=torch.uint8, device=self.device)
                except torch.OutOfMemoryError:
                    continue
            self._check(_lib.rrt_set_path_buffer(self._h, C.c_void_p(buf.data_ptr()), size),
                        "rrt_set_path_buffer")
            self._path = buf
            return size
        return 0

    def count_paths(self) -> dict:
        """The counting walk of rrt_count_paths: intersections and the path
        buffer sizes they need."""
        hits, need, one = C.c_int64(0), C.c_size_t(0), C.c_size_t(0)
        self._call("rrt_count_paths", C.byref(hits), C.byref(need), C.byref(one))
        return dict(hits=int(hits.value), bytes_paths=int(need.value),
                    bytes_one_walk=int(one.value))

    def _plan_paths(self):
        """After a new tree: give the context a path buffer when the paths are
        to be recorded.  A buffer already there is kept (the library records
        into it, in one walk when there is room) unless a recording did not
        fit it since it was sized."""
        if self.record_paths == 0:
            return
        unfit = self.recording_stats()[4]
        if self._path is not None and unfit == self._unfit_seen:
            return
        self._unfit_seen = unfit
        cnt = self.count_paths()
        have = 0 if self._path is None else self._path.numel()
        budget = self.path_budget or int(0.6 * (self._free_bytes() + have))
        need, one = cnt["bytes_paths"], cnt["bytes_one_walk"]
        # room for the one-walk pool and, after it, for the reverse mode's
        # transposed paths (32 bytes per intersection while they are built)
        want = max(one, 5 * need)
        if self.record_paths == 1:
            # required: at least the paths, unless an explicit budget says no
            # (then the library reports RRT_E_WORKSPACE)
            size = min(want, budget if self.path_budget else max(budget, need))
        elif self.n_halo > 1:
            # a batch whose paths do not fit at once is solved in groups of
            # halos whose paths fit the buffer
            size = min(want, budget)
        else:
            size = min(want, budget) if need <= budget else 0
        # smaller sizes when the device cannot hand out that much: the paths
        # with the one-walk pool, then the paths alone (a batch: half as much)
        smaller = [f for f in (one, need) if f < size] or ([size // 2] if self.n_halo > 1 else [])
        self.set_path_buffer(size, smaller)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.rrt_destroy(self._h)
            self._h = None
        self._ws = None
        self._path = None

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
        if n >= 1:
            self._ensure_ws(n=n, n_halo=1)
        self._call("rrt_set_particles", n, _ptr(pos), _ptr(h), _ptr(mu), _ptr(nH), _ptr(T),
                   _ptr(xi))
        self._keep = [pos, h, mu, nH, T, xi]      # copied by the library; kept until synced
        self.n = n
        self.n_halo = 1

    def set_tuning(self, **kw):
        """Launch knobs: trace_block, packet (1 or 64), path_group, leaf, adjoint_scatter (0/1),
        tiles (0/1), keep_columns (0/1), one_pass (0, 1 or a pool size in chunks),
        packet_queue (0/1)."""
        for k, v in kw.items():
            self._call("rrt_set_tuning", TUNE_KEYS[k], int(v))

    def set_update_rule(self, tau_skip: float = 0.0, tau_case_b: float = float("inf"),
                        relative: bool = False, n_blocks: int = 1):
        """The paper's update rule for iterate(): frozen thin particles, case B
        above a tau_eff threshold, relative convergence, density-ordered blocks.
        Defaults restore the order-independent case A update."""
        self._call("rrt_set_update_rule", float(tau_skip), float(tau_case_b),
                   int(bool(relative)), int(n_blocks))

    def evolve(self, dt: float, n_steps: int):
        """Non-equilibrium evolution: n_steps of dt seconds at the rate of each
        step's current state.  Returns x (input order)."""
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._call("rrt_evolve", float(dt), int(n_steps), _ptr(x))
        return x

    def set_scheme(self, near_far):
        """The paper's near/far scheme (True or 1) or the plain scheme (False or 0)."""
        v = int(near_far)
        self._call("rrt_set_scheme", v)
        self._ensure_ws()                      # the near columns

    def near_columns(self):
        """Near total-hydrogen columns [n, n_ray] of the last compute_columns."""
        out = torch.empty(self.n, self.n_ray, dtype=torch.float64, device=self.device)
        self._call("rrt_get_near_columns", _ptr(out))
        return out

    def set_halos(self, offsets):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self._ensure_ws(n_halo=off.size - 1)
        self._call("rrt_set_halos", off.size - 1, off.ctypes.data)
        self.n_halo = off.size - 1

    def iterate_halos(self, max_iter: int, tol: float, per_launch: int = 8, want_x: bool = True):
        x = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_x else None
        its = np.zeros(self.n_halo, np.int32)
        rc = self._call("rrt_iterate_halos", int(max_iter), float(tol), int(per_launch), _ptr(x),
                        its.ctypes.data)
        return dict(x=x, halo_iters=its, converged=(rc == RRT_OK))

    def set_rays(self, dirs):
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        if d.shape[0] >= 1:
            self._ensure_ws(n_ray=d.shape[0])
        self._call("rrt_set_rays", d.shape[0], d.ctypes.data)
        self.n_ray = d.shape[0]

    def set_spectrum(self, sigma, w):
        s = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64))
        ww = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        if s.shape != ww.shape:
            raise ValueError("sigma and w must have the same length")
        if s.size >= 1:
            self._ensure_ws(n_bins=s.size)
        self._call("rrt_set_spectrum", s.size, s.ctypes.data, ww.ctypes.data)
        self.n_bins = s.size
        self.sigma = s

    def build_tree(self):
        self._call("rrt_build_tree")
        self._keep = []
        self._plan_paths()

    # -- the path ---------------------------------------------------------
    def compute_columns(self, want_N: bool = True, count: bool = True):
        N = torch.empty((self.n, self.n_ray), dtype=torch.float64, device=self.device) \
            if want_N else None
        hits = C.c_int64(0)
        self._call("rrt_compute_columns", _ptr(N), C.byref(hits) if count else None)
        return N, (hits.value if count else None)

    def compute_gamma(self):
        lnG = torch.empty(self.n, dtype=torch.float64, device=self.device)
        G = torch.empty_like(lnG)
        tau = torch.empty(self.n, dtype=torch.float32, device=self.device)
        self._call("rrt_compute_gamma", _ptr(lnG), _ptr(G), _ptr(tau))
        return lnG, G, tau

    def update_equilibrium(self):
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        md = C.c_double(0)
        self._call("rrt_update_equilibrium", _ptr(x), C.byref(md))
        return x, md.value

    def iterate(self, max_iter: int, tol: float, want_x: bool = True):
        x = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_x else None
        it = C.c_int32(0)
        md = C.c_double(0)
        rc = self._call("rrt_iterate_equilibrium", int(max_iter), float(tol), _ptr(x),
                        C.byref(it), C.byref(md))
        return dict(x=x, iters=it.value, max_dx=md.value, converged=(rc == RRT_OK))

    def convergence(self) -> dict:
        """Per sweep of the last iterate(): the largest change and the numbers of
        particles whose change was below tol, absolutely and relative to x."""
        m = C.c_int32(0)
        self._call("rrt_get_convergence", 0, C.byref(m), None, None, None)
        k = m.value
        md, na, nr = np.zeros(k), np.zeros(k, np.int64), np.zeros(k, np.int64)
        self._call("rrt_get_convergence", k, C.byref(m), md.ctypes.data, na.ctypes.data,
                   nr.ctypes.data)
        return dict(max_dx=md, n_abs=na, n_rel=nr)

    # -- reverse mode -----------------------------------------------------
    def set_density(self, n_H):
        nH = self._dev(n_H, torch.float32)
        if nH.numel() != self.n:
            raise ValueError("n_H must have n entries")
        self._call("rrt_set_density", _ptr(nH))
        torch.cuda.current_stream(self.device).synchronize()

    def forward(self, K: int):
        """Exactly K iterations from the thin state; keeps the iterates."""
        if int(K) > self._K:
            self._K = int(K)
            self._ensure_ws()
        lnG = torch.empty(self.n, dtype=torch.float64, device=self.device)
        x = torch.empty_like(lnG)
        self._call("rrt_forward", int(K), _ptr(lnG), _ptr(x))
        self.generation = getattr(self, "generation", 0) + 1
        return lnG, x

    def backward(self, dL_dlnG=None, dL_dx=None):
        """Returns (dL/dw as float64 numpy [n_bins], dL/dn_H as a float64 tensor [n])."""
        gl = None if dL_dlnG is None else self._dev(dL_dlnG, torch.float64)
        gx = None if dL_dx is None else self._dev(dL_dx, torch.float64)
        nb = self.sigma.size
        dw = np.zeros(nb, np.float64)
        dn = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._call("rrt_backward", _ptr(gl), _ptr(gx), dw.ctypes.data, _ptr(dn))
        return dw, dn

    def set_state(self, x=None):
        xs = None if x is None else self._dev(x, torch.float64)
        self._call("rrt_set_state", _ptr(xs))
        if xs is not None:
            torch.cuda.current_stream(self.device).synchronize()

    def get_state(self):
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        lnG, G = torch.empty_like(x), torch.empty_like(x)
        tau = torch.empty(self.n, dtype=torch.float32, device=self.device)
        self._call("rrt_get_state", _ptr(x), _ptr(lnG), _ptr(G), _ptr(tau))
        return dict(x=x, lnG=lnG, G=G, tau=tau)

    # -- inspection -------------------------------------------------------
    def tree(self) -> dict:
        nn = C.c_int64(0)
        self._call("rrt_get_tree", 0, C.byref(nn), None, None, None, None, None, None, None)
        m = nn.value
        lo = np.zeros((m, 3), np.float32)
        hi = np.zeros((m, 3), np.float32)
        skip = np.zeros(m, np.int32)
        first = np.zeros(m, np.int32)
        count = np.zeros(m, np.int32)
        perm = np.zeros(self.n, np.int32)
        codes = np.zeros(self.n, np.uint64)
        self._call("rrt_get_tree", m, C.byref(nn), lo.ctypes.data, hi.ctypes.data,
                   skip.ctypes.data, first.ctypes.data, count.ctypes.data, perm.ctypes.data,
                   codes.ctypes.data)
        out = dict(n_nodes=m, lo=lo, hi=hi, skip=skip, first=first, count=count, perm=perm,
                   codes=codes)
        if self.n_halo > 1:
            root = np.zeros(self.n_halo, np.int32)
            end = np.zeros(self.n_halo, np.int32)
            self._call("rrt_get_halo_roots", root.ctypes.data, end.ctypes.data)
            out.update(seg_root=root, seg_end=end)
        return out

    def hits(self):
        off = np.zeros(self.n * self.n_ray + 1, np.int64)
        self._call("rrt_get_hits", 0, off.ctypes.data, None, None)
        total = int(off[-1])
        self._ensure_ws()
        self._grow_ws(self.workspace_info()["ws_used"] + 8 * (total + off.size) + (64 << 20))
        hj = np.zeros(max(total, 1), np.int32)
        hi = np.zeros(max(total, 1), np.int32)
        self._call("rrt_get_hits", total, off.ctypes.data, hj.ctypes.data, hi.ctypes.data)
        return off, hj[:total], hi[:total]

    def hits_rows(self, sources):
        """Hit lists of every ray of the given sources (input indices), from
        the wave-cooperative walk: (row_off [n_src * n_ray + 1], hit_j, hit_img,
        hit_fac) with the rays of sources[i] at rows i * n_ray + k."""
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int64))
        off = np.zeros(src.size * self.n_ray + 1, np.int64)
        self._call("rrt_get_hits_rows", src.size, src.ctypes.data, 0, off.ctypes.data, None, None,
                   None)
        total = int(off[-1])
        hj = np.zeros(max(total, 1), np.int32)
        hi = np.zeros(max(total, 1), np.int32)
        hf = np.zeros(max(total, 1), np.float32)
        self._call("rrt_get_hits_rows", src.size, src.ctypes.data, total, off.ctypes.data,
                   hj.ctypes.data, hi.ctypes.data, hf.ctypes.data)
        return off, hj[:total], hi[:total], hf[:total]

    def path_rows(self, sources):
        """The recorded paths of every ray of the given sources: (row_off,
        hit_j, hit_fac) laid out as in hits_rows."""
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int64))
        off = np.zeros(src.size * self.n_ray + 1, np.int64)
        self._call("rrt_get_path_rows", src.size, src.ctypes.data, 0, off.ctypes.data, None,
                   None)
        total = int(off[-1])
        hj = np.zeros(max(total, 1), np.int32)
        hf = np.zeros(max(total, 1), np.float32)
        self._call("rrt_get_path_rows", src.size, src.ctypes.data, total, off.ctypes.data,
                   hj.ctypes.data, hf.ctypes.data)
        return off, hj[:total], hf[:total]

    def recording_stats(self) -> np.ndarray:
        """Path recordings: [one walk, one walk + fallback walk, after a count,
        count + record walks, did not fit]."""
        out = np.zeros(N_REC_STATS, np.int64)
        self._call("rrt_get_recording_stats", out.ctypes.data, N_REC_STATS)
        return out

    def trace_stats(self) -> dict:
        out = np.zeros(6, np.int64)
        self._call("rrt_trace_stats", out.ctypes.data)
        return dict(rays=int(out[0]), packet_node_visits=int(out[1]),
                    ray_node_visits=int(out[2]), packet_leaf_visits=int(out[3]),
                    pair_tests=int(out[4]), hits=int(out[5]))

    def enable_timing(self, on: bool = True):
        self._call("rrt_enable_timing", 1 if on else 0)

    def reset_timing(self):
        self._call("rrt_reset_timing")

    def timing(self) -> dict:
        out = np.zeros(16)
        self._call("rrt_get_timing", out.ctypes.data, 16)
        cnt = np.zeros(2, np.int64)
        self._call("rrt_get_counters", cnt.ctypes.data)
        return dict(trace_ms=out[0], rate_ms=out[1], build_ms=out[2], n_trace=int(out[3]),
                    record_ms=out[4], path_ms=out[5], n_path=int(out[6]),
                    path_hits=int(out[7]), tile_ms=out[8], n_tile=int(out[9]),
                    tile_build_ms=out[10], tile_set_total=int(out[11]),
                    chunk_walk_ms=out[12], n_chunk_walk=int(out[13]), compact_ms=out[14],
                    other_walk_ms=out[15], last_hits=int(cnt[0]), total_hits=int(cnt[1]))

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
