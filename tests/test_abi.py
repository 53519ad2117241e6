"""The C-ABI library loads and exports every entry point include/rrt.h declares
(no GPU work: nothing here launches a kernel)."""
import os
import re

import numpy as np

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rrt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rrt_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_path():
    names = _declared()
    for need in ["rrt_create", "rrt_destroy", "rrt_set_particles", "rrt_set_rays",
                 "rrt_set_spectrum", "rrt_build_tree", "rrt_compute_columns",
                 "rrt_compute_gamma", "rrt_update_equilibrium", "rrt_iterate_equilibrium",
                 "rrt_last_error"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_1304_4235_amd as P
    lib = P.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(P.SIGNATURES)
    assert lib.rrt_version() >= 10000


def test_library_healpix_matches_generator():
    import paper_1304_4235_amd as P
    for ns in (1, 2, 3, 8):
        np.testing.assert_allclose(P.healpix_dirs(ns), W.healpix_dirs(ns), atol=2e-15, rtol=0)


def test_library_rejects_bad_healpix():
    import paper_1304_4235_amd as P
    out = np.zeros((12, 3))
    assert P.lib().rrt_healpix_dirs(0, out.ctypes.data) == -1
