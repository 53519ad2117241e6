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


def _header_text():
    txt = open(os.path.join(ROOT, "include", "rrt.h")).read()
    return re.sub(r"/\*.*?\*/", "", txt, flags=re.S)


def test_params_struct_matches_header():
    import ctypes as C
    from paper_1304_4235_amd.rrt import Params
    body = re.search(r"typedef struct \{(.*?)\}\s*rrt_params;", _header_text(), flags=re.S)
    assert body
    ctype = {"double": C.c_double, "int64_t": C.c_int64, "int32_t": C.c_int32}
    fields = []
    for typ, name, count in re.findall(r"(\w+)\s+(\w+)(?:\[(\d+)\])?\s*;", body.group(1)):
        t = ctype[typ]
        fields.append((name, t * int(count) if count else t))
    assert [f[0] for f in Params._fields_] == [f[0] for f in fields]
    for (_, got), (_, want) in zip(Params._fields_, fields):
        assert C.sizeof(got) == C.sizeof(want)
    assert C.sizeof(Params) == sum(C.sizeof(t) for _, t in fields)


def test_enums_match_header():
    from paper_1304_4235_amd.rrt import ERRORS, TUNE_KEYS
    txt = _header_text()
    tune = {m[0].lower(): int(m[1]) for m in re.findall(r"RRT_TUNE_(\w+)\s*=\s*(\d+)", txt)}
    # the binding's name for the adjoint knob says which form it picks
    tune["adjoint_scatter"] = tune.pop("adjoint")
    assert tune == TUNE_KEYS
    errs = {-int(v): "RRT_E_" + n for n, v in re.findall(r"RRT_E_(\w+)\s*=\s*-(\d+)", txt)}
    assert errs == ERRORS
