"""The C-ABI library loads without a GPU and exports every function include/mg.h declares."""

import ctypes
import os
import re

import paper_1406_5369_amd as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "mg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ["mg_setup", "mg_vcycle", "mg_solve", "mg_residual_norm", "mg_destroy", "mg_strerror",
                     "mg_level_smooth", "mg_level_residual_restrict", "mg_level_prolong_correct",
                     "mg_level_coarsest", "mg_level_ir_update"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(mg.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    lib = mg.lib()
    for n in declared():
        assert getattr(lib, n).argtypes is not None or n in ("mg_strerror",), n


def test_status_strings_without_gpu():
    assert mg.strerror(0) == "ok"
    assert "diverged" in mg.strerror(mg.MG_EDIVERGED)
    assert mg.strerror(12345) == "unknown status"


def test_params_defaults_follow_the_paper():
    p = mg.Params(dim=3, n=33)
    assert (p.nu1, p.nu2, p.omega, p.smoother) == (2, 2, 1.0, mg.SMOOTH_RBGS)
    assert mg.Params(dim=2, n=9, smoother=mg.SMOOTH_JACOBI).omega == 0.8
