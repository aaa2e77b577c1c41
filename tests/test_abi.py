"""Host-side checks of the C ABI: the library loads and exports every function
declared in include/wcmg.h; the ctypes parameter struct matches the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wcmg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wcmg_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("wcmg_create", "wcmg_set_gauge", "wcmg_setup", "wcmg_refine", "wcmg_apply_D", "wcmg_restrict",
              "wcmg_prolong", "wcmg_solve", "wcmg_get_coarse_op", "wcmg_coarse_apply"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1904_08678_amd import wcmg
    if not os.path.exists(wcmg.library_path):
        pytest.skip("library not built")
    lib = ctypes.CDLL(wcmg.library_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_params_struct_matches_defaults():
    from paper_1904_08678_amd import wcmg
    if not os.path.exists(wcmg.library_path):
        pytest.skip("library not built")
    p = wcmg.default_params()
    assert tuple(p.dims) == (8, 8, 8, 8)
    assert p.outer_tol == 1e-10 and p.coarse_tol == 0.05 and p.kcycle_tol == 0.1
    assert p.n_levels == 2 and p.relax_sweeps == 20 and p.post_smooth == 4 and p.outer_restart == 20
    assert ctypes.sizeof(wcmg.Params) == 200  # sizeof(wcmg_params) from the C compiler


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1904_08678_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "wcmg_oracle" not in src, f
