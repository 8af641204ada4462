"""The C-ABI library loads and exports every entry point include/dfmm.h declares.

No GPU is needed: only argument validation paths that return before any HIP
call are exercised.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dfmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dfmm_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_1712_07739_amd as pk

    return pk.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    import paper_1712_07739_amd as pk

    assert set(pk.ENTRY_POINTS) == set(names)


def test_params_struct_matches_header_defaults(L):
    import paper_1712_07739_amd as pk

    p = pk.default_params()
    assert (p.order, p.depth, p.n_quad, p.n_circle, p.precision) == (5, 4, 3, 64, 0)
    assert abs(p.c11 - 3.5) < 1e-15 and abs(p.c12 - 1.5) < 1e-15 and p.c44 == 1.0
    assert p.box_size == 1.1 and list(p.box_lo) == [-0.05] * 3
    assert (p.m2l_mode, p.aniso_kernel, p.lsq_degree, p.leaf_max, p.freq_chunks) == (0, 0, 0, 0, 0)
    # layout: 2 ints, 4 doubles, 3 doubles, 1 double, 8 ints
    assert ctypes.sizeof(pk.Params) == 8 + 8 * 8 + 32


@pytest.mark.parametrize("field,value", [
    ("order", 1), ("order", 9), ("depth", 1), ("depth", 11), ("n_quad", 0), ("n_circle", 7),
    ("c44", -1.0), ("core_a", -1e-3), ("box_size", 0.0), ("precision", 3), ("m2l_mode", 2),
    ("aniso_kernel", 5), ("lsq_degree", 5), ("lsq_degree", -2), ("leaf_max", -1), ("freq_chunks", -1),
])
def test_setup_rejects_bad_parameters_before_touching_the_gpu(L, field, value):
    import paper_1712_07739_amd as pk

    p = pk.default_params()
    setattr(p, field, value)
    h = ctypes.c_void_p()
    rc = L.dfmm_fmm_setup(ctypes.byref(p), None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert len(L.dfmm_last_error()) > 0


def test_null_arguments_and_status_strings(L):
    assert L.dfmm_plan_info(None, None, 0) == -1
    assert L.dfmm_tree_set_timing(None, 1) == -1
    assert L.dfmm_fmm_forces(None, None, None, None, None, None) == -1
    assert L.dfmm_tree_check_positions(None, None, None, None) == -1
    L.dfmm_tree_destroy(None)
    L.dfmm_plan_destroy(None)
    for s, txt in ((0, b"ok"), (-4, b"point outside the root cube"), (-5, b"non-finite coordinate")):
        assert L.dfmm_status_string(s) == txt


def test_product_package_does_not_reference_the_oracle():
    """The product path never imports, loads or calls the oracle."""
    pkg = os.path.join(ROOT, "paper_1712_07739_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt and "dfmm_oracle" not in txt, f
