"""CPU-side checks of the C ABI: the library loads and exports every function
that include/lp_unwrap.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lp_unwrap.h")
LIB = os.path.join(ROOT, "paper_2203_13675_amd", "liblp_unwrap.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\([^;{]*\)\s*;",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2203_13675_amd import build_lib
        build_lib.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    for must in ("lp_unwrap_create", "lp_unwrap_solve", "lp_unwrap_batch", "lp_unwrap_destroy",
                 "lp_unwrap_status_string", "lpu_apply_A", "lpu_precond_apply"):
        assert must in names, names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_lists_every_export():
    from paper_2203_13675_amd import binding
    assert sorted(binding.EXPORTED) == declared_functions()


def test_status_strings_and_defaults(lib):
    lib.lp_unwrap_status_string.restype = ctypes.c_char_p
    for code in (0, 1, -1, -2, -3, -4, -5, 77):
        s = lib.lp_unwrap_status_string(code)
        assert s is not None and len(s) > 0
    from paper_2203_13675_amd import binding
    o = binding.default_options()
    # the paper's stopping parameters (Section 3) are the defaults
    assert o.k_max == 500 and o.outer_tol == 1e-6 and o.eps_cg == 0.005
    assert o.l_max == 0 and o.residual_period == 0       # 0 -> 2MN and floor(sqrt(MN))
    assert o.ssor_omega == 1.0


def test_struct_layouts_match_header():
    """Field order and sizes of the ctypes mirrors follow the header."""
    from paper_2203_13675_amd import binding
    text = open(HEADER).read()
    for cls, cname in ((binding.LpuOptions, "lpu_options"), (binding.LpuStats, "lpu_stats"),
                       (binding.LpuMap, "lpu_map"), (binding.LpuTuning, "lpu_tuning")):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), text, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            parts = decl.replace("*", " ").split()
            names = " ".join(parts[1:]) if parts[0] != "const" else " ".join(parts[2:])
            if parts[0] in ("long",):
                names = " ".join(parts[2:])
            fields += [x.strip() for x in names.split(",")]
        assert [f for f, _ in cls._fields_] == fields, (cname, fields)


def test_default_tuning(lib):
    from paper_2203_13675_amd import binding
    t = binding.LpuTuning()
    lib.lpu_default_tuning(ctypes.byref(t))
    assert t.as_dict() == {"tile_rows": 16, "grid": 16384, "dct_grid": 2048, "use_graph": 1,
                           "max_batch_iters": 64}
