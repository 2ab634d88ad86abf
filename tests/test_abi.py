"""The C ABI library loads on a CPU-only host and exports every symbol the
header declares; the oracle and the product path stay separate."""
import ast
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(hyb(?:1d)?_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_header_symbols():
    from paper_1601_02708_amd import hyb
    lib = hyb.load()
    declared = header_functions()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(hyb.SIGNATURES) == declared
    out = subprocess.run(["nm", "-D", "--defined-only", hyb.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (hyb(?:1d)?_\w+)", out))
    assert set(declared) <= exported


def test_query_sizes_without_gpu():
    import ctypes
    from paper_1601_02708_amd import hyb
    lib = hyb.load()
    lat = hyb.HybLattice()
    lat.N, lat.precision, lat.eta = 2048, hyb.HYB_FP32, 10
    mesh = hyb.HybMesh(128, 4094.0, 0.0, 1, 1, None)
    fb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.hyb_query(ctypes.addressof(mesh), ctypes.addressof(lat), ctypes.addressof(fb),
                         ctypes.addressof(wb)) == hyb.HYB_OK
    assert fb.value >= 9 * 2048 * 2048 * 4 and fb.value % 256 == 0
    assert wb.value > 2048 * 2048 * 10
    lat.N = 2
    assert lib.hyb_query(None, ctypes.addressof(lat), ctypes.addressof(fb), ctypes.addressof(wb)) == hyb.HYB_EINVAL


def _imports(path):
    tree = ast.parse(open(path).read())
    names = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            names |= {a.name for a in node.names}
        elif isinstance(node, ast.ImportFrom):
            names.add(node.module or "")
            names |= {f"{node.module}.{a.name}" for a in node.names}
    return names


def test_product_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_1601_02708_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            assert not any(n.split(".")[0] == "oracle" for n in _imports(os.path.join(pkg, fn))), fn
    for fn in os.listdir(os.path.join(pkg, "csrc")):
        assert "oracle" not in open(os.path.join(pkg, "csrc", fn)).read().lower(), fn


def test_oracle_never_imports_product_kernels():
    od = os.path.join(ROOT, "oracle")
    for fn in os.listdir(od):
        if fn.endswith(".py"):
            for n in _imports(os.path.join(od, fn)):
                assert not n.startswith("paper_1601_02708_amd.hyb"), (fn, n)
                assert not n.startswith("paper_1601_02708_amd.csrc"), (fn, n)
        if fn.endswith(".c"):
            assert "hyb.h" not in open(os.path.join(od, fn)).read()


def test_hybrid1d_sizes_without_gpu():
    """The 1-D set-up of Sec. 7.1 (table row h_c = 1.25e-3, h_f = 6.25e-4,
    L_ov = 1e-2): 1/2 + L_ov/2 = 0.505 is node 404 of the coarse grid, the
    fine grid has 0.505 / 6.25e-4 = 808 cells, eta = 4; spacings that do not
    fit the interface points are rejected."""
    from paper_1601_02708_amd import hyb
    nc, nf, eta, xf0, ws = hyb.hybrid1d_sizes(1.25e-3, 6.25e-4, 1e-2, 10)
    assert (nc, nf, eta) == (405, 809, 4) and abs(xf0 - 0.495) < 1e-15 and ws % 256 == 0
    with pytest.raises(hyb.HybError):
        hyb.hybrid1d_sizes(1.25e-3, 5e-4, 1e-2, 10)          # (h_c / h_f)^2 not an integer
    with pytest.raises(hyb.HybError):
        hyb.hybrid1d_sizes(3e-3, 1.5e-3, 1e-2, 10)           # interface points off the grids
