"""CPU checks of the C ABI boundary and of the oracle / product separation.

No compute call is made here (there is no GPU); the library is loaded and its
exported symbols are compared with the declarations in include/*.h.
"""

import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2111_00113_amd")
LIB = os.path.join(PKG, "libsgmres.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(sgmres_\w+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_solver_entry_points():
    names = declared_functions()
    for required in ("sgmres_solve", "sgmres_solve_transposed", "sgmres_solve_ex", "sgmres_arnoldi_cycle",
                     "sgmres_sketched_lsq", "sgmres_basis_combine", "sgmres_sketch_apply",
                     "sgmres_sketch_pattern", "sgmres_residual", "sgmres_csr_transpose"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgmres.so not built")
def test_library_loads_and_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sgmres_\w+)", out))
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgmres.so not built")
def test_library_is_gfx950_code():
    # the embedded device code object names its target triple
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_oracle_and_product_share_no_code():
    prod = glob.glob(os.path.join(PKG, "**", "*.*"), recursive=True)
    for path in prod:
        if not path.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
            continue
        text = open(path, errors="ignore").read()
        assert not re.search(r"^\s*(import|from)\s+oracle\b", text, flags=re.M), path
        assert "sgmres_oracle" not in text and "liboracle" not in text, path
    for path in glob.glob(os.path.join(ROOT, "oracle", "*.*")):
        if not path.endswith((".py", ".c", ".h")):
            continue
        text = open(path, errors="ignore").read()
        assert "paper_2111_00113_amd" not in text and "sgmres.h" not in text, path


def test_binding_raises_without_gpu_tensors():
    torch = pytest.importorskip("torch")
    import paper_2111_00113_amd as sg

    with pytest.raises(TypeError):
        sg.sgmres.__dict__["_check_dev"](torch.zeros(3, dtype=torch.float64))
