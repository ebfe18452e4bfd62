"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments on the host, and plans the nested
dissection correctly."""
import ctypes
import os
import re

import pytest

import paper_2408_03571_amd as hs
from paper_2408_03571_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helmschwarz.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:hs_status|int64_t|void|const char\*)\s+(hs_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


@pytest.mark.parametrize("n,k,bc", [(4, 10.0, 1), (3, 10.0, 1), (65, 0.0, 1), (65, 10.0, 7), (64, 1.0, 0)])
def test_assemble_rejects_bad_arguments(n, k, bc):
    lib = _lib.load()
    out = ctypes.c_void_p()
    assert lib.hs_assemble(n, k, bc, None, ctypes.byref(out)) == _lib.HS_EINVAL
    assert not out.value
    assert len(lib.hs_last_error()) > 0


def test_assemble_sizes():
    P = hs.hs_assemble(65, 20.0, hs.HS_BC_DIRICHLET)
    assert hs.hs_problem_size(P) == 63 * 63
    Q = hs.hs_assemble(257, 80.0, hs.HS_BC_SOMMERFELD)
    assert hs.hs_problem_size(Q) == 257 * 257


@pytest.mark.parametrize("n,nsub,overlap,ratio,variant,prec,msg", [
    (65, 0, 2, 2, 1, 0, "nsub"), (65, 4, -1, 2, 1, 0, "overlap"), (65, 4, 2, 3, 1, 0, "power of two"),
    (65, 4, 2, 128, 1, 0, "divisible"), (65, 4, 2, 2, 5, 0, "variant"), (65, 4, 2, 2, 1, 9, "prec"),
    (65, 40, 2, 2, 1, 0, "narrower"), (257, 2, 2, 2, 1, 0, "longer than 72"), (65, 70, 0, 2, 1, 0, "empty"),
])
def test_setup_rejects_bad_arguments(n, nsub, overlap, ratio, variant, prec, msg):
    """All of these are rejected on the host before any device work, so they
    run on a machine without a GPU."""
    P = hs.hs_assemble(n, 20.0, hs.HS_BC_SOMMERFELD)
    lib = _lib.load()
    out = ctypes.c_void_p()
    st = lib.hs_setup_schwarz(P.handle, nsub, overlap, ratio, variant, prec, None, ctypes.byref(out))
    assert st == _lib.HS_EINVAL
    assert msg in lib.hs_last_error().decode()


@pytest.mark.parametrize("basis", [-1, 2, 7])
def test_setup_rejects_unknown_basis(basis):
    P = hs.hs_assemble(65, 20.0, hs.HS_BC_SOMMERFELD)
    lib = _lib.load()
    out = ctypes.c_void_p()
    st = lib.hs_setup_schwarz_ex(P.handle, 4, 2, 2, 1, 0, basis, None, ctypes.byref(out))
    assert st == _lib.HS_EINVAL
    assert "basis" in lib.hs_last_error().decode()
    assert not out.value


def test_gmres_workspace_grows_with_maxit():
    P = hs.hs_assemble(65, 20.0, hs.HS_BC_SOMMERFELD)
    a = hs.hs_gmres_workspace_bytes(P, 10)
    b = hs.hs_gmres_workspace_bytes(P, 20)
    assert b > a >= 21 * 65 * 65 * 16
    with pytest.raises(hs.HSError):
        hs.hs_gmres_workspace_bytes(P, 0)


@pytest.mark.parametrize("ncx,ncy,reach,leaf", [(31, 31, 2, 8), (33, 33, 2, 8), (65, 65, 2, 8),
                                                (17, 17, 3, 8), (33, 33, 3, 6), (5, 7, 2, 4), (1, 1, 2, 8),
                                                (40, 9, 2, 5), (129, 129, 2, 8), (33, 33, 1, 8),
                                                (81, 81, 1, 8), (7, 5, 1, 3)])
def test_nested_dissection_plan(ncx, ncy, reach, leaf):
    st = hs.hs_nd_plan_check(ncx, ncy, reach, leaf)
    assert st["fronts"] >= 1
    assert st["max_nF"] == st["max_nF"]


def test_nested_dissection_precision_config_sizes():
    """Coarse grid of the n = 1025, H = 2h workload: the largest front must fit
    the kernels' limits (separator of 2 x 513 nodes)."""
    st = hs.hs_nd_plan_check(513, 513, 2, 8)
    assert st["max_nI"] <= 1152 and st["max_nB"] <= 2048
