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
    (65, 0, 2, 2, 1, 0, "nsub"), (65, (4, 0), 2, 2, 1, 0, "nsub_y"), (65, (0, 4), 2, 2, 1, 0, "nsub_x"),
    (65, 4, -1, 2, 1, 0, "overlap"), (65, 4, 2, 3, 1, 0, "power of two"),
    (65, 4, 2, 128, 1, 0, "divisible"), (65, 4, 2, 2, 5, 0, "variant"), (65, 4, 2, 2, 1, 9, "prec"),
    (65, 40, 2, 2, 1, 0, "narrower"), (65, (4, 40), 2, 2, 1, 0, "narrower"), (257, 2, 2, 2, 1, 0, "longer than 96"), (193, 2, 2, 2, 1, 0, "longer than 96"),
    (65, 70, 0, 2, 1, 0, "empty"),
])
def test_setup_rejects_bad_arguments(n, nsub, overlap, ratio, variant, prec, msg):
    """All of these are rejected on the host before any device work (the size
    query and the set-up run the same validation; the set-up is handed a
    workspace address that must never be touched), so they run on a machine
    without a GPU."""
    P = hs.hs_assemble(n, 20.0, hs.HS_BC_SOMMERFELD)
    lib = _lib.load()
    nsx, nsy = (nsub, nsub) if isinstance(nsub, int) else nsub
    nb = ctypes.c_size_t()
    st = lib.hs_schwarz_workspace_bytes_ex(P.handle, nsx, nsy, overlap, ratio, variant, prec, 0, ctypes.byref(nb))
    assert st == _lib.HS_EINVAL
    assert msg in lib.hs_last_error().decode()
    out = ctypes.c_void_p()
    st = lib.hs_setup_schwarz(P.handle, nsx, nsy, overlap, ratio, variant, prec, ctypes.c_void_p(1 << 40),
                              ctypes.c_size_t(1 << 50), None, ctypes.byref(out))
    assert st == _lib.HS_EINVAL
    assert msg in lib.hs_last_error().decode()
    assert not out.value


@pytest.mark.parametrize("basis", [-1, 2, 7])
def test_setup_rejects_unknown_basis(basis):
    P = hs.hs_assemble(65, 20.0, hs.HS_BC_SOMMERFELD)
    lib = _lib.load()
    out = ctypes.c_void_p()
    st = lib.hs_setup_schwarz_ex(P.handle, 4, 4, 2, 2, 1, 0, basis, ctypes.c_void_p(1 << 40), ctypes.c_size_t(1 << 50),
                                 None, ctypes.byref(out))
    assert st == _lib.HS_EINVAL
    assert "basis" in lib.hs_last_error().decode()
    assert not out.value


@pytest.mark.parametrize("ws,nbytes,msg", [(None, 1 << 50, "NULL"), (1 << 40 | 128, 1 << 50, "aligned"),
                                           (1 << 40, 4096, "too small")])
def test_setup_rejects_bad_workspaces(ws, nbytes, msg):
    """A missing, misaligned or short workspace is refused before any device
    work (the address is never dereferenced)."""
    P = hs.hs_assemble(65, 20.0, hs.HS_BC_SOMMERFELD)
    lib = _lib.load()
    out = ctypes.c_void_p()
    st = lib.hs_setup_schwarz(P.handle, 4, 4, 2, 2, 1, 0, ctypes.c_void_p(ws) if ws else None,
                              ctypes.c_size_t(nbytes), None, ctypes.byref(out))
    assert st == _lib.HS_EINVAL
    assert msg in lib.hs_last_error().decode()
    assert not out.value


def test_schwarz_workspace_sizes():
    """The workspace query (host only) against what it must hold: it covers
    the local factors and the coarse factor the set-up stores, grows with the
    problem, and its variant-free form is the largest of the exact ones."""
    lib = _lib.load()

    def ex(P, nsx, nsy, variant, prec, basis, ratio=2):
        nb = ctypes.c_size_t()
        assert lib.hs_schwarz_workspace_bytes_ex(P.handle, nsx, nsy, 2, ratio, variant, prec, basis,
                                                 ctypes.byref(nb)) == 0
        return nb.value

    P = hs.hs_assemble(257, 80.0, hs.HS_BC_SOMMERFELD)
    ras = ex(P, 4, 4, hs.HS_RAS2, hs.HS_C64, hs.HS_COARSE_BEZIER)
    shs = ex(P, 4, 4, hs.HS_SHS2, hs.HS_C64, hs.HS_COARSE_BEZIER)
    p1 = ex(P, 4, 4, hs.HS_RAS2, hs.HS_C64, hs.HS_COARSE_P1)
    assert shs - ras >= 2 * 257 * 257 * 16       # SHS2 keeps e and r - A e
    assert p1 < ras                               # 9-point coarse rows instead of 25
    assert hs.hs_schwarz_workspace_bytes(P, 4, 2, 2, hs.HS_C64) == max(ras, shs, p1)
    # complex128 factors: twice the local factor bytes (68^2 per line, 68 lines, 16 subdomains of 4 x 4)
    c128 = ex(P, 4, 4, hs.HS_RAS2, hs.HS_C128, hs.HS_COARSE_BEZIER)
    assert c128 - ras >= 16 * 68 * 68 * 68 * 8 * 0.9
    # rectangular decompositions plan their own blocks
    assert ex(P, 4, 8, hs.HS_RAS2, hs.HS_C64, hs.HS_COARSE_BEZIER) != ras
    # HS_C64X / HS_C64S add a complex128 copy of the factors to the set-up scratch
    assert ex(P, 4, 4, hs.HS_RAS2, hs.HS_C64X, hs.HS_COARSE_BEZIER) > ras
    Q = hs.hs_assemble(513, 160.0, hs.HS_BC_SOMMERFELD)
    assert ex(Q, 8, 8, hs.HS_RAS2, hs.HS_C64, hs.HS_COARSE_BEZIER) > 3 * ras


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


def test_nested_dissection_pivot_inverse_storage():
    """A front of at most 64 unknowns keeps one triangle of its complex-symmetric
    pivot inverse G = F_II^-1 (|I|(|I|+1)/2 entries), a larger front all of it
    (|I|^2): one front of 8 x 8 and one of 9 x 9 nodes.  The per-level counts
    add up to the plan's."""
    assert hs.hs_nd_plan_check(8, 8, 2, 8)["g_elems"] == 64 * 65 // 2
    assert hs.hs_nd_plan_check(9, 9, 2, 9)["g_elems"] == 81 * 81
    st = hs.hs_nd_plan_check(129, 129, 2, 8)
    L = hs.hs_nd_plan_level_stats(129, 129, 2)
    assert sum(lv["g_entries"] for lv in L) == st["g_elems"]
    assert sum(lv["v_entries"] for lv in L) == st["v_elems"]


def test_nested_dissection_precision_config_sizes():
    """Coarse grid of the n = 1025, H = 2h workload: the largest front must fit
    the kernels' limits (separator of 2 x 513 nodes)."""
    st = hs.hs_nd_plan_check(513, 513, 2, 8)
    assert st["max_nI"] <= 1152 and st["max_nB"] <= 2048


def test_nested_dissection_subtree_split():
    """The deepest levels of the n = 1025 coarse solve (coarse grid 513 x 513)
    are solved by subtree: from depth 8 down, one workgroup per front at
    depth 8 (256) with all its descendants, every front of them within the
    subtree kernels' limits (|I| <= 64, |B| <= 320, at most 5 depths); the
    levels above keep launches of their own.  Smaller plans put at least
    their leaves in subtrees."""
    L = hs.hs_nd_plan_level_stats(513, 513, 2)
    sub = [lv for lv, s in enumerate(L) if s["subtree_workgroups"]]
    assert sub == list(range(8, len(L))) and len(sub) <= 5
    assert L[8]["subtree_workgroups"] == L[8]["fronts"] == 256
    for lv, s in enumerate(L):
        if lv in sub:
            assert s["fwd_workgroups"] == 0 and s["bwd_workgroups"] == 0
            assert s["max_nI"] <= 64 and s["max_nB"] <= 320
        else:
            assert s["bwd_workgroups"] > 0 and s["subtree_workgroups"] == 0
    for nc in (17, 33, 65, 129):
        L = hs.hs_nd_plan_level_stats(nc, nc, 2)
        assert L[-1]["subtree_workgroups"] >= 1
