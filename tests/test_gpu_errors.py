"""Error paths of the HIP path reached on the device, through the C ABI.

Both conditions are built from the host: every kernel runs to its normal end
and the status is read back by the host.
  HS_ESINGULAR  MP-1 (Sec. 2, Dirichlet) at n = 5 with k^2 = 64: the 3 x 3
                interior operator is 16 (4 I - adjacency) - 64 I = -16
                adjacency, whose first grid-line block is -16 times the
                adjacency of a three-node path, a singular matrix of small
                integers.  Its Gauss-Jordan inversion meets an exact zero
                pivot, which the local factorisation reports.
  HS_ENAN       a right-hand side holding a NaN: ||b|| is not finite, the
                solve stops before its first iteration; in a batch only that
                instance fails and the others converge.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2408_03571_amd as hs  # noqa: E402
from paper_2408_03571_amd import _lib  # noqa: E402
from oracle import problem  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


def test_singular_local_block_reports_esingular():
    A = problem.assemble(5, problem.DIRICHLET, k=8.0).toarray()
    # the premise, checked on the oracle's matrix: the operator and its first
    # line block are exactly singular integer matrices
    assert np.array_equal(A, np.round(A.real))
    assert np.linalg.matrix_rank(A) < A.shape[0]
    assert np.linalg.matrix_rank(A[:3, :3]) == 2
    P = hs.hs_assemble(5, 8.0, hs.HS_BC_DIRICHLET)
    with pytest.raises(hs.HSError) as e:
        hs.hs_setup_schwarz(P, 1, 2, 2, hs.HS_RAS2, hs.HS_C128)
    assert e.value.status == hs.HS_ESINGULAR
    assert "subdomain 0" in str(e.value)
    # the same problem at a regular wavenumber sets up
    P2 = hs.hs_assemble(5, 7.0, hs.HS_BC_DIRICHLET)
    hs.hs_setup_schwarz(P2, 1, 2, 2, hs.HS_RAS2, hs.HS_C128)


def test_nan_right_hand_side_reports_enan():
    n = 65
    P = hs.hs_assemble(n, 20.0, hs.HS_BC_SOMMERFELD)
    M = hs.hs_setup_schwarz(P, 4, 2, 2, hs.HS_RAS2, hs.HS_C128)
    f = problem.rhs(n, problem.SOMMERFELD)
    f[17] = np.nan
    b = torch.from_numpy(f).to(DEV)
    x = torch.zeros_like(b)
    for ortho in (hs.HS_ORTHO_DCGS2, hs.HS_ORTHO_MGS):
        with pytest.raises(hs.HSError) as e:
            hs.hs_gmres_solve(P, M, b, x, tol=1e-6, maxit=50, ortho=ortho)
        assert e.value.status == hs.HS_ENAN
        assert "non-finite" in str(e.value)
    # the preconditioner is unharmed: a finite right-hand side solves
    f[17] = 0.0
    st, _ = hs.hs_gmres_solve(P, M, torch.from_numpy(f).to(DEV), x, tol=1e-6, maxit=200)
    assert st["converged"]


def test_nan_instance_of_a_batch_fails_alone():
    ns = [65, 97, 65]
    Ps = [hs.hs_assemble(n, 0.3 * (n - 1), hs.HS_BC_SOMMERFELD) for n in ns]
    Ms = [hs.hs_setup_schwarz(P, 3, 2, 2, hs.HS_RAS2, hs.HS_C64) for P in Ps]
    B = hs.hs_batch_create(Ms)
    fs = [problem.rhs(n, problem.SOMMERFELD) for n in ns]
    fs[1][5] = np.nan
    b = torch.from_numpy(np.concatenate(fs)).to(DEV)
    x = torch.zeros_like(b)
    maxit = 200
    nbytes = hs.hs_batch_gmres_workspace_bytes(B, maxit)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    st = (hs.GmresStats * 3)()
    opts = hs.GmresOpts(hs.HS_ORTHO_DCGS2, 1, 0, hs.HS_C128)
    status = _lib.load().hs_batch_gmres_solve(B.handle, ctypes.c_void_p(b.data_ptr()),
                                              ctypes.c_void_p(x.data_ptr()), 1e-6, maxit, ctypes.byref(opts),
                                              ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(nbytes),
                                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), st)
    torch.cuda.synchronize()
    assert status == hs.HS_ENAN
    assert st[0].converged and st[2].converged and not st[1].converged
    assert st[0].relres_true <= 1e-6 and st[2].relres_true <= 1e-6
