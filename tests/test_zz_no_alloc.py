"""The allocation-free application of M^{-1} (hs_apply_Minv_noalloc) against
hs_apply_Minv, through the C ABI.

Both run the same kernels in the same order over the same factors; only the
buffers an application writes and reads back differ (the library's static
scratch array instead of the preconditioner's own), so the results must be
equal bit for bit.  Calls follow each other with inputs of different sizes,
so each call finds the previous call's contents in the array.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2408_03571_amd as hs  # noqa: E402
from workloads import random_vector  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"
LIMIT = 64 << 20


def setup(n, nsub, ratio, variant, prec):
    k = 0.3125 * (n - 1)
    P = hs.hs_assemble(n, k, hs.HS_BC_SOMMERFELD)
    M = hs.hs_setup_schwarz(P, nsub, 2, ratio, variant, prec)
    return P, M


def both(P, M, seed):
    N = hs.hs_problem_size(P)
    r = torch.from_numpy(random_vector(N, seed=seed)).to(DEV)
    z_ref = torch.zeros_like(r)
    z_new = torch.full_like(r, complex(np.nan, np.nan))
    hs.hs_apply_Minv(M, r, z_ref)
    hs.hs_apply_Minv_noalloc(M, r, z_new)
    torch.cuda.synchronize()
    return z_ref.cpu().numpy(), z_new.cpu().numpy()


@pytest.mark.parametrize("variant,prec", [(hs.HS_RAS2, hs.HS_C64), (hs.HS_AS2, hs.HS_C128),
                                          (hs.HS_SHS2, hs.HS_C64)])
def test_noalloc_apply_equals_apply_larger_then_smaller(variant, prec):
    big = setup(257, 4, 2, variant, prec)
    small = setup(129, 3, 4, variant, prec)
    for (P, M), seed in ((big, 1), (small, 2), (big, 3)):
        assert hs.hs_precond_get_info(M)["apply_work_bytes"] <= LIMIT
        ref, new = both(P, M, seed)
        assert np.all(np.isfinite(new))
        assert np.array_equal(ref.view(np.float64), new.view(np.float64))


def test_noalloc_apply_covers_the_full_size_configuration():
    # n = 1025, 16 x 16 subdomains, H = 2h, RAS2: the limit the header states
    for prec in (hs.HS_C64, hs.HS_C128):
        P, M = setup(1025, 16, 2, hs.HS_RAS2, prec)
        assert hs.hs_precond_get_info(M)["apply_work_bytes"] <= LIMIT
        ref, new = both(P, M, 7)
        assert np.array_equal(ref.view(np.float64), new.view(np.float64))
        del M


def test_noalloc_apply_rejects_a_preconditioner_above_the_limit():
    # SHS2 keeps two fine-grid vectors per application: at n = 1537 that alone
    # is 75.6 MB, above the 64 MiB array
    P, M = setup(1537, 24, 8, hs.HS_SHS2, hs.HS_C64)
    assert hs.hs_precond_get_info(M)["apply_work_bytes"] > LIMIT
    r = torch.zeros(hs.hs_problem_size(P), dtype=torch.complex128, device=DEV)
    z = torch.zeros_like(r)
    with pytest.raises(hs.HSError) as e:
        hs.hs_apply_Minv_noalloc(M, r, z)
    assert e.value.status == hs.HS_EINVAL
    assert "static limit" in str(e.value)
    # the refusal left the array usable
    Ps, Ms = setup(129, 3, 2, hs.HS_RAS2, hs.HS_C64)
    ref, new = both(Ps, Ms, 5)
    assert np.array_equal(ref.view(np.float64), new.view(np.float64))
