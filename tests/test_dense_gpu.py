"""The dense TSQR step (section "Post-processing") on plain matrices, against
the oracle's textbook Householder QR (needs an MI355X)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_00525_amd as F
    F.lib()
    return F


from _parity import colscaled, relf as _relf


@pytest.mark.parametrize("variant", [0, 1, 2])
# n = 17..31: the shared-tile step in 4-column blocks with a partly filled
# last block and a wholly idle last wave
@pytest.mark.parametrize("n", [1, 5, 8, 13, 16, 17, 19, 21, 24, 25, 27, 31, 32, 35, 40, 41, 64, 65, 100, 128])
def test_single_workgroup_matches_householder(F, oracle_lib, n, variant):
    import torch
    tpw = 2
    rows = F.debug_dense_rows(n, variant, tpw) - 37     # several tiles and a ragged tail
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((rows, n)) * 10.0 ** rng.uniform(-3, 3, n)
    R = F.debug_dense_step(torch.as_tensor(A).cuda(), 1, tpw, variant).cpu().numpy()
    ref, _ = oracle_lib.householder_r(np.asfortranarray(A))
    assert np.all(np.tril(R, -1) == 0.0)
    assert np.all(np.diag(R) >= 0)
    assert _relf(R, ref) <= 1e-12
    # every column against its own norm (column scales span 10^-3..10^3)
    assert colscaled(R, ref) <= 1e-12


@pytest.mark.parametrize("n", [7, 16, 17, 21, 25, 31, 32, 37, 48, 96, 128])
def test_many_workgroups_preserve_gram(F, oracle_lib, n):
    import torch
    wg = 9
    rows = wg * F.debug_dense_rows(n, 0, 1) - 5
    rng = np.random.default_rng(7 + n)
    A = rng.standard_normal((rows, n))
    S = F.debug_dense_step(torch.as_tensor(A).cuda(), wg, 1, 0).cpu().numpy()
    assert S.shape == (wg * n, n)
    for b in range(wg):
        assert np.allclose(np.tril(S[b * n:(b + 1) * n], -1), 0.0)
    Ghi, Glo = oracle_lib.gram_ld(np.asfortranarray(A))
    assert _relf(S.T @ S, Ghi + Glo) <= 1e-13


@pytest.mark.parametrize("n", [10, 23, 29, 40])
def test_rank_deficient_and_zero_columns(F, oracle_lib, n):
    import torch
    rows = F.debug_dense_rows(n, 0, 2) - 7      # one workgroup, a ragged last tile
    rng = np.random.default_rng(3)
    A = rng.standard_normal((rows, n))
    A[:, 3] = 0.0
    A[:, 7] = 2.0 * A[:, 1]
    if 16 < n <= 32:
        # inside a 4-column block of the shared-tile step, and in its last
        # (partly filled) block
        A[:, 17] = 0.0
        A[:, 18] = A[:, 16] - A[:, 5]
        A[:, n - 1] = -A[:, n - 2]
    if n > 32:
        # the same inside the last column block of the shared-tile step
        A[:, 35] = 0.0
        A[:, 38] = -A[:, 33]
    R = F.debug_dense_step(torch.as_tensor(A).cuda(), 1, 2, 0).cpu().numpy()
    assert np.all(np.isfinite(R))
    Ghi, Glo = oracle_lib.gram_ld(np.asfortranarray(A))
    assert _relf(R.T @ R, Ghi + Glo) <= 1e-13


def test_coverage_is_checked(F):
    import torch
    A = torch.zeros((F.debug_dense_rows(16, 0, 1) + 1, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(F.FigaroError):
        F.debug_dense_step(A, 1, 1, 0)
