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


# figaro_tsqr: the whole post-processing QR (every level) of a plain matrix.
# Sizes: one tile, one workgroup with a ragged tile, several levels, and a
# first level at its workgroup cap (many tiles per workgroup); column scales
# 10^U[-3,3] so that every column is compared against its own norm.
TSQR_CASES = [(1, 1), (1, 5000), (7, 0), (7, 3), (7, 100), (8, 70001), (16, 1024), (16, 200003),
              (17, 129), (24, 50000), (32, 128), (32, 300001), (40, 90001), (41, 777), (64, 20000),
              (100, 5000), (128, 40000)]


@pytest.mark.parametrize("n,rows", TSQR_CASES)
def test_tsqr_matches_householder(F, oracle_lib, n, rows):
    import torch
    rng = np.random.default_rng(1000 * n + rows % 997)
    A = rng.standard_normal((rows, n)) * 10.0 ** rng.uniform(-3, 3, n)
    R = F.tsqr(torch.as_tensor(A).cuda()).cpu().numpy()
    assert np.all(np.tril(R, -1) == 0.0)
    assert np.all(np.diag(R) >= 0)
    if rows < n:     # R is not unique: compare R^T R
        Ghi, Glo = oracle_lib.gram_ld(np.asfortranarray(A))
        assert _relf(R.T @ R, Ghi + Glo) <= 1e-13 if rows else np.all(R == 0)
        return
    ref, _ = oracle_lib.householder_r(np.asfortranarray(A))
    err, cerr = _relf(R, ref), colscaled(R, ref)
    print(f"[tsqr] n={n} rows={rows} rel_err={err:.2e} colscaled={cerr:.2e}", flush=True)
    assert err <= 1e-10
    assert cerr <= 1e-10


def test_tsqr_leading_dimension_and_workspace(F, oracle_lib):
    """A submatrix view (leading dimension larger than the rows) and an
    explicitly passed workspace of exactly the reported size."""
    import torch
    rng = np.random.default_rng(5)
    big = torch.as_tensor(np.asfortranarray(rng.standard_normal((90000, 40)))).cuda()
    A = big[:80000, 3:30]          # column-major storage, leading dimension 90000
    nbytes = F.tsqr_workspace_bytes(80000, 27)
    ws = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    R = F.tsqr(A, workspace=ws).cpu().numpy()
    ref, _ = oracle_lib.householder_r(np.asfortranarray(A.cpu().numpy()))
    assert _relf(R, ref) <= 1e-10
    assert colscaled(R, ref) <= 1e-10
