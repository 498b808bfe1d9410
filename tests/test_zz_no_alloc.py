"""figaro_tsqr_noalloc (the post-processing QR with the library's static
device array instead of a workspace) against figaro_tsqr on the same inputs:
two calls in a row on one GPU, the second with a smaller input, so the second
call reuses an array that still holds the first call's partial R's.  The
results must be bit for bit those of figaro_tsqr (same levels, same kernels)
and within 1e-10 of the oracle's Householder R, column by column (needs an
MI355X)."""
import numpy as np
import pytest

from _parity import colscaled, relf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_00525_amd as F
    F.lib()
    return F


def _matrix(rows, n, seed):
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((rows, n)) * 10.0 ** rng.uniform(-3, 3, n))


# (n, first rows, second rows): the shared-tile kernel with several levels,
# the narrow per-wave kernel, and a wide matrix whose first level sits at the
# workgroup cap of the array (8 MiB / 2 / (8 n^2) = 52 workgroups at n = 100)
@pytest.mark.parametrize("n,rows1,rows2", [(32, 300001, 50000), (16, 200003, 1024), (100, 60000, 5000)])
def test_noalloc_matches_workspace_entry_point(F, oracle_lib, n, rows1, rows2):
    import torch
    for k, rows in enumerate((rows1, rows2)):
        Ah = _matrix(rows, n, 17 * n + k)
        A = torch.as_tensor(Ah).cuda()            # column-major storage
        print(f"[noalloc] n={n} rows={rows} call={k + 1}", flush=True)
        Rn = F.tsqr_noalloc(A)
        Rw = F.tsqr(A)
        torch.cuda.synchronize()
        Rn, Rw = Rn.cpu().numpy(), Rw.cpu().numpy()
        assert np.array_equal(Rn, Rw), (n, rows)
        ref, _ = oracle_lib.householder_r(Ah)
        err, cerr = relf(Rn, ref), colscaled(Rn, ref)
        print(f"[noalloc] n={n} rows={rows} rel_err={err:.2e} colscaled={cerr:.2e}", flush=True)
        assert err <= 1e-10
        assert cerr <= 1e-10


def test_noalloc_rejects_unsupported_width(F):
    import torch
    A = torch.zeros((10, 129), dtype=torch.float64, device="cuda").t().contiguous().t()
    with pytest.raises(F.FigaroError) as e:
        F.tsqr_noalloc(A)
    assert e.value.name == "EUNSUPPORTED"
