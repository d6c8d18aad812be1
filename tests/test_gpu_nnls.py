"""GPU parity of SNMF's right factor (Section 4, Alg. SNMF, last step):
per-column nonnegative least squares on the compressed matrix, against the
oracle (brute force over all supports for small r, Lawson-Hanson through
scipy on sampled columns at the 10000 x 100000 separable workload's size),
through the C ABI.  The NNLS optimum is unique (B[:, K] has full column
rank), so the comparison is element by element: 1e-10 relative to the
column's largest entry for FP64 inputs."""
import numpy as np
import pytest

from oracle import cnmf_oracle as O
from paper_1505_04650_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1505_04650_amd import api  # noqa: E402

DEV = torch.device("cuda", 0)


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def assert_columns_close(H, ref, tol):
    scale = np.maximum(np.abs(ref).max(axis=0), 1e-300)
    err = (np.abs(H - ref).max(axis=0) / scale).max()
    assert err < tol, err


@pytest.mark.parametrize("r,k,n", [(1, 4, 50), (6, 15, 300), (10, 14, 200), (9, 40, 777)])
def test_nnls_matches_bruteforce(r, k, n):
    g = np.random.default_rng(100 + r + k)
    B = g.standard_normal((k, n))
    K = g.choice(n, size=r, replace=False).astype(np.int64)
    H, info = api.snmf_nnls(dev(B), dev(K, torch.int64), want_info=True)
    H = host(H)
    C = B[:, K]
    ref = np.stack([O.nnls_bruteforce(C, B[:, j]) for j in range(n)], axis=1)
    assert_columns_close(H, ref, 1e-10)
    inf = host(info)
    assert inf[0] == 0 and inf[2] == 0
    assert (H >= 0).all()
    # the selected columns reproduce themselves: h = e_i
    assert np.abs(H[np.arange(r), K] - 1.0).max() < 1e-10


def test_nnls_fp32_input_and_padded_ld():
    g = np.random.default_rng(5)
    k, n, r = 20, 1000, 12
    Bf = g.standard_normal((k, n + 24)).astype(np.float32)
    Bd = dev(Bf, torch.float32)[:, :n]           # ldb = n + 24
    K = g.choice(n, size=r, replace=False).astype(np.int64)
    H = host(api.snmf_nnls(Bd, dev(K, torch.int64)))
    ref = O.snmf_right_factor(Bf[:, :n].astype(np.float64), K)
    assert_columns_close(H, ref, 1e-10)


def test_nnls_recovers_planted_factor_after_selection():
    A, planted = WL.separable_matrix(500, 4000, 8, 0.0, seed=31)
    K, _, B = api.select(dev(A), 8, 18, 2, None, want_B=True, seed=32)
    Kh = host(K)
    assert sorted(Kh.tolist()) == list(planted)
    H = host(api.snmf_nnls(B, K))
    # A = A[:, K] H exactly (W has full column rank and H is the planted factor)
    assert np.linalg.norm(A - A[:, Kh] @ H) < 1e-10 * np.linalg.norm(A)


def test_nnls_full_size_separable_sampled_columns():
    """10000 x 100000 separable workload (two-sided sketch, k 30, q 2):
    H on all 100000 columns of the GPU's B; 400 sampled columns (and the
    planted ones) against Lawson-Hanson on the same B."""
    w = WL.WORKLOADS["separable_fp32_10000x100000"]
    A, planted = WL.separable_on_device(w.m, w.n, w.r, w.sep_noise, 400, DEV)
    K, _, B = api.select(A, w.r, w.k, w.q, sides="both", want_B=True, seed=401)
    del A
    H, info = api.snmf_nnls(B, K, want_info=True)
    Bh, Kh, H = host(B).astype(np.float64), host(K), host(H)
    assert sorted(Kh.tolist()) == planted.tolist()
    inf = host(info)
    assert inf[0] == 0 and inf[2] == 0
    g = np.random.default_rng(402)
    cols = np.unique(np.concatenate([g.choice(w.n, size=400, replace=False), Kh]))
    ref = O.snmf_right_factor(Bh[:, cols], [int(np.where(cols == kk)[0][0]) for kk in Kh])
    assert_columns_close(H[:, cols], ref, 1e-9)
