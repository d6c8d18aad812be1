"""GPU tests of the device-drawn test matrices (Alg. 1's first step), the
CholeskyQR2 breakdown fallback on rank-deficient samples (k > rank A), and
SPA's tie rule, through the C ABI.

* Generator: the device's Philox4x32-10 + Box-Muller matrices match the
  oracle side's own implementation of the same published definitions to a
  few ulp, and a seeded sketch equals the oracle fed the host-drawn matrices
  to 1e-10.
* Breakdown: for an exactly rank-r A with k > r several orthonormal bases
  are correct (their trailing columns are arbitrary), so projectors and
  residuals are compared, never the trailing columns.
* SPA: exactly tied column norms must resolve to the lowest index, as the
  oracle does.
"""
import numpy as np
import pytest

from oracle import cnmf_oracle as O
from oracle import philox as P
from paper_1505_04650_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1505_04650_amd import _lib as L  # noqa: E402
from paper_1505_04650_amd import api  # noqa: E402

DEV = torch.device("cuda", 0)


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sin_max_angle(Q1, Q2):
    """sin of the largest principal angle between span(Q1) and span(Q2)
    (orthonormal columns): the 2-norm of Q1's part outside span(Q2), which
    unlike sqrt(1 - cos^2) stays accurate for tiny angles."""
    return float(np.linalg.norm(Q1 - Q2 @ (Q2.T @ Q1), 2))


# --------------------------------------------------------------------------
# generator
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed,mid,rows,cols", [(0, 0, 1000, 20), (0xDEADBEEF12345678, 1, 777, 61),
                                                (12345, 17, 4099, 128), (2 ** 63 + 5, 3, 1, 1)])
def test_gaussian_matches_host_generator(seed, mid, rows, cols):
    got = host(api.gaussian(rows, cols, seed, mid))
    ref = P.gaussian_matrix(seed, mid, rows, cols)
    # a few ulp of the pair's radius (the transcendental functions of the two
    # libraries may differ in the last bits)
    pairs = (cols + 1) // 2
    full = P.gaussian_matrix(seed, mid, rows, 2 * pairs).reshape(rows, pairs, 2)
    rho = np.repeat(np.sqrt((full ** 2).sum(axis=2)), 2, axis=1)[:, :cols]
    assert np.all(np.abs(got - ref) <= 4 * np.spacing(np.maximum(1.0, rho)))


def test_gaussian_large_row_index():
    """Rows far from 0 use the row counter word (no wrap into other rows)."""
    rows, cols = 300000, 3
    got = host(api.gaussian(rows, cols, 99, 0))
    ref = P.gaussian_matrix(99, 0, rows, cols)
    assert np.abs(got - ref).max() <= 4 * np.spacing(8.0)


def test_seeded_sketch_matches_oracle_on_regenerated_test_matrices():
    w = WL.WORKLOADS["plain_fp64_1000x500"]
    inp = WL.make_inputs(w)
    A = inp["A"]
    m, n = A.shape
    seed = 0x1234ABCD5678
    out = api.sketch(dev(A), w.r, w.k, w.q, None, None, want_ac=True, seed=seed)
    oml = P.gaussian_matrix(seed, 0, n, w.k)
    omr = P.gaussian_matrix(seed, 1, m, w.k)
    ref = O.sketch(A, oml, omr, w.q)
    for name in ("L", "R", "B", "At", "Ac"):
        got = host(getattr(out, name))
        assert rel(got, ref[name]) < 1e-10, name
        assert np.abs(got - ref[name]).max() < 1e-10 * np.abs(ref[name]).max(), name
    st = host(out.stats)
    assert st[0] < 1e-13 and st[1] < 1e-13 and st[2] == 0 and st[3] == 0


def test_seeded_factorize_equals_explicit_test_matrices():
    """A seeded factorisation is the one run on the library's own matrices."""
    w = WL.WORKLOADS["plain_fp64_1000x500"]
    inp = WL.make_inputs(w, m=400, n=300)
    A = dev(inp["A"])
    m, n = inp["A"].shape
    seed = 77
    oml, omr = api.gaussian(n, w.k, seed, 0), api.gaussian(m, w.k, seed, 1)
    kw = dict(iters=20, lam=30.0, phi=30.0)
    f1 = api.factorize(A, w.r, w.k, w.q, dev(inp["U1"]), dev(inp["V1"]), None, None, seed=seed, **kw)
    f2 = api.factorize(A, w.r, w.k, w.q, dev(inp["U1"]), dev(inp["V1"]), oml, omr, **kw)
    assert np.array_equal(host(f1.U), host(f2.U))
    assert np.array_equal(host(f1.V), host(f2.V))


# --------------------------------------------------------------------------
# rank-deficient samples: exactly rank-r A with k > r
# --------------------------------------------------------------------------

def _exact_rank(m, n, r, seed):
    g = np.random.default_rng(seed)
    return g.random((m, r)) @ g.random((r, n))


@pytest.mark.parametrize("q", [0, 4])
@pytest.mark.parametrize("m,n,r,k", [(1000, 500, 10, 20), (700, 900, 30, 100)])
def test_rank_deficient_sketch_fp64(m, n, r, k, q):
    A = _exact_rank(m, n, r, seed=m + r)
    g = np.random.default_rng(k)
    oml, omr = g.standard_normal((n, k)), g.standard_normal((m, k))
    out = api.sketch(dev(A), r, k, q, dev(oml), dev(omr), want_ac=True, seed=5)
    Lg, Rg, Bg, Atg = host(out.L), host(out.R), host(out.B), host(out.At)
    st = host(out.stats)
    # the fallback acted and resolved every breakdown
    assert st[2] > 0 and st[3] == 0
    api.synchronize()
    # orthonormal bases (Section 2's guarantee needs them), both sides
    assert np.abs(Lg.T @ Lg - np.eye(k)).max() < 1e-13
    assert np.abs(Rg @ Rg.T - np.eye(k)).max() < 1e-13
    assert st[0] < 1e-13 and st[1] < 1e-13
    # projectors and residuals (sigma_{r+1} = 0: the sketch captures A)
    nA = np.linalg.norm(A)
    assert np.linalg.norm(A - Lg @ (Lg.T @ A)) <= 1e-13 * nA
    assert np.linalg.norm(A - (A @ Rg.T) @ Rg) <= 1e-13 * nA
    assert np.linalg.norm(A - Lg @ Bg) <= 1e-13 * nA
    assert np.linalg.norm(A - Lg @ Atg @ Rg) <= 1e-13 * nA
    # the oracle's (Householder) bases give the same projections of A
    ref = O.sketch(A, oml, omr, q)
    assert np.linalg.norm(Lg @ (Lg.T @ A) - ref["L"] @ (ref["L"].T @ A)) <= 1e-13 * nA
    assert np.linalg.norm(A @ Rg.T @ Rg - A @ ref["R"].T @ ref["R"]) <= 1e-13 * nA
    # the leading r columns span range(A) on both sides
    assert sin_max_angle(Lg[:, :r], ref["L"][:, :r]) < 1e-10


def test_rank_deficient_sketch_fp32():
    m, n, r, k = 3000, 1200, 20, 40
    A = _exact_rank(m, n, r, seed=3).astype(np.float32)
    A64 = A.astype(np.float64)
    g = np.random.default_rng(4)
    oml, omr = g.standard_normal((n, k)), g.standard_normal((m, k))
    out = api.sketch(dev(A, torch.float32), r, k, 4, dev(oml), dev(omr), seed=6)
    st = host(out.stats)
    assert st[3] == 0 and st[0] < 1e-12 and st[1] < 1e-12
    Lg, Rg = host(out.L), host(out.R)
    nA = np.linalg.norm(A64)
    assert np.linalg.norm(A64 - Lg @ (Lg.T @ A64)) <= 2e-6 * nA
    assert np.linalg.norm(A64 - (A64 @ Rg.T) @ Rg) <= 2e-6 * nA


def test_rank_deficient_select_recovers_planted():
    """Separable A without noise (rank exactly r) and k > r: SPA on the
    completed basis still returns the planted columns."""
    A, planted = WL.separable_matrix(600, 5000, 10, 0.0, seed=21)
    K, _, B = api.select(dev(A), 10, 25, 2, None, want_B=True, seed=22)
    Kg = host(K).astype(np.int64).tolist()
    assert sorted(Kg) == list(planted)
    assert Kg == O.spa(host(B), 10)


def test_nan_input_reports_unresolved_breakdown():
    g = np.random.default_rng(8)
    A = g.random((300, 200))
    A[17, 33] = np.nan
    out = api.sketch(dev(A), 5, 10, 1, None, None, seed=1)
    st = host(out.stats)
    assert st[3] > 0
    with pytest.raises(L.CnmfError) as e:
        api.synchronize()
    assert e.value.status == L.CNMF_EBREAKDOWN
    # reported once: the count is cleared, and a clean call leaves it clear
    api.synchronize()
    out = api.sketch(dev(g.random((300, 200))), 5, 10, 1, None, None, seed=1)
    assert host(out.stats)[3] == 0
    api.synchronize()


# --------------------------------------------------------------------------
# SPA tie rule (lowest index wins), exact ties
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spa_exact_ties_take_lowest_index(dtype):
    k, n = 12, 4001
    g = np.random.default_rng(31)
    B = 0.1 * g.random((k, n))
    # unit directions scaled to exactly tied norms; duplicates of a column,
    # and two orthogonal columns of equal norm, far apart in index
    e = np.eye(k)
    B[:, 900] = 3.0 * e[0]
    B[:, 3000] = 3.0 * e[0]          # duplicate of column 900
    B[:, 2500] = 3.0 * e[1]          # same norm, orthogonal
    B[:, 77] = 2.0 * e[2]
    B[:, 3999] = 2.0 * e[3]
    B[:, 1500] = 2.0 * e[3]          # duplicate, lower index than 3999
    Bq = host(dev(B, dtype))         # the values the GPU sees
    K, _ = api.spa(dev(B, dtype), 5)
    Kg = host(K).astype(np.int64).tolist()
    Kref = O.spa(Bq, 5)
    assert Kref[:4] == [900, 2500, 77, 1500]
    assert Kg == Kref


# --------------------------------------------------------------------------
# SRHT test matrices (Section 2, remark after Thm. 3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed,mid,rows,cols", [(0, 0, 1000, 20), (0xDEADBEEF12345678, 1, 777, 61),
                                                (5, 2, 128, 128), (9, 3, 5, 5), (31, 0, 100000, 30)])
def test_srht_matches_host_generator(seed, mid, rows, cols):
    """Bit for bit: signs, sampled columns (including the probing after 64
    taken draws when every column of a small Hadamard matrix is sampled)
    and the scale 1 / sqrt(cols)."""
    got = host(api.srht(rows, cols, seed, mid))
    ref = P.srht_matrix(seed, mid, rows, cols)
    assert np.array_equal(got, ref)


def test_srht_sketch_matches_oracle():
    w = WL.WORKLOADS["plain_fp64_1000x500"]
    A = WL.make_inputs(w)["A"]
    m, n = A.shape
    seed = 4242
    out = api.sketch(dev(A), w.r, w.k, w.q, None, None, want_ac=True, seed=seed, test_matrix="srht")
    ref = O.sketch(A, P.srht_matrix(seed, 0, n, w.k), P.srht_matrix(seed, 1, m, w.k), w.q)
    for name in ("L", "R", "B", "At", "Ac"):
        got = host(getattr(out, name))
        assert rel(got, ref[name]) < 1e-10, name
    assert host(out.stats)[3] == 0


@pytest.mark.parametrize("q", [0, 2])
def test_srht_sketch_captures_the_range_like_gaussian(q):
    """Same projection error as the Gaussian test matrix to a few percent
    (20000 x 5000 recipe at reduced size, FP32)."""
    w = WL.WORKLOADS["nmf_fp32_20000x5000"]
    A = WL.make_inputs(w, m=4000, n=3000)["A"]
    Ad = dev(A, torch.float32)
    A64 = A.astype(np.float64)
    res = {}
    for kind in ("gaussian", "srht"):
        Lg = host(api.sketch(Ad, w.r, w.k, q, None, None, sides="left", seed=77, test_matrix=kind).L)
        res[kind] = np.linalg.norm(A64 - Lg @ (Lg.T @ A64)) / np.linalg.norm(A64)
    assert res["srht"] <= 1.05 * res["gaussian"]
