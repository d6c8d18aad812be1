"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances: FP64 paths 1e-10 relative, both in the Frobenius norm and
element by element (max |difference| <= 1e-10 max |reference|, so that small
entries cannot hide behind the large ones); FP32 paths are judged
by their relative-residual gap to the oracle (<= 1e-3) plus orthonormality
and subspace angles; SPA indices are compared exactly.
"""
import math

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
    return t.detach().cpu().double().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def close64(a, b, tol=1e-10):
    """FP64 parity: relative Frobenius difference and element-wise difference
    (scaled by the largest reference entry) both within tol."""
    assert a.shape == b.shape
    fro = rel(a, b)
    elem = float(np.abs(a - b).max() / np.abs(b).max())
    return fro < tol and elem < tol


def sin_max_angle(Q1, Q2):
    """sin of the largest principal angle between span(Q1) and span(Q2)."""
    s = np.linalg.svd(Q1.T @ Q2, compute_uv=False)
    return math.sqrt(max(0.0, 1.0 - float(s.min()) ** 2))


# --------------------------------------------------------------------------
# the dominant kernel: one streaming pass
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(1037, 523, 21), (64, 64, 16), (3001, 2999, 128), (257, 4099, 37), (5, 7, 3)])
def test_range_product_matches_matmul(dtype, shape):
    m, n, kx = shape
    g = np.random.default_rng(m + n + kx)
    A = g.standard_normal((m, n))
    X = g.standard_normal((n, kx))
    Z = g.standard_normal((m, kx))
    Ad = dev(A, dtype)
    Y = host(api.range_product(Ad, dev(X, dtype)))
    W = host(api.range_product(Ad, dev(Z, dtype), trans=True))
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    # reference products in FP64 on the same (rounded) inputs
    Ar = host(Ad)
    Xr = host(dev(X, dtype))
    Zr = host(dev(Z, dtype))
    assert rel(Y, Ar @ Xr) < tol
    assert rel(W, Ar.T @ Zr) < tol


def test_range_product_padded_lda():
    g = np.random.default_rng(5)
    big = dev(g.standard_normal((300, 260)), torch.float32)
    A = big[:, :250]  # lda = 260 (row-major view)
    X = dev(g.standard_normal((250, 40)), torch.float32)
    Y = host(api.range_product(A, X))
    assert rel(Y, host(A) @ host(X)) < 2e-6


@pytest.mark.parametrize("shape", [(300, 4100, 128), (513, 2048, 96), (777, 1000, 112), (2000, 516, 60),
                                   (1200, 3000, 128), (257, 132, 16), (5, 36, 48), (20000, 5000, 120)])
def test_range_product_fp32_lds_ring_shapes(shape):
    """FP32 rows that are 16-byte aligned (n % 4 == 0) take the LDS-ring pass
    kernels: ragged row tiles (256), ragged K chunks (32), every operand
    width class, several split counts.  Element-wise against the FP64
    product of the same FP32 inputs, within the FP32 accumulation bound."""
    m, n, kx = shape
    g = np.random.default_rng(m * 3 + n + kx)
    A = g.random((m, n)).astype(np.float32)
    X = (g.random((n, kx)) - 0.5).astype(np.float32)
    Z = (g.random((m, kx)) - 0.5).astype(np.float32)
    Ad = dev(A, torch.float32)
    Y = host(api.range_product(Ad, dev(X, torch.float32)))
    W = host(api.range_product(Ad, dev(Z, torch.float32), trans=True))
    A64, X64, Z64 = A.astype(np.float64), X.astype(np.float64), Z.astype(np.float64)
    for got, ref, mag, kdim in ((Y, A64 @ X64, np.abs(A64) @ np.abs(X64), n),
                                (W, A64.T @ Z64, np.abs(A64.T) @ np.abs(Z64), m)):
        bound = 2.0 * kdim * 2.0 ** -24 * mag + 1e-30
        assert np.all(np.abs(got - ref) <= bound)


def test_range_product_fp32_padded_aligned_lda():
    """lda > n with 16-byte aligned rows (the LDS-ring kernels read only the
    first n columns of each row)."""
    g = np.random.default_rng(6)
    big = dev(g.standard_normal((300, 264)), torch.float32)
    A = big[:, :256]   # lda = 264, n = 256
    X = dev(g.standard_normal((256, 40)), torch.float32)
    Z = dev(g.standard_normal((300, 40)), torch.float32)
    assert rel(host(api.range_product(A, X)), host(A) @ host(X)) < 2e-6
    assert rel(host(api.range_product(A, Z, trans=True)), host(A).T @ host(Z)) < 2e-6


# --------------------------------------------------------------------------
# FP64 path at the 1000 x 500 workload: 1e-10 against the oracle
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1():
    w = WL.WORKLOADS["plain_fp64_1000x500"]
    inp = WL.make_inputs(w)
    sk = O.sketch(inp["A"], inp["Omega_L"], inp["Omega_R"], w.q)
    lam = float(np.linalg.svd(sk["At"], compute_uv=False)[w.r - 1])
    adm = O.admm(sk["At"], sk["L"], sk["R"], inp["U1"], inp["V1"], lam, lam, 1.0, w.iters)
    res = O.rel_residual(inp["A"], adm["U"], adm["V"])
    return w, inp, sk, lam, adm, res


def test_sketch_fp64_parity(c1):
    w, inp, sk, *_ = c1
    out = api.sketch(dev(inp["A"]), w.r, w.k, w.q, dev(inp["Omega_L"]), dev(inp["Omega_R"]), want_ac=True)
    for name in ("L", "R", "B", "At", "Ac"):
        got = host(getattr(out, name))
        assert close64(got, sk[name]), name
    st = host(out.stats)
    assert st[0] < 1e-13 and st[1] < 1e-13 and st[2] == 0


def test_factorize_admm_fp64_parity(c1):
    w, inp, sk, lam, adm, res = c1
    f = api.factorize(dev(inp["A"]), w.r, w.k, w.q, dev(inp["U1"]), dev(inp["V1"]), dev(inp["Omega_L"]),
                      dev(inp["Omega_R"]), method="admm", iters=w.iters, lam=lam, phi=lam)
    U, V = host(f.U), host(f.V)
    assert close64(U, adm["U"])
    assert close64(V, adm["V"])
    assert abs(float(host(f.rel_residual)[0]) - res) <= 1e-10 * res


# The r x r solves across block counts (r up to 64) and sketch widths (k up to
# 128): one and two 16-row strips of X per wave, up to the largest shapes the
# single-workgroup solve holds in LDS.  The 16437-row shapes have more than
# 240 64-row sweeps on one side, so its row-update blocks take two sweeps
# each (129 blocks of 128 rows, the last one ragged).  Each launch of the
# iteration also sums its solve's partials in workgroups of its own, with 1,
# 2 or 4 groups of 16 elements each, the fewest that keep the launch within
# one workgroup per CU on a 256-CU device: one group for the small shapes,
# two for r 64 / k 74 and up, four at 20000 rows with r 48 / k 80; with 240
# row-update blocks (15360 rows) the sums are too slow beside the solve and
# run as separate launches instead.
@pytest.mark.parametrize("m,n,r,k", [(420, 300, 5, 9), (500, 400, 37, 47), (500, 400, 48, 80), (500, 400, 64, 74),
                                     (500, 400, 20, 100), (500, 400, 64, 112), (500, 400, 48, 128),
                                     (16437, 150, 10, 20), (150, 16437, 12, 22), (20000, 150, 48, 80),
                                     (150, 15360, 20, 40), (15360, 150, 32, 60)])
def test_factorize_admm_fp64_solve_shapes(m, n, r, k):
    A = WL.nmf_matrix(m, n, r, 0.05, seed=31 + r, dtype=np.float64)
    g = np.random.default_rng(41 + k)
    oml, omr = g.standard_normal((n, k)), g.standard_normal((m, k))
    U1, V1 = WL.init_factors(float(A.mean()), m, n, r, 51 + r)
    q, iters = 1, 15
    sk = O.sketch(A, oml, omr, q)
    lam = float(np.linalg.svd(sk["At"], compute_uv=False)[r - 1])
    ref = O.admm(sk["At"], sk["L"], sk["R"], U1, V1, lam, 0.7 * lam, 1.0, iters)
    f = api.factorize(dev(A), r, k, q, dev(U1), dev(V1), dev(oml), dev(omr), method="admm", iters=iters, lam=lam,
                      phi=0.7 * lam)
    assert close64(host(f.U), ref["U"])
    assert close64(host(f.V), ref["V"])


@pytest.mark.parametrize("sides", ["left", "right"])
@pytest.mark.parametrize("q", [0, 1, 3])
def test_sketch_one_sided_ragged_fp64(sides, q):
    g = np.random.default_rng(100 + q)
    m, n, r, k = 613, 389, 7, 19
    A = g.random((m, r)) @ g.random((r, n)) + np.abs(0.01 * g.standard_normal((m, n)))
    oml, omr = g.standard_normal((n, k)), g.standard_normal((m, k))
    out = api.sketch(dev(A), r, k, q, dev(oml), dev(omr), sides=sides)
    if sides == "left":
        ref = O.sketch(A, oml, None, q)
        assert close64(host(out.L), ref["L"])
        assert close64(host(out.B), ref["B"])
    else:
        Rref = O.range_finder(A.T, omr, q).T
        assert close64(host(out.R), Rref)


# --------------------------------------------------------------------------
# FP32 path (the 20000 x 5000 workload's recipe at reduced size, and full)
# --------------------------------------------------------------------------

def _fp32_case(m, n, iters):
    w = WL.WORKLOADS["nmf_fp32_20000x5000"]
    inp = WL.make_inputs(w, m=m, n=n)
    A64 = inp["A"].astype(np.float64)            # the FP32-rounded values
    sk = O.sketch(A64, inp["Omega_L"], inp["Omega_R"], w.q)
    lam = float(np.linalg.svd(sk["At"], compute_uv=False)[w.r - 1])
    return w, inp, A64, sk, lam


def test_factorize_admm_fp32_reduced_size():
    w, inp, A64, sk, lam = _fp32_case(4000, 1500, 60)
    iters = 60
    adm = O.admm(sk["At"], sk["L"], sk["R"], inp["U1"], inp["V1"], lam, lam, 1.0, iters)
    res_o = O.rel_residual(A64, adm["U"], adm["V"])
    Ad = dev(inp["A"], torch.float32)
    f = api.factorize(Ad, w.r, w.k, w.q, dev(inp["U1"]), dev(inp["V1"]), dev(inp["Omega_L"]), dev(inp["Omega_R"]),
                      iters=iters, lam=lam, phi=lam, want_sketch=True)
    Lg = host(f.sketch.L)
    assert np.abs(Lg.T @ Lg - np.eye(w.k)).max() < 1e-5
    assert sin_max_angle(Lg[:, : w.r], sk["L"][:, : w.r]) < 1e-3
    res_g = float(host(f.rel_residual)[0])
    assert abs(res_g - res_o) <= 1e-3
    # the residual is computed in FP64 from the GPU factors
    assert abs(res_g - O.rel_residual(A64, host(f.U), host(f.V))) < 1e-6


# --------------------------------------------------------------------------
# SPA (Alg. SNMF): indices bit-exact
# --------------------------------------------------------------------------

def test_spa_on_given_matrix_is_exact():
    g = np.random.default_rng(7)
    B = g.standard_normal((30, 20011))
    K, sc = api.spa(dev(B), 20, want_scores=True)
    Kref, gaps = O.spa(B, 20, return_gaps=True)
    assert min(gaps) > 1e-9
    assert host(K).astype(np.int64).tolist() == Kref


def test_select_separable_recovers_planted_fp64():
    A, planted = WL.separable_matrix(700, 6000, 12, 1e-4, seed=9)
    g = np.random.default_rng(10)
    om = g.standard_normal((6000, 22))
    K, _, B = api.select(dev(A), 12, 22, 2, dev(om), want_B=True)
    Kg = host(K).astype(np.int64).tolist()
    Bref = O.sketch(A, om, None, 2)["B"]
    assert close64(host(B), Bref)
    assert Kg == O.spa(Bref, 12)
    assert sorted(Kg) == list(planted)


def test_select_separable_fp32_two_sided():
    A, planted = WL.separable_matrix(1200, 9000, 15, 1e-3, seed=11)
    g = np.random.default_rng(12)
    om, omr = g.standard_normal((9000, 25)), g.standard_normal((1200, 25))
    Ad = dev(A, torch.float32)
    K, _, B = api.select(Ad, 15, 25, 2, dev(om), dev(omr), sides="both", want_B=True)
    Kg = host(K).astype(np.int64).tolist()
    assert sorted(Kg) == list(planted)
    # same decision on the GPU's own B taken by the oracle's SPA
    assert Kg == O.spa(host(B), 15)


# --------------------------------------------------------------------------
# Alg. 2 (compressed MU) and the uncompressed comparators
# --------------------------------------------------------------------------

def test_factorize_mu_fp64_parity(c1):
    w, inp, sk, *_ = c1
    iters = 60
    ref = O.mu(sk["Ac"], sk["B"], sk["L"], sk["R"], inp["U1"], inp["V1"], iters, 1e-16)
    f = api.factorize(dev(inp["A"]), w.r, w.k, w.q, dev(inp["U1"]), dev(inp["V1"]), dev(inp["Omega_L"]),
                      dev(inp["Omega_R"]), method="mu", iters=iters, mu_eps=1e-16)
    assert close64(host(f.U), ref["X"])
    assert close64(host(f.V), ref["Y"])
    res = O.rel_residual(inp["A"], ref["X"], ref["Y"])
    assert abs(float(host(f.rel_residual)[0]) - res) <= 1e-10 * res


@pytest.fixture(scope="module")
def small_full():
    g = np.random.default_rng(200)
    m, n, r = 613, 389, 7
    A = g.random((m, r)) @ g.random((r, n)) + np.abs(0.01 * g.standard_normal((m, n)))
    U1, V1 = WL.init_factors(A.mean(), m, n, r, 201)
    lam = float(np.linalg.svd(A, compute_uv=False)[r - 1])
    return A, U1, V1, r, lam


def test_factorize_admm_full_fp64_parity(small_full):
    A, U1, V1, r, lam = small_full
    ref = O.admm_uncompressed(A, U1, V1, lam, 1.3 * lam, 1.0, 40)
    f = api.factorize(dev(A), r, r + 1, 0, dev(U1), dev(V1), method="admm_full", iters=40, lam=lam, phi=1.3 * lam)
    assert close64(host(f.U), ref["U"])
    assert close64(host(f.V), ref["V"])


def test_factorize_mu_full_fp64_parity(small_full):
    A, U1, V1, r, _ = small_full
    ref = O.mu_uncompressed(A, U1, V1, 40, 1e-16)
    f = api.factorize(dev(A), r, r + 1, 0, dev(U1), dev(V1), method="mu_full", iters=40, mu_eps=1e-16)
    assert close64(host(f.U), ref["X"])
    assert close64(host(f.V), ref["Y"])


@pytest.mark.parametrize("method", ["mu", "admm_full", "mu_full"])
def test_factorize_fp32_methods_residual_gap(method):
    w, inp, A64, sk, lam = _fp32_case(3000, 1200, 30)
    iters = 30
    if method == "mu":
        ref = O.mu(sk["Ac"], sk["B"], sk["L"], sk["R"], inp["U1"], inp["V1"], iters, 1e-16)
        U, V = ref["X"], ref["Y"]
    elif method == "admm_full":
        ref = O.admm_uncompressed(A64, inp["U1"], inp["V1"], lam, lam, 1.0, iters)
        U, V = ref["U"], ref["V"]
    else:
        ref = O.mu_uncompressed(A64, inp["U1"], inp["V1"], iters, 1e-16)
        U, V = ref["X"], ref["Y"]
    res_o = O.rel_residual(A64, U, V)
    f = api.factorize(dev(inp["A"], torch.float32), w.r, w.k, w.q, dev(inp["U1"]), dev(inp["V1"]),
                      dev(inp["Omega_L"]), dev(inp["Omega_R"]), method=method, iters=iters, lam=lam, phi=lam,
                      mu_eps=1e-16)
    res_g = float(host(f.rel_residual)[0])
    assert abs(res_g - res_o) <= 1e-3


# --------------------------------------------------------------------------
# The separable workload at full size (10000 x 100000, r 20, k 30, q 2,
# two-sided): generated on the device with the same recipe, SPA must return
# exactly the planted columns, and the oracle's SPA on the GPU's B must make
# the same choices in the same order.
# --------------------------------------------------------------------------

def separable_on_device(m, n, r, noise, seed):
    return WL.separable_on_device(m, n, r, noise, seed, DEV)


def test_select_separable_full_size_two_sided():
    w = WL.WORKLOADS["separable_fp32_10000x100000"]
    A, planted = separable_on_device(w.m, w.n, w.r, w.sep_noise, seed=300)
    g = np.random.default_rng(301)
    om, omr = g.standard_normal((w.n, w.k)), g.standard_normal((w.m, w.k))
    K, score, B = api.select(A, w.r, w.k, w.q, dev(om), dev(omr), sides="both", want_scores=True, want_B=True)
    Kg = host(K).astype(np.int64).tolist()
    assert sorted(Kg) == planted.tolist()
    Kref, gaps = O.spa(host(B), w.r, return_gaps=True)
    assert Kg == Kref
    assert min(gaps) > 1e-5   # the decisions are not tie-sensitive
