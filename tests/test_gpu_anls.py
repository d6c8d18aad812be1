"""GPU parity of compressed alternating NNLS (Section 3,
Eq. alternateLS_nmf_compressed) and its uncompressed form, through the C ABI.

Every half-step has a unique minimiser (the k x r matrices have full column
rank here), so the GPU's active-set solver must reproduce the oracle's
iterates: FP64 to 1e-10 (Frobenius and element-wise), FP32 by the
relative-residual gap (<= 1e-3).  At the 20000 x 5000 size, where the oracle
would take hours, the last half-step is checked by its optimality
conditions on sampled columns.
"""
import numpy as np
import pytest
import scipy.optimize

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


def close64(a, b, tol=1e-10):
    assert a.shape == b.shape
    fro = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    elem = float(np.abs(a - b).max() / np.abs(b).max())
    return fro < tol and elem < tol


def _nmf_input(m, n, r, seed, noise=0.01):
    g = np.random.default_rng(seed)
    A = g.random((m, r)) @ g.random((r, n)) + np.abs(noise * g.standard_normal((m, n)))
    U1, V1 = WL.init_factors(A.mean(), m, n, r, seed + 1)
    return A, U1, V1


def test_anls_fp64_parity_plain_workload():
    """1000 x 500, r 10, k 20, q 4 (the FP64 workload), 30 iterations."""
    w = WL.WORKLOADS["plain_fp64_1000x500"]
    inp = WL.make_inputs(w)
    sk = O.sketch(inp["A"], inp["Omega_L"], inp["Omega_R"], w.q)
    iters = 30
    ref = O.anls(sk["Ac"], sk["B"], sk["L"], sk["R"], inp["V1"], iters)
    f = api.factorize(dev(inp["A"]), w.r, w.k, w.q, dev(inp["U1"]), dev(inp["V1"]), dev(inp["Omega_L"]),
                      dev(inp["Omega_R"]), method="anls", iters=iters)
    assert close64(host(f.U), ref["X"])
    assert close64(host(f.V), ref["Y"])
    res = O.rel_residual(inp["A"], ref["X"], ref["Y"])
    assert abs(float(host(f.rel_residual)[0]) - res) <= 1e-10 * res
    api.synchronize()                      # every problem finished


@pytest.mark.parametrize("m,n,r,k", [(300, 200, 5, 15), (257, 190, 12, 22), (211, 333, 17, 27),
                                     (400, 150, 30, 40), (180, 260, 33, 45), (350, 300, 50, 60),
                                     (300, 280, 64, 74)])
def test_anls_fp64_parity_ragged_ranks(m, n, r, k):
    """Every specialisation of the wave solver (r rounded up to 8, 16, 24, 32,
    48, 64), ragged row counts."""
    A, U1, V1 = _nmf_input(m, n, r, seed=m + r)
    g = np.random.default_rng(k)
    oml, omr = g.standard_normal((n, k)), g.standard_normal((m, k))
    sk = O.sketch(A, oml, omr, 2)
    iters = 4
    ref = O.anls(sk["Ac"], sk["B"], sk["L"], sk["R"], V1, iters)
    f = api.factorize(dev(A), r, k, 2, dev(U1), dev(V1), dev(oml), dev(omr), method="anls", iters=iters)
    assert close64(host(f.U), ref["X"])
    assert close64(host(f.V), ref["Y"])


def test_anls_full_fp64_parity():
    A, U1, V1 = _nmf_input(613, 389, 7, seed=210)
    iters = 25
    ref = O.anls_uncompressed(A, V1, iters)
    f = api.factorize(dev(A), 7, 8, 0, dev(U1), dev(V1), method="anls_full", iters=iters)
    assert close64(host(f.U), ref["X"])
    assert close64(host(f.V), ref["Y"])


@pytest.mark.parametrize("method", ["anls", "anls_full"])
def test_anls_recovers_the_planted_factor(method):
    """A = W H exactly with V0 = H: one iteration gives U = W and V = H (the
    unique minimisers; zero residual)."""
    g = np.random.default_rng(220)
    m, n, r, k = 500, 300, 6, 16
    W, H = g.random((m, r)), g.random((r, n))
    A = W @ H
    U0 = np.full((m, r), 0.5)
    f = api.factorize(dev(A), r, k, 2, dev(U0), dev(H), None, None, method=method, iters=1, seed=3)
    assert np.abs(host(f.U) - W).max() < 1e-9
    assert np.abs(host(f.V) - H).max() < 1e-9
    assert float(host(f.rel_residual)[0]) < 1e-12


def test_anls_iterates_do_not_depend_on_the_warm_start():
    """U0 only seeds the first half-step's active sets."""
    A, U1, V1 = _nmf_input(400, 300, 9, seed=230)
    kw = dict(method="anls", iters=6, seed=11)
    f1 = api.factorize(dev(A), 9, 19, 2, dev(U1), dev(V1), None, None, **kw)
    f2 = api.factorize(dev(A), 9, 19, 2, dev(np.zeros_like(U1)), dev(V1), None, None, **kw)
    f3 = api.factorize(dev(A), 9, 19, 2, dev(np.ones_like(U1)), dev(V1), None, None, **kw)
    U1g, U2g, U3g = host(f1.U), host(f2.U), host(f3.U)
    assert np.abs(U1g - U2g).max() <= 1e-10 * np.abs(U1g).max()
    assert np.abs(U1g - U3g).max() <= 1e-10 * np.abs(U1g).max()


@pytest.mark.parametrize("method", ["anls", "anls_full"])
def test_anls_fp32_residual_gap(method):
    w = WL.WORKLOADS["nmf_fp32_20000x5000"]
    inp = WL.make_inputs(w, m=2000, n=900)
    A64 = inp["A"].astype(np.float64)
    iters = 10
    r = 20
    V1 = inp["V1"][:r]
    U1 = inp["U1"][:, :r]
    g = np.random.default_rng(240)
    k = r + 10
    oml, omr = g.standard_normal((900, k)), g.standard_normal((2000, k))
    if method == "anls":
        sk = O.sketch(A64, oml, omr, w.q)
        ref = O.anls(sk["Ac"], sk["B"], sk["L"], sk["R"], V1, iters)
    else:
        ref = O.anls_uncompressed(A64, V1, iters)
    res_o = O.rel_residual(A64, ref["X"], ref["Y"])
    f = api.factorize(dev(inp["A"], torch.float32), r, k, w.q, dev(U1), dev(V1), dev(oml), dev(omr),
                      method=method, iters=iters)
    res_g = float(host(f.rel_residual)[0])
    assert abs(res_g - res_o) <= 1e-3


def test_anls_full_size_last_half_step_is_optimal():
    """20000 x 5000, r 50, k 60, q 4, FP32 storage: V after the last
    iteration solves its NNLS problems against L^T U (checked in FP64 on the
    host for sampled columns, from the GPU's own L, B and U)."""
    w = WL.WORKLOADS["nmf_fp32_20000x5000"]
    gen = torch.Generator(device=DEV)
    gen.manual_seed(250)
    m, n, r, k = w.m, w.n, w.r, w.k
    Wf = torch.rand((m, r), generator=gen, device=DEV, dtype=torch.float32)
    Hf = torch.rand((r, n), generator=gen, device=DEV, dtype=torch.float32)
    A = Wf @ Hf + (0.05 * torch.randn((m, n), generator=gen, device=DEV, dtype=torch.float32)).abs()
    c = float(np.sqrt(4.0 * float(A.mean()) / r))
    U0 = c * torch.rand((m, r), generator=gen, device=DEV, dtype=torch.float64)
    V0 = c * torch.rand((r, n), generator=gen, device=DEV, dtype=torch.float64)
    f = api.factorize(A, r, k, w.q, U0, V0, None, None, method="anls", iters=5, seed=7, want_sketch=True)
    api.synchronize()
    Lg, Bg, Ug, Vg = host(f.sketch.L), host(f.sketch.B), host(f.U), host(f.V)
    C = Lg.T @ Ug                                   # k x r
    cols = np.random.default_rng(251).choice(n, 300, replace=False)
    Hs, Bs = Vg[:, cols], Bg[:, cols]
    grad = C.T @ (C @ Hs - Bs)                      # gradient of 1/2 ||C h - b||^2
    scale = np.abs(C.T @ Bs).max()
    assert Hs.min() >= 0
    # FP32 storage of U, V, B, L: optimality to a few 1e-6 of the scale
    assert grad.min() > -2e-5 * scale
    assert np.abs(grad * Hs).max() < 2e-5 * scale * np.abs(Hs).max()
    # and the sampled columns equal Lawson-Hanson's minimisers (FP64, on the
    # host) to the FP32 storage accuracy of V
    for j in range(20):
        ref, _ = scipy.optimize.nnls(C, Bs[:, j])
        assert np.abs(Hs[:, j] - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    res = float(host(f.rel_residual)[0])
    assert 0 < res < 0.05
