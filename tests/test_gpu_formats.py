"""GPU parity of the two other input formats, through the C ABI:

* dense A in host memory, streamed through the device in row blocks (the
  paper's big-data setting, Section 2.1: A larger than the device's memory;
  only the k-column sketches stay resident).  Small row blocks with a ragged
  last block exercise the double-buffered copies; the results must equal the
  oracle's (FP64, 1e-10) and, to rounding, the device-resident path's.
* sparse A in compressed-row form (the paper's sparse synthetic inputs,
  Section 5.1): products with A and with its transpose built on the device;
  the oracle runs on the same matrix densified.
"""
import numpy as np
import pytest

from oracle import cnmf_oracle as O
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


def pinned(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).pin_memory()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def close64(a, b, tol=1e-10):
    assert a.shape == b.shape
    fro = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    elem = float(np.abs(a - b).max() / np.abs(b).max())
    return fro < tol and elem < tol


@pytest.fixture(scope="module")
def c1():
    w = WL.WORKLOADS["plain_fp64_1000x500"]
    inp = WL.make_inputs(w)
    sk = O.sketch(inp["A"], inp["Omega_L"], inp["Omega_R"], w.q)
    lam = float(np.linalg.svd(sk["At"], compute_uv=False)[w.r - 1])
    return w, inp, sk, lam


# --------------------------------------------------------------------------
# dense A in host memory
# --------------------------------------------------------------------------

@pytest.mark.parametrize("block_rows", [128, 333, 0])
def test_host_streamed_sketch_fp64(c1, block_rows):
    """1000 x 500 FP64, q 4, two-sided: blocks of 128 (7 full + 104), 333
    (odd size) and the default (one block)."""
    w, inp, sk, _ = c1
    A = inp["A"]
    out = api.sketch(pinned(A), w.r, w.k, w.q, dev(inp["Omega_L"]), dev(inp["Omega_R"]), want_ac=True,
                     block_rows=block_rows)
    res = api.sketch(dev(A), w.r, w.k, w.q, dev(inp["Omega_L"]), dev(inp["Omega_R"]), want_ac=True)
    for name in ("L", "R", "B", "At", "Ac"):
        assert close64(host(getattr(out, name)), sk[name]), name
    # the projection of A is the device-resident path's to rounding (the
    # trailing basis columns are sensitive to the summation order; the
    # projection is not)
    Lh, Ld = host(out.L), host(res.L)
    assert np.linalg.norm(Lh @ (Lh.T @ A) - Ld @ (Ld.T @ A)) <= 1e-13 * np.linalg.norm(A)
    st = host(out.stats)
    assert st[0] < 1e-13 and st[1] < 1e-13 and st[3] == 0


def test_host_streamed_factorize_admm_fp64(c1):
    w, inp, sk, lam = c1
    iters = 40
    ref = O.admm(sk["At"], sk["L"], sk["R"], inp["U1"], inp["V1"], lam, lam, 1.0, iters)
    f = api.factorize(pinned(inp["A"]), w.r, w.k, w.q, dev(inp["U1"]), dev(inp["V1"]), dev(inp["Omega_L"]),
                      dev(inp["Omega_R"]), iters=iters, lam=lam, phi=lam, block_rows=96)
    assert close64(host(f.U), ref["U"])
    assert close64(host(f.V), ref["V"])
    res = O.rel_residual(inp["A"], ref["U"], ref["V"])
    assert abs(float(host(f.rel_residual)[0]) - res) <= 1e-10 * res


def test_host_streamed_uncompressed_mu_fp64():
    """The uncompressed comparators stream A twice per iteration."""
    g = np.random.default_rng(400)
    m, n, r = 613, 389, 7
    A = g.random((m, r)) @ g.random((r, n)) + np.abs(0.01 * g.standard_normal((m, n)))
    U1, V1 = WL.init_factors(A.mean(), m, n, r, 401)
    ref = O.mu_uncompressed(A, U1, V1, 20, 1e-16)
    f = api.factorize(pinned(A), r, r + 1, 0, dev(U1), dev(V1), method="mu_full", iters=20, mu_eps=1e-16,
                      block_rows=100)
    assert close64(host(f.U), ref["X"])
    assert close64(host(f.V), ref["Y"])


def test_host_streamed_select_fp32_equals_device_path():
    A, planted = WL.separable_matrix(3000, 20000, 12, 1e-3, seed=402, dtype=np.float32)
    kw = dict(sides="both", seed=403, want_B=True)
    Kh, _, Bh = api.select(pinned(A, torch.float32), 12, 22, 2, block_rows=700, **kw)
    Kd, _, Bd = api.select(dev(A, torch.float32), 12, 22, 2, **kw)
    assert sorted(host(Kh).astype(np.int64).tolist()) == list(planted)
    assert torch.equal(Kh, Kd)
    Bh, Bd = host(Bh), host(Bd)
    assert np.abs(Bh - Bd).max() <= 1e-5 * np.abs(Bd).max()


# --------------------------------------------------------------------------
# sparse A (CSR)
# --------------------------------------------------------------------------

def csr(rowptr, colind, vals, m, n, dtype=torch.float64):
    return torch.sparse_csr_tensor(torch.as_tensor(rowptr, device=DEV), torch.as_tensor(colind.astype(np.int64),
                                   device=DEV), torch.as_tensor(vals, dtype=dtype, device=DEV), size=(m, n))


def to_csr(A):
    mask = A != 0
    rowptr = np.zeros(A.shape[0] + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(mask.sum(axis=1))
    rows, cols = np.nonzero(mask)
    return rowptr, cols.astype(np.int32), A[rows, cols]


@pytest.fixture(scope="module")
def sparse_case():
    m, n, r, k = 2000, 1500, 10, 20
    _, _, _, A = WL.sparse_nmf_matrix(m, n, r, 0.1, seed=410)
    # empty rows (first, inner, last) and empty columns
    A[[0, 17, 1999], :] = 0.0
    A[:, [3, 1499]] = 0.0
    rowptr, colind, vals = to_csr(A)
    g = np.random.default_rng(411)
    oml, omr = g.standard_normal((n, k)), g.standard_normal((m, k))
    sk = O.sketch(A, oml, omr, 2)
    return m, n, r, k, rowptr, colind, vals, A, oml, omr, sk


def test_csr_sketch_fp64(sparse_case):
    m, n, r, k, rowptr, colind, vals, A, oml, omr, sk = sparse_case
    assert (np.diff(rowptr) == 0).any()            # some rows are empty
    out = api.sketch(csr(rowptr, colind, vals, m, n), r, k, 2, dev(oml), dev(omr), want_ac=True)
    for name in ("L", "R", "B", "At", "Ac"):
        assert close64(host(getattr(out, name)), sk[name]), name
    api.synchronize()


@pytest.mark.parametrize("method", ["admm", "anls"])
def test_csr_factorize_fp64(sparse_case, method):
    m, n, r, k, rowptr, colind, vals, A, oml, omr, sk = sparse_case
    U1, V1 = WL.init_factors(max(A.mean(), 1e-3), m, n, r, 412)
    iters = 15
    lam = float(np.linalg.svd(sk["At"], compute_uv=False)[r - 1])
    if method == "admm":
        ref = O.admm(sk["At"], sk["L"], sk["R"], U1, V1, lam, lam, 1.0, iters)
        Ur, Vr = ref["U"], ref["V"]
    else:
        ref = O.anls(sk["Ac"], sk["B"], sk["L"], sk["R"], V1, iters)
        Ur, Vr = ref["X"], ref["Y"]
    f = api.factorize(csr(rowptr, colind, vals, m, n), r, k, 2, dev(U1), dev(V1), dev(oml), dev(omr),
                      method=method, iters=iters, lam=lam, phi=lam)
    assert close64(host(f.U), Ur)
    assert close64(host(f.V), Vr)
    # the residual from the nonzeros and the Gram matrices equals the dense one
    res = O.rel_residual(A, Ur, Vr)
    assert abs(float(host(f.rel_residual)[0]) - res) <= 1e-9 * res


def test_csr_uncompressed_anls_fp64():
    m, n, r = 700, 525, 6
    rowptr, colind, vals, A = WL.sparse_nmf_matrix(m, n, r, 0.2, seed=420)
    A = np.abs(A)
    vals = np.abs(vals)
    U1, V1 = WL.init_factors(A.mean(), m, n, r, 421)
    ref = O.anls_uncompressed(A, V1, 8)
    f = api.factorize(csr(rowptr, colind, vals, m, n), r, r + 1, 0, dev(U1), dev(V1), method="anls_full",
                      iters=8)
    assert close64(host(f.U), ref["X"])
    assert close64(host(f.V), ref["Y"])


def test_csr_fp32_residual_gap():
    m, n, r, k = 4000, 3000, 16, 26
    rowptr, colind, vals, A = WL.sparse_nmf_matrix(m, n, r, 0.1, seed=430, dtype=np.float32)
    A64 = A.astype(np.float64)
    g = np.random.default_rng(431)
    oml, omr = g.standard_normal((n, k)), g.standard_normal((m, k))
    U1, V1 = WL.init_factors(A64.mean(), m, n, r, 432)
    sk = O.sketch(A64, oml, omr, 2)
    lam = float(np.linalg.svd(sk["At"], compute_uv=False)[r - 1])
    ref = O.admm(sk["At"], sk["L"], sk["R"], U1, V1, lam, lam, 1.0, 30)
    res_o = O.rel_residual(A64, ref["U"], ref["V"])
    f = api.factorize(csr(rowptr, colind, vals, m, n, torch.float32), r, k, 2, dev(U1), dev(V1), dev(oml),
                      dev(omr), iters=30, lam=lam, phi=lam)
    assert abs(float(host(f.rel_residual)[0]) - res_o) <= 1e-3
    # the GPU's own factors give the residual it reports (FP64 on the host)
    assert abs(float(host(f.rel_residual)[0]) - O.rel_residual(A64, host(f.U), host(f.V))) <= 1e-6


def test_csr_bad_column_index_is_reported(sparse_case):
    m, n, r, k, rowptr, colind, vals, A, oml, omr, sk = sparse_case
    bad = colind.copy()
    bad[7] = n + 3                                  # outside [0, n): skipped and counted
    ci = torch.as_tensor(bad, device=DEV)
    inp = L.cnmf_input(0, L.CNMF_F64, m, n, n, L.CNMF_CSR, 0, 0, 0, len(vals), 0)
    rp = torch.as_tensor(rowptr, device=DEV)
    vv = dev(vals)
    inp.data_dev, inp.rowptr_dev, inp.colind_dev = vv.data_ptr(), rp.data_ptr(), ci.data_ptr()
    h = api.default_handle()
    Lt = torch.empty((m, k), dtype=torch.float64, device=DEV)
    d = api._sketch_desc(r, k, 2, L.CNMF_LEFT, dev(oml), None, "f64", "f64", 0)
    out = L.cnmf_sketch_out(api._ptr(Lt), None, None, None, None, None)
    import ctypes as C
    L.check(h._lib.cnmf_sketch(h.raw, C.byref(inp), C.byref(d), C.byref(out)), h.raw)
    with pytest.raises(L.CnmfError) as e:
        api.synchronize()
    assert e.value.status == L.CNMF_EBREAKDOWN
    api.synchronize()


def test_csr_without_nonzeros():
    """nnz = 0: the products are zero, the fallback completes the bases with
    Gaussian columns (orthonormal), the factorisation's residual is 0."""
    m, n, r, k = 300, 200, 4, 10
    A = torch.sparse_csr_tensor(torch.zeros(m + 1, dtype=torch.int64, device=DEV),
                                torch.zeros(0, dtype=torch.int64, device=DEV),
                                torch.zeros(0, dtype=torch.float64, device=DEV), size=(m, n))
    out = api.sketch(A, r, k, 1, None, None, seed=4)
    Lg = host(out.L)
    assert np.abs(Lg.T @ Lg - np.eye(k)).max() < 1e-13
    assert np.abs(host(out.B)).max() == 0.0
    U1, V1 = WL.init_factors(0.1, m, n, r, 5)
    f = api.factorize(A, r, k, 1, dev(U1), dev(V1), None, None, iters=3, lam=1.0, phi=1.0, seed=4)
    assert float(host(f.rel_residual)[0]) == 0.0
    api.synchronize()


def test_host_block_larger_than_the_matrix(c1):
    w, inp, sk, _ = c1
    out = api.sketch(pinned(inp["A"]), w.r, w.k, w.q, dev(inp["Omega_L"]), dev(inp["Omega_R"]),
                     block_rows=10 ** 6)
    assert close64(host(out.L), sk["L"])
