"""Host-side checks of the C ABI: the library loads without a GPU, exports
every symbol the header declares, and rejects invalid arguments before any
device work."""
import ctypes as C
import os
import re

import pytest

from paper_1505_04650_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "cnmf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:cnmf|snmf)_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libcnmf.so is not built (run python -m paper_1505_04650_amd.build)")
    return L.load()


def test_exports_every_declared_symbol(lib):
    syms = header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(syms) == sorted(L.EXPORTED)


def test_version_and_status_strings(lib):
    assert lib.cnmf_version().startswith(b"cnmf-mi355x")
    assert lib.cnmf_status_string(L.CNMF_EINVAL) == b"invalid argument"


def _desc(r=10, k=20, q=2, sides=L.CNMF_BOTH, method=L.CNMF_ADMM, iters=10, prec=L.CNMF_F32):
    sk = L.cnmf_sketch_desc(r, k, q, sides, prec, prec, 0, C.c_void_p(16), C.c_void_p(16))
    return L.cnmf_factorize_desc(sk, method, iters, 1.0, 1.0, 1.0, 0.0, C.c_void_p(16), C.c_void_p(16))


def test_workspace_bytes_is_host_only_and_grows(lib):
    out = C.c_size_t()
    d = _desc()
    assert lib.cnmf_workspace_bytes(2000, 1000, C.byref(d), C.byref(out)) == L.CNMF_OK
    small = out.value
    assert lib.cnmf_workspace_bytes(20000, 5000, C.byref(d), C.byref(out)) == L.CNMF_OK
    assert out.value > small > 0


@pytest.mark.parametrize("r,k,m,n", [(0, 5, 100, 100), (10, 10, 100, 100), (10, 200, 1000, 1000),
                                     (10, 20, 100, 15)])
def test_workspace_bytes_rejects_bad_shapes(lib, r, k, m, n):
    out = C.c_size_t()
    d = _desc(r=r, k=k)
    assert lib.cnmf_workspace_bytes(m, n, C.byref(d), C.byref(out)) == L.CNMF_EINVAL
    assert len(lib.cnmf_last_error(None)) > 0


def test_calls_without_handle_or_data_fail_cleanly(lib):
    A = L.cnmf_input(C.c_void_p(0), L.CNMF_F32, 100, 50, 50)
    sk = L.cnmf_sketch_desc(5, 10, 1, L.CNMF_BOTH, L.CNMF_F32, L.CNMF_F32, 0, None, None)
    out = L.cnmf_sketch_out()
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(sk), C.byref(out)) == L.CNMF_EINVAL
    A.data_dev = C.c_void_p(16)
    A.lda = 40
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(sk), C.byref(out)) == L.CNMF_EINVAL
    assert b"lda" in lib.cnmf_last_error(None)
    A.lda = 50
    # NULL test matrices are valid (drawn on the device from the seed): only the handle is missing
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(sk), C.byref(out)) == L.CNMF_EINVAL
    assert b"handle" in lib.cnmf_last_error(None)
    sk.omega_left_dev = C.c_void_p(16)
    sk.omega_right_dev = C.c_void_p(16)
    sk.k = 51
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(sk), C.byref(out)) == L.CNMF_EINVAL  # k > min(m, n)
    sk.k = 10
    sk.pass_dtype = L.CNMF_F64
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(sk), C.byref(out)) == L.CNMF_EINVAL  # F64 pass, F32 input
    sk.pass_dtype = L.CNMF_F32
    # everything valid but no handle
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(sk), C.byref(out)) == L.CNMF_EINVAL
    assert b"handle" in lib.cnmf_last_error(None)


def test_factorize_parameter_checks(lib):
    A = L.cnmf_input(C.c_void_p(16), L.CNMF_F32, 100, 50, 50)
    out = L.cnmf_factorize_out()
    d = _desc(r=5, k=10)
    d.lambda_ = 0.0
    assert lib.cnmf_factorize(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_EINVAL
    d.lambda_ = 1.0
    d.sk.sides = L.CNMF_LEFT
    assert lib.cnmf_factorize(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_EINVAL
    d.sk.sides = L.CNMF_BOTH
    d.iters = -1
    assert lib.cnmf_factorize(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_EINVAL


@pytest.mark.parametrize("r,k,ok", [(64, 112, True), (48, 128, True), (64, 113, False), (64, 128, False)])
def test_admm_solve_lds_limit(lib, r, k, ok):
    # the r x r solves of one iteration run in one workgroup's LDS
    A = L.cnmf_input(C.c_void_p(16), L.CNMF_F32, 2000, 1000, 1000)
    d = _desc(r=r, k=k)
    out = L.cnmf_factorize_out()
    st = lib.cnmf_factorize(None, C.byref(A), C.byref(d), C.byref(out))
    if ok:
        assert st == L.CNMF_EINVAL and b"handle" in lib.cnmf_last_error(None)
    else:
        assert st == L.CNMF_ENOTSUP and b"LDS" in lib.cnmf_last_error(None)
    d.method = L.CNMF_MU
    assert lib.cnmf_factorize(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_EINVAL


def test_gaussian_and_synchronize_argument_checks(lib):
    out = C.c_void_p(16)
    assert lib.cnmf_gaussian(None, 1, 0, 10, 4, out, 4) == L.CNMF_EINVAL
    assert b"handle" in lib.cnmf_last_error(None)
    assert lib.cnmf_synchronize(None) == L.CNMF_EINVAL


def test_seeded_sketch_workspace_holds_the_test_matrices(lib):
    """NULL test matrices are drawn into the workspace: (m + n) k doubles more."""
    given, seeded = _desc(r=50, k=60, q=4), _desc(r=50, k=60, q=4)
    seeded.sk.omega_left_dev = None
    seeded.sk.omega_right_dev = None
    a, b = C.c_size_t(), C.c_size_t()
    assert lib.cnmf_workspace_bytes(20000, 5000, C.byref(given), C.byref(a)) == L.CNMF_OK
    assert lib.cnmf_workspace_bytes(20000, 5000, C.byref(seeded), C.byref(b)) == L.CNMF_OK
    assert b.value - a.value >= 8 * (20000 + 5000) * 60


def test_snmf_nnls_argument_checks(lib):
    p = C.c_void_p(16)
    assert lib.snmf_nnls(None, p, L.CNMF_F32, 30, 100, 100, 20, p, p, 100, None) == L.CNMF_EINVAL
    assert b"handle" in lib.cnmf_last_error(None)
    assert lib.snmf_nnls(None, p, L.CNMF_F32, 30, 100, 100, 31, p, p, 100, None) == L.CNMF_EINVAL   # r > k
    assert lib.snmf_nnls(None, p, L.CNMF_F32, 30, 100, 100, 20, p, p, 99, None) == L.CNMF_EINVAL    # ldh < n
    assert lib.snmf_nnls(None, p, L.CNMF_F32, 100, 100, 100, 65, p, p, 100, None) == L.CNMF_ENOTSUP
    assert lib.snmf_nnls(None, None, L.CNMF_F32, 30, 100, 100, 20, p, p, 100, None) == L.CNMF_EINVAL


def test_python_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(FileNotFoundError):
        L._lib_backup = L._lib
        try:
            L._lib = None
            L.load(str(tmp_path / "missing.so"))
        finally:
            L._lib = L._lib_backup


def test_precision_combinations(lib):
    """Reduced-precision passes need an FP32 input; B and the last range
    pass need at least BF16; the workspace grows by the A / A^T copies."""
    A = L.cnmf_input(C.c_void_p(16), L.CNMF_F32, 100, 50, 50)
    sk = L.cnmf_sketch_desc(5, 10, 1, L.CNMF_BOTH, L.CNMF_FP8_E4M3, L.CNMF_FP8_E4M3, 0, C.c_void_p(16),
                            C.c_void_p(16))
    out = L.cnmf_sketch_out()
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(sk), C.byref(out)) == L.CNMF_ENOTSUP
    assert b"BF16" in lib.cnmf_last_error(None)
    sk.final_dtype = L.CNMF_BF16
    # valid combination: fails only for the missing handle
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(sk), C.byref(out)) == L.CNMF_EINVAL
    assert b"handle" in lib.cnmf_last_error(None)
    A64 = L.cnmf_input(C.c_void_p(16), L.CNMF_F64, 100, 50, 50)
    assert lib.cnmf_sketch(None, C.byref(A64), C.byref(sk), C.byref(out)) == L.CNMF_EINVAL
    sizes = {}
    for name, p, f in (("f32", L.CNMF_F32, L.CNMF_F32), ("bf16", L.CNMF_BF16, L.CNMF_BF16),
                       ("fp8", L.CNMF_FP8_E4M3, L.CNMF_BF16), ("fp8f32", L.CNMF_FP8_E4M3, L.CNMF_F32)):
        d = _desc(r=50, k=60, q=4)
        d.sk.pass_dtype, d.sk.final_dtype = p, f
        o = C.c_size_t()
        assert lib.cnmf_workspace_bytes(20000, 5000, C.byref(d), C.byref(o)) == L.CNMF_OK
        sizes[name] = o.value
    mn = 20000 * 5000
    assert sizes["bf16"] >= 4 * mn                         # BF16 A and A^T copies
    assert sizes["fp8"] >= 6 * mn                          # FP8 copies + the BF16 ones for the final passes
    assert sizes["fp8f32"] >= 2 * mn
    assert sizes["fp8"] > sizes["bf16"] > sizes["f32"]


def test_lowp_range_product_argument_checks(lib):
    A = L.cnmf_input(C.c_void_p(16), L.CNMF_F32, 100, 50, 50)
    X = C.c_void_p(16)
    assert lib.cnmf_range_product_lowp(None, C.byref(A), 0, L.CNMF_F32, X, 8, X) == L.CNMF_EINVAL
    assert lib.cnmf_range_product_lowp(None, C.byref(A), 0, L.CNMF_BF16, X, 0, X) == L.CNMF_EINVAL
    assert lib.cnmf_range_product_lowp(None, C.byref(A), 2, L.CNMF_BF16, X, 8, X) == L.CNMF_EINVAL
    A64 = L.cnmf_input(C.c_void_p(16), L.CNMF_F64, 100, 50, 50)
    assert lib.cnmf_range_product_lowp(None, C.byref(A64), 0, L.CNMF_BF16, X, 8, X) == L.CNMF_EINVAL
    assert lib.cnmf_range_product_lowp(None, C.byref(A), 0, L.CNMF_FP8_E4M3, X, 8, X) == L.CNMF_EINVAL
    assert b"handle" in lib.cnmf_last_error(None)


def test_anls_method_checks(lib):
    """Alternating NNLS: a known method; compressed form needs both sides;
    unknown method numbers are refused."""
    A = L.cnmf_input(C.c_void_p(16), L.CNMF_F32, 2000, 1000, 1000)
    out = L.cnmf_factorize_out()
    d = _desc(method=L.CNMF_ANLS)
    st = lib.cnmf_factorize(None, C.byref(A), C.byref(d), C.byref(out))
    assert st == L.CNMF_EINVAL and b"handle" in lib.cnmf_last_error(None)
    d.sk.sides = L.CNMF_LEFT
    assert lib.cnmf_factorize(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_EINVAL
    assert b"sides" in lib.cnmf_last_error(None)
    d = _desc(method=6)
    assert lib.cnmf_factorize(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_EINVAL
    assert b"unknown method" in lib.cnmf_last_error(None)
    # the compressed form keeps Ac = A R^T in its workspace, the full form two pass operands
    a, b, c = C.c_size_t(), C.c_size_t(), C.c_size_t()
    assert lib.cnmf_workspace_bytes(20000, 5000, C.byref(_desc(r=50, k=60, method=L.CNMF_ADMM)), C.byref(a)) == 0
    assert lib.cnmf_workspace_bytes(20000, 5000, C.byref(_desc(r=50, k=60, method=L.CNMF_ANLS)), C.byref(b)) == 0
    assert lib.cnmf_workspace_bytes(20000, 5000, C.byref(_desc(r=50, k=60, method=L.CNMF_ANLS_FULL)),
                                    C.byref(c)) == 0
    assert b.value > a.value and c.value > 0


def test_input_format_checks(lib):
    """Unknown formats, CSR without its index arrays, a negative block size
    and reduced-precision passes on a non-dense input are refused before
    anything runs."""
    out = L.cnmf_sketch_out()
    d = _desc().sk
    A = L.cnmf_input(C.c_void_p(16), L.CNMF_F32, 2000, 1000, 1000, 7)
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_EINVAL
    assert b"format" in lib.cnmf_last_error(None)
    A = L.cnmf_input(C.c_void_p(16), L.CNMF_F32, 2000, 1000, 1000, L.CNMF_CSR, 0, None, None, 10, 0)
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_EINVAL
    assert b"rowptr" in lib.cnmf_last_error(None)
    A = L.cnmf_input(C.c_void_p(16), L.CNMF_F32, 2000, 1000, 1000, L.CNMF_DENSE_HOST, 0, None, None, 0, -5)
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_EINVAL
    assert b"block_rows" in lib.cnmf_last_error(None)
    A = L.cnmf_input(C.c_void_p(16), L.CNMF_F32, 2000, 1000, 1000, L.CNMF_DENSE_HOST)
    d.pass_dtype = L.CNMF_BF16
    d.final_dtype = L.CNMF_BF16
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_ENOTSUP
    assert b"dense on the device" in lib.cnmf_last_error(None)


def test_test_matrix_kind_checks(lib):
    out = L.cnmf_sketch_out()
    d = _desc().sk
    d.test_matrix = 5
    A = L.cnmf_input(C.c_void_p(16), L.CNMF_F32, 2000, 1000, 1000)
    assert lib.cnmf_sketch(None, C.byref(A), C.byref(d), C.byref(out)) == L.CNMF_EINVAL
    assert b"test_matrix" in lib.cnmf_last_error(None)
    assert lib.cnmf_srht(None, 1, 0, 100, 10, C.c_void_p(16), 10) == L.CNMF_EINVAL
    assert b"handle" in lib.cnmf_last_error(None)
