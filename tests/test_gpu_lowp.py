"""Precision form of the range-finder passes (BF16 / FP8 E4M3 operands, FP32
accumulation, FP64 CholeskyQR2), through the C ABI.

Two levels:
  * the pass kernel against a host emulation of its rounding: A and the
    operand are rounded exactly as the kernels round them (BF16 round to
    nearest even; FP8 E4M3 with a power-of-two scale per 128x128 tile of A
    and a power-of-two column scale for the operand), the product of the rounded
    values is taken in FP64, and the GPU's FP32 accumulation must agree to
    a bound derived from the FP32 unit roundoff;
  * the whole sketch / factorisation against the FP64 oracle: the error of
    every result is measured, and the residual-type results must match the
    oracle's to a relative-residual gap of 1e-3.
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
TILE = 128


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# --------------------------------------------------------------------------
# host emulation of the roundings (independent of the library)
# --------------------------------------------------------------------------

def bf16(x):
    """float32 -> bfloat16 (round to nearest even), returned as float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def e4m3(x):
    """Round to OCP FP8 E4M3 (bias 7, 3 mantissa bits, subnormal quantum
    2^-9, largest finite 448), round to nearest even; |x| <= 448 here."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    _, e = np.frexp(np.where(a > 0, a, 1.0))       # a = f 2^e, f in [0.5, 1)
    ex = np.maximum(e - 1, -6)                      # unbiased exponent, clamped to the normal minimum
    q = np.ldexp(1.0, ex - 3)                       # spacing of the binade
    r = np.round(a / q) * q                         # numpy rounds halves to even
    assert r.max(initial=0.0) <= 448.0
    return np.sign(x) * r


def tile_exponent(tmax):
    """Smallest e with tmax / 2^e <= 448 (written from that definition: a
    search from above), clamped to [-126, 127]."""
    e = 127
    while e > -126 and tmax / 2.0 ** (e - 1) <= 448.0:
        e -= 1
    return e


def quant_a_fp8(A32):
    """A (float32) -> dequantised FP8 copy with per-tile power-of-two scales."""
    m, n = A32.shape
    out = np.empty((m, n), dtype=np.float64)
    for i0 in range(0, m, TILE):
        for j0 in range(0, n, TILE):
            t = A32[i0:i0 + TILE, j0:j0 + TILE]
            tmax = float(np.abs(t).max())
            e = tile_exponent(tmax) if tmax > 0 else 0
            q = e4m3(t.astype(np.float64) * 2.0 ** -e)
            out[i0:i0 + TILE, j0:j0 + TILE] = q * 2.0 ** e
    return out


def quant_x(X64, kind):
    x32 = X64.astype(np.float32)
    if kind == "bf16":
        return bf16(x32)
    out = np.empty_like(X64)
    for c in range(X64.shape[1]):
        mx = np.abs(X64[:, c]).max()
        s = 1.0
        if mx > 0:
            _, e = np.frexp(256.0 / mx)
            s = math.ldexp(1.0, int(e) - 1)
        out[:, c] = e4m3((X64[:, c] * s).astype(np.float32)) / s
    return out


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
@pytest.mark.parametrize("shape", [(1037, 523, 21), (300, 4099, 128), (257, 129, 16), (5, 7, 3), (128, 256, 48)])
def test_lowp_pass_matches_emulated_rounding(kind, shape):
    m, n, kx = shape
    g = np.random.default_rng(m * 7 + n + kx)
    # nonnegative data with a spread of magnitudes per tile, plus exact zeros
    A32 = (g.random((m, n)) * np.exp(g.standard_normal((m, 1)))).astype(np.float32)
    A32[:, :: 11] = 0.0
    X = g.standard_normal((n, kx))
    Z = g.standard_normal((m, kx))
    Ad = dev(A32, torch.float32)
    Y = host(api.range_product_lowp(Ad, dev(X), trans=False, pass_dtype=kind))
    W = host(api.range_product_lowp(Ad, dev(Z), trans=True, pass_dtype=kind))
    Aq = bf16(A32) if kind == "bf16" else quant_a_fp8(A32)
    Xq, Zq = quant_x(X, kind), quant_x(Z, kind)
    # FP32 accumulation: |error| <= c * n * u * (|A| |X|), u = 2^-24, plus
    # one rounding per 128-column chunk.  The FP8 MFMA itself does not add
    # its products exactly: it aligns a group of products to the group's
    # largest exponent and keeps about 13 bits below it (measured on gfx950:
    # a product of -110 next to one of 114688 entered the sum as -104, and
    # -3.375 next to 114688 vanished), while the accumulator it adds them to
    # keeps FP32 precision (2^20 + 1 stays exact).  Every 128-column chunk is
    # one instruction, so that loss is bounded per chunk; 2^-9 of the chunk's
    # |A| |X| covers it.
    for got, ref, bound in ((Y, Aq @ Xq, np.abs(Aq) @ np.abs(Xq)), (W, Aq.T @ Zq, np.abs(Aq.T) @ np.abs(Zq))):
        kdim = n if got is Y else m
        tol = 4.0 * (kdim + 2 * (kdim // TILE + 1)) * 2.0 ** -24 + (2.0 ** -9 if kind == "fp8" else 0.0)
        assert np.all(np.abs(got - ref) <= tol * bound + 1e-30)
    if kind == "fp8":
        # the chunk loss is small on average: far below one FP8 rounding (2^-4)
        err = np.abs(Y - Aq @ Xq) / (np.abs(Aq) @ np.abs(Xq) + 1e-30)
        assert float(np.median(err)) < 2.0 ** -12


def test_lowp_rounding_is_not_fp32():
    """The pass really runs in the reduced type: the FP8 result differs from
    the FP32 product by the FP8 rounding, not by FP32 rounding."""
    g = np.random.default_rng(3)
    A32 = g.random((512, 384)).astype(np.float32)
    X = g.standard_normal((384, 16))
    Ad = dev(A32, torch.float32)
    exact = A32.astype(np.float64) @ X
    y8 = host(api.range_product_lowp(Ad, dev(X), pass_dtype="fp8"))
    y16 = host(api.range_product_lowp(Ad, dev(X), pass_dtype="bf16"))
    e8, e16 = rel(y8, exact), rel(y16, exact)
    assert 1e-3 < e8 < 0.1
    assert 1e-5 < e16 < 1e-2
    assert e8 > 4 * e16


# --------------------------------------------------------------------------
# whole sketch against the FP64 oracle (the 100000 x 20000 precision recipe
# at reduced size: r = 100, k = 120, q = 4, FP32 storage)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def prec_case():
    w = WL.WORKLOADS["precision_100000x20000"]
    m, n = 6000, 2400
    inp = WL.make_inputs(w, m=m, n=n, want_init=False)
    A64 = inp["A"].astype(np.float64)
    sk = O.sketch(A64, inp["Omega_L"], inp["Omega_R"], w.q)
    return w, inp, A64, sk


def _proj_res_left(A, L):
    return float(np.linalg.norm(A - L @ (L.T @ A)) / np.linalg.norm(A))


def _proj_res_right(A, R):
    return float(np.linalg.norm(A - (A @ R.T) @ R) / np.linalg.norm(A))


@pytest.mark.parametrize("pass_dtype,final_dtype", [("f32", "f32"), ("bf16", "bf16"), ("fp8", "bf16"), ("fp8", "f32"),
                                                    ("bf16", "f32")])
def test_sketch_lowp_vs_fp64_oracle(prec_case, pass_dtype, final_dtype):
    w, inp, A64, sk = prec_case
    out = api.sketch(dev(inp["A"], torch.float32), w.r, w.k, w.q, dev(inp["Omega_L"]), dev(inp["Omega_R"]),
                     pass_dtype=pass_dtype, final_dtype=final_dtype)
    L, R, B, At = host(out.L), host(out.R), host(out.B), host(out.At)
    st = host(out.stats)
    # FP64 CholeskyQR2 restores orthonormality to FP32 storage level
    assert st[0] < 1e-5 and st[1] < 1e-5 and st[2] == 0
    errs = {}
    # per-result errors against the oracle
    errs["L_top_r_sin"] = float(np.sqrt(max(0.0, 1 - np.linalg.svd(L[:, : w.r].T @ sk["L"][:, : w.r],
                                                                    compute_uv=False).min() ** 2)))
    errs["B_vs_LtA"] = rel(B, L.T @ A64)          # B against the product of the GPU's own L
    errs["At_vs_BRt"] = rel(At, (L.T @ A64) @ R.T)
    rl_g, rl_o = _proj_res_left(A64, L), _proj_res_left(A64, sk["L"])
    rr_g, rr_o = _proj_res_right(A64, R), _proj_res_right(A64, sk["R"])
    errs["left_residual_gap"] = abs(rl_g - rl_o)
    errs["right_residual_gap"] = abs(rr_g - rr_o)
    print(f"\n[{pass_dtype}/{final_dtype}] " + " ".join(f"{k}={v:.3e}" for k, v in errs.items()))
    assert errs["left_residual_gap"] <= 1e-3
    assert errs["right_residual_gap"] <= 1e-3
    # the final pass precision bounds the sketch products
    fin_tol = 2e-2 if final_dtype == "bf16" else 1e-5
    assert errs["B_vs_LtA"] < fin_tol
    assert errs["At_vs_BRt"] < fin_tol
    assert errs["L_top_r_sin"] < 0.05


@pytest.mark.parametrize("pass_dtype", ["bf16", "fp8"])
def test_factorize_lowp_residual_gap(pass_dtype):
    """Compressed ADMM on a reduced-precision sketch: the relative residual
    is within 1e-3 of the FP64 oracle's on the same inputs."""
    w = WL.WORKLOADS["nmf_fp32_20000x5000"]
    inp = WL.make_inputs(w, m=5000, n=2000)
    A64 = inp["A"].astype(np.float64)
    sk = O.sketch(A64, inp["Omega_L"], inp["Omega_R"], w.q)
    lam = float(np.linalg.svd(sk["At"], compute_uv=False)[w.r - 1])
    iters = 60
    adm = O.admm(sk["At"], sk["L"], sk["R"], inp["U1"], inp["V1"], lam, lam, 1.0, iters)
    res_o = O.rel_residual(A64, adm["U"], adm["V"])
    f = api.factorize(dev(inp["A"], torch.float32), w.r, w.k, w.q, dev(inp["U1"]), dev(inp["V1"]),
                      dev(inp["Omega_L"]), dev(inp["Omega_R"]), iters=iters, lam=lam, phi=lam,
                      pass_dtype=pass_dtype, final_dtype="bf16")
    res_g = float(host(f.rel_residual)[0])
    print(f"\n[{pass_dtype}] residual gpu={res_g:.6e} oracle={res_o:.6e} gap={abs(res_g - res_o):.3e}")
    assert abs(res_g - res_o) <= 1e-3


def test_final_fp8_is_refused():
    g = np.random.default_rng(1)
    A = dev(g.random((300, 200)), torch.float32)
    om, omr = dev(g.standard_normal((200, 20))), dev(g.standard_normal((300, 20)))
    with pytest.raises(Exception, match="BF16"):
        api.sketch(A, 10, 20, 1, om, omr, pass_dtype="fp8", final_dtype="fp8")
