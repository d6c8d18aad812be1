"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each checks a defining property,
a closed form, a theorem's bound, a special case that reduces to a library
routine, or an invariant derived from the update rules.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

from oracle import cnmf_oracle as O
from paper_1505_04650_amd import workloads as WL


def rng(s):
    return np.random.default_rng(s)


# --------------------------------------------------------------------------
# Alg. 1 (Section 2)
# --------------------------------------------------------------------------

def test_orth_plus_defining_properties():
    """Q^T Q = I and Y = Q T with T upper triangular, diag(T) > 0 (unique QR)."""
    Y = rng(1).standard_normal((300, 17))
    Q = O.orth_plus(Y)
    T = Q.T @ Y
    assert np.abs(Q.T @ Q - np.eye(17)).max() < 1e-14
    assert np.abs(np.tril(T, -1)).max() < 1e-13
    assert np.all(np.diag(T) > 0)
    assert np.abs(Q @ np.triu(T) - Y).max() < 1e-13


@pytest.mark.parametrize("q", [0, 1])
def test_range_finder_equals_literal_power_scheme(q):
    """Alg. 1 as printed, (A A^T)^q A Omega then one QR, equals the
    re-orthonormalised iteration when the spectrum is flat enough that the
    literal product is well conditioned."""
    g = rng(2 + q)
    A = g.standard_normal((80, 60))
    Om = g.standard_normal((60, 12))
    literal = O.orth_plus(np.linalg.matrix_power(A @ A.T, q) @ A @ Om)
    assert np.abs(O.range_finder(A, Om, q) - literal).max() < 1e-11


@pytest.mark.parametrize("q", [0, 2, 4])
def test_exact_rank_r_is_captured(q):
    """sigma_{r+1} = 0 for an exactly rank-r nonnegative A, so with k >= r the
    projection residual of Eq. (compression_approximation) vanishes."""
    g = rng(10 + q)
    m, n, r, k = 300, 200, 6, 16
    A = g.random((m, r)) @ g.random((r, n))
    L = O.range_finder(A, g.standard_normal((n, k)), q)
    assert np.abs(L.T @ L - np.eye(k)).max() < 1e-14
    res = np.linalg.norm(A - L @ (L.T @ A)) / np.linalg.norm(A)
    assert res < 1e-13


def test_full_width_sketch_reproduces_a():
    g = rng(20)
    A = g.random((50, 30))
    L = O.range_finder(A, g.standard_normal((30, 30)), 1)
    assert np.abs(L @ (L.T @ A) - A).max() < 1e-12


def _decaying(m, n, seed, decay=0.7):
    g = rng(seed)
    U, _ = np.linalg.qr(g.standard_normal((m, n)))
    V, _ = np.linalg.qr(g.standard_normal((n, n)))
    s = decay ** np.arange(n)
    return (U * s) @ V.T, s


def test_theorem1_expected_frobenius_bound():
    """Thm. 1 (q = 0): E||A - QQ^T A||_F <= (1 + r/(r_ov - 1))^(1/2) (sum_{j>r} s_j^2)^(1/2)."""
    m, n, r, rov = 120, 80, 8, 4
    A, s = _decaying(m, n, 30, decay=0.85)
    tail = math.sqrt(float(np.sum(s[r:] ** 2)))
    errs = []
    for seed in range(40):
        Q = O.range_finder(A, rng(1000 + seed).standard_normal((n, r + rov)), 0)
        errs.append(np.linalg.norm(A - Q @ (Q.T @ A)))
    mean = float(np.mean(errs))
    assert mean <= math.sqrt(1 + r / (rov - 1)) * tail
    assert mean >= tail * (1 - 1e-12)           # never below the optimum of rank r


def test_theorem3_power_scheme_spectral_bound():
    """Thm. 3: E||A - PA||_2 <= c^(1/(2w+1)) sigma_{r+1}; the error falls with w."""
    m, n, r, rov = 150, 100, 6, 4
    A, s = _decaying(m, n, 31, decay=0.9)
    k = r + rov
    c = 1 + math.sqrt(r / (rov + 1)) + math.e * math.sqrt(k) / rov * math.sqrt(min(m, n) - r)
    means = []
    for w in range(4):
        errs = []
        for seed in range(20):
            Q = O.range_finder(A, rng(2000 + seed).standard_normal((n, k)), w)
            errs.append(np.linalg.norm(A - Q @ (Q.T @ A), 2))
        mean = float(np.mean(errs))
        assert mean <= c ** (1.0 / (2 * w + 1)) * s[r]
        assert mean >= s[k] * (1 - 1e-12)
        means.append(mean)
    assert means[0] > means[1] > means[2] >= means[3] * (1 - 1e-9)


def test_small_sketches_norms_and_exact_case():
    """||L^T A R^T||_F <= ||A||_F (orthogonal projections), with equality when
    A lies in range(L) x range(R^T); B = L^T A and At = L^T A R^T shapes."""
    g = rng(40)
    m, n, k = 90, 70, 9
    A = g.random((m, n))
    s = O.sketch(A, g.standard_normal((n, k)), g.standard_normal((m, k)), q=1)
    assert s["B"].shape == (k, n) and s["At"].shape == (k, k) and s["Ac"].shape == (m, k)
    assert np.linalg.norm(s["At"]) <= np.linalg.norm(A)
    assert np.abs(s["R"] @ s["R"].T - np.eye(k)).max() < 1e-14
    # A of rank 4 lies in both ranges once k >= 4
    A4 = g.random((m, 4)) @ g.random((4, n))
    s4 = O.sketch(A4, g.standard_normal((n, k)), g.standard_normal((m, k)), q=1)
    assert abs(np.linalg.norm(s4["At"]) - np.linalg.norm(A4)) < 1e-12 * np.linalg.norm(A4)


def test_ac_is_the_projection_of_a_onto_the_right_basis():
    """Ac = A R^T (Alg. 2's compressed data): Ac R is the orthogonal projection
    of A's rows onto range(R^T), so the remainder is orthogonal to R's rows,
    ||Ac||_F <= ||A||_F, and an A lying in range(R^T) is reproduced exactly;
    L^T Ac equals At (both are L^T A R^T).  A slip such as A L, A R or R A^T
    fails one of these."""
    g = rng(41)
    m, n, k = 90, 70, 9
    A = g.random((m, n))
    s = O.sketch(A, g.standard_normal((n, k)), g.standard_normal((m, k)), q=1)
    Ac, R, L = s["Ac"], s["R"], s["L"]
    assert Ac.shape == (m, k)
    assert np.abs((A - Ac @ R) @ R.T).max() < 1e-12 * np.abs(A).max()
    assert np.linalg.norm(Ac) <= np.linalg.norm(A) * (1 + 1e-14)
    assert np.abs(L.T @ Ac - s["At"]).max() < 1e-12 * np.abs(s["At"]).max()
    A4 = g.random((m, 4)) @ g.random((4, n))
    s4 = O.sketch(A4, g.standard_normal((n, k)), g.standard_normal((m, k)), q=1)
    assert np.linalg.norm(A4 - s4["Ac"] @ s4["R"]) <= 1e-13 * np.linalg.norm(A4)


# --------------------------------------------------------------------------
# Alg. 3 (Appendix B)
# --------------------------------------------------------------------------

def _small_problem(seed=50, m=60, n=45, r=4, k=10, q=2, noise=0.01):
    g = rng(seed)
    A = g.random((m, r)) @ g.random((r, n)) + np.abs(noise * g.standard_normal((m, n)))
    s = O.sketch(A, g.standard_normal((n, k)), g.standard_normal((m, k)), q=q)
    U1, V1 = WL.init_factors(A.mean(), m, n, r, seed + 1)
    lam = float(np.linalg.svd(s["At"], compute_uv=False)[r - 1])
    return A, s, U1, V1, lam


def test_admm_projection_invariants_every_iteration():
    """With xi = 1: U = max(t, 0), Lam = lam min(t, 0) for t = L Xt + Lam_prev/lam,
    hence Lam <= 0 <= U and Lam o U = 0 after every iteration (same for V, Phi)."""
    A, s, U1, V1, lam = _small_problem()
    out = O.admm(s["At"], s["L"], s["R"], U1, V1, lam, lam, 1.0, 30, history=True)
    Lprev = np.zeros_like(U1)
    Pprev = np.zeros_like(V1)
    for h in out["history"]:
        scale_l = lam * (np.abs(h["LX"]).max() + 1)
        scale_p = lam * (np.abs(h["YR"]).max() + 1)
        assert h["U"].min() >= 0 and h["V"].min() >= 0
        assert h["Lam"].max() <= 1e-14 * scale_l and h["Phi"].max() <= 1e-14 * scale_p
        assert np.abs(h["Lam"] * h["U"]).max() <= 1e-13 * scale_l * (np.abs(h["U"]).max() + 1)
        assert np.abs(h["Phi"] * h["V"]).max() <= 1e-13 * scale_p * (np.abs(h["V"]).max() + 1)
        t = h["LX"] + Lprev / lam
        assert np.abs(h["U"] + h["Lam"] / lam - t).max() <= 1e-13 * (np.abs(t).max() + 1)
        Lprev, Pprev = h["Lam"], h["Phi"]


def _lagrangian(At, L, R, Xt, Yt, U, V, Lam, Phi, lam, phi):
    """Augmented Lagrangian of the compressed problem with 1/2 on the data
    term (the reading under which the printed closed forms are minimisers)."""
    r1 = At - Xt @ Yt
    cu = L @ Xt - U
    cv = Yt @ R - V
    return (0.5 * np.sum(r1 * r1) + np.sum(Lam * cu) + lam / 2 * np.sum(cu * cu)
            + np.sum(Phi * cv) + phi / 2 * np.sum(cv * cv))


def test_admm_closed_forms_are_lagrangian_minimisers():
    """Each Xt / Yt update is the stationary point of the Lagrangian in that
    block with the others fixed (checked by central differences, which are
    exact for a quadratic), so a dropped term, a sign or a transpose in the
    closed forms fails here."""
    A, s, U1, V1, lam = _small_problem(seed=60)
    phi = 1.7 * lam
    At, L, R = s["At"], s["L"], s["R"]
    out = O.admm(At, L, R, U1, V1, lam, phi, 1.0, 6, history=True)
    U, V = U1.copy(), V1.copy()
    Lam, Phi = np.zeros_like(U1), np.zeros_like(V1)
    Yt = V1 @ R.T
    g = rng(61)
    for h in out["history"]:
        Xt = h["Xt"]
        for _ in range(3):
            E = g.standard_normal(Xt.shape)
            e = 1e-3
            d = (_lagrangian(At, L, R, Xt + e * E, Yt, U, V, Lam, Phi, lam, phi)
                 - _lagrangian(At, L, R, Xt - e * E, Yt, U, V, Lam, Phi, lam, phi)) / (2 * e)
            base = _lagrangian(At, L, R, Xt, Yt, U, V, Lam, Phi, lam, phi)
            assert abs(d) <= 1e-8 * (abs(base) + 1)
        Ytn = h["Yt"]
        for _ in range(3):
            E = g.standard_normal(Ytn.shape)
            e = 1e-3
            d = (_lagrangian(At, L, R, Xt, Ytn + e * E, U, V, Lam, Phi, lam, phi)
                 - _lagrangian(At, L, R, Xt, Ytn - e * E, U, V, Lam, Phi, lam, phi)) / (2 * e)
            base = _lagrangian(At, L, R, Xt, Ytn, U, V, Lam, Phi, lam, phi)
            assert abs(d) <= 1e-8 * (abs(base) + 1)
        # U and V are the nonnegative minimisers of their blocks: projected
        # stationarity of lam/2 ||L Xt - U||^2 + Lam.(L Xt - U) over U >= 0
        gU = -(Lam + lam * (L @ Xt - h["U"]))
        assert np.all(gU[h["U"] > 0] == pytest.approx(0, abs=1e-10 * (np.abs(gU).max() + 1)))
        assert gU[h["U"] == 0].min(initial=0) >= -1e-10 * (np.abs(gU).max() + 1)
        Yt, U, V, Lam, Phi = Ytn, h["U"], h["V"], h["Lam"], h["Phi"]


def test_admm_with_identity_bases_is_uncompressed_admm():
    """L = I_m, R = I_n turns Alg. 3 into the uncompressed ADMM (At = A)."""
    g = rng(70)
    m, n, r = 25, 18, 3
    A = g.random((m, r)) @ g.random((r, n))
    U1, V1 = WL.init_factors(A.mean(), m, n, r, 71)
    a = O.admm(A, np.eye(m), np.eye(n), U1, V1, 2.0, 3.0, 1.0, 40)
    b = O.admm_uncompressed(A, U1, V1, 2.0, 3.0, 1.0, 40)
    assert np.abs(a["U"] - b["U"]).max() < 1e-12
    assert np.abs(a["V"] - b["V"]).max() < 1e-12


def test_admm_rank_one_reaches_the_svd_floor():
    """For A > 0 the best rank-1 approximation is nonnegative (Perron), so the
    NMF optimum with r = 1 equals the SVD floor (sum_{j>=2} s_j^2)^(1/2)/||A||."""
    g = rng(80)
    A = g.random((40, 30)) + 0.1
    s = np.linalg.svd(A, compute_uv=False)
    floor = math.sqrt(float(np.sum(s[1:] ** 2))) / np.linalg.norm(A)
    U1, V1 = WL.init_factors(A.mean(), 40, 30, 1, 81)
    out = O.admm_uncompressed(A, U1, V1, s[0], s[0], 1.0, 600)
    assert O.rel_residual(A, out["U"], out["V"]) == pytest.approx(floor, rel=1e-7)
    # compressed, with k covering the whole column space
    sk = O.sketch(A, g.standard_normal((30, 30)), g.standard_normal((40, 30)), q=1)
    out = O.admm(sk["At"], sk["L"], sk["R"], U1, V1, s[0], s[0], 1.0, 600)
    assert O.rel_residual(A, out["U"], out["V"]) == pytest.approx(floor, rel=1e-7)


def test_admm_kkt_at_convergence():
    """Prop. 1: a converged sequence is a KKT point (the KKT system written
    with L^T Lam and Phi R^T, the dimensionally consistent forms)."""
    g = rng(90)
    m, n, r, k = 40, 30, 3, 8
    A = g.random((m, r)) @ g.random((r, n))
    s = O.sketch(A, g.standard_normal((n, k)), g.standard_normal((m, k)), q=2)
    U1, V1 = WL.init_factors(A.mean(), m, n, r, 91)
    lam = float(np.linalg.svd(s["At"], compute_uv=False)[r - 1])
    o = O.admm(s["At"], s["L"], s["R"], U1, V1, lam, lam, 1.0, 3000)
    Xt, Yt, U, V, Lam, Phi = o["Xt"], o["Yt"], o["U"], o["V"], o["Lam"], o["Phi"]
    L, R, At = s["L"], s["R"], s["At"]
    sc = np.linalg.norm(At) ** 2
    assert np.linalg.norm((Xt @ Yt - At) @ Yt.T + L.T @ Lam) <= 1e-6 * sc
    assert np.linalg.norm(Xt.T @ (Xt @ Yt - At) + Phi @ R.T) <= 1e-6 * sc
    assert np.linalg.norm(L @ Xt - U) <= 1e-6 * np.linalg.norm(U)
    assert np.linalg.norm(Yt @ R - V) <= 1e-6 * np.linalg.norm(V)
    assert O.rel_residual(A, U, V) < 1e-5


# --------------------------------------------------------------------------
# Alg. 2 with Ding et al. Eq. (8)
# --------------------------------------------------------------------------

def test_mu_half_steps_never_increase_their_objectives():
    """Alg. 2 requires ||Ac - X_{k+1} Yc_k|| <= ||Ac - X_k Yc_k|| and
    ||B - Xh_{k+1} Y_{k+1}|| <= ||B - Xh_{k+1} Y_k||; the semi-NMF rule is
    monotone (Ding et al. 2010, Thm. 1)."""
    A, s, U1, V1, _ = _small_problem(seed=100)
    L, R, Ac, B = s["L"], s["R"], s["Ac"], s["B"]
    out = O.mu(Ac, B, L, R, U1, V1, 60, 1e-300, history=True)
    X, Y = U1, V1
    for tag, Xn, Yn in out["history"]:
        if tag == "X":
            before = np.linalg.norm(Ac - X @ (Y @ R.T))
            after = np.linalg.norm(Ac - Xn @ (Y @ R.T))
        else:
            Xh = L.T @ X
            before = np.linalg.norm(B - Xh @ Y)
            after = np.linalg.norm(B - Xh @ Yn)
        assert after <= before * (1 + 1e-12)
        X, Y = Xn, Yn
    assert out["X"].min() >= 0 and out["Y"].min() >= 0


def test_mu_fixed_point_satisfies_complementarity():
    """Approaching a fixed point of the X-step, X o grad_X -> 0 (the KKT
    complementarity of the nonnegative least-squares half-step); MU converges
    sublinearly, so the check is a steady decrease plus a loose bound."""
    g = rng(110)
    m, n, r = 30, 20, 3
    A = g.random((m, r)) @ g.random((r, n))
    U1, V1 = WL.init_factors(A.mean(), m, n, r, 111)
    comp = []
    for iters in (250, 1000, 4000):
        o = O.mu_uncompressed(A, U1, V1, iters, 1e-300)
        X, Y = o["X"], o["Y"]
        gX = X @ (Y @ Y.T) - A @ Y.T
        comp.append(np.abs(X * gX).max() / (np.abs(A @ Y.T).max() * np.abs(X).max()))
    assert comp[0] > comp[1] > comp[2]
    assert comp[2] < 1e-4
    assert O.rel_residual(A, X, Y) < 3e-3


# --------------------------------------------------------------------------
# SPA on the compressed matrix (Section 4, Alg. SNMF)
# --------------------------------------------------------------------------

def test_spa_recovers_planted_columns_of_a_separable_matrix():
    """Near-separable A: SPA on A and on B = L^T A return the planted set, in
    the same order (norm invariance under orthonormal Q, Section 4)."""
    r = 10
    A, planted = WL.separable_matrix(400, 3000, r, 1e-4, seed=120)
    K_full = O.spa(A, r)
    assert sorted(K_full) == list(planted)
    L = O.range_finder(A, rng(121).standard_normal((3000, r + 10)), 2)
    K_comp = O.spa(L.T @ A, r)
    assert K_comp == K_full


def test_spa_order_equals_column_pivoted_qr():
    """SPA's greedy choice is the pivot rule of QR with column pivoting, so its
    order equals LAPACK's first r pivots on a generic matrix."""
    B = rng(130).standard_normal((12, 400))
    _, _, piv = scipy.linalg.qr(B, pivoting=True, mode="economic")
    assert O.spa(B, 8) == list(piv[:8])


def test_spa_invariant_under_orthonormal_basis_of_the_range():
    g = rng(140)
    A = g.random((200, 6)) @ g.random((6, 500))
    L = O.orth_plus(A @ g.standard_normal((500, 9)))
    assert O.spa(L.T @ A, 6) == O.spa(A, 6)


def test_spa_ties_choose_lowest_index():
    B = np.zeros((3, 6))
    B[0, 4] = B[0, 1] = 2.0        # equal norms at columns 1 and 4
    B[1, 5] = 1.0
    assert O.spa(B, 2)[0] == 1


# --------------------------------------------------------------------------
# Residual and NNLS
# --------------------------------------------------------------------------

def test_rel_residual_closed_forms():
    g = rng(150)
    U, V = g.random((70, 5)), g.random((5, 40))
    assert O.rel_residual(U @ V, U, V, block_rows=16) < 1e-15
    A = g.random((70, 40))
    ref = np.linalg.norm(A - U @ V) / np.linalg.norm(A)
    assert O.rel_residual(A, U, V, block_rows=16) == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("seed", range(5))
def test_nnls_bruteforce_matches_lawson_hanson(seed):
    g = rng(160 + seed)
    C = g.standard_normal((15, 6))
    b = g.standard_normal(15)
    h = O.nnls_bruteforce(C, b)
    ref, _ = scipy.optimize.nnls(C, b)
    assert np.abs(h - ref).max() < 1e-10


def test_snmf_right_factor_equals_bruteforce_and_kkt():
    """Each column of H solves its NNLS problem: equal to the brute-force
    minimiser over all supports (r = 6), and the KKT conditions hold
    (h >= 0, gradient >= 0, complementarity)."""
    g = rng(170)
    k, n, r = 12, 40, 6
    B = g.standard_normal((k, n))
    K = [3, 17, 0, 25, 9, 31]
    H = O.snmf_right_factor(B, K)
    C = B[:, K]
    for j in range(n):
        assert np.abs(H[:, j] - O.nnls_bruteforce(C, B[:, j])).max() < 1e-10
    assert (H >= 0).all()
    grad = C.T @ (C @ H - B)                   # gradient of 1/2 ||C h - b||^2
    assert (grad > -1e-10).all()
    assert np.abs(grad * H).max() < 1e-10


def test_snmf_right_factor_recovers_the_planted_factor():
    """A = W [I_r H'] P exactly separable: with K the planted columns and a
    basis Q of range(W), B = Q^T A gives H = [I_r H'] P exactly (W has full
    column rank, so the NNLS optimum is the true nonnegative factor)."""
    A, planted = WL.separable_matrix(300, 800, 7, 0.0, seed=171)
    g = rng(172)
    s = O.sketch(A, g.standard_normal((800, 12)), None, q=1)
    K = O.spa(s["B"], 7)
    assert sorted(K) == list(planted)
    H = O.snmf_right_factor(s["B"], K)
    assert np.linalg.norm(A - A[:, K] @ H) < 1e-10 * np.linalg.norm(A)
    assert np.abs(H[np.arange(7), K] - 1.0).max() < 1e-10       # the selected columns map to themselves


# --------------------------------------------------------------------------
# Section 3, Eq. alternateLS_nmf_compressed: alternating NNLS
# --------------------------------------------------------------------------

def _half_step_problem(tag, X, Y, L, R, Ac, B):
    """Matrix and right-hand sides of the half-step that produced ``tag``:
    rows of X against (Y R^T)^T, or columns of Y against L^T X."""
    if tag == "X":
        return (Y @ R.T).T, Ac.T          # k x r, k x m
    return L.T @ X, B                     # k x r, k x n


def test_anls_half_steps_satisfy_nnls_kkt():
    """Every half-step is minimised to the end: for each row of X (column of
    Y), h >= 0, the gradient C^T (C h - b) >= 0 and h o gradient = 0, the
    optimality conditions of the convex subproblem."""
    A, s, U1, V1, _ = _small_problem(seed=180)
    L, R, Ac, B = s["L"], s["R"], s["Ac"], s["B"]
    out = O.anls(Ac, B, L, R, V1, 8, history=True)
    X, Y = U1, V1
    for tag, Xn, Yn in out["history"]:
        C, rhs = _half_step_problem(tag, X, Y, L, R, Ac, B)
        H = Xn.T if tag == "X" else Yn
        grad = C.T @ (C @ H - rhs)
        scale = np.abs(C.T @ rhs).max()
        assert (H >= 0).all()
        assert grad.min() > -1e-10 * scale
        assert np.abs(grad * H).max() < 1e-10 * scale * max(1.0, np.abs(H).max())
        X, Y = Xn, Yn


def test_anls_equals_bruteforce_on_tiny_problems():
    """r = 3: every row of X and column of Y equals the minimiser found by
    enumerating all supports."""
    A, s, U1, V1, _ = _small_problem(seed=181, m=14, n=11, r=3, k=6)
    L, R, Ac, B = s["L"], s["R"], s["Ac"], s["B"]
    out = O.anls(Ac, B, L, R, V1, 3, history=True)
    X, Y = U1, V1
    for tag, Xn, Yn in out["history"]:
        C, rhs = _half_step_problem(tag, X, Y, L, R, Ac, B)
        H = Xn.T if tag == "X" else Yn
        for j in range(rhs.shape[1]):
            assert np.abs(H[:, j] - O.nnls_bruteforce(C, rhs[:, j])).max() < 1e-10
        X, Y = Xn, Yn


def test_anls_half_steps_do_at_least_as_well_as_mu():
    """An exact minimiser cannot lose to any feasible point: from the same
    Y, the ANLS X-step's objective is at most the MU X-step's, and both are
    at most the objective before the step (Alg. 2's requirement)."""
    A, s, U1, V1, _ = _small_problem(seed=182)
    L, R, Ac, B = s["L"], s["R"], s["Ac"], s["B"]
    Yc = V1 @ R.T
    x_anls = O.anls(Ac, B, L, R, V1, 1, history=True)["history"][0][1]
    x_mu = O.mu(Ac, B, L, R, U1, V1, 1, 1e-300, history=True)["history"][0][1]
    before = np.linalg.norm(Ac - U1 @ Yc)
    f_mu = np.linalg.norm(Ac - x_mu @ Yc)
    f_anls = np.linalg.norm(Ac - x_anls @ Yc)
    assert f_anls <= f_mu * (1 + 1e-12) and f_mu <= before * (1 + 1e-12)
    assert f_anls < 0.999 * f_mu          # and it is strictly better here


def test_anls_objectives_never_increase():
    """Alg. 2's monotonicity, for the compressed objectives and, with
    identity bases, for ||A - X Y||_F itself."""
    A, s, U1, V1, _ = _small_problem(seed=183)
    L, R, Ac, B = s["L"], s["R"], s["Ac"], s["B"]
    out = O.anls(Ac, B, L, R, V1, 15, history=True)
    X, Y = U1, V1
    first = True
    for tag, Xn, Yn in out["history"]:
        if tag == "X":
            before = np.linalg.norm(Ac - X @ (Y @ R.T))
            after = np.linalg.norm(Ac - Xn @ (Y @ R.T))
        else:
            before = np.linalg.norm(B - (L.T @ X) @ Y)
            after = np.linalg.norm(B - (L.T @ X) @ Yn)
        if not first:                      # U1 is not the previous X-step's output
            assert after <= before * (1 + 1e-12)
        first = False
        X, Y = Xn, Yn
    full = O.anls(A, A, None, None, V1, 10, history=True)["history"]
    objs = [np.linalg.norm(A - Xn @ Yn) for _, Xn, Yn in full]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(objs, objs[1:]))


@pytest.mark.parametrize("compressed", [True, False])
def test_anls_recovers_the_planted_factor_in_one_half_step(compressed):
    """A = W H exactly, rank r, W and H of full rank and nonnegative: with
    Y = H the X-step's unique minimiser is W (zero residual is reachable
    and the matrix has full column rank); the compressed X-step too, since
    R's rows span the row space of A when k >= r."""
    g = rng(184)
    m, n, r, k = 80, 60, 5, 9
    W, H = g.random((m, r)), g.random((r, n))
    A = W @ H
    if compressed:
        s = O.sketch(A, g.standard_normal((n, k)), g.standard_normal((m, k)), q=1)
        out = O.anls(s["Ac"], s["B"], s["L"], s["R"], H, 1)
    else:
        out = O.anls_uncompressed(A, H, 1)
    assert np.abs(out["X"] - W).max() < 1e-10
    assert np.abs(out["Y"] - H).max() < 1e-9
