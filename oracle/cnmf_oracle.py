"""Plain FP64 CPU oracle for compressed NMF (Tepper & Sapiro, "Compressed
Nonnegative Matrix Factorization is Fast and Accurate", arXiv:1505.04650).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this module.  The product (the HIP
library and its Python binding) never imports, calls or links anything here,
and this module imports nothing from the product.

Everything is NumPy/SciPy in float64.  Every function follows one passage of
the paper and cites it by section / algorithm / equation.  Library primitives
(matmul, Householder QR, Cholesky solves) serve as single steps; there is no
blocking, fusion or reordering beyond what the cited definition states.

Readings of passages that are silent or garbled (each also listed in the
design notes):
  * Alg. 1's power scheme (AA^T)^w A Omega followed by one QR is computed as
    re-orthonormalised subspace iteration; with the diag(T) >= 0 convention
    it is the same Q in exact arithmetic (see ``range_finder``).
  * The QR sign convention is diag(T) >= 0 (``orth_plus``).
  * ADMM (Appendix B, Alg. 3) is implemented with its printed closed forms;
    these are the minimisers of the Lagrangian with a 1/2 in front of the
    data term (the printed Lagrangian drops it).
  * MU is the semi-NMF rule of Ding, Li & Jordan (2010), Eq. (8), applied to
    each compressed half-step of Alg. 2.  The paper cites it without printing
    it; the rule is restated here from that publication.
  * Alternating NNLS (Eq. alternateLS_nmf_compressed) is the argmin form, the
    one the paper runs with an active-set NNLS solver (its "respectively"
    pairs the solvers with the two forms the other way round).  Each
    subproblem has a unique minimiser when its k x r matrix has full column
    rank, so any exact NNLS solver gives the same iterates; ``anls`` uses
    Lawson-Hanson.
  * SPA (Araujo et al. 2001; Gillis & Vavasis 2014) uses squared Euclidean
    column norms, lowest index on ties, 0-based indices.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

__all__ = [
    "orth_plus", "range_finder", "sketch", "admm", "mu", "spa",
    "rel_residual", "nnls_bruteforce", "admm_uncompressed", "mu_uncompressed",
    "snmf_right_factor", "anls", "anls_uncompressed",
]


# ---------------------------------------------------------------------------
# Section 2, Alg. 1 (structured random compression)
# ---------------------------------------------------------------------------

def orth_plus(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(Y) from a Householder QR (Alg. 1, QR step).

    Alg. 1 asks for "an orthogonal basis obtained using the QR decomposition"
    and fixes no signs.  Reading: columns are signed so that the triangular
    factor has a nonnegative diagonal, which makes Q unique for full column
    rank Y.
    """
    Y = np.asarray(Y, dtype=np.float64)
    Q, T = np.linalg.qr(Y, mode="reduced")
    s = np.sign(np.diag(T))
    s[s == 0] = 1.0
    return Q * s[None, :]


def range_finder(A: np.ndarray, Omega: np.ndarray, q: int) -> np.ndarray:
    """Alg. 1: Q = orth((A A^T)^q A Omega), m x k.

    Computed as subspace iteration with an orthonormalisation after every
    product: Q <- orth(A Omega); q times { Qt <- orth(A^T Q); Q <- orth(A Qt) }.
    Each triangular factor has a positive diagonal, so their product does
    too, and by uniqueness of the QR factorisation this Q equals
    orth((A A^T)^q A Omega) in exact arithmetic.
    """
    A = np.asarray(A, dtype=np.float64)
    Q = orth_plus(A @ Omega)
    for _ in range(int(q)):
        Qt = orth_plus(A.T @ Q)
        Q = orth_plus(A @ Qt)
    return Q


def sketch(A, Omega_L, Omega_R=None, q: int = 0):
    """Two-sided compression of Section 3 (text before Eq. alternate_nmf_compressed).

    L = Alg. 1 on A (m x k); R = (Alg. 1 on A^T)^T (k x n), each with its own
    Gaussian test matrix.  Small sketches:
        B  = L^T A       (k x n)   ("A-hat", also SNMF's compressed matrix)
        At = L^T A R^T   (k x k)   ("A-tilde", Alg. 3)
        Ac = A R^T       (m x k)   ("A-check", Alg. 2)
    With Omega_R None only the left side (L, B) is produced.
    """
    A = np.asarray(A, dtype=np.float64)
    out = {}
    L = range_finder(A, Omega_L, q)
    out["L"] = L
    out["B"] = L.T @ A
    if Omega_R is not None:
        R = range_finder(A.T, Omega_R, q).T
        out["R"] = R
        out["At"] = out["B"] @ R.T
        out["Ac"] = A @ R.T
    return out


# ---------------------------------------------------------------------------
# Appendix B, Alg. 3 (ADMM on the two-sided compressed problem)
# ---------------------------------------------------------------------------

def _spd_right_solve(RHS: np.ndarray, M: np.ndarray) -> np.ndarray:
    """RHS @ inv(M) for symmetric positive definite M (Cholesky)."""
    c = scipy.linalg.cho_factor(M, lower=False)
    return scipy.linalg.cho_solve(c, RHS.T).T


def _spd_left_solve(M: np.ndarray, RHS: np.ndarray) -> np.ndarray:
    """inv(M) @ RHS for symmetric positive definite M (Cholesky)."""
    c = scipy.linalg.cho_factor(M, lower=False)
    return scipy.linalg.cho_solve(c, RHS)


def admm(At, L, R, U1, V1, lam: float, phi: float, xi: float = 1.0,
         iters: int = 100, history: bool = False):
    """Alg. 3 (Appendix B): ADMM for NMF with structured random compression.

    Inputs: At = L^T A R^T (k x k); L (m x k) with orthonormal columns, or None
    for L = I_m; R (k x n) with orthonormal rows, or None for R = I_n; initial
    U1 (m x r), V1 (r x n); penalties lam, phi > 0; step xi.
    With L = I and R = I this is the uncompressed ADMM of Xu et al. (2012).

    Per iteration, in the box's order:
      Xt  <- (At Yt^T + lam L^T U - L^T Lam) (Yt Yt^T + lam I)^-1
      Yt  <- (Xt^T Xt + phi I)^-1 (Xt^T At + phi V R^T - Phi R^T)
      U   <- P+(L Xt + Lam / lam)
      V   <- P+(Yt R + Phi / phi)
      Lam <- Lam + xi lam (L Xt - U)
      Phi <- Phi + xi phi (Yt R - V)
    Initialisation: Yt = V1 R^T, Lam = 0, Phi = 0.  Returns U, V (the
    nonnegative outputs) and the final state.
    """
    At = np.asarray(At, dtype=np.float64)
    U = np.array(U1, dtype=np.float64)
    V = np.array(V1, dtype=np.float64)
    m, r = U.shape
    n = V.shape[1]
    Lm = (lambda X: X) if L is None else (lambda X: L @ X)          # L X
    LTm = (lambda X: X) if L is None else (lambda X: L.T @ X)       # L^T X
    Rm = (lambda Y: Y) if R is None else (lambda Y: Y @ R)          # Y R
    RTm = (lambda Y: Y) if R is None else (lambda Y: Y @ R.T)       # Y R^T
    I = np.eye(r)
    Yt = RTm(V)
    Lam = np.zeros((m, r))
    Phi = np.zeros((r, n))
    Xt = None
    hist = []
    for _ in range(int(iters)):
        Xt = _spd_right_solve(At @ Yt.T + lam * LTm(U) - LTm(Lam), Yt @ Yt.T + lam * I)
        Yt = _spd_left_solve(Xt.T @ Xt + phi * I, Xt.T @ At + phi * RTm(V) - RTm(Phi))
        LX = Lm(Xt)
        YR = Rm(Yt)
        U = np.maximum(LX + Lam / lam, 0.0)
        V = np.maximum(YR + Phi / phi, 0.0)
        Lam = Lam + xi * lam * (LX - U)
        Phi = Phi + xi * phi * (YR - V)
        if history:
            hist.append(dict(U=U.copy(), V=V.copy(), Lam=Lam.copy(), Phi=Phi.copy(),
                             Xt=Xt.copy(), Yt=Yt.copy(), LX=LX, YR=YR))
    out = dict(U=U, V=V, Lam=Lam, Phi=Phi, Xt=Xt, Yt=Yt)
    if history:
        out["history"] = hist
    return out


def admm_uncompressed(A, U1, V1, lam, phi, xi=1.0, iters=100):
    """Uncompressed ADMM (Xu et al. 2012): Alg. 3 with L = I_m, R = I_n, At = A."""
    return admm(A, None, None, U1, V1, lam, phi, xi, iters)


# ---------------------------------------------------------------------------
# Section 3, Alg. 2 with the multiplicative rule of Ding et al. (2010), Eq. (8)
# ---------------------------------------------------------------------------

def _pos(M):
    return (np.abs(M) + M) / 2.0


def _neg(M):
    return (np.abs(M) - M) / 2.0


def mu(Ac, B, L, R, X1, Y1, iters: int = 100, eps: float = 1e-16, history=False):
    """Alg. 2 (compressed alternating NMF) with semi-NMF multiplicative updates.

    Ding, Li & Jordan (2010), Eq. (8): for data D ~ F G^T with G >= 0 and F of
    any sign, G <- G o sqrt(((D^T F)^+ + G (F^T F)^-) / ((D^T F)^- + G (F^T F)^+)),
    with M^+ = (|M| + M)/2 and M^- = (|M| - M)/2.  It is needed because the
    compressed matrices have mixed signs.  Alg. 2 applies it to
      X-step: || Ac - X Yc ||,  Yc = Y R^T          (D = Ac^T, F = Yc^T, G = X)
      Y-step: || B  - Xh Y ||,  Xh = L^T X          (D = B,    F = Xh,   G = Y^T)
    with Ac = A R^T (m x k) and B = L^T A (k x n).  ``eps`` is added to each
    denominator.  L None means I_m and R None means I_n (then Ac = B = A).
    """
    X = np.array(X1, dtype=np.float64)
    Y = np.array(Y1, dtype=np.float64)
    hist = []
    for _ in range(int(iters)):
        Yc = Y if R is None else Y @ R.T                    # r x k
        N = Ac @ Yc.T                                        # m x r
        G = Yc @ Yc.T                                        # r x r
        X = X * np.sqrt((_pos(N) + X @ _neg(G)) / (_neg(N) + X @ _pos(G) + eps))
        if history:
            hist.append(("X", X.copy(), Y.copy()))
        Xh = X if L is None else L.T @ X                     # k x r
        N2 = B.T @ Xh                                        # n x r
        G2 = Xh.T @ Xh                                       # r x r
        Yt = Y.T * np.sqrt((_pos(N2) + Y.T @ _neg(G2)) / (_neg(N2) + Y.T @ _pos(G2) + eps))
        Y = Yt.T
        if history:
            hist.append(("Y", X.copy(), Y.copy()))
    out = dict(X=X, Y=Y)
    if history:
        out["history"] = hist
    return out


def mu_uncompressed(A, X1, Y1, iters=100, eps=1e-16):
    """Uncompressed multiplicative updates: ``mu`` with L = I, R = I, Ac = B = A."""
    return mu(A, A, None, None, X1, Y1, iters, eps)


# ---------------------------------------------------------------------------
# Section 4, Alg. SNMF: extreme columns of B = Q^T A by SPA
# ---------------------------------------------------------------------------

def spa(B, r: int, return_gaps: bool = False):
    """Successive projection algorithm on the columns of B (k x n).

    r times: s_j = sum_i Rm_ij^2; p = smallest j attaining max s; append p;
    u = Rm[:, p] / sqrt(s_p); Rm <- Rm - u (u^T Rm).  Returns the 0-based
    indices in selection order (Alg. SNMF indexes columns in [0, n)).
    With return_gaps, also the relative gap between the best and the
    second-best score at each step (how tie-sensitive the choice was).
    """
    Rm = np.array(B, dtype=np.float64)
    K = []
    gaps = []
    for _ in range(int(r)):
        s = np.einsum("ij,ij->j", Rm, Rm)
        p = int(np.argmax(s))                 # first index attaining the max
        K.append(p)
        if return_gaps:
            s2 = np.delete(s, p)
            gaps.append(float((s[p] - s2.max()) / s[p]) if s2.size and s[p] > 0 else 1.0)
        u = Rm[:, p] / math.sqrt(s[p])
        Rm = Rm - np.outer(u, u @ Rm)
    if return_gaps:
        return K, gaps
    return K


# ---------------------------------------------------------------------------
# Reported error (Section 5: relative reconstruction error)
# ---------------------------------------------------------------------------

def rel_residual(A, U, V, block_rows: int = 4096) -> float:
    """||A - U V||_F / ||A||_F, sums of squares accumulated per row block in
    float64 and the block sums added with math.fsum."""
    A = np.asarray(A)
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    num, den = [], []
    for i0 in range(0, A.shape[0], block_rows):
        a = np.asarray(A[i0:i0 + block_rows], dtype=np.float64)
        d = a - U[i0:i0 + block_rows] @ V
        num.append(float(np.einsum("ij,ij->", d, d)))
        den.append(float(np.einsum("ij,ij->", a, a)))
    return math.sqrt(math.fsum(num)) / math.sqrt(math.fsum(den))


# ---------------------------------------------------------------------------
# Section 4, Eq. (snmf_right_factor_col): tiny NNLS by enumeration
# ---------------------------------------------------------------------------

def nnls_bruteforce(C, b):
    """min_{h >= 0} ||b - C h||_2 by enumerating every support S (r <= 12).

    For each S, solve unconstrained least squares on the columns in S; keep
    the solutions that are nonnegative; return the one with smallest residual.
    """
    C = np.asarray(C, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = C.shape[1]
    best_h = np.zeros(r)
    best = float(b @ b)
    for mask in range(1, 1 << r):
        S = [j for j in range(r) if mask >> j & 1]
        hS, *_ = np.linalg.lstsq(C[:, S], b, rcond=None)
        if np.all(hS >= 0):
            h = np.zeros(r)
            h[S] = hS
            res = b - C @ h
            val = float(res @ res)
            if val < best:
                best, best_h = val, h
    return best_h


def snmf_right_factor(B, K):
    """Section 4, Alg. SNMF, last step: the right factor H (r x n) of
    separable NMF, A ~ A[:, K] H, computed on the compressed matrix
    B = Q^T A column by column (Eq. snmf_right_factor_col):
        H[:, j] = argmin_{h >= 0} ||B[:, j] - B[:, K] h||_2.
    Each column is one nonnegative least-squares problem, solved here by
    the Lawson-Hanson active-set method (scipy.optimize.nnls) as a library
    step.  (The paper writes h in R^{r + r_ov}; with |K| = r it is R^r.)
    """
    import scipy.optimize
    B = np.asarray(B, dtype=np.float64)
    C = B[:, list(K)]
    H = np.zeros((C.shape[1], B.shape[1]))
    for j in range(B.shape[1]):
        H[:, j], _ = scipy.optimize.nnls(C, B[:, j])
    return H


# ---------------------------------------------------------------------------
# Section 3, Eq. alternateLS_nmf_compressed: alternating nonnegative least
# squares on the compressed matrices (the paper runs it with an active-set
# NNLS solver)
# ---------------------------------------------------------------------------

def anls(Ac, B, L, R, Y1, iters: int = 100, history: bool = False):
    """Compressed alternating nonnegative least squares (Section 3,
    Eq. alternateLS_nmf_compressed_X and _Y), each half-step minimised to
    the end:
      X <- argmin_{X >= 0} || Ac - X (Y R^T) ||_F      (Ac = A R^T, m x k)
      Y <- argmin_{Y >= 0} || B  - (L^T X) Y ||_F      (B  = L^T A, k x n)
    Both problems separate: row i of X is the NNLS problem with matrix
    (Y R^T)^T (k x r) and right-hand side Ac[i]; column j of Y the NNLS
    problem with matrix L^T X (k x r) and right-hand side B[:, j].  Each is
    solved by the Lawson-Hanson active-set method (scipy.optimize.nnls) as a
    library step.  Only Y1 enters: the first X-step depends on Y alone.
    L None means I_m and R None means I_n (then Ac = B = A).
    """
    import scipy.optimize
    Ac = np.asarray(Ac, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    Y = np.array(Y1, dtype=np.float64)
    r = Y.shape[0]
    X = np.zeros((Ac.shape[0], r))
    hist = []
    for _ in range(int(iters)):
        Yc = Y if R is None else Y @ R.T                    # r x k
        CX = Yc.T                                            # k x r
        for i in range(Ac.shape[0]):
            X[i], _ = scipy.optimize.nnls(CX, Ac[i])
        if history:
            hist.append(("X", X.copy(), Y.copy()))
        CY = X if L is None else L.T @ X                     # k x r
        Y = np.empty((r, B.shape[1]))
        for j in range(B.shape[1]):
            Y[:, j], _ = scipy.optimize.nnls(CY, B[:, j])
        if history:
            hist.append(("Y", X.copy(), Y.copy()))
    out = dict(X=X, Y=Y)
    if history:
        out["history"] = hist
    return out


def anls_uncompressed(A, Y1, iters=100):
    """Uncompressed alternating NNLS (Section 3, Eq. alternateLS_nmf):
    ``anls`` with L = I, R = I, Ac = B = A."""
    return anls(A, A, None, None, Y1, iters)
