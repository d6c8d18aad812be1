"""Pins of the host test-matrix generators (oracle side): Gaussian and SRHT.

The generator is Philox4x32-10 (Salmon et al., SC'11) followed by the
Box-Muller transform; the device implements the same definitions on its own.
Pins: the published known-answer vectors, the counter layout of the matrix
recipe, and the distribution (moments, Kolmogorov-Smirnov against the normal
CDF, independence of the pair members and of the streams).
"""
import os

import numpy as np
import pytest
import scipy.stats

from oracle import philox as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for w in rows:
        out = P.philox4x32_10(np.array([w[:4]], dtype=np.uint64), (w[4], w[5]))[0]
        assert [int(v) for v in out] == w[6:]


def test_matrix_entry_uses_counter_pair_row_id():
    """Entry (0, 0) / (0, 1) of matrix 0 under seed 0 is the Box-Muller pair of
    the all-zero counter and key (the first known-answer vector)."""
    w = _kat()[0][6:]
    a = ((w[1] << 32) | w[0]) >> 11
    b = ((w[3] << 32) | w[2]) >> 11
    u1 = (a + 1) * 2.0 ** -53
    u2 = b * 2.0 ** -53
    rho = np.sqrt(-2.0 * np.log(u1))
    z = P.gaussian_matrix(0, 0, 1, 2)[0]
    assert z[0] == rho * np.cos(P.TWO_PI * u2) and z[1] == rho * np.sin(P.TWO_PI * u2)
    # the key is (seed low, seed high): seed 0xffffffffffffffff with the all-ones
    # counter is the second vector (pair 0xffffffff is out of range, so use the
    # raw generator)
    w2 = _kat()[1]
    out = P.philox4x32_10(np.array([w2[:4]], dtype=np.uint64), (0xFFFFFFFF, 0xFFFFFFFF))[0]
    assert [int(v) for v in out] == w2[6:]


def test_gaussian_distribution():
    z = P.gaussian_matrix(12345, 0, 2000, 101).ravel()
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert abs(scipy.stats.kurtosis(z)) < 5.0 * np.sqrt(24.0 / n)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3


def test_pairs_and_streams_are_independent():
    z = P.gaussian_matrix(7, 1, 50000, 2)
    n = z.shape[0]
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 5.0 / np.sqrt(n)
    a = P.gaussian_matrix(7, 0, 300, 40).ravel()
    b = P.gaussian_matrix(7, 1, 300, 40).ravel()
    c = P.gaussian_matrix(8, 0, 300, 40).ravel()
    for x, y in ((a, b), (a, c)):
        assert abs(np.corrcoef(x, y)[0, 1]) < 5.0 / np.sqrt(a.size)
        assert not np.any(x == y)


def test_prefix_and_odd_widths_are_consistent():
    full = P.gaussian_matrix(99, 3, 37, 12)
    assert np.array_equal(P.gaussian_matrix(99, 3, 37, 11), full[:, :11])
    assert np.array_equal(P.gaussian_matrix(99, 3, 20, 12), full[:20])
    assert np.array_equal(P.gaussian_matrix(99, 3, 37, 12), full)


# --------------------------------------------------------------------------
# SRHT test matrices (Section 2, remark after Thm. 3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("rows,cols", [(64, 10), (100, 20), (257, 37), (5, 5)])
def test_srht_is_signed_sampled_hadamard(rows, cols):
    """Omega = D H[:rows, S] / sqrt(k) with H the Sylvester-Hadamard matrix
    of the padded size (the library's construction), D = diag(+-1), S a
    selection of distinct columns."""
    import scipy.linalg
    seed, mid = 1234567, 3
    Om = P.srht_matrix(seed, mid, rows, cols)
    p = 1
    while p < rows:
        p *= 2
    S = P.srht_columns(seed, mid, rows, cols)
    assert len(set(S)) == cols and all(0 <= s < p for s in S)
    H = scipy.linalg.hadamard(p).astype(np.float64)
    Hs = H[:rows][:, S] / np.sqrt(cols)
    d = Om[:, 0] / Hs[:, 0]
    assert set(np.unique(d)) <= {-1.0, 1.0}
    assert np.array_equal(Om, d[:, None] * Hs)
    assert np.all(np.abs(Om) == 1.0 / np.sqrt(cols))


def test_srht_columns_are_orthogonal_for_power_of_two_rows():
    """Distinct Hadamard columns are orthogonal: Omega^T Omega = (p / k) I."""
    Om = P.srht_matrix(99, 0, 128, 24)
    assert np.abs(Om.T @ Om - (128 / 24) * np.eye(24)).max() < 1e-13


def test_srht_signs_and_samples_are_spread():
    """Signs are balanced and the sampled columns cover the padded range."""
    Om = P.srht_matrix(7, 1, 4096, 64)
    assert abs(float(np.mean(np.sign(Om[:, 1])))) < 0.1
    S = np.array(P.srht_columns(7, 1, 4096, 64))
    assert S.min() < 512 and S.max() > 3584
    assert len(set(S.tolist())) == 64
