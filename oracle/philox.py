"""Host re-implementation of the Gaussian test-matrix generator (Alg. 1's
first step: draw a Gaussian random matrix), for the oracle side.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this module; the product has its own
device implementation of the same published definitions and shares no code
with this one.

Definitions (each side implements them from the publications):
  * Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
    Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 4 x 32-bit
    counter and a 2 x 32-bit key; each of 10 rounds multiplies counter words
    0 and 2 by the constants 0xD2511F53 and 0xCD9E8D57, and mixes the high
    halves of the products with the other two words and the round key; the
    key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) between
    rounds.
  * The Box-Muller transform (Box and Muller, 1958) turns two uniforms into
    two independent standard normals: rho = sqrt(-2 ln u1),
    (z0, z1) = (rho cos 2 pi u2, rho sin 2 pi u2).

The subsampled randomized Hadamard transform (SRHT) test matrix that the
paper names as an alternative to the Gaussian one (Section 2, remark after
Thm. 3; Halko, Martinsson and Tropp 2011, Sec. 4.6; Tropp 2011): for
`rows` rows padded to p = 2^ceil(log2 rows), Omega = D H S / sqrt(k) with D
a diagonal of random signs, H the p x p Walsh-Hadamard (Sylvester) matrix
with entries (-1)^popcount(i & j), and S the selection of k distinct
columns drawn uniformly; entry (i, c) = d_i (-1)^popcount(i & s_c) / sqrt(k).
Randomness (a reading of its own): d_i = -1 when bit 0 of word x0 of the
counter (0, i, matrix_id, 1) is set; s_c is drawn in order c = 0, 1, ...
from the words x0 of the counters (c, t, matrix_id, 2), t = 0, 1, ...,
masked to [0, p), the first value not taken by s_0..s_{c-1}; after 64
taken draws, the first free index at or after the last draw (cyclically).

The matrix recipe (a reading of its own, as the paper fixes no generator):
entry (i, j) of test matrix `matrix_id` drawn with `seed` comes from the
counter (j // 2, i, matrix_id, 0) under the key (seed mod 2^32, seed div
2^32); with the four output words x0..x3,
    u1 = (((x1 << 32) | x0) >> 11 + 1) 2^-53      in (0, 1]
    u2 = (((x3 << 32) | x2) >> 11) 2^-53          in [0, 1)
and the entry is z0 for even j, z1 for odd j.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)
TWO_PI = 6.283185307179586   # the double nearest 2 pi


def philox4x32_10(counters: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 of each row of `counters` (N x 4, uint32) under `key`
    (two uint32 words); returns N x 4 uint32 output words."""
    c = np.asarray(counters, dtype=np.uint64).reshape(-1, 4)
    c0, c1, c2, c3 = (c[:, i].copy() for i in range(4))
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0          # < 2^64: exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def gaussian_matrix(seed: int, matrix_id: int, rows: int, cols: int) -> np.ndarray:
    """rows x cols FP64 matrix of iid N(0, 1) entries by the recipe above."""
    pairs = (cols + 1) // 2
    i = np.repeat(np.arange(rows, dtype=np.uint64), pairs)
    p = np.tile(np.arange(pairs, dtype=np.uint64), rows)
    ctr = np.stack([p, i, np.full_like(p, matrix_id), np.zeros_like(p)], axis=1)
    x = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)).astype(np.uint64)
    a = ((x[:, 1] << np.uint64(32)) | x[:, 0]) >> np.uint64(11)
    b = ((x[:, 3] << np.uint64(32)) | x[:, 2]) >> np.uint64(11)
    u1 = (a + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    rho = np.sqrt(-2.0 * np.log(u1))
    th = TWO_PI * u2
    z = np.stack([rho * np.cos(th), rho * np.sin(th)], axis=1).reshape(rows, 2 * pairs)
    return np.ascontiguousarray(z[:, :cols])


def _words0(seed: int, ctrs) -> np.ndarray:
    x = philox4x32_10(np.asarray(ctrs, dtype=np.uint64).reshape(-1, 4), (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    return x[:, 0].astype(np.uint64)


def srht_columns(seed: int, matrix_id: int, rows: int, cols: int) -> list:
    """The k = cols distinct sampled Hadamard column indices s_c in [0, p)."""
    p = 1
    while p < rows:
        p *= 2
    taken = []
    for c in range(cols):
        v = None
        for t in range(64):
            cand = int(_words0(seed, [c, t, matrix_id, 2])[0]) & (p - 1)
            if cand not in taken:
                v = cand
                break
        if v is None:
            v = cand
            while v in taken:
                v = (v + 1) % p
        taken.append(v)
    return taken


def srht_matrix(seed: int, matrix_id: int, rows: int, cols: int) -> np.ndarray:
    """rows x cols FP64 SRHT test matrix by the recipe above."""
    s = np.array(srht_columns(seed, matrix_id, rows, cols), dtype=np.int64)
    i = np.arange(rows, dtype=np.uint64)
    ctr = np.stack([np.zeros_like(i), i, np.full_like(i, matrix_id), np.ones_like(i)], axis=1)
    d = np.where(_words0(seed, ctr) & np.uint64(1), -1.0, 1.0)
    bits = np.bitwise_and(np.arange(rows, dtype=np.int64)[:, None], s[None, :])
    par = np.array([[bin(int(v)).count("1") & 1 for v in row] for row in bits], dtype=np.int64)
    return d[:, None] * np.where(par == 1, -1.0, 1.0) / np.sqrt(cols)
