"""Matrices of the method and the blockwise 2-D transform (oracle; test
infrastructure only).

Notation follows the paper: T is the 16x16 matrix with entries in {0, +1, -1}
(Section 2), S the orthogonalising diagonal, C_hat = S T the orthogonal
approximation, C the exact DCT-II.  Block coefficients of a 16x16 block A are
B = C_hat A C_hat^T (Section 4); the integer part is Z = T A T^T so that
B = S Z S.
"""
from __future__ import annotations

import math

import numpy as np

N = 16

# Section 2: the proposed multiplierless matrix T, entries in {0, +1, -1}.
T = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1],
    [1, 1, 1, 1, 1, 1, 1, 1, -1, -1, -1, -1, -1, -1, -1, -1],
    [1, 1, 1, 0, 0, -1, -1, -1, -1, -1, -1, 0, 0, 1, 1, 1],
    [1, 1, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, -1, -1],
    [1, 0, 0, -1, -1, 0, 0, 1, 1, 0, 0, -1, -1, 0, 0, 1],
    [1, 1, -1, -1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1],
    [1, 0, -1, -1, 1, 1, 0, -1, -1, 0, 1, 1, -1, -1, 0, 1],
    [0, 0, -1, 1, 1, -1, -1, 1, -1, 1, 1, -1, -1, 1, 0, 0],
    [1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1],
    [1, -1, -1, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 1, 1, -1],
    [1, -1, 0, 1, -1, 0, 1, -1, -1, 1, 0, -1, 1, 0, -1, 1],
    [0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0],
    [0, -1, 1, 0, 0, 1, -1, 0, 0, -1, 1, 0, 0, 1, -1, 0],
    [1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1],
    [0, -1, 1, -1, 1, -1, 1, 0, 0, 1, -1, 1, -1, 1, -1, 0],
    [1, -1, 0, 0, -1, 1, -1, 1, -1, 1, -1, 1, 0, 0, 1, -1],
], dtype=np.int64)


def wht() -> np.ndarray:
    """The 16x16 Walsh-Hadamard matrix in natural (Sylvester) order,
    H_1 = [1], H_2k = [[H_k, H_k], [H_k, -H_k]]: a comparison transform of
    Table 2 that the kernels also accept in place of T."""
    h = np.array([[1]], dtype=np.int64)
    while h.shape[0] < N:
        h = np.block([[h, h], [h, -h]])
    return h


def row_norms(t: np.ndarray = T) -> np.ndarray:
    """n_i = (T T^T)_ii, the squared row norms of T (Section 2: T T^T is
    diagonal, which is what makes the orthogonalisation possible)."""
    return np.diag(t @ t.T).copy()


def s_diag(t: np.ndarray = T) -> np.ndarray:
    """Diagonal of S = diag(1/sqrt(n_i)) in float64 (Section 2)."""
    return 1.0 / np.sqrt(row_norms(t).astype(np.float64))


def c_hat(t: np.ndarray = T) -> np.ndarray:
    """C_hat = S T, the orthogonal approximation (Section 2), float64."""
    return s_diag(t)[:, None] * t.astype(np.float64)


def dct_matrix(n: int = N) -> np.ndarray:
    """Exact orthonormal DCT-II matrix: C[k, m] = a_k cos(pi (2m+1) k / (2n)),
    a_0 = sqrt(1/n), a_k = sqrt(2/n) otherwise.  The paper compares against
    "the exact DCT" without printing it; this is the standard orthonormal
    definition, and its Table 2 coding measures reproduce from it."""
    k = np.arange(n)[:, None].astype(np.float64)
    m = np.arange(n)[None, :].astype(np.float64)
    c = np.cos(np.pi * (2.0 * m + 1.0) * k / (2.0 * n))
    a = np.full((n, 1), math.sqrt(2.0 / n))
    a[0, 0] = math.sqrt(1.0 / n)
    return a * c


# ----------------------------------------------------------------------------
# Eq. (1): T = P2 M4 M3 M2 P1 M1, built from the paper's description of each
# factor.  These matrices exist so that the tests can check the product
# against T and count the additions of Table 1; the transforms below do not
# use them.

def _ident(n):
    return np.eye(n, dtype=np.int64)


def _counter_ident(n):
    return np.fliplr(np.eye(n, dtype=np.int64))


def _butterfly(n):
    """[[I, J], [J, -I]] of order n, with I, J of order n/2 (J is the
    counter-identity)."""
    h = n // 2
    top = np.hstack([_ident(h), _counter_ident(h)])
    bot = np.hstack([_counter_ident(h), -_ident(h)])
    return np.vstack([top, bot])


def _block_diag(*blocks):
    n = sum(b.shape[0] for b in blocks)
    out = np.zeros((n, n), dtype=np.int64)
    o = 0
    for b in blocks:
        k = b.shape[0]
        out[o:o + k, o:o + k] = b
        o += k
    return out


def factor_M1():
    return _butterfly(16)


def factor_P1():
    q = np.array([
        [0, 0, 1, 0, 0, 0, 0],
        [0, 0, 0, 1, 0, 0, 0],
        [0, 0, 0, 0, 0, 0, 1],
        [0, 0, 0, 0, 0, 1, 0],
        [0, 0, 0, 0, 1, 0, 0],
        [0, 1, 0, 0, 0, 0, 0],
        [1, 0, 0, 0, 0, 0, 0],
    ], dtype=np.int64)
    return _block_diag(_ident(9), q)


def factor_M2():
    return _block_diag(_butterfly(8), _butterfly(8))


def factor_M3():
    a = [[1, 0, 0, 1], [0, 1, 1, 0], [0, -1, 1, 0], [1, 0, 0, -1]]
    b = [[0, 1, 1, 1], [-1, -1, 0, 1], [-1, 1, -1, 0], [1, 0, -1, 1]]
    c = [[1, 0, 0, 1], [0, 1, 1, 0], [0, -1, 1, 0], [-1, 0, 0, 1]]
    d = [[0, 1, 1, 1], [1, 1, 0, -1], [1, -1, 1, 0], [1, 0, -1, 1]]
    return _block_diag(*(np.array(x, dtype=np.int64) for x in (a, b, c, d)))


def factor_M4():
    h2 = np.array([[1, 1], [1, -1]], dtype=np.int64)
    return _block_diag(h2, _ident(6), h2, _ident(6))


# Eq. (1): P2 in cycle notation.  The printed cycles close by repeating their
# first element; read without the repetition they are (0)(1 8)(2 4 3 11 10 7
# 12)(5 9 13 14 6)(15).  A cycle (a b ...) maps a to b; output i of P2 is
# input sigma(i).  This reading (the other direction does not) reproduces T.
P2_CYCLES = [[0], [1, 8], [2, 4, 3, 11, 10, 7, 12], [5, 9, 13, 14, 6], [15]]


def p2_sigma(cycles=P2_CYCLES) -> np.ndarray:
    sigma = np.arange(N)
    for cyc in cycles:
        for a, b in zip(cyc, cyc[1:] + cyc[:1]):
            sigma[a] = b
    return sigma


def factor_P2(cycles=P2_CYCLES):
    sigma = p2_sigma(cycles)
    p = np.zeros((N, N), dtype=np.int64)
    p[np.arange(N), sigma] = 1
    return p


def factors():
    """Eq. (1) factors in application order: M1, P1, M2, M3, M4, P2."""
    return [factor_M1(), factor_P1(), factor_M2(), factor_M3(), factor_M4(), factor_P2()]


def additions(m: np.ndarray) -> int:
    """Additions needed to apply a {0, +1, -1} matrix: each output row with k
    non-zero entries costs k - 1 additions/subtractions (Section 3.1)."""
    nnz = np.count_nonzero(m, axis=1)
    return int(np.sum(np.maximum(nnz - 1, 0)))


# ----------------------------------------------------------------------------
# Blockwise 2-D transform (Section 4: B_k = C~ A_k C~^T, A'_k = C~^T B'_k C~).

def forward_int(blocks: np.ndarray, t: np.ndarray = T) -> np.ndarray:
    """Z = T A T^T for every 16x16 block (int64, exact)."""
    a = np.asarray(blocks, dtype=np.int64)
    return t @ a @ t.T


def scale(z: np.ndarray, t: np.ndarray = T) -> np.ndarray:
    """B = S Z S, i.e. B_uv = s_u s_v Z_uv (float64): the orthonormal
    coefficients C_hat A C_hat^T."""
    s = s_diag(t)
    return np.asarray(z, dtype=np.float64) * (s[:, None] * s[None, :])


def forward_real(blocks: np.ndarray) -> np.ndarray:
    """B = C_hat A C_hat^T computed directly in float64."""
    c = c_hat()
    return c @ np.asarray(blocks, dtype=np.float64) @ c.T


def inverse_real(b: np.ndarray, t: np.ndarray = T) -> np.ndarray:
    """A' = C_hat^T B' C_hat in float64 (Section 4)."""
    c = c_hat(t)
    return c.T @ np.asarray(b, dtype=np.float64) @ c


def inverse_weights(t: np.ndarray = T) -> np.ndarray:
    """w_i = 48 / n_i.  Since C_hat^T S = T^T S^2 = T^T diag(1/n), the inverse
    of integer coefficients Z' (with B' = S Z' S) is
        A' = T^T diag(1/n) Z' diag(1/n) T = (T^T W Z' W T) / 2304,
    with W = diag(w) and 2304 = 48^2.  All w_i are integers (3, 4 or 6)."""
    n = row_norms(t)
    assert np.all(48 % n == 0)
    return 48 // n


def inverse_int_numerator(z_kept: np.ndarray, t: np.ndarray = T) -> np.ndarray:
    """Exact integer numerator N = T^T (w w^T * Z') T of A' = N / 2304."""
    w = inverse_weights(t)
    wz = (w[:, None] * w[None, :]) * np.asarray(z_kept, dtype=np.int64)
    return t.T @ wz @ t


def dct_forward(blocks: np.ndarray) -> np.ndarray:
    """Exact DCT-II coefficients C A C^T in float64 (comparison transform)."""
    c = dct_matrix()
    return c @ np.asarray(blocks, dtype=np.float64) @ c.T


def dct_inverse(b: np.ndarray) -> np.ndarray:
    c = dct_matrix()
    return c.T @ np.asarray(b, dtype=np.float64) @ c
