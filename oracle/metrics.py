"""Similarity and coding measures of Section 3 (Table 2) in float64 (oracle;
test infrastructure only).  ``c`` is the exact DCT matrix, ``ct`` the
approximation under test (for the proposed method, C_hat = S T)."""
from __future__ import annotations

import math

import numpy as np


def markov_covariance(n: int = 16, rho: float = 0.95) -> np.ndarray:
    """R_ij = rho^|i-j| (first-order Markov model, Section 3.2)."""
    i = np.arange(n)
    return rho ** np.abs(i[:, None] - i[None, :]).astype(np.float64)


def dct_distortion(c: np.ndarray, ct: np.ndarray) -> float:
    """d2 = 1 - (1/N) ||diag(C C~^T)||^2."""
    d = np.diag(c @ ct.T)
    return float(1.0 - (d @ d) / c.shape[0])


def total_error_energy(c: np.ndarray, ct: np.ndarray) -> float:
    """epsilon = pi ||C - C~||_F^2."""
    return float(math.pi * np.sum((c - ct) ** 2))


def mse(c: np.ndarray, ct: np.ndarray, rho: float = 0.95) -> float:
    """MSE = (1/N) tr((C - C~) R (C - C~)^T)."""
    d = c - ct
    return float(np.trace(d @ markov_covariance(c.shape[0], rho) @ d.T) / c.shape[0])


def coding_gain(ct: np.ndarray, rho: float = 0.95) -> float:
    """C_g = 10 log10( (1/N) sum s_ii / (prod s_ii sqrt(sum_j c~_ij^2))^(1/N) ),
    s = C~ R C~^T."""
    n = ct.shape[0]
    s = ct @ markov_covariance(n, rho) @ ct.T
    num = np.trace(s) / n
    terms = np.diag(s) * np.sqrt(np.sum(ct * ct, axis=1))
    den = math.exp(np.sum(np.log(terms)) / n)
    return float(10.0 * math.log10(num / den))


def transform_efficiency(ct: np.ndarray, rho: float = 0.95) -> float:
    """eta = sum |s_ii| / sum_ij |s_ij| * 100."""
    s = ct @ markov_covariance(ct.shape[0], rho) @ ct.T
    return float(np.sum(np.abs(np.diag(s))) / np.sum(np.abs(s)) * 100.0)


def table2_row(c: np.ndarray, ct: np.ndarray, rho: float = 0.95) -> dict:
    return {
        "d2": dct_distortion(c, ct),
        "epsilon": total_error_energy(c, ct),
        "mse": mse(c, ct, rho),
        "cg": coding_gain(ct, rho),
        "eta": transform_efficiency(ct, rho),
    }
