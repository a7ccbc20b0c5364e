"""RI factor tensors K^Q_ij (written B here, [N_aux][N][N]).

eq:K_ijQ defines K^Q_ij = sum_A (ij|A) V^{-1/2}_{AQ}, so that the 4-index
integrals factor as v_ijkl = sum_Q K^Q_ij K^Q_kl (eq:vKQKQ).  The synthetic
stand-in supplies K directly from a Gaussian model of the chain (V = I), or,
for the screened front end (eq:V_ijA, then the second eq:K_ijQ), the same
Gaussian model as (ij|A) with a Gaussian metric V.
"""
from __future__ import annotations

import numpy as np


def synthetic_b(x: np.ndarray, xq: np.ndarray, amp: float, a: float, c: float) -> np.ndarray:
    """B^Q_ij = amp exp(-a (x_i-x_j)^2) exp(-c (x_Q - (x_i+x_j)/2)^2)."""
    x = np.asarray(x, dtype=np.float64)
    xq = np.asarray(xq, dtype=np.float64)
    dij = x[:, None] - x[None, :]
    mij = 0.5 * (x[:, None] + x[None, :])
    bond = amp * np.exp(-a * dij * dij)
    out = np.empty((xq.shape[0], x.shape[0], x.shape[0]))
    for q in range(xq.shape[0]):
        d = xq[q] - mij
        out[q] = bond * np.exp(-c * d * d)
    return out


def inverse_sqrt_spd(v: np.ndarray) -> np.ndarray:
    """V^{-1/2} of a symmetric positive definite V by its eigendecomposition."""
    w, u = np.linalg.eigh(v)
    if w.min() <= 0:
        raise ValueError("V is not positive definite")
    return (u / np.sqrt(w)) @ u.T


def b_from_three_index(ija: np.ndarray, v: np.ndarray | None) -> np.ndarray:
    """eq:K_ijQ: K^Q_ij = sum_A (ij|A) V^{-1/2}_{AQ}; V = None means V = I."""
    if v is None:
        return np.array(ija, dtype=np.float64, copy=True)
    vis = inverse_sqrt_spd(v)
    return np.einsum("aij,aq->qij", ija, vis, optimize=True)


def screen_three_index(ija: np.ndarray, eps_prime: float) -> np.ndarray:
    """eq:V_ijA: (ij|A)^L keeps (ij|A) where |(ij|A)| >= (eps' / N) M_j, with
    M_j the largest |(ij|A)| over i and A for that j, and is zero elsewhere.
    ija is [N_aux][N][N] (A, i, j); N is the basis size."""
    ija = np.asarray(ija, dtype=np.float64)
    n = ija.shape[1]
    out = np.zeros_like(ija)
    for j in range(n):
        col = ija[:, :, j]
        m_j = float(np.max(np.abs(col)))
        thr = eps_prime / n * m_j
        out[:, :, j] = np.where(np.abs(col) >= thr, col, 0.0)
    return out


def four_index(b: np.ndarray) -> np.ndarray:
    """eq:vKQKQ: v_ijkl = sum_Q K^Q_ij K^Q_kl (tiny N only)."""
    n = b.shape[1]
    flat = b.reshape(b.shape[0], n * n)
    return (flat.T @ flat).reshape(n, n, n, n)
