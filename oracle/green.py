"""Finite-temperature Green's function of a one-body Hamiltonian.

eq:Gij defines G_ij(tau) = -<T a_i(tau) a_j^dagger>; for the non-interacting
problem (eq:G0, with the Fock matrix F, overlap S and chemical potential mu)
it is, for 0 < tau < beta, with F C = S C eps, C^T S C = I, e~ = eps - mu and
f = 1 / (1 + exp(beta e~)):

  G(tau)        = -C diag((1 - f) exp(-e~ tau)) C^T
  G(beta - tau) = -C diag(f exp(e~ tau)) C^T

so G(0+) + G(beta-) = -S^{-1} (the anticommutator eq:Smatrix) and the
particle number is N_e = -2 sum_ij G_ij(beta-) S_ij (Section III).  The
weights are evaluated in log form so that exp(beta |e~|) never overflows:
ln(1 - f) = -softplus(-beta e~), ln f = -softplus(beta e~).

The paper's tau grid is not specified; this project uses Gauss-Legendre
nodes mapped to [0, beta].
"""
from __future__ import annotations

import numpy as np


def softplus(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def tau_grid(beta: float, ntau: int):
    """Gauss-Legendre nodes and weights on [0, beta] (ascending)."""
    x, w = np.polynomial.legendre.leggauss(int(ntau))
    return 0.5 * beta * (1.0 + x), 0.5 * beta * w


def orbitals(f: np.ndarray, s: np.ndarray | None = None):
    """Generalised eigenpairs F C = S C eps with C^T S C = I (ascending eps)."""
    f = np.asarray(f, dtype=np.float64)
    if s is None:
        return np.linalg.eigh(f)
    ws, us = np.linalg.eigh(s)
    x = (us / np.sqrt(ws)) @ us.T          # S^{-1/2}
    e, y = np.linalg.eigh(x @ f @ x)
    return e, x @ y


def midgap_mu(eps: np.ndarray, n_occ: int) -> float:
    """Chemical potential halfway between the HOMO and the LUMO."""
    return 0.5 * (float(eps[n_occ - 1]) + float(eps[n_occ]))


def occupations(eps: np.ndarray, mu: float, beta: float) -> np.ndarray:
    return np.exp(-softplus(beta * (eps - mu)))


def green_tau(eps: np.ndarray, c: np.ndarray, mu: float, beta: float, tau):
    """(G(tau), G(beta - tau)) for each tau in (0, beta); arrays [ntau][N][N]."""
    tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
    et = eps - mu
    g = np.empty((tau.shape[0], c.shape[0], c.shape[0]))
    gb = np.empty_like(g)
    for t, tv in enumerate(tau):
        lw = -et * tv - softplus(-beta * et)          # ln[(1-f) e^{-e~ tau}]
        lb = et * tv - softplus(beta * et)            # ln[f e^{e~ tau}]
        g[t] = -(c * np.exp(lw)) @ c.T
        gb[t] = -(c * np.exp(lb)) @ c.T
    return g, gb


def electron_count(eps: np.ndarray, c: np.ndarray, mu: float, beta: float,
                   s: np.ndarray | None = None) -> float:
    """N_e = -2 sum_ij G_ij(beta-) S_ij."""
    f = occupations(eps, mu, beta)
    g_beta = -(c * f) @ c.T
    s = np.eye(c.shape[0]) if s is None else s
    return float(-2.0 * np.sum(g_beta * s))
