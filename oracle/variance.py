"""Exact variance of the pair estimator of eq:sigma_2 under different
distributions of the stochastic vectors (test infrastructure, like the rest
of oracle/).

For one pair (theta for the first vertex, theta' for the second) the energy
contribution sum_t w_t Tr(Sigma_s(tau_t) Gbar(tau_t)) of selfenergy.sigma_pair
is a polynomial in the vectors:

  e = sum_ab x_ab th_a th_b + sum_cd y_cd th'_c th'_d
      + sum_abcd W_ab,cd th_a th_b th'_c th'_d,

with x from Sigma[S_xi, D], y from Sigma[D, S_eta] and W from
Sigma[S_xi, S_eta].  Writing q = vec(th th^T), q' = vec(th' th'^T), every
unbiased distribution has E[q] = u = vec(I), and its fourth moments
M4[(ab),(a'b')] = E[th_a th_b th_a' th_b'] fix the variance exactly:

  E[e]   = x.u + y.u + u^T W u
  E[e^2] = x^T M4 x + y^T M4 y + tr(W^T M4 W M4) + 2 (x.u)(y.u)
           + 2 x^T M4 W u + 2 y^T M4 W^T u.

Distributions (all with E[th th^T] = I):
* +-1 (Section II): M4 = d_ab d_a'b' + d_aa' d_bb' + d_ab' d_ba' - 2 d_abab'.
* k = 1 importance draws th = e_Q / sqrt(p_Q): M4 = d_{a=b=a'=b'} / p_a.
* stratified (classes Q mod K, class c drawn with probability pi_c, +-1 /
  sqrt(pi_c) on its members): the +-1 pattern restricted to one class,
  divided by pi_c, summed over classes.

W uses the energy of eq:sigma for one bilinear piece on each vertex,
Tr(Sigma[a(x)b, c(x)d] Gbar) = 2 Tr(b G c Gb) Tr(a G d Gb) - Tr(a G c Gb b G d Gb).
"""
from __future__ import annotations

import numpy as np

from . import selfenergy as se
from .split import Split

VERTEX = (("L", "S"), ("S", "L"), ("S", "S"))   # the stochastic vertex of eq:RS-SRI


def _factors(b: np.ndarray, split: Split):
    kl = split.kl_dense()
    return {"L": kl, "S": b - kl}


def pair_forms(b: np.ndarray, split: Split, g: np.ndarray, gb: np.ndarray, w: np.ndarray):
    """(x [A][A], y [A][A], W [A*A][A*A]) of the quadratic and quartic parts
    of the pair energy, summed over the tau quadrature with weights w."""
    k = _factors(b, split)
    na = b.shape[0]
    x = np.zeros((na, na))
    y = np.zeros((na, na))
    wt = np.zeros((na, na, na, na))
    for t in range(g.shape[0]):
        gt, gbt = g[t], gb[t]
        m = {}
        tr1 = {}
        for s1 in "LS":
            for s2 in "LS":
                mm = np.einsum("xij,jk,ykl,lm->xyim", k[s1], gt, k[s2], gbt, optimize=True)
                m[s1 + s2] = mm                                   # K^s1_x G K^s2_y Gb
                tr1[s1 + s2] = np.einsum("xyii->xy", mm)
        for sa, sb in VERTEX:
            for sc, sd in VERTEX:
                # 2 Tr(b G c Gb) Tr(a G d Gb) - Tr(a G c Gb b G d Gb), indices (a, b, c, d)
                direct = 2.0 * np.einsum("bc,ad->abcd", tr1[sb + sc], tr1[sa + sd])
                exch = np.einsum("acij,bdji->abcd", m[sa + sc], m[sb + sd], optimize=True)
                wt += w[t] * (direct - exch)
        for sa, sb in VERTEX:
            for a in range(na):
                for c in range(na):
                    x[a, c] += w[t] * np.sum(se.sigma_d_right(split, k[sa][a], k[sb][c], gt, gbt) * gbt.T)
                    y[a, c] += w[t] * np.sum(se.sigma_d_left(split, k[sa][a], k[sb][c], gt, gbt) * gbt.T)
    return x, y, wt.reshape(na * na, na * na)


def m4_pm1(na: int, members=None) -> np.ndarray:
    """Fourth moments of +-1 vectors (on `members` only, if given)."""
    idx = np.arange(na) if members is None else np.asarray(members)
    out = np.zeros((na, na, na, na))
    for a in idx:
        for b in idx:
            out[a, a, b, b] += 1.0
            out[a, b, a, b] += 1.0
            out[a, b, b, a] += 1.0
        out[a, a, a, a] -= 2.0
    return out.reshape(na * na, na * na)


def m4_importance(p: np.ndarray) -> np.ndarray:
    na = p.shape[0]
    out = np.zeros((na, na, na, na))
    for a in range(na):
        out[a, a, a, a] = 1.0 / p[a]
    return out.reshape(na * na, na * na)


def m4_stratified(pi: np.ndarray, nclass: int, na: int) -> np.ndarray:
    return sum(m4_pm1(na, np.arange(c, na, nclass)) / pi[c] for c in range(nclass))


def mean_var(x: np.ndarray, y: np.ndarray, wm: np.ndarray, m4: np.ndarray):
    """Exact mean and variance of e for independent vectors with moments m4."""
    na = x.shape[0]
    u = np.eye(na).reshape(-1)
    xv, yv = x.reshape(-1), y.reshape(-1)
    mean = xv @ u + yv @ u + u @ wm @ u
    e2 = (xv @ m4 @ xv + yv @ m4 @ yv + np.trace(wm.T @ m4 @ wm @ m4) + 2.0 * (xv @ u) * (yv @ u)
          + 2.0 * xv @ m4 @ wm @ u + 2.0 * yv @ m4 @ wm.T @ u)
    return float(mean), float(e2 - mean * mean)


def mixture_terms(x: np.ndarray, y: np.ndarray, wm: np.ndarray, pieces):
    """For moments M4 = sum_j P_j / r_j (r on the simplex), the variance is
    sum_jk C_jk / (r_j r_k) + sum_j c_j / r_j + const - mean^2.  pieces: the
    P_j.  Returns (C, c, const, mean)."""
    na = x.shape[0]
    u = np.eye(na).reshape(-1)
    xv, yv = x.reshape(-1), y.reshape(-1)
    wu, wtu = wm @ u, wm.T @ u
    mean = float(xv @ u + yv @ u + u @ wm @ u)
    a = [wm.T @ p @ wm for p in pieces]                        # tr(W^T P_j W P_k) = sum(A_j * P_k^T)
    cmat = np.array([[float(np.sum(a[j] * pieces[k].T)) for k in range(len(pieces))] for j in range(len(pieces))])
    cvec = np.array([float(xv @ p @ xv + yv @ p @ yv + 2.0 * xv @ p @ wu + 2.0 * yv @ p @ wtu) for p in pieces])
    const = 2.0 * float(xv @ u) * float(yv @ u)
    return cmat, cvec, const, mean


def mixture_var(terms, r: np.ndarray) -> float:
    cmat, cvec, const, mean = terms
    inv = 1.0 / r
    return float(inv @ cmat @ inv + cvec @ inv + const - mean * mean)


def importance_terms(x: np.ndarray, y: np.ndarray, wm: np.ndarray):
    """mixture_terms for k = 1 importance draws (piece j: the single moment
    E[th_j^4] = 1 / p_j), without forming the pieces."""
    na = x.shape[0]
    u = np.eye(na).reshape(-1)
    d = np.arange(na) * (na + 1)                                # index of (a, a)
    wd = wm[np.ix_(d, d)]
    wu, wtu = (wm @ u)[d], (wm.T @ u)[d]
    xd, yd = x[np.arange(na), np.arange(na)], y[np.arange(na), np.arange(na)]
    mean = float(x.reshape(-1) @ u + y.reshape(-1) @ u + u @ wm @ u)
    cvec = xd * xd + yd * yd + 2.0 * xd * wu + 2.0 * yd * wtu
    const = 2.0 * float(x.reshape(-1) @ u) * float(y.reshape(-1) @ u)
    return wd * wd, cvec, const, mean
