"""Second-order self-energy and its RS-SRI estimator.

eq:sigma (second-order Born, closed shell):

  Sigma_ij(tau) = sum_{klmnpq} v_imqk (2 v_lpnj - v_nplj)
                  G_kl(tau) G_mn(tau) G_pq(beta - tau)

eq:sigma_2 replaces the first v by the RS-SRI form eq:RS-SRI averaged over
theta, and the second v (both its direct and its exchange use) by the same
form averaged over an independent set theta'.  Every vertex is then a sum of
bilinear pieces a (x) b (v_imqk = a_im b_qk), and for one bilinear piece on
each vertex eq:sigma collapses (sum over m,n and over k,l,p,q) to

  Sigma[a(x)b, c(x)d] = 2 Tr(b G c Gb) (a G d) - a G c Gb b G d,

with Gb = G(beta - tau).  The brute-force evaluation of eq:sigma below is
the definition itself; the bilinear form is checked against it.

The deterministic vertex D = sum_Q K^{L,Q} (x) K^{L,Q} acts through the
Coulomb/exchange-like map on a matrix W,

  JK(W) = 2 sum_Q Tr(K^{L,Q} W) K^{L,Q} - sum_Q K^{L,Q} W K^{L,Q},

because summing the bilinear form over Q gives
  Sigma[D, c(x)d] = JK(G c Gb) (G d)   and   Sigma[a(x)b, D] = (a G) JK(Gb b G).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .split import Split

Term = Tuple[np.ndarray, np.ndarray, float]   # (a, b, coefficient): coef * a (x) b


def sigma_bruteforce(v1: np.ndarray, v2: np.ndarray, g: np.ndarray, gb: np.ndarray) -> np.ndarray:
    """eq:sigma with first vertex v1 and second vertex v2, summed literally."""
    w = 2.0 * v2 - v2.transpose(2, 1, 0, 3)      # w_lpnj = 2 v_lpnj - v_nplj
    return np.einsum("imqk,lpnj,kl,mn,pq->ij", v1, w, g, g, gb, optimize="optimal")


def sigma_bilinear(a, b, c, d, g, gb) -> np.ndarray:
    """eq:sigma for v1 = a (x) b and v2 = c (x) d."""
    ag = a @ g
    cgb = c @ gb
    direct = 2.0 * np.trace(b @ g @ cgb) * (ag @ d)
    exchange = ag @ cgb @ b @ g @ d
    return direct - exchange


def sigma_terms(terms1: Sequence[Term], terms2: Sequence[Term], g, gb) -> np.ndarray:
    """eq:sigma for v1 = sum coef*a(x)b and v2 = sum coef*c(x)d (bilinearity)."""
    n = g.shape[0]
    out = np.zeros((n, n))
    for a, b, ca in terms1:
        for c, d, cc in terms2:
            out += (ca * cc) * sigma_bilinear(a, b, c, d, g, gb)
    return out


def jk(split: Split, w: np.ndarray) -> np.ndarray:
    """JK(W) = 2 sum_Q Tr(K^L_Q W) K^L_Q - sum_Q K^L_Q W K^L_Q on the supports."""
    out = np.zeros_like(w)
    for s, k in zip(split.support, split.blocks):
        if s.shape[0] == 0:
            continue
        ws = w[np.ix_(s, s)]
        t = float(np.sum(k * ws.T))              # Tr(k W_SS)
        out[np.ix_(s, s)] += 2.0 * t * k - k @ ws @ k
    return out


def sigma_d_left(split: Split, c, d, g, gb) -> np.ndarray:
    """Sigma[D, c (x) d] = sum_Q Sigma[K_Q (x) K_Q, c (x) d]."""
    return jk(split, g @ c @ gb) @ (g @ d)


def sigma_d_right(split: Split, a, b, g, gb) -> np.ndarray:
    """Sigma[a (x) b, D] = sum_Q Sigma[a (x) b, K_Q (x) K_Q]."""
    return (a @ g) @ jk(split, gb @ b @ g)


def sigma_dd(split: Split, g, gb, q_rows=None) -> np.ndarray:
    """Sigma[D, D] = sum_{Q,Q'} Sigma[K_Q (x) K_Q, K_Q' (x) K_Q'] on blocks.

    For each pair: M = k_Q G[S_Q,S_Q'] k_Q', T = M Gb[S_Q',S_Q]; the pair adds
    2 Tr(T) M - T M to Sigma[S_Q, S_Q'] (the bilinear form restricted to the
    supports).  q_rows restricts the first index Q to a subset (partial sums,
    used only to time the oracle on a sample)."""
    n = g.shape[0]
    naux = split.naux
    wmax = max(split.wmax, 1)
    idx = np.zeros((naux, wmax), dtype=np.int64)
    kb = np.zeros((naux, wmax, wmax))
    for q, (s, k) in enumerate(zip(split.support, split.blocks)):
        idx[q, :s.shape[0]] = s
        kb[q, :s.shape[0], :s.shape[0]] = k
    out = np.zeros((n, n))
    for q in (range(naux) if q_rows is None else q_rows):
        if split.support[q].shape[0] == 0:
            continue
        iq = idx[q]
        gqq = g[iq][:, idx].transpose(1, 0, 2)            # [Q'][a][b] = G[S_Q(a), S_Q'(b)]
        gbqq = gb[idx][:, :, iq]                           # [Q'][c][d] = Gb[S_Q'(c), S_Q(d)]
        m = np.matmul(np.matmul(kb[q][None], gqq), kb)     # k_Q G k_Q'
        t = np.matmul(m, gbqq)
        tr = np.trace(t, axis1=1, axis2=2)
        cblk = 2.0 * tr[:, None, None] * m - np.matmul(t, m)   # [Q'][a][d]
        strip = np.zeros((wmax, n))
        np.add.at(strip, (slice(None), idx.reshape(-1)),
                  cblk.transpose(1, 0, 2).reshape(wmax, -1))
        np.add.at(out, iq, strip)
    return out


def jk_dense_b(b: np.ndarray, w: np.ndarray) -> np.ndarray:
    """JK with the full factors: 2 sum_Q Tr(B_Q W) B_Q - sum_Q B_Q W B_Q."""
    t = np.einsum("qij,ji->q", b, w)
    return 2.0 * np.einsum("q,qij->ij", t, b) - np.einsum("qij,jk,qkl->il", b, w, b)


def sigma_ri(b: np.ndarray, g, gb) -> np.ndarray:
    """Deterministic RI-GF2: eq:sigma with v = sum_Q B_Q (x) B_Q on both vertices
    (O(N_aux^2 N^3), small chains only)."""
    n = g.shape[0]
    out = np.zeros((n, n))
    for q in range(b.shape[0]):
        out += jk_dense_b(b, g @ b[q] @ gb) @ (g @ b[q])
    return out


def s_terms(xl: np.ndarray, xs: np.ndarray) -> List[Term]:
    """The stochastic vertex of eq:RS-SRI for one vector:
    R^L (x) R^S + R^S (x) R^L + R^S (x) R^S."""
    return [(xl, xs, 1.0), (xs, xl, 1.0), (xs, xs, 1.0)]


def sigma_pair(split: Split, xl, xs, yl, ys, g, gb) -> np.ndarray:
    """One-pair estimate of eq:sigma_2 minus its deterministic D x D part:
    Sigma[D, S_eta] + Sigma[S_xi, D] + Sigma[S_xi, S_eta], where S_xi is built
    from theta (first vertex) and S_eta from theta' (second vertex)."""
    t1 = s_terms(xl, xs)
    t2 = s_terms(yl, ys)
    out = sigma_terms(t1, t2, g, gb)
    for c, d, coef in t2:
        out += coef * sigma_d_left(split, c, d, g, gb)
    for a, b_, coef in t1:
        out += coef * sigma_d_right(split, a, b_, g, gb)
    return out
