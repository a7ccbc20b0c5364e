"""Self-consistent GF2 on either side of the self-energy (Section III).

The steps around Sigma(tau) that make GF2 self-consistent:

* Matsubara transforms (eq:GFT, eq:Ginverse): X(i w_n) = int_0^beta
  e^{i w_n tau} X(tau) dtau with odd frequencies w_n = (2n+1) pi / beta, and
  X(tau) = (1/beta) sum_n e^{-i w_n tau} X(i w_n).  Real symmetric X(tau)
  gives X(-i w) = conj X(i w), so only n >= 0 is kept and the inverse sum
  is (2/beta) sum_{n>=0} Re[e^{-i w_n tau} X(i w_n)].
* Dyson's equation (eq:dyson) with the non-interacting G0 (eq:G0):
  G(i w) = [(mu + i w) S - F - Sigma(i w)]^{-1}.
* The Fock matrix (eq:F) with the density P = -2 G(beta-):
  F_ij = h_ij + sum_kl P_kl (v_ijkl - v_ilkj / 2), v from the RI factors
  (eq:vKQKQ), i.e. F = h + J[P] - K[P]/2 with J = sum_Q B_Q Tr(B_Q P) and
  K = sum_Q B_Q P B_Q.
* The chemical potential that conserves N_e = -2 sum_ij G_ij(beta-) S_ij.

Readings (where the paper leaves the numerics open):
* Sigma(tau) -> Sigma(i w) is the quadrature on the tau grid of the
  self-energy (Gauss-Legendre; exact to the grid's order for the smooth
  Sigma(tau) at frequencies well below n_tau / beta).
* G(i w) -> G(tau) subtracts the non-interacting G0 of the same F and mu,
  whose tau form is known in closed form: G(tau) = G0(tau) + (2/beta)
  sum_{n < n_w} Re[e^{-i w_n tau} (G - G0)(i w_n)]; the difference decays
  as 1/w^2, so the truncation error falls as 1/n_w.
* mu is found by bisection on N_e(mu) at fixed Sigma(i w) (N_e increases
  with mu) to a fixed bracket width.
* The synthetic chain supplies F, not h: h = F_tb - J[P0] + K[P0]/2 with P0
  the density of the tight-binding F_tb, so that the first Fock build
  reproduces F_tb.

Test infrastructure only, like the rest of oracle/.
"""
from __future__ import annotations

import numpy as np

from . import green


def matsubara(beta: float, nw: int) -> np.ndarray:
    """Odd Matsubara frequencies w_n = (2n+1) pi / beta, n = 0 .. nw-1."""
    return (2.0 * np.arange(nw) + 1.0) * np.pi / beta


def tau_to_iw(x_tau: np.ndarray, tau: np.ndarray, w: np.ndarray, omegas: np.ndarray) -> np.ndarray:
    """eq:GFT by the tau quadrature: X(i w_n) = sum_t w_t e^{i w_n tau_t} X(tau_t)."""
    ph = np.exp(1j * omegas[:, None] * tau[None, :]) * w[None, :]          # [nw][ntau]
    nt, n, m = x_tau.shape
    x = x_tau.reshape(nt, n * m)
    return (ph.real @ x + 1j * (ph.imag @ x)).reshape(-1, n, m)


def g0_iw(f: np.ndarray, s: np.ndarray, mu: float, omegas: np.ndarray) -> np.ndarray:
    """eq:G0: [(mu + i w) S - F]^{-1} per frequency."""
    out = np.empty((len(omegas),) + f.shape, dtype=np.complex128)
    for k, wn in enumerate(omegas):
        out[k] = np.linalg.inv((mu + 1j * wn) * s - f)
    return out


def dyson(f: np.ndarray, s: np.ndarray, mu: float, sigma_iw: np.ndarray, omegas: np.ndarray) -> np.ndarray:
    """eq:dyson: G(i w) = [G0(i w)^{-1} - Sigma(i w)]^{-1}."""
    out = np.empty((len(omegas),) + f.shape, dtype=np.complex128)
    for k, (wn, sg) in enumerate(zip(omegas, sigma_iw)):
        out[k] = np.linalg.inv((mu + 1j * wn) * s - f - sg)
    return out


def iw_to_tau(diff_iw: np.ndarray, omegas: np.ndarray, beta: float, tau: np.ndarray) -> np.ndarray:
    """eq:Ginverse for a difference that decays at high frequency:
    (2/beta) sum_n Re[e^{-i w_n tau} X(i w_n)] for each tau (tau in [0, beta])."""
    ph = np.exp(-1j * np.outer(np.atleast_1d(tau), omegas))                 # [ntau][nw]
    nw, n, m = diff_iw.shape
    return (2.0 / beta) * np.real(ph @ diff_iw.reshape(nw, n * m)).reshape(-1, n, m)


def green_tau_dyson(f, s, mu, beta, sigma_iw, omegas, tau):
    """G(tau) and G(beta - tau) of the Dyson G: the closed-form G0(tau) of
    (F, S, mu) plus the back-transformed G - G0.  Returns (G, Gbar, G(beta-))."""
    e, c = green.orbitals(f, s)
    g0, g0b = green.green_tau(e, c, mu, beta, tau)
    _, g0beta = green.green_tau(e, c, mu, beta, [0.0])          # G0(beta - 0) = G0(beta-)
    d = dyson(f, s, mu, sigma_iw, omegas) - g0_iw(f, s, mu, omegas)
    g = g0 + iw_to_tau(d, omegas, beta, tau)
    gb = g0b + iw_to_tau(d, omegas, beta, beta - np.asarray(tau))
    gbeta = g0beta[0] + iw_to_tau(d, omegas, beta, [beta])[0]
    return g, gb, gbeta


def electron_count(gbeta: np.ndarray, s: np.ndarray) -> float:
    """N_e = -2 sum_ij G_ij(beta-) S_ij (Section III)."""
    return float(-2.0 * np.sum(gbeta * s))


def g_beta_minus(f, s, mu, beta, sigma_iw, omegas) -> np.ndarray:
    e, c = green.orbitals(f, s)
    _, g0beta = green.green_tau(e, c, mu, beta, [0.0])
    d = dyson(f, s, mu, sigma_iw, omegas) - g0_iw(f, s, mu, omegas)
    return g0beta[0] + iw_to_tau(d, omegas, beta, [beta])[0]


def tune_mu(f, s, beta, sigma_iw, omegas, n_elec, lo, hi, steps=60):
    """Bisection on mu in [lo, hi] for N_e(mu) = n_elec at fixed Sigma(i w):
    `steps` halvings of the bracket, the midpoint of the last bracket."""
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if electron_count(g_beta_minus(f, s, mid, beta, sigma_iw, omegas), s) < n_elec:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def fock(h: np.ndarray, b: np.ndarray, p: np.ndarray) -> np.ndarray:
    """eq:F with the RI factors: F = h + J[P] - K[P]/2, J = sum_Q B_Q Tr(B_Q P),
    K = sum_Q B_Q P B_Q (P = -2 G(beta-) the spin-summed density)."""
    j = np.einsum("qij,q->ij", b, np.einsum("qkl,lk->q", b, p))
    k = np.einsum("qik,kl,qlj->ij", b, p, b)
    return h + j - 0.5 * k


def core_hamiltonian(f_tb: np.ndarray, b: np.ndarray, p0: np.ndarray) -> np.ndarray:
    """h = F_tb - J[P0] + K[P0]/2: the first Fock build returns F_tb."""
    return 2.0 * f_tb - fock(f_tb, b, p0)
