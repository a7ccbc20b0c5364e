"""Quasiparticle energies from the self-energy (the Conclusions' excited-
state direction; the paper gives no method, so this module states one).

* The diagonal of the self-energy in the orbital basis of F (F c_k = S c_k
  eps_k, c^T S c = 1) on the first M Matsubara frequencies, by the same tau
  quadrature as eq:GFT:  s_k(i w_n) = sum_t w_t e^{i w_n tau_t} (c_k^T
  Sigma(tau_t) c_k).
* Its analytic continuation by the M-point Pade approximant in Thiele's
  continued-fraction form with the Vidberg-Serene recursion for the
  coefficients (J. Low Temp. Phys. 29, 179 (1977)): g_0(z_i) = u_i,
  g_p(z) = (g_{p-1}(z_{p-1}) - g_{p-1}(z)) / ((z - z_{p-1}) g_{p-1}(z)),
  a_p = g_p(z_p) (a vanishing a_p ends the fraction: later a are zero),
  and C(z) = a_0 / (1 + a_1 (z - z_0) / (1 + a_2 (z - z_1) / (1 + ...)))
  evaluated by the three-term recurrence of its convergents.
* The quasiparticle equation in the diagonal approximation,
  E = eps_k + Re s_k(E - mu + i eta), solved by fixed-point iteration from
  E = eps_k (frequencies are measured from mu, as in eq:dyson's
  (mu + i w) S), stopped when |E_new - E| <= 1e-13 (at most `iters` steps).

Test infrastructure only, like the rest of oracle/.
"""
from __future__ import annotations

import numpy as np

from . import green


def sigma_mo_diag_iw(sigma_tau, f, s, tau, w, omegas):
    """s_k(i w_n) for every orbital k of (F, S): [n_w][N] complex."""
    e, c = green.orbitals(f, s)
    diag = np.einsum("ik,tij,jk->tk", c, sigma_tau, c)                   # [ntau][N]
    ph = np.exp(1j * np.outer(omegas, tau)) * w[None, :]                 # [n_w][ntau]
    return ph @ diag, e


def pade_coefficients(z: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Thiele continued-fraction coefficients a_p through the points (z_i, u_i)."""
    m = len(z)
    g = np.array(u, dtype=np.complex128)          # g[i] holds g_p(z_i) for i >= p
    a = np.zeros(m, dtype=np.complex128)
    a[0] = g[0]
    for p in range(1, m):
        if a[p - 1] == 0:                         # the fraction ends: later terms vanish
            break
        prev = g[p - 1]                           # g_{p-1}(z_{p-1})
        for i in range(p, m):
            g[i] = (prev - g[i]) / ((z[i] - z[p - 1]) * g[i])
        a[p] = g[p]
    return a


def pade_eval(z_pts: np.ndarray, a: np.ndarray, z: complex) -> complex:
    """C(z) from the convergent recurrence A_{p} = A_{p-1} + (z - z_{p-1}) a_p
    A_{p-2} (and B likewise), A_{-1} = 0, A_0 = a_0, B_{-1} = B_0 = 1."""
    a_m2, a_m1 = 0.0 + 0.0j, complex(a[0])
    b_m2, b_m1 = 1.0 + 0.0j, 1.0 + 0.0j
    for p in range(1, len(a)):
        t = (z - z_pts[p - 1]) * a[p]
        a_m2, a_m1 = a_m1, a_m1 + t * a_m2
        b_m2, b_m1 = b_m1, b_m1 + t * b_m2
    return a_m1 / b_m1


def qp_energies(sigma_tau, f, s, mu, beta, tau, w, n_pade, eta, iters=200):
    """E_k for every orbital: (E [N], converged [N] bool)."""
    omegas = (2.0 * np.arange(n_pade) + 1.0) * np.pi / beta
    siw, eps = sigma_mo_diag_iw(sigma_tau, f, s, tau, w, omegas)
    z = 1j * omegas
    out = np.empty(len(eps))
    ok = np.zeros(len(eps), dtype=bool)
    for k in range(len(eps)):
        a = pade_coefficients(z, siw[:, k])
        e = eps[k]
        for _ in range(iters):
            e_new = eps[k] + pade_eval(z, a, complex(e - mu, eta)).real
            done = abs(e_new - e) <= 1e-13
            e = e_new
            if done:
                ok[k] = True
                break
        out[k] = e
    return out, ok
