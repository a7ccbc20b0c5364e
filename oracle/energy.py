"""Correlation energy from the self-energy, and estimator statistics.

eq:corr gives the correlation energy per electron as (1/N_e) times the
tau-integral of Tr(Sigma(tau) G(beta - tau)).  As printed it lacks the sign
and factor that make it the Galitskii-Migdal energy; the reading used here
is fixed by the textbook limit it must reach: for the one-shot
non-interacting G and beta -> infinity, the closed-shell second-order energy
must equal the textbook MP2 energy (checked by ``mp2_energy`` against the
quadrature in the tests).  With Sigma of eq:sigma that gives

  E_corr,total = -GM_FACTOR * int_0^beta Tr[Sigma(tau) G(beta - tau)] dtau

and E_corr per electron = E_corr,total / N_e.  The tau integral is the
quadrature sum over the tau grid.
"""
from __future__ import annotations

import numpy as np

from .green import occupations

# int Tr(Sigma Gb) -> -2 E_MP2 in the zero-temperature limit: the (occ, occ,
# virt, virt) and (virt, virt, occ, occ) index classes of the closed form
# each give -E_MP2.  The test suite pins this against the textbook
# closed-shell MP2 formula.
GM_FACTOR = 0.5


def trace_product(a: np.ndarray, bt: np.ndarray) -> float:
    """Tr(A B) = sum_ij A_ij B_ji."""
    return float(np.sum(a * bt.T))


def energy_integrand(sigma: np.ndarray, gb: np.ndarray) -> np.ndarray:
    """Tr(Sigma(tau_t) G(beta - tau_t)) for every tau point."""
    return np.array([trace_product(s, g) for s, g in zip(sigma, gb)])


def energy_total(sigma: np.ndarray, gb: np.ndarray, w: np.ndarray) -> float:
    return -GM_FACTOR * float(np.dot(w, energy_integrand(sigma, gb)))


def sample_energies(e_det: np.ndarray, e_samples: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Per-pair total energies E_s = -GM sum_t w_t (Tr(Sigma_det Gb) + e_s(tau_t)).

    e_det: [ntau]; e_samples: [ns][ntau] with e_s(tau) = Tr(Sigma_s Gb)."""
    return -GM_FACTOR * (e_samples + e_det[None, :]) @ w


def mean_stderr(es: np.ndarray):
    es = np.asarray(es, dtype=np.float64)
    m = float(np.mean(es))
    if es.shape[0] < 2:
        return m, float("nan")
    return m, float(np.std(es, ddof=1) / np.sqrt(es.shape[0]))


# ---------------------------------------------------------------------------
# Molecular-orbital closed forms (independent of the tau grid).
# ---------------------------------------------------------------------------

def mo_factors(b: np.ndarray, c: np.ndarray) -> np.ndarray:
    """B in the orbital basis: C^T B_Q C."""
    return np.einsum("ai,qab,bj->qij", c, b, c, optimize=True)


def mo_eri(b: np.ndarray, c: np.ndarray) -> np.ndarray:
    bm = mo_factors(b, c)
    n = c.shape[1]
    flat = bm.reshape(bm.shape[0], n * n)
    return (flat.T @ flat).reshape(n, n, n, n)


def sigma_mo(b, eps, c, mu, beta, tau) -> np.ndarray:
    """Sigma^MO_xy(tau) = -sum_kmp (xm|pk)[2(kp|my) - (mp|ky)]
    (1-f_k)(1-f_m) f_p exp(-(e~_k + e~_m - e~_p) tau): eq:sigma with the
    diagonal orbital-basis G."""
    from .green import softplus
    v = mo_eri(b, c)
    et = eps - mu
    out = []
    for tv in np.atleast_1d(tau):
        wk = np.exp(-et * tv - softplus(-beta * et))      # (1-f) e^{-e~ tau}
        wp = np.exp(et * tv - softplus(beta * et))        # f e^{e~ tau}
        inner = 2.0 * v - v.transpose(2, 1, 0, 3)          # [k p m y] -> 2(kp|my)-(mp|ky)
        s = -np.einsum("xmpk,kpmy,k,m,p->xy", v, inner, wk, wk, wp, optimize=True)
        out.append(s)
    return np.array(out)


def energy_integral_mo(b, eps, c, mu, beta) -> float:
    """int_0^beta Tr(Sigma(tau) G(beta - tau)) dtau in closed form:
    sum_{kmpx} (xm|pk)[2(kp|mx) - (mp|kx)] (1-f_k)(1-f_m) f_p f_x
    (1 - exp(-beta D)) / D with D = e~_k + e~_m - e~_p - e~_x.

    The occupation product and the kernel are combined in log form so that
    large beta neither overflows nor loses the classes where exp(-beta D)
    cancels the occupations."""
    from .green import softplus
    v = mo_eri(b, c)
    et = eps - mu
    lf = -softplus(beta * et)           # ln f
    l1f = -softplus(-beta * et)         # ln (1 - f)
    inner = 2.0 * v - v.transpose(2, 1, 0, 3)
    num = np.einsum("xmpk,kpmx->kmpx", v, inner, optimize=True)
    d = (et[:, None, None, None] + et[None, :, None, None]
         - et[None, None, :, None] - et[None, None, None, :])
    lo = (l1f[:, None, None, None] + l1f[None, :, None, None]
          + lf[None, None, :, None] + lf[None, None, None, :])
    tiny = np.abs(d) * beta < 1e-12
    pos = d > 0
    dsafe = np.where(tiny, 1.0, d)
    with np.errstate(over="ignore", under="ignore", invalid="ignore"):
        kpos = np.exp(lo) * (-np.expm1(-beta * dsafe)) / dsafe
        kneg = np.exp(lo - beta * dsafe) * (-np.expm1(beta * dsafe)) / (-dsafe)
    val = np.where(tiny, beta * np.exp(lo), np.where(pos, kpos, kneg))
    return float(np.sum(num * val))


def mp2_energy(b, eps, c, n_occ) -> float:
    """Textbook closed-shell MP2: sum_ijab (ia|jb)[2(ia|jb) - (ib|ja)]
    / (e_i + e_j - e_a - e_b)."""
    v = mo_eri(b, c)
    o = slice(0, n_occ)
    vv = slice(n_occ, c.shape[1])
    iajb = v[o, vv, o, vv]
    ibja = iajb.transpose(0, 3, 2, 1)
    eo, ev = eps[:n_occ], eps[n_occ:]
    den = eo[:, None, None, None] - ev[None, :, None, None] + eo[None, None, :, None] - ev[None, None, None, :]
    return float(np.sum(iajb * (2.0 * iajb - ibja) / den))
