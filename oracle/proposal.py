"""Importance proposal over the auxiliary index (a project form, not in the
paper; it changes how the stochastic orbitals of Section II are drawn, not
what they estimate).

Stochastic vectors theta = (1/sqrt(k)) sum_{j<k} e_j u_{Q_j} / sqrt(p_{Q_j})
with Q_j ~ p and e_j = +-1 satisfy E[theta theta^T] = I for any p > 0, which
is all the unbiasedness of eq:abgd_l and eq:RS-SRI needs.  k = 1 is the
default.  p comes from a small network over per-Q features:

  p = (1 - alpha) softmax(z) + alpha / N_aux,
  z_Q = w2 . tanh(W1 phi_Q + b1)          (hidden width 128)

trained to match per-Q contribution magnitudes t_Q that the method itself
produces (KL(t/sum t || softmax z) summed over training chains).

Per-Q contributions use the energy of eq:sigma with one bilinear vertex on
each side, e[a(x)a, b(x)b](tau) = 2 Tr(a G b Gb)^2 - Tr((a G b Gb)^2),
integrated over tau: P(a, b) = sum_t w_t e(tau_t).  With S_Q = B_Q (x) B_Q -
K_Q (x) K_Q the stochastic vertex a single index Q carries,

  d_QQ' = P(B_Q,B_Q') - P(B_Q,K_Q') - P(K_Q,B_Q') + P(K_Q,K_Q')
  cL_Q  = sum_R [P(K_R, B_Q) - P(K_R, K_Q)]
  cR_Q  = sum_R [P(B_Q, K_R) - P(K_Q, K_R)]
  t_Q   = |cL_Q| + |cR_Q| + sum_Q' |d_QQ'|

B_Q enters on its numerical support: elements below TARGET_SUPPORT_REL times
max|B| are dropped for the target tables only.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import rng as _rng

HIDDEN = 128
D_IN = 4
TARGET_SUPPORT_REL = 1e-10
END_SCALE = 4.0
NORM_FLOOR = 1e-30


# ---------------------------------------------------------------------------
# Features
# ---------------------------------------------------------------------------

def raw_features(x: np.ndarray, xq: np.ndarray, b: np.ndarray, kl: np.ndarray,
                 density: np.ndarray) -> np.ndarray:
    """phi_Q = (tanh(d_end/4), ln||B_Q||_F, ln(||B_Q - K_Q||_F + 1e-30),
    sum_ij B_Q,ij P_ij) with d_end the distance of x_Q to the nearer chain end
    and P the density matrix."""
    d_end = np.minimum(xq - x[0], x[-1] - xq)
    f1 = np.tanh(d_end / END_SCALE)
    f2 = np.log(np.sqrt(np.einsum("qij,qij->q", b, b)) + NORM_FLOOR)
    bs = b - kl
    f3 = np.log(np.sqrt(np.einsum("qij,qij->q", bs, bs)) + NORM_FLOOR)
    f4 = np.einsum("qij,ij->q", b, density)
    return np.stack([f1, f2, f3, f4], axis=1)


def density_matrix(eps, c, mu, beta) -> np.ndarray:
    """P = -2 G(beta-) = 2 C diag(f) C^T."""
    from .green import occupations
    f = occupations(eps, mu, beta)
    return 2.0 * (c * f) @ c.T


# ---------------------------------------------------------------------------
# Per-Q contribution tables and targets
# ---------------------------------------------------------------------------

def truncate(b: np.ndarray, rel: float = TARGET_SUPPORT_REL) -> np.ndarray:
    m = np.max(np.abs(b))
    return np.where(np.abs(b) >= rel * m, b, 0.0)


def pair_energy(a: np.ndarray, bb: np.ndarray, g, gb, w) -> float:
    """P(a, b) = sum_t w_t [2 Tr(a G b Gb)^2 - Tr((a G b Gb)^2)]."""
    tot = 0.0
    for t in range(w.shape[0]):
        m = a @ g[t] @ bb @ gb[t]
        tr = np.trace(m)
        tot += w[t] * (2.0 * tr * tr - float(np.sum(m * m.T)))
    return tot


def pair_tables(bt: np.ndarray, kl: np.ndarray, g, gb, w):
    """P over every (Q, Q') for the four factor choices: returns dict of
    [N_aux][N_aux] arrays keyed 'BB', 'BK', 'KB', 'KK'."""
    naux = bt.shape[0]
    src = {"B": bt, "K": kl}
    out = {}
    for key in ("BB", "BK", "KB", "KK"):
        x, y = src[key[0]], src[key[1]]
        tab = np.zeros((naux, naux))
        for q in range(naux):
            for r in range(naux):
                tab[q, r] = pair_energy(x[q], y[r], g, gb, w)
        out[key] = tab
    return out


def targets_from_tables(tab) -> np.ndarray:
    d = tab["BB"] - tab["BK"] - tab["KB"] + tab["KK"]
    cl = np.sum(tab["KB"] - tab["KK"], axis=0)      # sum over R of P(K_R, B_Q) - P(K_R, K_Q)
    cr = np.sum(tab["BK"] - tab["KK"], axis=1)      # sum over R of P(B_Q, K_R) - P(K_Q, K_R)
    return np.abs(cl) + np.abs(cr) + np.sum(np.abs(d), axis=1)


# ---------------------------------------------------------------------------
# Network, loss, gradients, optimiser
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Mlp:
    w1: np.ndarray      # [HIDDEN][D_IN]
    b1: np.ndarray      # [HIDDEN]
    w2: np.ndarray      # [HIDDEN]
    mean: np.ndarray    # [D_IN] feature standardisation
    std: np.ndarray     # [D_IN]


def init_mlp(seed: int, mean: np.ndarray, std: np.ndarray) -> Mlp:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights from counter stream 2:
    word(seed, 2, 0, q) for q over w1 (row-major), then b1, then w2."""
    nw1, nb1, nw2 = HIDDEN * D_IN, HIDDEN, HIDDEN
    u = _rng.uniform_from_word(_rng.words(seed, 2, 0, np.arange(nw1 + nb1 + nw2)))
    r = 2.0 * u - 1.0
    w1 = r[:nw1].reshape(HIDDEN, D_IN) / np.sqrt(D_IN)
    b1 = r[nw1:nw1 + nb1] / np.sqrt(D_IN)
    w2 = r[nw1 + nb1:] / np.sqrt(HIDDEN)
    return Mlp(w1, b1, w2, np.asarray(mean, float), np.asarray(std, float))


def forward(m: Mlp, phi: np.ndarray):
    """Logits z[N_aux] and the hidden activations (for backprop)."""
    xs = (phi - m.mean) / m.std
    h = np.tanh(xs @ m.w1.T + m.b1)
    return h @ m.w2, (xs, h)


def softmax(z: np.ndarray) -> np.ndarray:
    e = np.exp(z - np.max(z))
    return e / np.sum(e)


def proposal(z: np.ndarray, alpha: float) -> np.ndarray:
    return (1.0 - alpha) * softmax(z) + alpha / z.shape[0]


def loss(m: Mlp, chains) -> float:
    """sum over chains of KL(t_hat || softmax(z)); chains = [(phi, t_hat)]."""
    tot = 0.0
    for phi, th in chains:
        z, _ = forward(m, phi)
        ls = z - np.max(z) - np.log(np.sum(np.exp(z - np.max(z))))
        nz = th > 0
        tot += float(np.sum(th[nz] * (np.log(th[nz]) - ls[nz])))
    return tot


def gradients(m: Mlp, chains):
    """Exact gradients of ``loss`` w.r.t. (w1, b1, w2) by backpropagation:
    dL/dz = softmax(z) - t_hat per chain."""
    gw1 = np.zeros_like(m.w1)
    gb1 = np.zeros_like(m.b1)
    gw2 = np.zeros_like(m.w2)
    for phi, th in chains:
        z, (xs, h) = forward(m, phi)
        dz = softmax(z) - th
        gw2 += h.T @ dz
        da = (dz[:, None] * m.w2[None, :]) * (1.0 - h * h)
        gw1 += da.T @ xs
        gb1 += np.sum(da, axis=0)
    return gw1, gb1, gw2


@dataclasses.dataclass
class AdamState:
    t: int
    m: list
    v: list


def adam_init(m: Mlp) -> AdamState:
    ps = [m.w1, m.b1, m.w2]
    return AdamState(0, [np.zeros_like(p) for p in ps], [np.zeros_like(p) for p in ps])


def adam_step(m: Mlp, st: AdamState, grads, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015) with bias correction, in place."""
    st.t += 1
    for i, (p, gr) in enumerate(zip([m.w1, m.b1, m.w2], grads)):
        st.m[i] = b1 * st.m[i] + (1 - b1) * gr
        st.v[i] = b2 * st.v[i] + (1 - b2) * gr * gr
        mh = st.m[i] / (1 - b1 ** st.t)
        vh = st.v[i] / (1 - b2 ** st.t)
        p -= lr * mh / (np.sqrt(vh) + eps)


def importance_theta(p: np.ndarray, seed: int, stream: int, ns: int, k: int = 1,
                     s0: int = 0) -> np.ndarray:
    """theta[s] = (1/sqrt(k)) sum_j e_j u_{Q_j} / sqrt(p_{Q_j}) with (Q_j, e_j)
    from the counter generator and the sequential CDF of p."""
    cdf = _rng.proposal_cdf(p)
    q, sgn = _rng.importance_draws(seed, stream, ns, k, cdf, s0)
    theta = np.zeros((ns, p.shape[0]))
    for s in range(ns):
        for j in range(k):
            theta[s, q[s, j]] += sgn[s, j] / np.sqrt(k * p[q[s, j]])
    return theta


# ---------------------------------------------------------------------------
# Stratified stochastic orbitals (project form)
# ---------------------------------------------------------------------------

def class_probabilities(p: np.ndarray, nclass: int) -> np.ndarray:
    """pi_c = sum of p_Q over the class Q = c (mod nclass), normalised; all
    sums sequential in index order (the class draw compares against them)."""
    p = np.asarray(p, dtype=np.float64)
    pi = [0.0] * nclass
    for q in range(p.shape[0]):
        pi[q % nclass] += float(p[q])
    tot = 0.0
    for c in range(nclass):
        tot += pi[c]
    return np.array([x / tot for x in pi])


def stratified_theta(p: np.ndarray, nclass: int, seed: int, stream: int, ns: int,
                     s0: int = 0) -> np.ndarray:
    """theta[s]: one class c ~ pi per vector (pi from class_probabilities),
    theta_Q = e_Q / sqrt(pi_c) for Q = c (mod nclass) with e_Q the +-1 orbital
    of the same (stream, s, Q), and 0 elsewhere.  E[theta theta^T] = I for
    any pi > 0: Q sits in exactly one class, drawn with probability pi_c, and
    distinct Q carry independent signs."""
    naux = p.shape[0]
    pi = class_probabilities(p, nclass)
    c = _rng.class_draws(seed, stream, ns, _rng.proposal_cdf(pi), s0)
    e = _rng.rademacher(seed, stream, ns, naux, s0)
    member = (np.arange(naux)[None, :] % nclass) == c[:, None]
    return np.where(member, e / np.sqrt(pi[c])[:, None], 0.0)
