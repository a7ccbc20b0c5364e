"""Writes n800_subset.npz: oracle values of the N = 800 chain on a subset of
its tau points and pairs, for the GPU parity test at the full size.

Problem: 400 dimers (N = 800, N_aux = 2400), beta = 100, eps = 1e-4, the
128-point Gauss-Legendre tau grid, +-1 stochastic orbitals from seed 0.
Subset: tau nodes {0, 1, 126, 127} (two at each end of [0, beta], where G or
G(beta - tau) is largest) and pairs s = 0..3.

Stored (FP64):
  tau_idx[4], tau[4], w[4]     the nodes and their quadrature weights
  e_det[4]                     Tr(Sigma[D,D](tau) Gbar(tau))
  es[4 pairs][4 tau]           Tr(Sigma_s(tau) Gbar(tau)), Sigma_s the one-pair
                               estimate of eq:sigma_2 without its D x D part
  pos[K][2]                    sampled (i, j) positions
  det_pos[4 tau][K]            Sigma[D,D](tau) at those positions
  sig_pos[4 pairs][4 tau][K]   Sigma_s(tau) at those positions
  nnz, wmax, kmax              the split (eq:K_L)

Only the oracle and the seeded input generator are called.  The factor
tensor (12 GB in FP64) is never formed: every Q slice is evaluated from the
geometry when the oracle asks for it.  About two minutes on 8 cores.

Usage: python tests/golden/make_n800_subset.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import chain_inputs as ci                                                  # noqa: E402
from oracle import energy, green, integrals, rng, selfenergy as se, split as sp   # noqa: E402

N_DIMER, BETA, NTAU, EPS, SEED = 400, 100.0, 128, 1e-4, 0
TAU_IDX = [0, 1, 126, 127]
PAIRS = [0, 1, 2, 3]
K_RANDOM, K_BAND = 256, 256


def positions(n):
    r = np.random.default_rng(800)
    rnd = r.integers(0, n, size=(K_RANDOM, 2))
    i = r.integers(0, n, size=K_BAND)
    j = np.clip(i + r.integers(-4, 5, size=K_BAND), 0, n - 1)
    return np.concatenate([rnd, np.stack([i, j], axis=1)]).astype(np.int64)


def main():
    t0 = time.time()
    geo = ci.chain_geometry(N_DIMER)
    n, naux = geo.n, geo.naux

    def b_slice(q):
        return integrals.synthetic_b(geo.x, geo.xq[q:q + 1], geo.amp, geo.a, geo.c)[0]

    f = ci.fock_tight_binding(geo.x)
    e, c = green.orbitals(f)
    mu = green.midgap_mu(e, n // 2)
    tau_all, w_all = green.tau_grid(BETA, NTAU)
    tau, w = tau_all[TAU_IDX], w_all[TAU_IDX]
    g, gb = green.green_tau(e, c, mu, BETA, tau)
    spl = sp.split_b(b_slice, EPS, naux)
    print(f"split: nnz {spl.nnz}, wmax {spl.wmax}, kmax {spl.kmax:.6e} ({time.time() - t0:.0f} s)", flush=True)

    th = rng.rademacher(SEED, 0, max(PAIRS) + 1, naux)[PAIRS]
    thp = rng.rademacher(SEED, 1, max(PAIRS) + 1, naux)[PAIRS]
    _, xl, xs = sp.r_vectors(b_slice, spl, th)
    _, yl, ys = sp.r_vectors(b_slice, spl, thp)
    print(f"R vectors ({time.time() - t0:.0f} s)", flush=True)

    pos = positions(n)
    nt = len(TAU_IDX)
    e_det = np.zeros(nt)
    det_pos = np.zeros((nt, pos.shape[0]))
    es = np.zeros((len(PAIRS), nt))
    sig_pos = np.zeros((len(PAIRS), nt, pos.shape[0]))
    for t in range(nt):
        det = se.sigma_dd(spl, g[t], gb[t])
        e_det[t] = energy.trace_product(det, gb[t])
        det_pos[t] = det[pos[:, 0], pos[:, 1]]
        for k in range(len(PAIRS)):
            sig = se.sigma_pair(spl, xl[k], xs[k], yl[k], ys[k], g[t], gb[t])
            es[k, t] = energy.trace_product(sig, gb[t])
            sig_pos[k, t] = sig[pos[:, 0], pos[:, 1]]
        print(f"tau {TAU_IDX[t]} done ({time.time() - t0:.0f} s)", flush=True)

    np.savez_compressed(os.path.join(HERE, "n800_subset.npz"), tau_idx=np.array(TAU_IDX), tau=tau, w=w,
                        e_det=e_det, es=es, pos=pos, det_pos=det_pos, sig_pos=sig_pos,
                        nnz=np.array(spl.nnz), wmax=np.array(spl.wmax), kmax=np.array(spl.kmax),
                        pairs=np.array(PAIRS))
    print(f"wrote n800_subset.npz ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
