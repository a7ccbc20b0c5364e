"""Shared seeded problem set-up for parity tests: the same synthetic chain is
handed to the oracle (CPU, FP64) and to the HIP library."""
import numpy as np

import chain_inputs as ci
from oracle import green, integrals, rng, selfenergy as se, split as sp


def chain(n_dimer, beta, ntau, eps):
    geo = ci.chain_geometry(n_dimer)
    f = ci.fock_tight_binding(geo.x)
    return dict(geo=geo, f=f, beta=beta, ntau=ntau, eps=eps, n=geo.n, naux=geo.naux)


def oracle_setup(pb):
    geo = pb["geo"]
    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    e, c = green.orbitals(pb["f"])
    mu = green.midgap_mu(e, geo.n // 2)
    tau, w = green.tau_grid(pb["beta"], pb["ntau"])
    g, gb = green.green_tau(e, c, mu, pb["beta"], tau)
    spl = sp.split_b(b, pb["eps"])
    return dict(b=b, e=e, c=c, mu=mu, tau=tau, w=w, g=g, gb=gb, split=spl)


def oracle_pairs(o, seed, ns, taus, pairs, theta=None, thetap=None):
    """Per-pair Sigma_s(tau) (unsymmetrised) for the listed tau and pair
    indices, and e_s(tau) = Tr(Sigma_s Gb)."""
    b, spl = o["b"], o["split"]
    naux = b.shape[0]
    if theta is None:
        theta = rng.rademacher(seed, 0, max(pairs) + 1, naux)
        thetap = rng.rademacher(seed, 1, max(pairs) + 1, naux)
    sel = np.array(sorted(set(pairs)))
    _, xl, xs = sp.r_vectors(b, spl, theta[sel])
    _, yl, ys = sp.r_vectors(b, spl, thetap[sel])
    pos = {s: i for i, s in enumerate(sel)}
    out = {}
    for t in taus:
        for s in pairs:
            i = pos[s]
            sig = se.sigma_pair(spl, xl[i], xs[i], yl[i], ys[i], o["g"][t], o["gb"][t])
            out[(t, s)] = sig
    return out


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))
