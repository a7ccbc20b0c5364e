"""Statistical pins of the oracle's estimator (Results section claims):
unbiased against deterministic RI, error falling as 1/sqrt(N_s), and a much
smaller error for RS-SRI than for SRI at equal N_s."""
import numpy as np
import pytest

import chain_inputs as ci
from oracle import energy, green, integrals, rng, selfenergy as se, split as sp


def _setup(n_dimer=10, beta=50.0, ntau=8, eps=1e-2):
    geo = ci.chain_geometry(n_dimer)
    b = integrals.synthetic_b(geo.x, geo.xq, geo.amp, geo.a, geo.c)
    f = ci.fock_tight_binding(geo.x)
    e, c = green.orbitals(f)
    mu = green.midgap_mu(e, geo.n // 2)
    tau, w = green.tau_grid(beta, ntau)
    g, gb = green.green_tau(e, c, mu, beta, tau)
    return geo, b, g, gb, w, sp.split_b(b, eps)


def _pair_energies(b, spl, g, gb, w, seed, ns, s0=0):
    th = rng.rademacher(seed, 0, ns, b.shape[0], s0)
    thp = rng.rademacher(seed, 1, ns, b.shape[0], s0)
    _, xl, xs = sp.r_vectors(b, spl, th)
    _, yl, ys = sp.r_vectors(b, spl, thp)
    es = np.zeros((ns, len(w)))
    for s in range(ns):
        for t in range(len(w)):
            sig = se.sigma_pair(spl, xl[s], xs[s], yl[s], ys[s], g[t], gb[t])
            es[s, t] = energy.trace_product(sig, gb[t])
    return energy.sample_energies(np.zeros(len(w)), es, w)


@pytest.fixture(scope="module")
def tiny():
    geo, b, g, gb, w, spl = _setup()
    e_ri = -energy.GM_FACTOR * sum(w[t] * energy.trace_product(se.sigma_ri(b, g[t], gb[t]), gb[t])
                                   for t in range(len(w)))
    e_dd = -energy.GM_FACTOR * sum(w[t] * energy.trace_product(se.sigma_dd(spl, g[t], gb[t]), gb[t])
                                   for t in range(len(w)))
    es = _pair_energies(b, spl, g, gb, w, seed=0, ns=256)
    return dict(b=b, g=g, gb=gb, w=w, spl=spl, e_ri=e_ri, e_dd=e_dd, es=es)


def test_estimator_unbiased_against_deterministic_ri(tiny):
    m, se_ = energy.mean_stderr(tiny["es"])
    target = tiny["e_ri"] - tiny["e_dd"]
    assert abs(m - target) < 4.0 * se_
    # the deterministic block dominates, the stochastic remainder is small
    assert abs(target) < 0.2 * abs(tiny["e_ri"])


def test_error_falls_as_inverse_sqrt_ns(tiny):
    es = tiny["es"]
    # stderr of means of blocks of 16 vs blocks of 64 pairs
    b16 = es.reshape(16, 16).mean(axis=1)
    b64 = es.reshape(4, 64).mean(axis=1)
    sig = np.std(es, ddof=1)
    assert abs(np.std(b16, ddof=1) / (sig / 4.0) - 1.0) < 0.5
    assert np.std(b64, ddof=1) < np.std(b16, ddof=1)


def test_rs_sri_error_much_smaller_than_sri(tiny):
    spl_sri = sp.split_b(tiny["b"], 1.5)             # empty large part: pure SRI
    es_sri = _pair_energies(tiny["b"], spl_sri, tiny["g"], tiny["gb"], tiny["w"], seed=3, ns=32)
    ratio = np.std(es_sri, ddof=1) / np.std(tiny["es"], ddof=1)
    assert ratio > 10.0
