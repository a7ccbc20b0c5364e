"""Parity of the estimator variants (control-variate form, double average)
with the oracle (oracle/variants.py) on the same seeded theta.

Bars as for the main path: FP64 1e-10 relative, FP32 1e-5."""
import numpy as np
import pytest

from oracle import energy, green, rng, selfenergy as se, split as sp, variants as va

from _problems import chain, oracle_setup, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2005_12338_amd import gf2
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gf2.Context(0)
    yield c
    c.close()


def _gpu(ctx, pb, dtype):
    geo = pb["geo"]
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=dtype)
    tau, w = green.tau_grid(pb["beta"], pb["ntau"])
    G, Gb, _ = ctx.green_tau(pb["f"], tau, pb["beta"], n_occ=geo.n // 2)
    spl = ctx.split(B, pb["eps"])
    return B, G, Gb, spl, w


@pytest.mark.parametrize("n_dimer,prec,tol", [(5, "fp64", 1e-10), (75, "fp32", 1e-5)])
def test_control_variate_form_matches_oracle(ctx, n_dimer, prec, tol):
    pb = chain(n_dimer, 50.0, 3, 1e-2)
    o = oracle_setup(pb)
    ns, seed = 3, 7
    B, G, Gb, spl, w = _gpu(ctx, pb, torch.float64 if prec == "fp64" else torch.float32)
    acc = torch.zeros_like(G)
    es = torch.zeros((ns, pb["ntau"]), dtype=torch.float64, device="cuda")
    ctx.sigma_stoch_cv(spl, B, G, Gb, acc, ns=ns, seed=seed, prec=prec, e_samples=es)
    naux = o["b"].shape[0]
    rt, rl, _ = sp.r_vectors(o["b"], o["split"], rng.rademacher(seed, 0, ns, naux))
    yt, yl, _ = sp.r_vectors(o["b"], o["split"], rng.rademacher(seed, 1, ns, naux))
    ref = np.zeros((pb["ntau"], pb["n"], pb["n"]))
    big = np.zeros_like(ref)
    es_ref = np.zeros((ns, pb["ntau"]))
    es_big = np.zeros((ns, pb["ntau"]))
    for t in range(pb["ntau"]):
        for s in range(ns):
            sig = va.sigma_pair_cv(rt[s], rl[s], yt[s], yl[s], o["g"][t], o["gb"][t])
            full = va.chain(rt[s], yt[s], o["g"][t], o["gb"][t])
            ref[t] += sig
            big[t] += full
            es_ref[s, t] = energy.trace_product(sig, o["gb"][t])
            es_big[s, t] = energy.trace_product(full, o["gb"][t])
    # the form is a difference of two chains that nearly cancel: the bar is
    # relative to the chains themselves (each computed in the path's precision)
    got, eg = acc.cpu().numpy(), es.cpu().numpy()
    print(f"{prec}: |dSigma| / max|Sigma_s| {rel(got, ref):.2e}, / max|chain| "
          f"{np.abs(got - ref).max() / np.abs(big).max():.2e}")
    assert np.abs(got - ref).max() < tol * np.abs(big).max()
    assert np.abs(eg - es_ref).max() < tol * np.abs(es_big).max()
    spl.free()


def test_double_average_matches_oracle(ctx):
    pb = chain(5, 50.0, 3, 1e-2)
    o = oracle_setup(pb)
    ns, seed = 3, 11
    B, G, Gb, spl, w = _gpu(ctx, pb, torch.float64)
    acc = torch.zeros_like(G)
    es = torch.zeros((ns * ns, pb["ntau"]), dtype=torch.float64, device="cuda")
    ctx.sigma_stoch_double(spl, B, G, Gb, acc, ns=ns, seed=seed, prec="fp64", e_samples=es)
    det = ctx.sigma_det(spl, G, Gb)
    Sigma = ctx.sigma_finalize(det, acc, ns * ns)
    e, _, s_err = ctx.energy_double(Sigma, Gb, w, pb["n"], es, ns)
    naux = o["b"].shape[0]
    _, xl, xs = sp.r_vectors(o["b"], o["split"], rng.rademacher(seed, 0, ns, naux))
    _, yl, ys = sp.r_vectors(o["b"], o["split"], rng.rademacher(seed, 1, ns, naux))
    sig_ref = np.zeros((pb["ntau"], pb["n"], pb["n"]))
    es_ref = np.zeros((ns * ns, pb["ntau"]))
    for t in range(pb["ntau"]):
        mean, per = va.sigma_double(o["split"], xl, xs, yl, ys, o["g"][t], o["gb"][t])
        dd = se.sigma_dd(o["split"], o["g"][t], o["gb"][t])
        sig_ref[t] = dd + 0.5 * (mean + mean.T)
        for i in range(ns):
            for j in range(ns):
                es_ref[i * ns + j, t] = energy.trace_product(per[i][j], o["gb"][t])
    assert rel(es.cpu().numpy(), es_ref) < 1e-10
    assert rel(Sigma.cpu().numpy(), sig_ref) < 1e-10
    e_ref = energy.energy_total(sig_ref, o["gb"], w)
    e_det = np.array([energy.trace_product(se.sigma_dd(o["split"], o["g"][t], o["gb"][t]), o["gb"][t])
                      for t in range(pb["ntau"])])
    tot = energy.sample_energies(e_det, es_ref, w).reshape(ns, ns)
    m_ref, s_ref = va.double_mean_stderr(tot)
    assert abs(e - e_ref) < 1e-10 * abs(e_ref)
    assert abs(m_ref - e_ref) < 1e-10 * abs(e_ref)
    assert abs(s_err - s_ref) < 1e-10 * s_ref
    spl.free()
