"""gf2_energy_noalloc (the entry point that allocates nothing) against
gf2_energy on the same device inputs: two calls in a row, the second with a
smaller problem, each equal to the allocating call (same kernels, same
order of summation: bitwise)."""
import numpy as np
import pytest

from oracle import green

from _problems import chain

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


def _run(ctx, n_dimer, ntau, ns):
    pb = chain(n_dimer, 50.0, ntau, 1e-2)
    geo = pb["geo"]
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float64)
    tau, w = green.tau_grid(pb["beta"], ntau)
    G, Gb, _ = ctx.green_tau(pb["f"], tau, pb["beta"], n_occ=geo.n // 2)
    spl = ctx.split(B, pb["eps"])
    Sigma, es = ctx.sigma_tau(spl, B, G, Gb, ns=ns, seed=3, prec="fp64")
    spl.free()
    return geo, Sigma, Gb, w, es


@pytest.mark.parametrize("with_samples", [True, False])
def test_noalloc_energy_equals_energy_on_two_calls(ctx, with_samples):
    for n_dimer, ntau, ns in ((10, 16, 8), (4, 6, 4)):      # the second call is smaller
        geo, Sigma, Gb, w, es = _run(ctx, n_dimer, ntau, ns)
        es_arg = es if with_samples else None
        e, epe, se = ctx.energy(Sigma, Gb, w, geo.n, es_arg)
        wd = torch.tensor(w, dtype=torch.float64, device="cuda")
        out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.energy_noalloc(Sigma, Gb, wd, geo.n, out, es_arg)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert got[0] == e and got[1] == epe and got[2] == se, (got, (e, epe, se))
        assert np.isfinite(got).all() and e < 0


def test_noalloc_energy_rejects_more_tau_than_its_scratch(ctx):
    from paper_2005_12338_amd import gf2
    n, ntau = 4, 513
    Sigma = torch.zeros((ntau, n, n), dtype=torch.float64, device="cuda")
    wd = torch.zeros(ntau, dtype=torch.float64, device="cuda")
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(gf2.Gf2Error) as ex:
        ctx.energy_noalloc(Sigma, Sigma, wd, 4.0, out)
    assert ex.value.code == gf2.GF2_E_ARG and "512" in str(ex.value)
