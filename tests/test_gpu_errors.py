"""Error paths of the C ABI, forced from the host, and two contexts driven
from two host threads.

Every condition here is produced by the arguments the host passes (a
non-finite value in an input, an allocation request no device can meet), so
every kernel still runs to completion normally."""
import threading

import numpy as np
import pytest

from oracle import green

from _problems import chain

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gf2mod():
    from paper_2005_12338_amd import gf2
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return gf2


def _inputs(ctx, n_dimer=5, ntau=4, eps=1e-2):
    pb = chain(n_dimer, 50.0, ntau, eps)
    geo = pb["geo"]
    B = ctx.build_B(geo.n, geo.naux, geom=geo, dtype=torch.float64)
    tau, w = green.tau_grid(pb["beta"], ntau)
    G, Gb, _ = ctx.green_tau(pb["f"], tau, pb["beta"], n_occ=geo.n // 2)
    return geo, B, G, Gb, w, eps


def _energy(ctx, seed=0, ns=4):
    geo, B, G, Gb, w, eps = _inputs(ctx)
    spl = ctx.split(B, eps)
    Sigma, es = ctx.sigma_tau(spl, B, G, Gb, ns=ns, seed=seed, prec="fp64")
    e = ctx.energy(Sigma, Gb, w, geo.n, es)
    spl.free()
    return e, Sigma.cpu().numpy()


def test_nan_in_g_is_a_numeric_error_and_the_context_survives(gf2mod):
    ctx = gf2mod.Context(0)
    geo, B, G, Gb, w, eps = _inputs(ctx)
    spl = ctx.split(B, eps)
    Gbad = G.clone()
    Gbad[1, 2, 3] = float("nan")
    with pytest.raises(gf2mod.Gf2Error) as ex:
        ctx.sigma_tau(spl, B, Gbad, Gb, ns=4, seed=0, prec="fp64")
    assert ex.value.code == gf2mod.GF2_E_NUMERIC
    Sigma, es = ctx.sigma_tau(spl, B, G, Gb, ns=4, seed=0, prec="fp64")   # a clean call still works
    assert torch.isfinite(Sigma).all()
    spl.free()
    ctx.close()


def test_nan_in_sigma_is_a_numeric_error_of_the_energy(gf2mod):
    ctx = gf2mod.Context(0)
    geo, B, G, Gb, w, eps = _inputs(ctx)
    Sigma = torch.zeros_like(G)
    Sigma[0, 0, 0] = float("inf")
    with pytest.raises(gf2mod.Gf2Error) as ex:
        ctx.energy(Sigma, Gb, w, geo.n)
    assert ex.value.code == gf2mod.GF2_E_NUMERIC
    ctx.close()


def test_oversized_scratch_request_is_nomem_and_the_context_survives(gf2mod):
    ctx = gf2mod.Context(0)
    import ctypes as C
    out = np.zeros(4, dtype=np.uint64)
    # 2^52 words (32 PiB): the device buffer is requested before anything is
    # launched or copied, and no device can provide it
    st = ctx.lib.gf2_rng_words(ctx.h, 0, 0, 0, 0, 1 << 52, out.ctypes.data_as(C.POINTER(C.c_uint64)))
    assert st == gf2mod.GF2_E_NOMEM
    assert b"allocation" in ctx.lib.gf2_last_error(ctx.h)
    from oracle import rng
    got = ctx.rng_words(7, 1, 3, 0, 64)              # the next call is unaffected
    assert np.array_equal(got, rng.words(7, 1, 3, np.arange(64, dtype=np.uint64)))
    e, _ = _energy(ctx)
    assert np.isfinite(e[0])
    ctx.close()


def test_argument_errors(gf2mod):
    ctx = gf2mod.Context(0)
    geo, B, G, Gb, w, eps = _inputs(ctx)
    spl = ctx.split(B, eps)
    with pytest.raises(gf2mod.Gf2Error) as ex:
        ctx.sigma_tau(spl, B, G, Gb, ns=0, seed=0, prec="fp64")
    assert ex.value.code == gf2mod.GF2_E_ARG
    with pytest.raises(gf2mod.Gf2Error) as ex:
        ctx.energy_adaptive(spl, B, G, Gb, w, torch.zeros_like(G), geo.n, 1e-3, batch=8, max_pairs=1)
    assert ex.value.code == gf2mod.GF2_E_ARG
    other = gf2mod.Context(0)
    with pytest.raises(gf2mod.Gf2Error) as ex:       # a split handle of another context
        other.sigma_tau(spl, B, G, Gb, ns=4, seed=0, prec="fp64")
    assert ex.value.code == gf2mod.GF2_E_STATE
    other.close()
    spl.free()
    ctx.close()


def test_two_contexts_on_two_threads(gf2mod):
    """Each thread owns a context and runs the whole path three times; every
    result equals the single-threaded one bitwise (FP64 path, fixed order)."""
    ref_ctx = gf2mod.Context(0)
    ref = {seed: _energy(ref_ctx, seed) for seed in (1, 2)}
    ref_ctx.close()
    torch.cuda.synchronize()
    errors, results = [], {}

    def work(seed):
        try:
            c = gf2mod.Context(0, stream=torch.cuda.Stream())
            out = []
            for _ in range(3):
                with torch.cuda.stream(c.stream):
                    out.append(_energy(c, seed))
                c.stream.synchronize()
            c.close()
            results[seed] = out
        except Exception as exc:      # reported on the main thread
            errors.append(exc)

    th = [threading.Thread(target=work, args=(s,)) for s in (1, 2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not errors, errors
    for seed in (1, 2):
        for e, sig in results[seed]:
            assert e == ref[seed][0]
            assert np.array_equal(sig, ref[seed][1])
