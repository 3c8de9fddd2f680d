"""GPU parity of stochastic relaxation (Sec. 1) against the oracle, and of
its driver mode against the sequence of half-sweeps it stands for."""
import numpy as np
import pytest

import inputs
import oracle as O
import paper_1209_4008_amd as gf
from gpu_helpers import TOL, download, oracle_input, say, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gf.Context()
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("prec,storage", [(gf.FP64, gf.R18), (gf.FP64, gf.R12),
                                          (gf.FP32, gf.R12)])
def test_sr_half_sweep_parity(ctx, prec, storage, gauge):
    dims = (4, 6, 4, 8)
    U = inputs.config0(dims, 0.6, 61)
    ref = oracle_input(U, prec, storage)
    for k, (p, omega) in enumerate([(0.3, 1.0), (0.7, 1.5), (0.0, 1.7), (1.0, 1.0)]):
        for par in (0, 1):
            f, g = upload(ctx, ref, prec, storage)
            ctx.sweep_sr(f, g, gauge, par, omega, p, 123, k)
            O.sweep_sr(ref, gauge, par, omega, p, 123, k)
            err = np.abs(download(ctx, f, g) - ref).max()
            assert err <= TOL[prec], (k, par, err)


def test_sr_driver_is_its_sweeps(ctx):
    dims = (8, 8, 8, 8)
    U = inputs.config0(dims, 0.3, 1)
    p = gf.fix_params(omega=1.0, theta_target=1e-12, max_sweeps=3000, check_every=50,
                      sr_prob=0.5, seed=77, flags=gf.FLAG_GRAPH)
    a, g = upload(ctx, U, gf.FP64, gf.R12)
    r = ctx.fix(a, g, gf.LANDAU, p)
    say("stochastic relaxation p=0.5: sweeps", r.sweeps)
    assert r.status == gf.OK and r.theta < 1e-12
    b, _ = upload(ctx, U, gf.FP64, gf.R12)
    for k in range(r.sweeps):
        if k % 50 == 0 and k > 0:
            ctx.reunitarize(b, g)
        for par in (0, 1):
            ctx.sweep_sr(b, g, gf.LANDAU, par, 1.0, 0.5, 77, k)
    if r.sweeps % 50 == 0 and r.sweeps > 0:
        ctx.reunitarize(b, g)
    assert np.array_equal(download(ctx, a, g), download(ctx, b, g))
    # the same gauge is reached as by overrelaxation (F of the FP64 oracle's OR run)
    ro = O.fix(oracle_input(U, gf.FP64, gf.R12), gf.LANDAU, 1.7, 1e-12, 3000, 50, 1)
    assert r.F == pytest.approx(ro["F"], rel=1e-9)


@pytest.mark.parametrize("nt", [0, 1, 2])
@pytest.mark.parametrize("tps", [1, 4])
def test_sr_variants(ctx, tps, nt):
    """Stochastic relaxation in every nontemporal mode and lanes per site."""
    dims = (4, 6, 8, 10)
    U = inputs.config0(dims, 0.6, 62)
    ctx.set_sweep_variant(gf.FP64, gf.R12, tps, nt)
    try:
        ref = oracle_input(U, gf.FP64, gf.R12)
        for par in (0, 1):
            f, g = upload(ctx, ref, gf.FP64, gf.R12)
            ctx.sweep_sr(f, g, gf.LANDAU, par, 1.2, 0.5, 321, 7)
            O.sweep_sr(ref, gf.LANDAU, par, 1.2, 0.5, 321, 7)
            assert np.abs(download(ctx, f, g) - ref).max() <= TOL[gf.FP64]
    finally:
        ctx.set_sweep_variant(gf.FP64, gf.R12, 0, -1)
