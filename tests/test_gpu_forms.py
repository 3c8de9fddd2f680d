"""GPU parity of the other forms of g^omega (Sec. 2: the power taken to first
or second order, and the exact power) against the oracle, per half-sweep and
through the drivers."""
import numpy as np
import pytest

import inputs
import oracle as O
import paper_1209_4008_amd as gf
from gpu_helpers import TOL, download, oracle_input, say, upload

pytestmark = pytest.mark.gpu

COMBOS = [(gf.FP64, gf.R18), (gf.FP64, gf.R12), (gf.FP32, gf.R18), (gf.FP32, gf.R12)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gf.Context()
    yield c
    torch.cuda.synchronize()
    c.close()


def _check(ctx, U, prec, storage, gauge, omega, form):
    ref = oracle_input(U, prec, storage)
    for par in (0, 1, 0):
        f, g = upload(ctx, ref, prec, storage)
        ctx.sweep_form(f, g, gauge, par, omega, form)
        O.sweep_form(ref, gauge, par, omega, form)
        err = np.abs(download(ctx, f, g) - ref).max()
        assert err <= TOL[prec], (par, err)


@pytest.mark.parametrize("form", [1, 2, 3])
@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("prec,storage", COMBOS)
@pytest.mark.parametrize("dims", [(6, 4, 2, 10), (4, 6, 8, 10)])
def test_form_half_sweep_parity(ctx, dims, prec, storage, gauge, form):
    U = inputs.config0(dims, 0.6, 71)
    say("form half-sweep", form, dims, prec, storage, gauge)
    _check(ctx, U, prec, storage, gauge, 1.7, form)


@pytest.mark.parametrize("nt", [0, 1, 2])
@pytest.mark.parametrize("tps", [1, 2, 4])
@pytest.mark.parametrize("prec", [gf.FP64, gf.FP32])
def test_form_variants(ctx, prec, tps, nt):
    """Every lanes-per-site / nontemporal variant with the exact power, and
    omega near 2 where the forms differ most."""
    U = inputs.config0((4, 6, 8, 10), 0.8, 72)
    ctx.set_sweep_variant(prec, gf.R12, tps, nt)
    try:
        for form in (1, 2, 3):
            _check(ctx, U, prec, gf.R12, gf.LANDAU, 1.95, form)
    finally:
        ctx.set_sweep_variant(prec, gf.R12, 0, -1)


def test_form_zero_is_gf_sweep(ctx):
    U = inputs.config0((4, 6, 8, 10), 0.6, 73)
    a, g = upload(ctx, U, gf.FP64, gf.R12)
    b, _ = upload(ctx, U, gf.FP64, gf.R12)
    ctx.sweep_form(a, g, gf.LANDAU, 0, 1.7, 0)
    ctx.sweep(b, g, gf.LANDAU, 0, 1.7)
    assert np.array_equal(download(ctx, a, g), download(ctx, b, g))


@pytest.mark.parametrize("form", [1, 2, 3])
def test_form_fix_matches_oracle(ctx, form):
    """gf_fix with or_form: same sweep count and F as the oracle's driver with
    the same form (config 0, FP64 12 reals, theta < 1e-12)."""
    dims = (8, 8, 8, 8)
    U = inputs.config0(dims, 0.3, 1)
    f, g = upload(ctx, U, gf.FP64, gf.R12)
    p = gf.fix_params(omega=1.7, theta_target=1e-12, max_sweeps=2000, check_every=100,
                      or_form=form, flags=gf.FLAG_GRAPH)
    r = ctx.fix(f, g, gf.LANDAU, p)
    ro = O.fix(oracle_input(U, gf.FP64, gf.R12), gf.LANDAU, 1.7, 1e-12, 2000, 100, 1, form=form)
    say("form", form, "sweeps gpu", r.sweeps, "oracle", ro["sweeps"])
    assert r.status == gf.OK and ro["converged"]
    assert r.sweeps == ro["sweeps"]
    assert r.F == pytest.approx(ro["F"], rel=1e-10)


@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
def test_form_mixed_tracked(ctx, gauge):
    """Mixed precision with or_form = 2 and g tracked: final F within 1e-10 of
    the FP64 oracle's fix with the same form."""
    dims = (8, 8, 8, 8)
    U = inputs.config0(dims, 0.3, 1)
    glo = gf.Geom.make(dims, gf.FP32, gf.R12)
    hi, ghi = upload(ctx, U, gf.FP64, gf.R12)
    lo = ctx.empty_field(glo)
    p = gf.fix_params(omega=1.7, theta_target=1e-13, theta_switch=1e-6, max_sweeps=4000,
                      check_every=100, or_form=2, flags=gf.FLAG_GRAPH)
    r = ctx.fix_mixed(lo, glo, hi, ghi, gauge, p)
    ro = O.fix(oracle_input(U, gf.FP64, gf.R12), gauge, 1.7, 1e-13, 4000, 100, 1, form=2)
    assert r.status == gf.OK and ro["converged"]
    assert r.F == pytest.approx(ro["F"], rel=1e-10)


def test_form_errors(ctx):
    U = inputs.config0((4, 4, 4, 4), 0.5, 1)
    f, g = upload(ctx, U, gf.FP64, gf.R12)
    before = download(ctx, f, g)
    for form in (-1, 4):
        with pytest.raises(gf.GFError) as e:
            ctx.sweep_form(f, g, gf.LANDAU, 0, 1.7, form)
        assert e.value.status == gf.ERR_ARG
    with pytest.raises(gf.GFError) as e:
        ctx.fix(f, g, gf.LANDAU, gf.fix_params(or_form=2, sr_prob=0.5))
    assert e.value.status == gf.ERR_UNSUPPORTED
    with pytest.raises(gf.GFError) as e:
        ctx.fix(f, g, gf.LANDAU, gf.fix_params(or_form=7))
    assert e.value.status == gf.ERR_ARG
    b = gf.Batch(ctx, [g], [f])
    try:
        with pytest.raises(gf.GFError) as e:
            b.run(gf.fix_params(or_form=1))
        assert e.value.status == gf.ERR_UNSUPPORTED
    finally:
        b.close()
    # rejected calls leave the field untouched
    assert np.array_equal(download(ctx, f, g), before)
