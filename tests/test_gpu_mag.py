"""GPU parity of the maximally Abelian gauge (GF_MAG) against the oracle: per
half-sweep from identical input (the kernel builds M from hand-derived
coefficient vectors, the oracle by polarising R evaluated with full products),
the measurement, and the drivers."""
import math

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


def _check(ctx, U, prec, storage, omega, form, steps=(0, 1, 0)):
    ref = oracle_input(U, prec, storage)
    for par in steps:
        f, g = upload(ctx, ref, prec, storage)
        ctx.sweep_form(f, g, gf.MAG, par, omega, form)
        O.mag_sweep(ref, par, omega, form)
        err = np.abs(download(ctx, f, g) - ref).max()
        assert err <= TOL[prec], (par, err)


# Parity per element needs a well-conditioned local problem: the maximiser is
# the top eigenvector of M, which moves by about |dM| / gap (Davis-Kahan), and
# where the two top eigenvalues (nearly) coincide several maximisers are
# equally valid and rounding decides between them. Near the maximally Abelian
# gauge the gaps are O(1); the inputs below (diagonal phases times exp(i eps H))
# have relative gaps >= 0.73 (eps 0.2) and >= 0.026 (eps 0.4). Rough fields are
# checked for validity instead (test_mag_rough_field_validity).
@pytest.mark.parametrize("eps", [0.2, 0.4])
@pytest.mark.parametrize("form", [0, 3])
@pytest.mark.parametrize("prec,storage", COMBOS)
@pytest.mark.parametrize("dims", [(6, 4, 2, 10), (4, 6, 8, 10)])
def test_mag_half_sweep_parity(ctx, dims, prec, storage, form, eps):
    U = inputs.abelian_noise(dims, 91, eps)
    say("mag half-sweep", dims, prec, storage, form, eps)
    _check(ctx, U, prec, storage, 1.7, form)


@pytest.mark.parametrize("prec,storage", [(gf.FP64, gf.R12), (gf.FP32, gf.R12)])
def test_mag_rough_field_validity(ctx, prec, storage):
    """Haar-scrambled rough field (small eigen-gaps at some sites): each GPU
    half-sweep keeps the links unitary and the plaquette, never lowers F_MAG,
    and agrees with the oracle on the bulk of the links."""
    dims = (4, 6, 8, 10)
    U = inputs.config0(dims, 0.6, 95)
    ref = oracle_input(U, prec, storage)
    f, g = upload(ctx, ref, prec, storage)
    F, P = ctx.empty_out(1), ctx.empty_out(1)
    ctx.functional(f, g, gf.MAG, F)
    ctx.plaquette(f, g, P)
    F0, P0 = F.item(), P.item()
    for par in (0, 1, 0, 1):
        ctx.sweep(f, g, gf.MAG, par, 1.7)
        O.mag_sweep(ref, par, 1.7, 0)
        ctx.functional(f, g, gf.MAG, F)
        assert F.item() >= F0 - (1e-14 if prec == gf.FP64 else 1e-6)
        F0 = F.item()
        got = download(ctx, f, g)
        close = np.abs(got - ref).reshape(-1, 9).max(axis=1) <= TOL[prec]
        say("  rough field: links within the bar %.4f" % close.mean())
        assert close.mean() > 0.9
        ref = got  # continue both from the GPU state
    ctx.plaquette(f, g, P)
    assert P.item() == pytest.approx(P0, abs=1e-13 if prec == gf.FP64 else 1e-5)
    M = download(ctx, f, g).reshape(-1, 3, 3)
    assert np.abs(M @ M.conj().transpose(0, 2, 1) - np.eye(3)).max() < (
        1e-13 if prec == gf.FP64 else 1e-5)


@pytest.mark.parametrize("nt", [0, 1, 2])
@pytest.mark.parametrize("tps", [1, 2, 4])
@pytest.mark.parametrize("prec", [gf.FP64, gf.FP32])
def test_mag_variants(ctx, prec, tps, nt):
    U = inputs.abelian_noise((4, 6, 8, 10), 92, 0.4)
    ctx.set_sweep_variant(prec, gf.R12, tps, nt)
    try:
        _check(ctx, U, prec, gf.R12, 1.0, 0, steps=(0, 1))
        _check(ctx, U, prec, gf.R12, 1.9, 2, steps=(1,))
    finally:
        ctx.set_sweep_variant(prec, gf.R12, 0, -1)


def test_mag_gf_sweep_equals_form_zero(ctx):
    U = inputs.config0((4, 6, 8, 10), 0.6, 93)
    a, g = upload(ctx, U, gf.FP64, gf.R12)
    b, _ = upload(ctx, U, gf.FP64, gf.R12)
    ctx.sweep(a, g, gf.MAG, 1, 1.7)
    ctx.sweep_form(b, g, gf.MAG, 1, 1.7, 0)
    assert np.array_equal(download(ctx, a, g), download(ctx, b, g))


@pytest.mark.parametrize("prec,storage", COMBOS)
def test_mag_measure_parity(ctx, prec, storage):
    dims = (6, 4, 8, 4)
    U = inputs.config0(dims, 0.7, 94)
    f, g = upload(ctx, U, prec, storage)
    ref = oracle_input(U, prec, storage)
    F, th = ctx.empty_out(1), ctx.empty_out(1)
    ctx.measure(f, g, gf.MAG, F, th)
    rtol = 1e-12 if prec == gf.FP64 else 1e-5
    assert F.item() == pytest.approx(O.mag_functional(ref), rel=rtol)
    assert th.item() == pytest.approx(O.mag_theta(ref), rel=rtol)


def test_mag_measure_closed_form(ctx):
    """One link rotated by (cos e, 0, sin e, 0) in subgroup (0, 2) of the unit
    field: F = 1 - 2 sin^2(e)/(12 V), theta = 2 sin^2(2e)/(3 V)."""
    dims = (4, 4, 2, 6)
    V = 4 * 4 * 2 * 6
    e = 0.31
    U = inputs.unit_field(dims)
    G = np.eye(3, dtype=np.complex128)
    G[0, 0], G[0, 2], G[2, 0], G[2, 2] = math.cos(e), math.sin(e), -math.sin(e), math.cos(e)
    U[2, 1, 0, 5, 3] = G
    f, g = upload(ctx, U, gf.FP64, gf.R18)
    F, th = ctx.empty_out(1), ctx.empty_out(1)
    ctx.measure(f, g, gf.MAG, F, th)
    assert F.item() == pytest.approx(1 - 2 * math.sin(e) ** 2 / (12 * V), rel=1e-15)
    assert th.item() == pytest.approx(2 * math.sin(2 * e) ** 2 / (3 * V), rel=1e-13)


def test_mag_fix_matches_oracle(ctx):
    dims = (4, 4, 4, 8)
    U = inputs.abelian_noise(dims, 96, 0.4)
    f, g = upload(ctx, U, gf.FP64, gf.R12)
    p = gf.fix_params(omega=1.7, theta_target=1e-12, max_sweeps=3000, check_every=50,
                      flags=gf.FLAG_GRAPH)
    r = ctx.fix(f, g, gf.MAG, p)
    ro = O.fix_mag(oracle_input(U, gf.FP64, gf.R12), 1.7, 1e-12, 3000, 50, 1)
    say("mag fix: gpu sweeps", r.sweeps, "oracle", ro["sweeps"])
    assert r.status == gf.OK and ro["converged"]
    assert r.sweeps == ro["sweeps"]
    assert r.F == pytest.approx(ro["F"], rel=1e-10)


def test_mag_mixed_tracked(ctx):
    dims = (4, 4, 4, 8)
    U = inputs.abelian_noise(dims, 97, 0.4)
    glo = gf.Geom.make(dims, gf.FP32, gf.R12)
    hi, ghi = upload(ctx, U, gf.FP64, gf.R12)
    lo = ctx.empty_field(glo)
    p = gf.fix_params(omega=1.7, theta_target=1e-13, theta_switch=1e-7, max_sweeps=3000,
                      check_every=50, flags=gf.FLAG_GRAPH)
    P0 = ctx.empty_out(1)
    ctx.plaquette(hi, ghi, P0)
    r = ctx.fix_mixed(lo, glo, hi, ghi, gf.MAG, p)
    ro = O.fix_mag(oracle_input(U, gf.FP64, gf.R12), 1.7, 1e-13, 3000, 50, 1)
    assert r.status == gf.OK and ro["converged"]
    assert r.F == pytest.approx(ro["F"], rel=1e-10)
    P1 = ctx.empty_out(1)
    ctx.plaquette(hi, ghi, P1)
    assert P1.item() == pytest.approx(P0.item(), abs=1e-13)


@pytest.mark.parametrize("seed", [1, 2])
def test_mag_abelian_copy_reaches_maximum(ctx, seed):
    U = inputs.abelian_gauge((4, 4, 4, 4), seed, eps=0.3)
    f, g = upload(ctx, U, gf.FP64, gf.R18)
    r = ctx.fix(f, g, gf.MAG, gf.fix_params(omega=1.7, theta_target=1e-24, max_sweeps=3000,
                                             check_every=20))
    assert r.status == gf.OK
    assert r.F == pytest.approx(1.0, abs=1e-12)


def test_mag_unsupported_paths(ctx):
    U = inputs.config0((4, 4, 4, 4), 0.5, 1)
    f, g = upload(ctx, U, gf.FP64, gf.R12)
    before = download(ctx, f, g)
    calls = [lambda: ctx.heatbath_half(f, g, gf.MAG, 0, 1.0, 1, 0),
             lambda: ctx.micro_half(f, g, gf.MAG, 0),
             lambda: ctx.sweep_sr(f, g, gf.MAG, 0, 1.0, 0.5, 1, 0),
             lambda: ctx.anneal_sweep(f, g, gf.MAG, 1.0, 1, 0, 1),
             lambda: ctx.fix(f, g, gf.MAG, gf.fix_params(sa_steps=10)),
             lambda: ctx.fix(f, g, gf.MAG, gf.fix_params(sr_prob=0.3))]
    for call in calls:
        with pytest.raises(gf.GFError) as e:
            call()
        assert e.value.status == gf.ERR_UNSUPPORTED
    with pytest.raises(gf.GFError):
        ctx.sweep(f, g, 3, 0, 1.7)
    assert np.array_equal(download(ctx, f, g), before)
