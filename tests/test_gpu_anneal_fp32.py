"""The FP32 annealing updates -- the path the mixed-precision driver, the
Coulomb workload and the batch run (Sec. 1: annealing as a preconditioner) --
against the FP64 oracle, per element, to the FP32 bar of 2e-5, from identical
input (the generator's field rounded to FP32 on both sides).

Microcanonical half-sweeps draw nothing: every element within 2e-5.

Heatbath half-sweeps draw the same Philox numbers as the oracle. The FP32
sampler can decide a Kennedy-Pendleton trial differently from the FP64 one
only where the trial's accept margin |(1 - lambda^2) - u4^2| lies within its
rounding of 0. For every site whose links differ from the oracle's by more
than 2e-5 the oracle enumerates each outcome that deciding such borderline
trials (margin < TAU) the other way gives; the GPU's 8 links must match one of
those outcomes to 2e-5. A site with no borderline trial has one outcome, the
exact one, so it is held to 2e-5 outright; the number of borderline sites is
reported and bounded.

The tracked kernels (the site transformations accumulated into the
gauge-transformation field, as in the mixed driver's FP32 phase) are held to
the same bar for the field and for g.
"""
import numpy as np
import pytest

import inputs
import oracle as O
import paper_1209_4008_amd as gf
from gpu_helpers import (download, heatbath_sites_check, oracle_input, say, site_errors,
                         upload)

pytestmark = pytest.mark.gpu

BAR = 2e-5
TAU = 1e-5
DIMS = (6, 4, 6, 10)  # 720 sites per parity: one ragged 2048-site tile
# 5120 sites per parity: two tiles and a ragged third
DIMS_TILES = (8, 8, 10, 16)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gf.Context()
    yield c
    torch.cuda.synchronize()
    c.close()


def check_heatbath(dims, U_in, got, ref, gauge, parity, T, seed, sweep, what):
    """every site of `parity` checked; returns (borderline sites, sites)"""
    sites, _ = site_errors(dims, got, ref, parity)
    border = heatbath_sites_check(dims, U_in, got, ref, gauge, T, seed, sweep, sites, BAR, TAU,
                                  what)
    return border, sites.size


VARIANTS = [(tps, nt) for tps in (1, 2, 4) for nt in (0, 1, 2)]


@pytest.mark.parametrize("tps,nt", VARIANTS)
@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("storage", [gf.R12, gf.R18])
def test_fp32_micro_half_per_element(ctx, storage, gauge, tps, nt):
    U = inputs.config0(DIMS, 0.5, 61)
    ref0 = oracle_input(U, gf.FP32, storage)
    ctx.set_anneal_variant(gf.FP32, storage, tps, nt)
    try:
        for parity in (0, 1):
            f, g = upload(ctx, U, gf.FP32, storage)
            ctx.micro_half(f, g, gauge, parity)
            got = download(ctx, f, g)
            ref = ref0.copy()
            O.micro_half(ref, gauge, parity)
            err = np.abs(got - ref).max()
            assert err <= BAR, (parity, err)
    finally:
        ctx.set_anneal_variant(gf.FP32, storage, 0, -1)


@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("storage", [gf.R12, gf.R18])
def test_fp32_micro_half_several_tiles(ctx, storage, gauge):
    """the built-in variant on a lattice of several tiles and a ragged one"""
    U = inputs.config0(DIMS_TILES, 0.5, 67)
    ref0 = oracle_input(U, gf.FP32, storage)
    for parity in (0, 1):
        f, g = upload(ctx, U, gf.FP32, storage)
        ctx.micro_half(f, g, gauge, parity)
        got = download(ctx, f, g)
        ref = ref0.copy()
        O.micro_half(ref, gauge, parity)
        err = np.abs(got - ref).max()
        assert err <= BAR, (parity, err)


@pytest.mark.parametrize("tps,nt", VARIANTS)
@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("storage", [gf.R12, gf.R18])
def test_fp32_heatbath_half_per_element(ctx, storage, gauge, tps, nt):
    U = inputs.config0(DIMS, 0.5, 62)
    ref0 = oracle_input(U, gf.FP32, storage)
    ctx.set_anneal_variant(gf.FP32, storage, tps, nt)
    border = total = 0
    try:
        for k, T in enumerate([1.45, 0.5, 0.05, 0.01]):
            for parity in (0, 1):
                f, g = upload(ctx, U, gf.FP32, storage)
                ctx.heatbath_half(f, g, gauge, parity, T, 901, k)
                got = download(ctx, f, g)
                ref = ref0.copy()
                assert O.heatbath_half(ref, gauge, parity, T, 901, k) == 0
                nb, ns = check_heatbath(DIMS, ref0, got, ref, gauge, parity, T, 901, k,
                                        f"hb T={T} p={parity}")
                border += nb
                total += ns
    finally:
        ctx.set_anneal_variant(gf.FP32, storage, 0, -1)
    assert border <= max(2, total // 500), (border, total)


def gauge_field(ctx, geom, G):
    import torch
    out = torch.empty(geom.volume * 18, dtype=torch.float64, device="cuda")
    ctx.gauge_unpack(geom, G, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.complex128).reshape(tuple(geom.dims) + (3, 3)).copy()


@pytest.mark.parametrize("tps", [1, 2, 4])
@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("storage", [gf.R12, gf.R18])
def test_fp32_tracked_micro_and_overrelaxation(ctx, storage, gauge, tps):
    """A tracked microcanonical half-sweep (RED) and a tracked overrelaxation
    half-sweep (BLACK), each from the input and g = 1: the field against the
    oracle's half-sweep and g against the oracle's site transformations."""
    U = inputs.config0(DIMS, 0.5, 63)
    ref0 = oracle_input(U, gf.FP32, storage)
    ctx.set_sweep_variant(gf.FP32, storage, tps, 0)
    ctx.set_anneal_variant(gf.FP32, storage, tps, 0)
    try:
        for kind, parity in ((O.MICRO, 0), (O.OR, 1)):
            f, geom = upload(ctx, U, gf.FP32, storage)
            G = ctx.empty_gauge(geom)
            ctx.gauge_unit(geom, G)
            if kind == O.MICRO:
                ctx.micro_half_tracked(f, G, geom, gauge, parity)
            else:
                ctx.sweep_tracked(f, G, geom, gauge, parity, 1.7)
            ref = ref0.copy()
            gref = O.half_sweep_g(ref, gauge, parity, kind, omega=1.7)
            errU = np.abs(download(ctx, f, geom) - ref).max()
            errg = np.abs(gauge_field(ctx, geom, G) - gref).max()
            say("tracked", "micro" if kind == O.MICRO else "OR", storage, gauge, tps,
                f"field {errU:.2e} g {errg:.2e}")
            assert errU <= BAR and errg <= BAR, (kind, errU, errg)
    finally:
        ctx.set_sweep_variant(gf.FP32, storage, 0, -1)
        ctx.set_anneal_variant(gf.FP32, storage, 0, -1)


@pytest.mark.parametrize("tps", [1, 2, 4])
@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("storage", [gf.R12, gf.R18])
def test_fp32_tracked_heatbath(ctx, storage, gauge, tps):
    """Tracked heatbath half-sweep from g = 1: the field as in the untracked
    check; g equal to the oracle's site transformation at every site whose
    draws were decided as in FP64, and at every site the field equal to the
    input transformed by the GPU's own g (eq. (4))."""
    U = inputs.config0(DIMS, 0.5, 64)
    ref0 = oracle_input(U, gf.FP32, storage)
    ctx.set_anneal_variant(gf.FP32, storage, tps, 0)
    try:
        for parity, T in ((0, 1.2), (1, 0.02)):
            f, geom = upload(ctx, U, gf.FP32, storage)
            G = ctx.empty_gauge(geom)
            ctx.gauge_unit(geom, G)
            ctx.heatbath_half_tracked(f, G, geom, gauge, parity, T, 77, 3)
            got = download(ctx, f, geom)
            ggpu = gauge_field(ctx, geom, G)
            ref = ref0.copy()
            gref = O.half_sweep_g(ref, gauge, parity, O.HEATBATH, param=T, seed=77, sweep=3)
            check_heatbath(DIMS, ref0, got, ref, gauge, parity, T, 77, 3, f"tracked hb T={T}")
            sites, err = site_errors(DIMS, got, ref, parity)
            exact = sites[err <= BAR]
            gd = np.abs(ggpu.reshape(-1, 3, 3)[exact] - gref.reshape(-1, 3, 3)[exact]).max()
            assert gd <= BAR, gd
            W = ref0.copy()
            O.gauge_transform(W, ggpu)
            assert np.abs(W - got).max() <= BAR
    finally:
        ctx.set_anneal_variant(gf.FP32, storage, 0, -1)


def test_fp32_heatbath_larger_lattice_borderline_rate(ctx):
    """8x8x10x16 (several tiles and a ragged one) at the temperatures of the
    annealing schedules, built-in variant: the per-site check and the rate of
    borderline sites."""
    dims = DIMS_TILES
    U = inputs.config0(dims, 0.4, 65)
    ref0 = oracle_input(U, gf.FP32, gf.R12)
    border = total = 0
    for k, T in enumerate([1.45, 1.0, 0.3, 0.1, 0.01]):
        for parity in (0, 1):
            f, g = upload(ctx, U, gf.FP32, gf.R12)
            ctx.heatbath_half(f, g, gf.COULOMB, parity, T, 5, k)
            got = download(ctx, f, g)
            ref = ref0.copy()
            O.heatbath_half(ref, gf.COULOMB, parity, T, 5, k)
            nb, ns = check_heatbath(dims, ref0, got, ref, gf.COULOMB, parity, T, 5, k,
                                    f"8x8x10x16 T={T} p={parity}")
            border += nb
            total += ns
    say("borderline sites", border, "of", total)
    assert border <= max(2, total // 1000), (border, total)


@pytest.mark.parametrize("tps", [1, 2, 4])
@pytest.mark.parametrize("storage", [gf.R12, gf.R18])
def test_fp32_tracked_accumulates_onto_g(ctx, storage, tps):
    """g(x) <- Gtot g(x) onto a g that is not 1: G starts as a Haar-random
    field from the generator (rounded to FP32 rows), one tracked half-sweep of
    each kind; g after = the oracle's site transformation times g before."""
    import torch
    U = inputs.config0(DIMS, 0.5, 66)
    h = inputs.haar_sites(DIMS, 91)
    ref0 = oracle_input(U, gf.FP32, storage)
    # what the FP32 rows of h hold, with row 2 rebuilt (the kernels' g)
    h32 = h.astype(np.complex64).astype(np.complex128)
    h32[..., 2, :] = np.conj(np.cross(h32[..., 0, :], h32[..., 1, :]))
    hc = torch.from_numpy(np.ascontiguousarray(h).view(np.float64).reshape(-1).copy()).to("cuda")
    ctx.set_sweep_variant(gf.FP32, storage, tps, 0)
    ctx.set_anneal_variant(gf.FP32, storage, tps, 0)
    try:
        for kind, parity in ((O.MICRO, 1), (O.OR, 0), (O.HEATBATH, 1)):
            f, geom = upload(ctx, U, gf.FP32, storage)
            G = ctx.empty_gauge(geom)
            ctx.gauge_pack(geom, hc, G)
            if kind == O.MICRO:
                ctx.micro_half_tracked(f, G, geom, gf.COULOMB, parity)
            elif kind == O.OR:
                ctx.sweep_tracked(f, G, geom, gf.COULOMB, parity, 1.7)
            else:
                ctx.heatbath_half_tracked(f, G, geom, gf.COULOMB, parity, 0.05, 3, 9)
            ref = ref0.copy()
            gh = O.half_sweep_g(ref, gf.COULOMB, parity, kind, omega=1.7, param=0.05, seed=3,
                                sweep=9)
            got_g = gauge_field(ctx, geom, G)
            want = gh @ h32
            if kind == O.HEATBATH:
                sites, err = site_errors(DIMS, download(ctx, f, geom), ref, parity)
                sel = np.ones(int(np.prod(DIMS)), dtype=bool)
                sel[sites[err > BAR]] = False  # borderline sites are checked elsewhere
                errg = np.abs(got_g.reshape(-1, 3, 3)[sel] - want.reshape(-1, 3, 3)[sel]).max()
            else:
                errg = np.abs(got_g - want).max()
            say("tracked accumulation", kind, storage, tps, f"g {errg:.2e}")
            assert errg <= BAR, (kind, errg)
    finally:
        ctx.set_sweep_variant(gf.FP32, storage, 0, -1)
        ctx.set_anneal_variant(gf.FP32, storage, 0, -1)
