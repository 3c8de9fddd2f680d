"""GPU parity of the drivers and of simulated annealing, plus sampled parity
at the full benchmark sizes."""
import numpy as np
import pytest

import inputs
import oracle as O
import paper_1209_4008_amd as gf
from gpu_helpers import (TOL, download, host_canon, oracle_input, say, site_parity, sites_links,
                         upload)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gf.Context()
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("storage", [gf.R18, gf.R12])
def test_fix_config0_matches_oracle(ctx, storage):
    """8^4, FP64, omega = 1.7, theta < 1e-12, max 2000 sweeps, check every 100."""
    U = inputs.config0((8, 8, 8, 8), 0.3, 1)
    say("fix config0 FP64", storage)
    f, g = upload(ctx, U, gf.FP64, storage)
    p = gf.fix_params(omega=1.7, theta_target=1e-12, max_sweeps=2000, check_every=100)
    r = ctx.fix(f, g, gf.LANDAU, p)
    ref = oracle_input(U, gf.FP64, storage)
    ro = O.fix(ref, gf.LANDAU, 1.7, 1e-12, 2000, 100, 1)
    assert r.status == gf.OK and ro["converged"]
    assert r.sweeps == ro["sweeps"]
    assert r.F == pytest.approx(ro["F"], rel=1e-10)
    assert r.theta < 1e-12
    assert np.abs(download(ctx, f, g) - ref).max() < 1e-9


def _mixed(ctx, U, gauge, flags, target=1e-14, switch=1e-6, max_sweeps=4000, check_every=100):
    glo = gf.Geom.make(U.shape[:4], gf.FP32, gf.R12)
    ghi = gf.Geom.make(U.shape[:4], gf.FP64, gf.R12)
    fhi, _ = upload(ctx, U, gf.FP64, gf.R12)
    flo = ctx.empty_field(glo)
    P0 = ctx.empty_out(1)
    ctx.plaquette(fhi, ghi, P0)
    p = gf.fix_params(omega=1.7, theta_target=target, theta_switch=switch,
                      max_sweeps=max_sweeps, check_every=check_every, flags=flags)
    r = ctx.fix_mixed(flo, glo, fhi, ghi, gauge, p)
    P1 = ctx.empty_out(1)
    ctx.plaquette(fhi, ghi, P1)
    return r, P0.item(), P1.item(), fhi, ghi


@pytest.mark.parametrize("switch", [1e-6, 1e-12])
@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
def test_fix_mixed_matches_fp64_oracle(ctx, gauge, switch):
    """FP32 phase with tracked g, FP64 phase on the original orbit: final F
    equals the FP64 oracle's to 1e-10, the plaquette is unchanged to 1e-13;
    also with the FP32 phase run on to theta < 1e-12 (the tracked g is then
    applied at FP32 precision, and the FP64 phase removes that)."""
    dims = (8, 8, 8, 8) if gauge == gf.LANDAU else (8, 6, 6, 6)
    U = inputs.config0(dims, 0.3, 1)
    r, P0, P1, fhi, ghi = _mixed(ctx, U, gauge, gf.FLAG_TIMING, switch=switch)
    ref = oracle_input(U, gf.FP64, gf.R12)
    ro = O.fix(ref, gauge, 1.7, 1e-14, 4000, 100, 1)
    say("mixed", gauge, "switch", switch, r.as_dict(), ro)
    assert r.status == gf.OK and ro["converged"]
    assert r.sweeps_lo > 0 and r.sweeps > r.sweeps_lo
    assert r.theta_at_switch < switch and r.theta < 1e-14
    assert r.F == pytest.approx(ro["F"], rel=1e-10)
    assert P1 == pytest.approx(P0, abs=1e-13)
    assert r.kernel_launches[0] == 2 * r.sweeps_lo
    assert r.kernel_launches[1] == 2 * (r.sweeps - r.sweeps_lo)
    if gauge == gf.COULOMB:
        F, th = ctx.empty_out(dims[0]), ctx.empty_out(dims[0])
        ctx.measure(fhi, ghi, gauge, F, th)
        assert np.allclose(F.cpu().numpy(), O.functional(ref, gauge)[1], rtol=1e-10)


@pytest.mark.parametrize("mixed", [False, True])
def test_fix_graph_replay_matches_eager(ctx, mixed):
    """Sweeps between checks replayed from a captured hipGraph give the same
    bits as eager launches (each replay is followed by an eager check)."""
    U = inputs.config0((8, 8, 8, 8), 0.3, 1)
    outs = []
    for flags in (0, gf.FLAG_GRAPH):
        if mixed:
            r, _, _, f, g = _mixed(ctx, U, gf.LANDAU, flags, check_every=20)
        else:
            f, g = upload(ctx, U, gf.FP64, gf.R12)
            r = ctx.fix(f, g, gf.LANDAU, gf.fix_params(omega=1.7, theta_target=1e-12,
                                                      max_sweeps=2000, check_every=20,
                                                      flags=flags))
        outs.append((r.sweeps, r.F, r.theta, download(ctx, f, g)))
    assert outs[0][0] == outs[1][0] and outs[0][1] == outs[1][1] and outs[0][2] == outs[1][2]
    assert np.array_equal(outs[0][3], outs[1][3])


def test_fix_mixed_untracked_carries_fp32_rounding(ctx):
    """Without tracking, the FP32 phase perturbs the gauge-invariant content
    at the FP32 rounding level: the plaquette moves and F differs from the
    FP64 oracle beyond 1e-10 but within 1e-6."""
    U = inputs.config0((8, 8, 8, 8), 0.3, 1)
    r, P0, P1, _, _ = _mixed(ctx, U, gf.LANDAU, gf.FLAG_NO_TRACK)
    ro = O.fix(oracle_input(U, gf.FP64, gf.R12), gf.LANDAU, 1.7, 1e-14, 4000, 100, 1)
    assert r.status == gf.OK
    assert r.F == pytest.approx(ro["F"], rel=1e-6)
    assert abs(P1 - P0) > 1e-12


@pytest.mark.parametrize("storage", [gf.R12, gf.R18])
def test_fp32_sweeps_stay_on_the_gauge_orbit(ctx, storage):
    """A gauge transformation (eq. (4)) leaves the plaquette unchanged, so 2600
    FP32 overrelaxation sweeps (the FP32 phase of the mixed 32^4 fix) may move
    it only by accumulated FP32 rounding, which averages out over the 6V
    plaquettes: here a few 1e-7. A projection of the 12-real links whose
    rounding is not neutral walks the field off its orbit instead (+5.7e-6
    over these sweeps when the rows were projected in FP32 arithmetic)."""
    import torch
    dims = (32, 32, 32, 32)
    canon = inputs.gpu_heatbath(dims, 6.0, 300, 2)
    g = gf.Geom.make(dims, gf.FP32, storage)
    U = ctx.empty_field(g)
    ctx.pack(g, canon, U)
    P0, P1 = ctx.empty_out(1), ctx.empty_out(1)
    ctx.plaquette(U, g, P0)
    for _ in range(26):
        for _ in range(100):
            ctx.sweep(U, g, gf.LANDAU, 0, 1.7)
            ctx.sweep(U, g, gf.LANDAU, 1, 1.7)
        ctx.reunitarize(U, g)
    ctx.plaquette(U, g, P1)
    F, th = ctx.empty_out(1), ctx.empty_out(1)
    ctx.measure(U, g, gf.LANDAU, F, th)
    torch.cuda.synchronize()
    say("FP32 orbit", storage, "plaquette change", P1.item() - P0.item(), "theta", th.item())
    assert th.item() < 1e-5  # the sweeps did fix the gauge
    assert abs(P1.item() - P0.item()) < 1e-6


@pytest.mark.parametrize("prec,storage", [(gf.FP64, gf.R18), (gf.FP64, gf.R12)])
def test_fix_coulomb_matches_oracle(ctx, prec, storage):
    dims = (8, 4, 6, 4)
    U = inputs.config0(dims, 0.4, 4)
    f, g = upload(ctx, U, prec, storage)
    p = gf.fix_params(omega=1.7, theta_target=1e-13, max_sweeps=3000, check_every=50)
    r = ctx.fix(f, g, gf.COULOMB, p)
    ref = oracle_input(U, prec, storage)
    ro = O.fix(ref, gf.COULOMB, 1.7, 1e-13, 3000, 50, 1)
    assert r.status == gf.OK and ro["converged"] and r.sweeps == ro["sweeps"]
    F, th = ctx.empty_out(dims[0]), ctx.empty_out(dims[0])
    ctx.measure(f, g, gf.COULOMB, F, th)
    assert np.allclose(F.cpu().numpy(), O.functional(ref, gf.COULOMB)[1], rtol=1e-10)
    assert np.all(th.cpu().numpy() < 1e-13)


@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("storage", [gf.R18, gf.R12])
def test_anneal_parity_fp64(ctx, gauge, storage):
    """FP64 heatbath and microcanonical half-sweeps, each from identical
    input: the same Philox draws and accept/reject decisions as the oracle.
    (Over several half-sweeps the annealing dynamics amplify last-bit
    differences like any chaotic map, so the bar is per half-sweep.)"""
    dims = (4, 4, 6, 4)
    U = inputs.config0(dims, 0.6, 21)
    ref = oracle_input(U, gf.FP64, storage)
    for k, T in enumerate([1.45, 0.8, 0.3, 0.01]):
        steps = [("hb", 0), ("hb", 1)] + [("mc", p) for _ in range(3) for p in (0, 1)]
        for kind, p in steps:
            f, g = upload(ctx, ref, gf.FP64, storage)
            if kind == "hb":
                ctx.heatbath_half(f, g, gauge, p, T, 777, k)
                capped = O.heatbath_half(ref, gauge, p, T, 777, k)
                assert capped == 0
            else:
                ctx.micro_half(f, g, gauge, p)
                O.micro_half(ref, gauge, p)
            err = np.abs(download(ctx, f, g) - ref).max()
            assert err <= 1e-12, (k, T, kind, p, err)


def test_anneal_sweep_is_its_half_sweeps(ctx):
    """gf_anneal_sweep = heatbath RED, BLACK, then n_micro microcanonical
    sweeps, bit for bit."""
    dims = (4, 6, 4, 8)
    U = inputs.config0(dims, 0.6, 22)
    a, g = upload(ctx, U, gf.FP32, gf.R12)
    b, _ = upload(ctx, U, gf.FP32, gf.R12)
    for k, T in enumerate([1.2, 0.5]):
        ctx.anneal_sweep(a, g, gf.COULOMB, T, 5, k, 3)
        for p in (0, 1):
            ctx.heatbath_half(b, g, gf.COULOMB, p, T, 5, k)
        for _ in range(3):
            for p in (0, 1):
                ctx.micro_half(b, g, gf.COULOMB, p)
    assert np.array_equal(download(ctx, a, g), download(ctx, b, g))


def test_anneal_fp32_statistics(ctx):
    """FP32 annealing with a reunitarisation after each step: the plaquette
    stays that of U = 1 (gauge transformations only) and a hot anneal
    disorders the field."""
    dims = (8, 8, 8, 8)
    U = inputs.unit_field(dims)
    f, g = upload(ctx, U, gf.FP32, gf.R12)
    for k in range(10):
        ctx.anneal_sweep(f, g, gf.LANDAU, 4.0, 3, k, 1)
        ctx.reunitarize(f, g)
    F, P = ctx.empty_out(1), ctx.empty_out(1)
    ctx.functional(f, g, gf.LANDAU, F)
    ctx.plaquette(f, g, P)
    assert F.item() < 0.5
    assert P.item() == pytest.approx(1.0, abs=1e-5)


def _full_size_input(dims, beta, sweeps, seed):
    import torch
    say("generating", dims, beta, sweeps, seed)
    d = inputs.gpu_heatbath(dims, beta, sweeps, seed)
    torch.cuda.synchronize()
    return host_canon(d, dims)


@pytest.mark.parametrize("dims,beta,seed", [((32, 32, 32, 32), 6.0, 2), ((48, 48, 48, 48), 6.2, 3)])
@pytest.mark.parametrize("prec", [gf.FP32, gf.FP64])
def test_full_size_sampled_parity(ctx, dims, beta, seed, prec):
    """One RED half-sweep at the benchmark sizes (12-real storage) in the
    launch configuration the benchmark times: the variant the autotuner picks
    on this field, as the benchmark does; 256 sampled sites recomputed by the
    oracle."""
    U = _full_size_input(dims, beta, 20, seed)
    f, g = upload(ctx, U, prec, gf.R12)
    try:
        variant, _ = ctx.autotune(g, gf.LANDAU, U_like=f)
        say("full size", dims, "precision", prec, "autotuned variant", variant)
        ctx.sweep(f, g, gf.LANDAU, 0, 1.7)
    finally:
        ctx.set_sweep_variant(prec, gf.R12, 0, -1)
    got = download(ctx, f, g)
    ref = oracle_input(U, prec, gf.R12)
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    cand = rng.choice(V, size=1024, replace=False)
    sites = [int(s) for s in cand if site_parity(dims, s) == 0][:256]
    O.update_sites(ref, gf.LANDAU, 1.7, sites)
    g4 = got.reshape(V, 4, 3, 3)
    r4 = ref.reshape(V, 4, 3, 3)
    err = max(np.abs(g4[s, mu] - r4[s, mu]).max() for s, mu in sites_links(dims, sites))
    assert err <= TOL[prec], err
    # and an untouched-parity property at any size: plaquette unchanged
    P0, P1 = ctx.empty_out(1), ctx.empty_out(1)
    f0, g0 = upload(ctx, U, prec, gf.R12)
    ctx.plaquette(f0, g0, P0)
    ctx.plaquette(f, g, P1)
    assert P1.item() == pytest.approx(P0.item(), abs=1e-12 if prec == gf.FP64 else 1e-5)


@pytest.mark.parametrize("storage,flags", [(gf.R18, 0), (gf.R12, 0), (gf.R12, gf.FLAG_GRAPH)])
def test_fix_coulomb_frozen_matches_oracle(ctx, storage, flags):
    """Coulomb with converged timeslices frozen: the same check at which each
    timeslice freezes as the oracle's freezing driver (through the count of
    frozen timeslice-sweeps), the same sweeps, the same fixed field."""
    dims = (8, 4, 6, 4)
    U = inputs.config0(dims, 0.8, 4)
    say("coulomb frozen", storage, flags)
    f, g = upload(ctx, U, gf.FP64, storage)
    p = gf.fix_params(omega=1.7, theta_target=1e-13, max_sweeps=3000, check_every=10,
                      flags=flags | gf.FLAG_FREEZE_TIMESLICES)
    r = ctx.fix(f, g, gf.COULOMB, p)
    ref = oracle_input(U, gf.FP64, storage)
    ro = O.fix_coulomb_frozen(ref, 1.7, 1e-13, 3000, 10, 1)
    say(r.as_dict(), ro)
    assert len(set(ro["frozen_at"].tolist())) > 3  # the timeslices freeze at different checks
    assert r.status == gf.OK and ro["converged"] and r.sweeps == ro["sweeps"]
    assert r.frozen_slice_sweeps == int(np.sum(ro["sweeps"] - ro["frozen_at"]))
    assert r.theta == pytest.approx(ro["theta"].max(), rel=1e-6)
    assert np.abs(download(ctx, f, g) - ref).max() < 1e-9
    F, th = ctx.empty_out(dims[0]), ctx.empty_out(dims[0])
    ctx.measure(f, g, gf.COULOMB, F, th)
    assert np.allclose(F.cpu().numpy(), ro["F"], rtol=1e-10)
    assert np.all(th.cpu().numpy() < 1e-13)


def test_fix_coulomb_frozen_mixed(ctx):
    """Freezing in both phases of the mixed driver (FP32 at theta_switch, FP64
    at the target): every theta_t below the target, F per timeslice equal to
    the FP64 oracle's, the plaquette unchanged."""
    dims = (8, 6, 6, 6)
    U = inputs.config0(dims, 0.3, 1)
    r, P0, P1, fhi, ghi = _mixed(ctx, U, gf.COULOMB, gf.FLAG_FREEZE_TIMESLICES | gf.FLAG_GRAPH,
                                 check_every=10)
    ref = oracle_input(U, gf.FP64, gf.R12)
    ro = O.fix(ref, gf.COULOMB, 1.7, 1e-14, 4000, 100, 1)
    say("mixed frozen", r.as_dict())
    assert r.status == gf.OK and r.theta < 1e-14 and r.frozen_slice_sweeps > 0
    F, th = ctx.empty_out(dims[0]), ctx.empty_out(dims[0])
    ctx.measure(fhi, ghi, gf.COULOMB, F, th)
    assert np.all(th.cpu().numpy() < 1e-14)
    assert np.allclose(F.cpu().numpy(), O.functional(ref, gf.COULOMB)[1], rtol=1e-10)
    assert P1 == pytest.approx(P0, abs=1e-13)


def test_fix_freeze_flag_errors(ctx):
    U = inputs.config0((4, 4, 4, 4), 0.3, 1)
    f, g = upload(ctx, U, gf.FP64, gf.R12)
    p = gf.fix_params(omega=1.7, theta_target=1e-12, max_sweeps=10, check_every=5,
                      flags=gf.FLAG_FREEZE_TIMESLICES)
    for gauge in (gf.LANDAU, gf.MAG):
        with pytest.raises(gf.GFError) as e:
            ctx.fix(f, g, gauge, p)
        assert e.value.status == gf.ERR_ARG


def test_fix_coulomb_frozen_partial_and_trivial(ctx):
    """Stopped at max_sweeps with some timeslices frozen: the same state as
    the oracle's freezing driver; an input that is already fixed freezes every
    timeslice at the first check and sweeps nothing."""
    dims = (8, 4, 6, 4)
    U = inputs.config0(dims, 0.8, 4)
    f, g = upload(ctx, U, gf.FP64, gf.R12)
    p = gf.fix_params(omega=1.7, theta_target=1e-13, max_sweeps=350, check_every=10,
                      flags=gf.FLAG_FREEZE_TIMESLICES | gf.FLAG_GRAPH)
    r = ctx.fix(f, g, gf.COULOMB, p)
    ref = oracle_input(U, gf.FP64, gf.R12)
    ro = O.fix_coulomb_frozen(ref, 1.7, 1e-13, 350, 10, 1)
    fa = ro["frozen_at"]
    assert not ro["converged"] and np.any(fa >= 0) and np.any(fa < 0)
    assert r.status == gf.NOT_CONVERGED and r.sweeps == 350
    assert r.frozen_slice_sweeps == int(np.sum(np.where(fa >= 0, 350 - fa, 0)))
    assert np.abs(download(ctx, f, g) - ref).max() < 1e-9
    # already fixed: the result of the run above, continued to convergence
    p.max_sweeps = 3000
    ctx.fix(f, g, gf.COULOMB, p)
    before = download(ctx, f, g)
    r2 = ctx.fix(f, g, gf.COULOMB, p)
    assert r2.status == gf.OK and r2.sweeps == 0 and r2.frozen_slice_sweeps == 0
    assert np.array_equal(download(ctx, f, g), before)
