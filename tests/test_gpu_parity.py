"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded input.

Bar: per half-sweep / sweep max-abs per link element <= 1e-12 (FP64) or
2e-5 (FP32) from identical input; F and theta relative <= 1e-12 (FP64);
final F of a full gauge fixing <= 1e-10 relative. Inputs come from the
seeded generators (inputs/), never from the GPU path.
"""
import numpy as np
import pytest

import inputs
import oracle as O
import paper_1209_4008_amd as gf
from gpu_helpers import (TOL, download, oracle_input, say, site_parity, sites_links, upload)

pytestmark = pytest.mark.gpu

COMBOS = [(gf.FP64, gf.R18), (gf.FP64, gf.R12), (gf.FP32, gf.R18), (gf.FP32, gf.R12)]
# (10, 8, 10, 14): 5600 sites per parity, two 2048-site tiles and a ragged third
DIMS = [(8, 8, 8, 8), (6, 4, 2, 10), (2, 2, 2, 2), (4, 6, 8, 10), (10, 8, 10, 14)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gf.Context()
    yield c
    torch.cuda.synchronize()
    c.close()


def test_philox_known_answers_and_oracle(ctx):
    torch = ctx.torch
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(1000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[0] = [0, 0, 0, 0]
    ctr[1] = [0xFFFFFFFF] * 4
    seed = 0
    d_ctr = torch.from_numpy(ctr.view(np.int32)).to("cuda")
    d_out = torch.zeros_like(d_ctr)
    ctx.philox(d_ctr, seed, d_out, ctr.shape[0])
    out = d_out.cpu().numpy().view(np.uint32)
    assert list(out[0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    for k in range(2, 1000, 97):
        assert list(out[k]) == O.philox4x32(list(ctr[k]), [seed, 0])
    seed = 0xFFFFFFFFFFFFFFFF
    ctx.philox(d_ctr, seed, d_out, 2)
    out = d_out.cpu().numpy().view(np.uint32)
    assert list(out[1]) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]


@pytest.mark.parametrize("prec,storage", COMBOS)
def test_pack_unpack_roundtrip(ctx, prec, storage):
    U = inputs.config0((4, 6, 2, 8), 0.4, 3)
    say("pack/unpack", prec, storage)
    f, g = upload(ctx, U, prec, storage)
    back = download(ctx, f, g)
    want = oracle_input(U, prec, storage)
    if prec == gf.FP64 and storage == gf.R18:
        assert np.array_equal(back, U)
    else:
        assert np.abs(back - want).max() <= (1e-15 if prec == gf.FP64 else 2e-7)


@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("prec,storage", COMBOS)
@pytest.mark.parametrize("dims", DIMS)
def test_half_sweep_parity(ctx, dims, prec, storage, gauge):
    U = inputs.config0(dims, 0.6, 11)
    say("half-sweep", dims, prec, storage, gauge)
    _half_sweep_check(ctx, U, prec, storage, gauge)


@pytest.mark.parametrize("nt", [0, 1, 2])
@pytest.mark.parametrize("tps", [1, 2, 4])
@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("prec,storage", COMBOS)
@pytest.mark.parametrize("dims", [(6, 4, 2, 10), (10, 8, 10, 14)])
def test_half_sweep_parity_variants(ctx, dims, prec, storage, gauge, tps, nt):
    """Every variant of the sweep kernel (lanes per site x nontemporal) against the oracle."""
    U = inputs.config0(dims, 0.6, 17)
    say("half-sweep variant", tps, nt, dims, prec, storage, gauge)
    ctx.set_sweep_variant(prec, storage, tps, nt)
    try:
        _half_sweep_check(ctx, U, prec, storage, gauge)
    finally:
        ctx.set_sweep_variant(prec, storage, 0, -1)


def _half_sweep_check(ctx, U, prec, storage, gauge):
    f, g = upload(ctx, U, prec, storage)
    ref = oracle_input(U, prec, storage)
    for p in (0, 1):
        ctx.sweep(f, g, gauge, p, 1.7)
        O.sweep(ref, gauge, p, 1.7)
        got = download(ctx, f, g)
        err = np.abs(got - ref).max()
        assert err <= TOL[prec], (p, err)
        # identical input for the next half-sweep
        f, g = upload(ctx, ref, prec, storage)


@pytest.mark.parametrize("prec,storage", [(gf.FP64, gf.R18), (gf.FP64, gf.R12)])
def test_sweep_trajectory(ctx, prec, storage):
    """Ten sweeps, each from the oracle's state, then ten without resync."""
    dims = (8, 4, 8, 4)
    U = inputs.config0(dims, 0.5, 12)
    ref = oracle_input(U, prec, storage)
    for k in range(10):
        f, g = upload(ctx, ref, prec, storage)
        ctx.sweep(f, g, gf.LANDAU, 0, 1.7)
        ctx.sweep(f, g, gf.LANDAU, 1, 1.7)
        O.sweep(ref, gf.LANDAU, 0, 1.7)
        O.sweep(ref, gf.LANDAU, 1, 1.7)
        assert np.abs(download(ctx, f, g) - ref).max() <= TOL[prec]
    for k in range(10):
        ctx.sweep(f, g, gf.LANDAU, 0, 1.7)
        ctx.sweep(f, g, gf.LANDAU, 1, 1.7)
        O.sweep(ref, gf.LANDAU, 0, 1.7)
        O.sweep(ref, gf.LANDAU, 1, 1.7)
    assert np.abs(download(ctx, f, g) - ref).max() <= 10 * TOL[prec]


@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("prec,storage", COMBOS)
def test_measure_parity(ctx, prec, storage, gauge):
    dims = (6, 4, 8, 4)
    U = inputs.config0(dims, 0.7, 13)
    f, g = upload(ctx, U, prec, storage)
    ref = oracle_input(U, prec, storage)
    n = dims[0] if gauge == gf.COULOMB else 1
    F, th = ctx.empty_out(n), ctx.empty_out(n)
    ctx.measure(f, g, gauge, F, th)
    F2, th2 = ctx.empty_out(n), ctx.empty_out(n)
    ctx.functional(f, g, gauge, F2)
    ctx.theta(f, g, gauge, th2)
    Fo = O.functional(ref, gauge)[1]
    tho = O.theta_A(ref, gauge)[1]
    rtol = 1e-12 if prec == gf.FP64 else 1e-5
    assert np.allclose(F.cpu().numpy(), Fo, rtol=rtol, atol=1e-14)
    assert np.allclose(th.cpu().numpy(), tho, rtol=rtol, atol=1e-14)
    assert np.array_equal(F.cpu().numpy(), F2.cpu().numpy())
    assert np.array_equal(th.cpu().numpy(), th2.cpu().numpy())


def test_measure_closed_form_single_link(ctx):
    """theta = 4 sin^2(e)/(3V) and F = 1 - (2 - 2cos e)/(12V) for one diagonal link."""
    dims = (4, 4, 6, 2)
    V = 4 * 4 * 6 * 2
    e = 0.37
    U = inputs.unit_field(dims)
    U[1, 2, 3, 1, 2] = np.diag([np.exp(1j * e), np.exp(-1j * e), 1.0])
    f, g = upload(ctx, U, gf.FP64, gf.R12)
    F, th = ctx.empty_out(1), ctx.empty_out(1)
    ctx.measure(f, g, gf.LANDAU, F, th)
    assert th.item() == pytest.approx(4 * np.sin(e) ** 2 / (3 * V), rel=1e-13)
    assert F.item() == pytest.approx(1 - (2 - 2 * np.cos(e)) / (12 * V), rel=1e-15)


@pytest.mark.parametrize("prec,storage", COMBOS)
def test_reunitarize_and_convert_parity(ctx, prec, storage):
    torch = ctx.torch
    dims = (4, 4, 4, 6)
    rng = np.random.default_rng(7)
    U = inputs.config0(dims, 0.5, 14)
    W = U + 1e-4 * (rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape))
    f, g = upload(ctx, W, prec, storage)
    ctx.reunitarize(f, g)
    ref = oracle_input(W, prec, storage)
    O.reunitarize(ref)
    tol = 1e-14 if prec == gf.FP64 else 1e-6
    assert np.abs(download(ctx, f, g) - ref).max() <= tol
    # conversion to FP64 R18 with and without the projection
    g2 = gf.Geom.make(dims, gf.FP64, gf.R18)
    f2 = ctx.empty_field(g2)
    f, g = upload(ctx, W, prec, storage)
    ctx.convert(g, f, g2, f2, reunitarize=True)
    assert np.abs(download(ctx, f2, g2) - ref).max() <= tol
    ctx.convert(g, f, g2, f2, reunitarize=False)
    assert np.abs(download(ctx, f2, g2) - oracle_input(W, prec, storage)).max() <= 1e-15
    with pytest.raises(gf.GFError):
        ctx.convert(g, f, g, f)  # overlapping buffers
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,storage", COMBOS)
def test_plaquette_parity(ctx, prec, storage):
    dims = (4, 6, 4, 8)
    U = inputs.config0(dims, 0.8, 15)
    f, g = upload(ctx, U, prec, storage)
    P = ctx.empty_out(1)
    ctx.plaquette(f, g, P)
    ref = O.plaquette(oracle_input(U, prec, storage))
    assert P.item() == pytest.approx(ref, rel=1e-13 if prec == gf.FP64 else 1e-6)


def test_determinism(ctx):
    dims = (8, 8, 8, 8)
    U = inputs.config0(dims, 0.6, 16)
    outs = []
    for _ in range(2):
        f, g = upload(ctx, U, gf.FP32, gf.R12)
        for k in range(5):
            ctx.sweep(f, g, gf.LANDAU, k % 2, 1.7)
        F, th = ctx.empty_out(1), ctx.empty_out(1)
        ctx.measure(f, g, gf.LANDAU, F, th)
        outs.append((download(ctx, f, g), F.item(), th.item()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1] and outs[0][2] == outs[1][2]


def test_argument_errors_on_gpu(ctx):
    U = inputs.config0((4, 4, 4, 4), 0.5, 1)
    f, g = upload(ctx, U, gf.FP64, gf.R18)
    for w in (0.5, 2.0, float("nan")):
        with pytest.raises(gf.GFError) as e:
            ctx.sweep(f, g, gf.LANDAU, 0, w)
        assert e.value.status == gf.ERR_ARG
    with pytest.raises(gf.GFError):
        ctx.sweep(f, g, gf.LANDAU, 2, 1.5)
    with pytest.raises(gf.GFError):
        ctx.sweep(f, g, 7, 0, 1.5)
    with pytest.raises(gf.GFError):
        ctx.sweep(f, gf.Geom.make((4, 4, 4, 3)), gf.LANDAU, 0, 1.5)
    with pytest.raises(gf.GFError):
        ctx.heatbath_half(f, g, gf.LANDAU, 0, 0.0, 1, 0)
    with pytest.raises(gf.GFError):
        ctx.sweep(None, g, gf.LANDAU, 0, 1.5)
    # the field is untouched by rejected calls
    assert np.array_equal(download(ctx, f, g), U)


@pytest.mark.parametrize("prec,storage", [(gf.FP64, gf.R12), (gf.FP32, gf.R12)])
def test_autotune_choice_and_parity_after(ctx, prec, storage):
    """The autotuner times the nine variants on a copy of the caller's field
    (graph-replayed blocks, median of interleaved rounds), leaves that field
    untouched, keeps the fastest for the field's size class only, and the
    tuned sweep still matches the oracle."""
    dims = (6, 4, 8, 10)
    U = inputs.config0(dims, 0.6, 18)
    f, g = upload(ctx, U, prec, storage)
    before = download(ctx, f, g)
    big = gf.Geom.make((72, 72, 72, 72), prec, storage)  # above 2 GiB: the other class
    big_before = ctx.sweep_variant_for(big)
    say("autotune", prec, storage)
    try:
        (tps, nt), table = ctx.autotune(g, gf.LANDAU, U_like=f)
        assert set(table) == {(t, n) for t in (1, 2, 4) for n in (0, 1, 2)}
        assert all(v > 0 for v in table.values())
        assert table[(tps, nt)] == min(table.values())
        assert ctx.sweep_variant_for(g) == (tps, nt)
        assert ctx.get_sweep_variant(prec, storage) == (tps, nt)
        assert ctx.sweep_variant_for(big) == big_before
        assert np.array_equal(download(ctx, f, g), before)
        _half_sweep_check(ctx, U, prec, storage, gf.LANDAU)
    finally:
        ctx.set_sweep_variant(prec, storage, 0, -1)


@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
def test_autotune_anneal_and_storage(ctx, gauge):
    """The annealing autotuner fills its own table (the sweep variant is left
    as it was); the storage axis returns the storage whose best variant is
    faster and tunes both; the caller's fields are untouched."""
    import torch
    dims = (6, 4, 8, 10)
    U = inputs.config0(dims, 0.6, 28)
    f, g = upload(ctx, U, gf.FP32, gf.R12)
    before = download(ctx, f, g)
    sweep_before = ctx.sweep_variant_for(g)
    try:
        (tps, nt), table = ctx.autotune_anneal(g, gauge, U_like=f, T=0.7)
        assert table[(tps, nt)] == min(table.values()) and all(v > 0 for v in table.values())
        assert ctx.anneal_variant_for(g) == (tps, nt)
        assert ctx.sweep_variant_for(g) == sweep_before
        assert np.array_equal(download(ctx, f, g), before)
        canon = torch.from_numpy(U.view(np.float64).reshape(-1).copy()).to("cuda")
        st, best = ctx.autotune_storage(g, gauge, canon)
        assert st in (gf.R12, gf.R18) and best[st] == min(best.values()) > 0
        say("storage axis", gauge, best)
    finally:
        for s_ in (gf.R12, gf.R18):
            ctx.set_sweep_variant(gf.FP32, s_, 0, -1)
        ctx.set_anneal_variant(gf.FP32, gf.R12, 0, -1)


@pytest.mark.parametrize("prec,storage", COMBOS)
def test_vanishing_subgroup_parts(ctx, prec, storage):
    """Uniform cyclic permutation field: all subgroup parts of K vanish, every
    subgroup is skipped, the field stays bit for bit, and the driver stops at
    this stationary point (F = 0, theta = 0) without a sweep."""
    dims = (4, 2, 4, 2)
    P = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], dtype=np.complex128)
    U = np.ascontiguousarray(np.broadcast_to(P, tuple(dims) + (4, 3, 3)))
    f, g = upload(ctx, U, prec, storage)
    for gauge in (gf.LANDAU, gf.COULOMB):
        for p in (0, 1):
            ctx.sweep(f, g, gauge, p, 1.7)
        assert np.array_equal(download(ctx, f, g), U)
    r = ctx.fix(f, g, gf.LANDAU, gf.fix_params(theta_target=1e-12, max_sweeps=100))
    assert r.status == gf.OK and r.sweeps == 0 and r.F == 0.0 and r.theta == 0.0


@pytest.mark.parametrize("tps", [1, 2, 4])
def test_nontemporal_modes_change_no_bit(ctx, tps):
    """The nontemporal modes are cache hints only: sweeps, the tracked mixed
    driver and a batch give the same bits under modes 0, 1 and 2."""
    dims = (4, 6, 8, 10)
    U = inputs.config0(dims, 0.5, 19)
    outs = []
    for nt in (0, 1, 2):
        say("nontemporal mode", nt, "lanes", tps)
        for prec in (gf.FP32, gf.FP64):
            ctx.set_sweep_variant(prec, gf.R12, tps, nt)
        try:
            res = []
            for prec in (gf.FP32, gf.FP64):
                f, g = upload(ctx, U, prec, gf.R12)
                for k in range(4):
                    ctx.sweep(f, g, gf.LANDAU, k % 2, 1.7)
                res.append(download(ctx, f, g))
            glo = gf.Geom.make(dims, gf.FP32, gf.R12)
            hi, ghi = upload(ctx, U, gf.FP64, gf.R12)
            lo = ctx.empty_field(glo)
            p = gf.fix_params(omega=1.7, theta_target=1e-12, theta_switch=1e-6, max_sweeps=3000,
                              check_every=100, flags=gf.FLAG_GRAPH)
            r = ctx.fix_mixed(lo, glo, hi, ghi, gf.LANDAU, p)
            res.append(download(ctx, hi, ghi))
            b_f, b_g = upload(ctx, U, gf.FP64, gf.R12)
            b = gf.Batch(ctx, [b_g], [b_f])
            try:
                rb = b.run(p)
            finally:
                b.close()
            res.append(download(ctx, b_f, b_g))
            res.append((r.sweeps, r.F, rb[0].sweeps, rb[0].F))
            outs.append(res)
        finally:
            for prec in (gf.FP32, gf.FP64):
                ctx.set_sweep_variant(prec, gf.R12, 0, -1)
    for other in outs[1:]:
        for a, b_ in zip(outs[0][:4], other[:4]):
            assert np.array_equal(a, b_)
        assert outs[0][4] == other[4]


def test_built_in_variant_follows_field_size(ctx):
    """Cached link accesses up to 2 GiB fields, streamed above, and FP64 one lane
    per site with the streamed accesses (no memory is touched: only the choice
    is queried); a set variant applies to every size."""
    small = gf.Geom.make((32, 32, 32, 32), gf.FP64, gf.R12)   # 0.4 GB
    big = gf.Geom.make((72, 72, 72, 72), gf.FP64, gf.R12)     # 10.3 GB
    big32 = gf.Geom.make((64, 64, 64, 64), gf.FP32, gf.R12)   # 3.2 GB
    assert ctx.sweep_variant_for(small) == (4, 0)
    assert ctx.sweep_variant_for(big) == (1, 1)
    assert ctx.sweep_variant_for(big32) == (2, 1)
    # the annealing updates: FP32 one lane per site, FP64 four
    assert ctx.anneal_variant_for(big32) == (1, 1)
    assert ctx.anneal_variant_for(small) == (4, 0)
    assert ctx.get_sweep_variant(gf.FP64, gf.R12) == (4, 0)
    ctx.set_sweep_variant(gf.FP64, gf.R12, 2, 2)
    try:
        assert ctx.sweep_variant_for(small) == (2, 2)
        assert ctx.sweep_variant_for(big) == (2, 2)
    finally:
        ctx.set_sweep_variant(gf.FP64, gf.R12, 0, -1)
