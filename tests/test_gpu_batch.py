"""GPU checks of the batch driver: lattices of uneven extents fixed together
give what each gives alone, and agree with the FP64 oracle."""
import numpy as np
import pytest

import inputs
import oracle as O
import paper_1209_4008_amd as gf
from gpu_helpers import download, host_canon, oracle_input, say, upload

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4, 4, 4), (6, 4, 4, 8), (8, 8, 8, 8), (4, 6, 6, 6), (2, 2, 2, 2)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gf.Context()
    yield c
    torch.cuda.synchronize()
    c.close()


def _inputs():
    return [inputs.config0(d, 0.3, 40 + k) for k, d in enumerate(SHAPES)]


def batch_vs_alone(ctx, Us, storage, sa):
    """the batch of Us against gf_fix_mixed on each lattice alone (seed + l),
    bit for bit, in the context's current sweep variants"""
    p = gf.fix_params(omega=1.7, theta_target=1e-13, theta_switch=1e-6, max_sweeps=4000,
                      check_every=25, sa_steps=sa, sa_micro=2, sa_T0=1.2, sa_T1=0.02,
                      seed=17, flags=gf.FLAG_GRAPH)
    fields, geoms = [], []
    for U in Us:
        f, g = upload(ctx, U, gf.FP64, storage)
        fields.append(f)
        geoms.append(g)
    b = gf.Batch(ctx, geoms, fields)
    res = b.run(p)
    b.close()
    for l, U in enumerate(Us):
        g = geoms[l]
        fhi, _ = upload(ctx, U, gf.FP64, storage)
        flo = ctx.empty_field(gf.Geom.make(g.dims, gf.FP32, gf.R12))
        pl = gf.fix_params(omega=1.7, theta_target=1e-13, theta_switch=1e-6, max_sweeps=4000,
                           check_every=25, sa_steps=sa, sa_micro=2, sa_T0=1.2, sa_T1=0.02,
                           seed=17 + l)
        r = ctx.fix_mixed(flo, gf.Geom.make(g.dims, gf.FP32, gf.R12), fhi, g, gf.LANDAU, pl)
        say("lattice", l, g.dims, "batch", res[l].sweeps, res[l].sweeps_lo, res[l].F,
            "alone", r.sweeps, r.sweeps_lo, r.F)
        assert res[l].status == gf.OK and r.status == gf.OK
        assert res[l].sweeps == r.sweeps and res[l].sweeps_lo == r.sweeps_lo
        assert res[l].F == pytest.approx(r.F, rel=1e-14)
        assert np.array_equal(download(ctx, fields[l], g), download(ctx, fhi, g))
    return res


@pytest.mark.parametrize("storage", [gf.R12, gf.R18])
@pytest.mark.parametrize("sa", [0, 60])
def test_batch_equals_individual_runs(ctx, storage, sa):
    batch_vs_alone(ctx, _inputs(), storage, sa)


@pytest.mark.parametrize("tps", [1, 2, 4])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_variants_equal_individual_runs(ctx, tps, mode):
    """every lanes-per-site x nontemporal variant of the batch kernels (set on
    the context for both phases) against the same variant on each lattice
    alone; the lattices converge at different checks, so the launch tables
    are rebuilt over the remaining lattices several times"""
    for prec in (gf.FP32, gf.FP64):
        ctx.set_sweep_variant(prec, gf.R12, tps, mode)
    try:
        batch_vs_alone(ctx, _inputs(), gf.R12, 30)
    finally:
        for prec in (gf.FP32, gf.FP64):
            ctx.set_sweep_variant(prec, gf.R12, 0, -1)


@pytest.mark.parametrize("storage", [gf.R12, gf.R18])
def test_batch_autotune(ctx, storage):
    """gf_batch_autotune: the caller's fields are untouched, each phase keeps
    the fastest of its nine timed variants on the context (these small
    lattices are in the first size class), and the batch then gives what
    each lattice gives alone in that variant"""
    Us = _inputs()
    fields, geoms = [], []
    for U in Us:
        f, g = upload(ctx, U, gf.FP64, storage)
        fields.append(f)
        geoms.append(g)
    before = [download(ctx, f, g) for f, g in zip(fields, geoms)]
    b = gf.Batch(ctx, geoms, fields)
    try:
        v32, v64, times = b.autotune()
    finally:
        b.close()
    try:
        say("batch autotune", storage, "FP32", v32, "FP64", v64)
        for ph, v in ((0, v32), (1, v64)):
            mine = {k[1:]: t for k, t in times.items() if k[0] == ph}
            assert len(mine) == 9 and all(t > 0 for t in mine.values())
            assert mine[v] == min(mine.values())
        assert ctx.get_sweep_variant(gf.FP32, gf.R12) == v32
        assert ctx.get_sweep_variant(gf.FP64, storage) == v64
        for f, g, want in zip(fields, geoms, before):
            assert np.array_equal(download(ctx, f, g), want)
        batch_vs_alone(ctx, Us, storage, 0)
    finally:
        ctx.set_sweep_variant(gf.FP32, gf.R12, 0, -1)
        ctx.set_sweep_variant(gf.FP64, storage, 0, -1)


def test_batch_of_many_small_lattices(ctx):
    """72 lattices of 2^4 ... 4^4 (the table search over the lattices runs
    seven levels deep) against the lattices alone"""
    shapes = [(2, 2, 2, 2), (2, 2, 2, 4), (4, 2, 2, 2), (2, 4, 2, 4), (4, 4, 4, 4), (4, 2, 4, 2)]
    Us = [inputs.config0(shapes[k % len(shapes)], 0.3, 300 + k) for k in range(72)]
    res = batch_vs_alone(ctx, Us, gf.R12, 0)
    say("many small lattices: sweeps", sorted(set(r.sweeps for r in res)))


def test_batch_matches_fp64_oracle(ctx):
    """Without annealing every lattice ends at the FP64 oracle's F (1e-10)."""
    Us = _inputs()
    fields, geoms = [], []
    for U in Us:
        f, g = upload(ctx, U, gf.FP64, gf.R12)
        fields.append(f)
        geoms.append(g)
    b = gf.Batch(ctx, geoms, fields)
    res = b.run(gf.fix_params(omega=1.7, theta_target=1e-13, theta_switch=1e-6,
                              max_sweeps=4000, check_every=25))
    b.close()
    for l, U in enumerate(Us):
        ro = O.fix(oracle_input(U, gf.FP64, gf.R12), gf.LANDAU, 1.7, 1e-13, 4000, 25, 1)
        assert ro["converged"] and res[l].status == gf.OK
        assert res[l].F == pytest.approx(ro["F"], rel=1e-10)


def test_batch_rejects_bad_input(ctx):
    U = inputs.config0((4, 4, 4, 4), 0.3, 1)
    f, g = upload(ctx, U, gf.FP64, gf.R12)
    f2, g2 = upload(ctx, U, gf.FP64, gf.R18)
    with pytest.raises(gf.GFError):
        gf.Batch(ctx, [g, g2], [f, f2])  # mixed storage
    with pytest.raises(gf.GFError) as e:
        gf.Batch(ctx, [g], [f], gauge=gf.COULOMB)
    assert e.value.status == gf.ERR_UNSUPPORTED
    f3, g3 = upload(ctx, U, gf.FP32, gf.R12)
    with pytest.raises(gf.GFError):
        gf.Batch(ctx, [g3], [f3])  # not FP64
    b = gf.Batch(ctx, [g], [f])
    try:
        with pytest.raises(gf.GFError) as e:
            b.run(gf.fix_params(omega=1.7, theta_target=1e-12, theta_switch=1e-6, max_sweeps=10,
                                check_every=5, flags=gf.FLAG_FREEZE_TIMESLICES))
        assert e.value.status == gf.ERR_UNSUPPORTED
    finally:
        b.close()


def test_batch_on_a_side_stream(ctx):
    """A context on a torch side stream (non-blocking with respect to the null
    stream) gives the same bits as one on the current stream: annealing, both
    phases and the lattice tables rewritten between them."""
    import torch
    Us = _inputs()
    p = gf.fix_params(omega=1.7, theta_target=1e-13, theta_switch=1e-6, max_sweeps=4000,
                      check_every=25, sa_steps=30, sa_micro=2, sa_T0=1.2, sa_T1=0.02,
                      seed=23, flags=gf.FLAG_GRAPH)
    outs = []
    side = torch.cuda.Stream()
    for c, s in ((ctx, None), (None, side)):
        own = c is None
        if own:
            c = gf.Context(stream=s)
        fields, geoms = [], []
        for U in Us:
            f, g = upload(c, U, gf.FP64, gf.R12)
            torch.cuda.synchronize()  # the staging tensor was allocated on the current stream
            fields.append(f)
            geoms.append(g)
        b = gf.Batch(c, geoms, fields)
        res = b.run(p)
        b.close()
        torch.cuda.synchronize()
        outs.append(([r.sweeps for r in res], [download(c, f, g) for f, g in zip(fields, geoms)]))
        if own:
            c.close()
    assert outs[0][0] == outs[1][0]
    for a, b2 in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b2)


def test_batch_gribov_shape_sampled_parity(ctx):
    """The Gribov-copy workload's shape: 64 Haar copies each of 16^4, 24^4 and
    12^3 x 24 (192 lattices, 28.1 M sites, 10.8 GB of FP64 12-real fields, so
    the built-in streamed mode), one FP64 sweep (RED then BLACK) through the
    batch driver; on 2 copies of each base, 16 BLACK sites and every RED
    neighbour they depend on are recomputed by the oracle from the same input,
    and the 8 links of each sampled BLACK site are compared to 1e-12."""
    import torch
    bases = [((16, 16, 16, 16), 5.8, 5), ((24, 24, 24, 24), 6.0, 6), ((24, 12, 12, 12), 5.9, 7)]
    copies = 64
    geoms, fields, owner, cps = [], [], [], []
    inputs_host = {}  # the generator's canonical fields of the sampled copies
    for k, (dims, beta, seed) in enumerate(bases):
        base = inputs.gpu_heatbath(dims, beta, 20, seed)
        g = gf.Geom.make(dims, gf.FP64, gf.R12)
        for cp in range(copies):
            c = base.clone()
            inputs.gpu_haar_copy(c, dims, 1000 + seed, cp)
            if cp in (0, 37):
                inputs_host[len(geoms)] = oracle_input(host_canon(c, dims), gf.FP64, gf.R12)
            f = ctx.empty_field(g)
            ctx.pack(g, c, f)
            geoms.append(g)
            fields.append(f)
            owner.append(k)
            cps.append(cp)
        del base
    torch.cuda.synchronize()
    picks = sorted(inputs_host)
    say("gribov-shape batch:", len(geoms), "lattices,", sum(g.volume for g in geoms), "sites")
    b = gf.Batch(ctx, geoms, fields)
    # theta_switch huge: the FP32 phase ends at its first check with g = 1, so
    # the FP64 fields enter the FP64 phase unchanged; then exactly one sweep
    res = b.run(gf.fix_params(omega=1.7, theta_target=0.0, theta_switch=1e30, max_sweeps=1,
                              check_every=1, reunit_at_check=0))
    b.close()
    assert all(r.sweeps == 1 for r in res)
    rng = np.random.default_rng(12)
    for l in picks:
        dims = geoms[l].dims
        V = int(np.prod(dims))
        got = download(ctx, fields[l], geoms[l]).reshape(V, 4, 3, 3)
        ref = inputs_host[l].copy()
        t, z, y, x = np.unravel_index(np.arange(V), dims)
        black = np.flatnonzero((t + z + y + x) % 2 == 1)
        sites = rng.choice(black, size=16, replace=False)
        red = set()
        for s in sites:
            st, sz, sy, sx = np.unravel_index(s, dims)
            for dt, dz, dy, dx in ((1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1)):
                for sign in (1, -1):
                    red.add(int(np.ravel_multi_index(((st + sign * dt) % dims[0],
                                                      (sz + sign * dz) % dims[1],
                                                      (sy + sign * dy) % dims[2],
                                                      (sx + sign * dx) % dims[3]), dims)))
        O.update_sites(ref, gf.LANDAU, 1.7, sorted(red))
        O.update_sites(ref, gf.LANDAU, 1.7, [int(s) for s in sites])
        r4 = ref.reshape(V, 4, 3, 3)
        err = 0.0
        for s in sites:
            st, sz, sy, sx = np.unravel_index(s, dims)
            err = max(err, np.abs(got[s] - r4[s]).max())
            for mu, (dt, dz, dy, dx) in enumerate(((1, 0, 0, 0), (0, 0, 0, 1), (0, 0, 1, 0),
                                                   (0, 1, 0, 0))):
                sb = int(np.ravel_multi_index(((st - dt) % dims[0], (sz - dz) % dims[1],
                                               (sy - dy) % dims[2], (sx - dx) % dims[3]), dims))
                err = max(err, np.abs(got[sb, mu] - r4[sb, mu]).max())
        say("lattice", l, dims, "copy", cps[l], "max err", err)
        assert err <= 1e-12, (l, err)
