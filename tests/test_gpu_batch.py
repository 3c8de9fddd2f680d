"""GPU checks of the batch driver: lattices of uneven extents fixed together
give what each gives alone, and agree with the FP64 oracle."""
import numpy as np
import pytest

import inputs
import oracle as O
import paper_1209_4008_amd as gf
from gpu_helpers import download, oracle_input, say, upload

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


@pytest.mark.parametrize("storage", [gf.R12, gf.R18])
@pytest.mark.parametrize("sa", [0, 60])
def test_batch_equals_individual_runs(ctx, storage, sa):
    Us = _inputs()
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
