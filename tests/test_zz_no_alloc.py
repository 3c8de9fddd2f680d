"""gf_measure_static, the measurement entry point that allocates nothing (its
per-block partial sums live in a fixed device array of the library, one per
GPU), against gf_measure on the same fields: F and theta bitwise equal, for
two calls in a row -- the second on a smaller lattice -- in every gauge; a
lattice beyond the array's size is refused before anything is enqueued."""
import numpy as np
import pytest

import inputs
import paper_1209_4008_amd as gf
from gpu_helpers import say, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gf.Context()
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB, gf.MAG])
def test_static_measure_matches_gf_measure(ctx, gauge):
    import torch
    big = (16, 16, 16, 32)
    cases = [(big, gf.FP64, gf.R12), ((4, 6, 4, 6), gf.FP32, gf.R18)]
    for dims, prec, st in cases:
        g = gf.Geom.make(dims, prec, st)
        f = ctx.empty_field(g)
        if dims == big:
            canon = inputs.gpu_config0(dims, 0.4, 71)
            ctx.pack(g, canon, f)
        else:
            f, g = upload(ctx, inputs.config0(dims, 0.4, 72), prec, st)
        n = dims[0] if gauge == gf.COULOMB else 1
        F0, t0 = ctx.empty_out(n), ctx.empty_out(n)
        F1, t1 = ctx.empty_out(n), ctx.empty_out(n)
        F1.fill_(float("nan"))
        t1.fill_(float("nan"))
        ctx.measure(f, g, gauge, F0, t0)
        ctx.measure_static(f, g, gauge, F1, t1)
        torch.cuda.synchronize()
        say("static measure", dims, gauge, F1[:2].tolist(), t1[:2].tolist())
        assert torch.equal(F0, F1) and torch.equal(t0, t1)
        assert torch.isfinite(F1).all() and torch.isfinite(t1).all()


def test_static_measure_refuses_lattices_beyond_its_array(ctx):
    g = gf.Geom.make((256, 256, 128, 128), gf.FP32, gf.R12)
    dummy = ctx.empty_out(8)
    with pytest.raises(gf.GFError) as e:
        ctx.measure_static(dummy, g, gf.LANDAU, dummy, dummy)
    assert e.value.status == gf.ERR_ARG and "static scratch" in str(e.value)
