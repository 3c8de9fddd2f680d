"""Checkpoint files (paper_1209_4008_amd/checkpoint.py): the format on the
CPU, and on the GPU that a run stopped, written, read back into a new buffer
and continued equals the run that never stopped, bit for bit (every link
element; the layout's padding sites are not part of the field), for the
annealing (draws keyed by the sweep index) and for the overrelaxation
driver."""
import json
import os

import numpy as np
import pytest

import inputs
import paper_1209_4008_amd as gf
from paper_1209_4008_amd import checkpoint as ck
from gpu_helpers import dev_canon, download, say


def test_format_round_trip(tmp_path):
    dims = (2, 2, 4, 2)
    U = inputs.config0(dims, 0.3, 3)
    links = np.ascontiguousarray(U).view(np.float64).reshape(-1)
    p = str(tmp_path / "c.npz")
    ck.write(p, links, dims, gf.FP32, gf.R12, {"gauge": "landau", "sweep": 7, "theta": [1.0, 0.5]})
    got, header = ck.read(p)
    assert np.array_equal(got, links)
    assert header["dims"] == list(dims) and header["precision"] == "fp32"
    assert header["storage"] == "r12" and header["state"]["sweep"] == 7
    g = ck.geom_of(header)
    assert (g.dims, g.prec, g.storage) == (dims, gf.FP32, gf.R12)
    with np.load(p, allow_pickle=False) as z:  # plain arrays only
        assert z["links"].dtype == np.float64 and json.loads(str(z["header"]))["format"] == 1


def test_format_rejects_bad_input(tmp_path):
    p = str(tmp_path / "c.npz")
    with pytest.raises(gf.GFError):
        ck.write(p, np.zeros(71), (1, 1, 1, 1), gf.FP64, gf.R18)
    with pytest.raises(gf.GFError):
        ck.write(p, np.zeros(72), (1, 1, 1, 1), 3, gf.R18)
    np.savez(p, links=np.zeros(72), header=np.array(json.dumps({"format": 99, "dims": [1, 1, 1, 1]})))
    with pytest.raises(gf.GFError):
        ck.read(p)
    np.savez(p, links=np.zeros(70), header=np.array(json.dumps({"format": 1, "dims": [1, 1, 1, 1]})))
    with pytest.raises(gf.GFError):
        ck.read(p)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gf.Context()
    yield c
    torch.cuda.synchronize()
    c.close()


def _anneal(ctx, U, g, steps, seed):
    for k in steps:
        ctx.anneal_sweep(U, g, gf.COULOMB, 1.2 - 0.1 * k, seed, k, 3)


@pytest.mark.gpu
@pytest.mark.parametrize("prec,storage", [(gf.FP32, gf.R12), (gf.FP64, gf.R18), (gf.FP64, gf.R12)])
def test_annealing_resumes_bit_for_bit(ctx, tmp_path, prec, storage):
    import torch
    dims = (6, 4, 8, 6)
    U = inputs.config0(dims, 0.6, 21)
    g = gf.Geom.make(dims, prec, storage)
    A = ctx.empty_field(g)
    ctx.pack(g, dev_canon(U, torch), A)
    B = A.clone()
    say("checkpoint anneal", prec, storage)
    _anneal(ctx, A, g, range(6), 11)
    _anneal(ctx, B, g, range(3), 11)
    p = str(tmp_path / "anneal.npz")
    ck.save(ctx, p, B, g, gauge="coulomb", seed=11, next_sweep=3)
    del B
    C, g2, state = ck.load(ctx, p)
    assert (g2.dims, g2.prec, g2.storage) == (g.dims, g.prec, g.storage)
    assert state == {"gauge": "coulomb", "seed": 11, "next_sweep": 3}
    _anneal(ctx, C, g2, range(state["next_sweep"], 6), state["seed"])
    assert np.array_equal(download(ctx, A, g), download(ctx, C, g))


@pytest.mark.gpu
def test_fix_resumes_bit_for_bit(ctx, tmp_path):
    """gf_fix in two calls of 200 sweeps (checks every 100, the field written
    and read back between them) equals one call of 400."""
    import torch
    dims = (8, 8, 8, 8)
    U = inputs.config0(dims, 0.3, 1)
    g = gf.Geom.make(dims, gf.FP64, gf.R12)
    A = ctx.empty_field(g)
    ctx.pack(g, dev_canon(U, torch), A)
    B = A.clone()
    ctx.fix(A, g, gf.LANDAU, gf.fix_params(omega=1.7, theta_target=0.0, max_sweeps=400,
                                            check_every=100))
    r = ctx.fix(B, g, gf.LANDAU, gf.fix_params(omega=1.7, theta_target=0.0, max_sweeps=200,
                                                check_every=100))
    p = str(tmp_path / "fix.npz")
    ck.save(ctx, p, B, g, sweeps=r.sweeps, theta=[r.theta])
    C = torch.empty_like(B)
    C, _, state = ck.load(ctx, p, C)
    assert state["sweeps"] == 200
    ctx.fix(C, g, gf.LANDAU, gf.fix_params(omega=1.7, theta_target=0.0, max_sweeps=200,
                                            check_every=100))
    assert np.array_equal(download(ctx, A, g), download(ctx, C, g))


@pytest.mark.gpu
def test_load_refuses_a_small_buffer(ctx, tmp_path):
    import torch
    dims = (2, 2, 2, 2)
    g = gf.Geom.make(dims, gf.FP64, gf.R18)
    U = ctx.empty_field(g)
    ctx.pack(g, dev_canon(inputs.config0(dims, 0.3, 2), torch), U)
    p = str(tmp_path / "s.npz")
    ck.save(ctx, p, U, g)
    with pytest.raises(gf.GFError):
        ck.load(ctx, p, U[:16])


@pytest.mark.gpu
def test_context_after_host_generators_in_a_fresh_process():
    """The host generators used before any GPU call (as the CPU-side tests do)
    must not keep a later Context from finding the GPU: a fresh process runs
    inputs.config0, then creates a Context and sweeps."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import inputs; U = inputs.config0((2, 2, 2, 2), 0.3, 1); "
            "import paper_1209_4008_amd as gf; print('bytes', gf.field_bytes(gf.Geom.make((2, 2, 2, 2)))); "
            "import torch; c = gf.Context(); g = gf.Geom.make((2, 2, 2, 2)); f = c.empty_field(g); "
            "c.pack(g, torch.from_numpy(U.view('float64').reshape(-1).copy()).to('cuda'), f); "
            "c.sweep(f, g, gf.LANDAU, 0, 1.7); torch.cuda.synchronize(); print('context ok')")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=240)
    say("fresh process:", r.stdout.strip(), r.stderr.strip()[-300:])
    assert r.returncode == 0 and "context ok" in r.stdout
