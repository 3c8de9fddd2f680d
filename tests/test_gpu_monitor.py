"""The unitarity monitor (gf_unitarity, GF_FLAG_MONITOR) and the drivers'
check log, against the oracle's definition of the deviation."""
import math

import numpy as np
import pytest

import inputs
import oracle as O
import paper_1209_4008_amd as gf
from gpu_helpers import download, oracle_input, say, upload

pytestmark = pytest.mark.gpu

COMBOS = [(gf.FP64, gf.R18), (gf.FP64, gf.R12), (gf.FP32, gf.R18), (gf.FP32, gf.R12)]
DIMS = (10, 8, 10, 14)  # several 2048-site tiles and a ragged one


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gf.Context()
    yield c
    torch.cuda.synchronize()
    c.close()


def gpu_unitarity(ctx, f, g):
    out = ctx.empty_out(1)
    ctx.unitarity(f, g, out)
    return out.item()


@pytest.mark.parametrize("prec,storage", COMBOS)
def test_unitarity_matches_oracle(ctx, prec, storage):
    """an SU(3) field, then links with a row scaled and a row tilted, each at
    a different site and direction (the last site of the lattice included)"""
    U = inputs.config0(DIMS, 0.4, 21)
    V = int(np.prod(DIMS))
    U4 = U.reshape(V, 4, 3, 3)
    for planted in (False, True):
        if planted:
            U4[V - 1, 3, 0, :] *= 1 + 4e-3
            U4[1234, 0, 1, :] += (3e-3 + 1e-3j) * U4[1234, 0, 0, :]
        f, g = upload(ctx, U, prec, storage)
        got = gpu_unitarity(ctx, f, g)
        want = O.unitarity(oracle_input(U, prec, storage))
        say("unitarity", prec, storage, "planted" if planted else "su3", got, want)
        assert abs(got - want) <= 1e-14 + 1e-12 * want, (got, want)
        if planted:
            assert got > 1e-3
        else:
            assert got < (1e-13 if prec == gf.FP64 else 1e-6)


def test_unitarity_of_nan_is_infinite(ctx):
    U = inputs.config0(DIMS, 0.4, 22)
    U.reshape(-1, 4, 3, 3)[777, 2, 1, 1] = np.nan
    f, g = upload(ctx, U, gf.FP64, gf.R18)
    assert gpu_unitarity(ctx, f, g) == math.inf


def test_fix_check_log_and_monitor(ctx):
    """one record per check, in order, the last one the result's F and theta;
    the monitor reads the field before the check's reunitarisation and changes
    nothing: the same sweeps, F and field as without it"""
    dims = (8, 8, 8, 8)
    U = inputs.config0(dims, 0.3, 23)
    runs = {}
    for flags in (0, gf.FLAG_MONITOR):
        f, g = upload(ctx, U, gf.FP64, gf.R12)
        log = gf.check_log(64)
        p = gf.fix_params(omega=1.7, theta_target=1e-12, max_sweeps=2000, check_every=50,
                          flags=flags | gf.FLAG_GRAPH, check_log=log)
        r = ctx.fix(f, g, gf.LANDAU, p)
        assert r.status == gf.OK
        recs = [log[k].as_dict() for k in range(r.check_log_n)]
        runs[flags] = (r, recs, download(ctx, f, g))
        assert r.check_log_n == r.checks
        assert [e["sweeps"] for e in recs] == [50 * k for k in range(r.checks)]
        assert recs[-1]["F"] == r.F and recs[-1]["theta"] == r.theta
        assert all(e["precision"] == "fp64" for e in recs)
        assert all(b["elapsed_ms"] >= a["elapsed_ms"] for a, b in zip(recs, recs[1:]))
        if flags:
            u = [e["unitarity"] for e in recs]
            say("FP64 12-real unitarity at the checks", min(u), max(u))
            assert max(u) < 1e-13 and r.unitarity_max == max(u)
        else:
            assert r.unitarity_max == -1 and all(e["unitarity"] == -1 for e in recs)
    (r0, l0, f0), (r1, l1, f1) = runs[0], runs[gf.FLAG_MONITOR]
    assert (r0.sweeps, r0.F, r0.theta) == (r1.sweeps, r1.F, r1.theta)
    assert np.array_equal(f0, f1)
    assert [(a["F"], a["theta"]) for a in l0] == [(b["F"], b["theta"]) for b in l1]


def test_mixed_check_log_and_a_full_log(ctx):
    """gf_fix_mixed: the FP32 phase's records first (their unitarity at the
    FP32 rounding level), then the FP64 phase's; a log shorter than the checks
    keeps the first ones"""
    dims = (8, 8, 8, 8)
    U = inputs.config0(dims, 0.3, 24)
    glo = gf.Geom.make(dims, gf.FP32, gf.R12)
    for cap in (64, 3):
        fhi, ghi = upload(ctx, U, gf.FP64, gf.R12)
        flo = ctx.empty_field(glo)
        log = gf.check_log(cap)
        p = gf.fix_params(omega=1.7, theta_target=1e-13, theta_switch=1e-6, max_sweeps=3000,
                          check_every=50, flags=gf.FLAG_MONITOR, check_log=log)
        r = ctx.fix_mixed(flo, glo, fhi, ghi, gf.LANDAU, p)
        assert r.status == gf.OK
        recs = [log[k].as_dict() for k in range(r.check_log_n)]
        assert r.check_log_n == min(cap, r.checks)
        prec = [e["precision"] for e in recs]
        assert prec == sorted(prec, key=lambda x: x != "fp32")  # fp32 records first
        for e in recs:
            assert e["unitarity"] < (1e-5 if e["precision"] == "fp32" else 1e-13), e
        if cap == 64:
            n32 = prec.count("fp32")
            assert n32 >= 2 and len(prec) > n32
            say("mixed: unitarity at FP32 checks", max(e["unitarity"] for e in recs[:n32]),
                "at FP64 checks", max(e["unitarity"] for e in recs[n32:]))
            assert r.unitarity_max == max(e["unitarity"] for e in recs)
