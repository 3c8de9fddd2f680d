"""Race freedom of the RED/BLACK decomposition (Sec. 2), shown on the kernels
themselves: the debug library libgf_debug.so is built from the same kernel
sources with every link-element load and store counted. In one half-sweep
every element of every link must be read exactly once and written exactly
once -- each link belongs to exactly one site of the swept parity, U_mu(x) to
x and U_mu(y) (y of the other parity) to y + mu, and a site reads and writes
only its own eight links -- so no two sites of a launch touch the same
element. Padding sites are never touched. The tracked update's
gauge-transformation field is read and written once at each site of the
swept parity and left alone at the others."""
import ctypes as C
import os

import numpy as np
import pytest

import inputs
import paper_1209_4008_amd as gf
from gpu_helpers import LAYOUT_TILE, say, upload

pytestmark = pytest.mark.gpu

DEBUG_LIB = os.path.join(os.path.dirname(gf.__file__), "libgf_debug.so")
DIMS = (10, 8, 10, 14)  # 5600 sites per parity: two 2048-site tiles and a ragged third


@pytest.fixture(scope="module")
def dbg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    assert os.path.exists(DEBUG_LIB), "libgf_debug.so is not built"
    L = C.CDLL(DEBUG_LIB)
    f = L.gf_debug_access_count
    f.restype = C.c_int32
    f.argtypes = [C.c_int32, C.POINTER(gf.Geom), C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    c = gf.Context()
    yield f, c
    torch.cuda.synchronize()
    c.close()


def expected_link_counts(geom):
    """1 at every element of the V/2 real sites of each parity block, 0 in
    the padding of the last tile"""
    nc = geom.storage // 2
    vh = geom.volume // 2
    W = LAYOUT_TILE
    vp = (vh + W - 1) // W * W
    h = np.arange(vp)
    real = (h < vh).astype(np.uint32)
    # element (p, mu, c, h) at p*4*NC*vp + (h//W)*W*4*NC + (mu*NC + c)*W + h%W
    out = np.zeros(8 * nc * vp, dtype=np.uint32)
    for p in range(2):
        for mu in range(4):
            for c in range(nc):
                off = p * 4 * nc * vp + (h // W) * W * 4 * nc + (mu * nc + c) * W + h % W
                out[off] = real
    return out


def expected_gauge_counts(geom, parity):
    vh = geom.volume // 2
    W = LAYOUT_TILE
    vp = (vh + W - 1) // W * W
    h = np.arange(vp)
    out = np.zeros(2 * 6 * vp, dtype=np.uint32)
    for c in range(6):
        off = parity * 6 * vp + (h // W) * W * 6 + c * W + h % W
        out[off] = (h < vh).astype(np.uint32)
    return out


CASES = [(upd, prec, st, gauge, tps)
         for upd in (0, 1, 2, 4)
         for prec in (gf.FP32, gf.FP64) for st in (gf.R12, gf.R18)
         for gauge in ((gf.LANDAU, gf.COULOMB) if upd != 4 else (gf.LANDAU,))
         for tps in (1, 2, 4)]


@pytest.mark.parametrize("upd,prec,st,gauge,tps", CASES)
def test_every_link_element_read_once_written_once(dbg, upd, prec, st, gauge, tps):
    import torch
    fn, ctx = dbg
    U = inputs.config0(DIMS, 0.4, 81)
    want = None
    for parity in (0, 1):
        f, geom = upload(ctx, U, prec, st)
        n = gf.field_bytes(geom) // (2 * prec)
        rd = torch.zeros(n, dtype=torch.int32, device="cuda")
        wr = torch.zeros(n, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        rc = fn(upd, C.byref(geom), gauge, parity, tps, C.c_void_p(f.data_ptr()), None,
                C.c_void_p(rd.data_ptr()), C.c_void_p(wr.data_ptr()), None, None,
                C.c_void_p(ctx.stream.cuda_stream))
        assert rc == 0
        if want is None:
            want = expected_link_counts(geom)
        r = rd.cpu().numpy().astype(np.uint32)
        w = wr.cpu().numpy().astype(np.uint32)
        assert np.array_equal(r, want), ("reads", int(r.max()), int((r != want).sum()))
        assert np.array_equal(w, want), ("writes", int(w.max()), int((w != want).sum()))


@pytest.mark.parametrize("st", [gf.R12, gf.R18])
@pytest.mark.parametrize("gauge", [gf.LANDAU, gf.COULOMB])
@pytest.mark.parametrize("tps", [1, 2, 4])
def test_tracked_update_counts(dbg, st, gauge, tps):
    import torch
    fn, ctx = dbg
    U = inputs.config0(DIMS, 0.4, 82)
    for parity in (0, 1):
        f, geom = upload(ctx, U, gf.FP32, st)
        G = ctx.empty_gauge(geom)
        ctx.gauge_unit(geom, G)
        n = gf.field_bytes(geom) // 8
        ng = gf.gauge_bytes(geom) // 8
        rd, wr = (torch.zeros(n, dtype=torch.int32, device="cuda") for _ in range(2))
        grd, gwr = (torch.zeros(ng, dtype=torch.int32, device="cuda") for _ in range(2))
        torch.cuda.synchronize()
        rc = fn(3, C.byref(geom), gauge, parity, tps, C.c_void_p(f.data_ptr()),
                C.c_void_p(G.data_ptr()), C.c_void_p(rd.data_ptr()), C.c_void_p(wr.data_ptr()),
                C.c_void_p(grd.data_ptr()), C.c_void_p(gwr.data_ptr()),
                C.c_void_p(ctx.stream.cuda_stream))
        assert rc == 0
        want = expected_link_counts(geom)
        assert np.array_equal(rd.cpu().numpy().astype(np.uint32), want)
        assert np.array_equal(wr.cpu().numpy().astype(np.uint32), want)
        gw = expected_gauge_counts(geom, parity)
        assert np.array_equal(grd.cpu().numpy().astype(np.uint32), gw)
        assert np.array_equal(gwr.cpu().numpy().astype(np.uint32), gw)
    say("tracked access counts", st, gauge, tps, "ok")
