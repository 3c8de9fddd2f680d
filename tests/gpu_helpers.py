"""Helpers shared by the GPU tests: moving canonical fields to and from the
device through the C ABI, and preparing the oracle's input from the same
generator output (never from the GPU path)."""
import sys

import numpy as np

import paper_1209_4008_amd as gf

TOL = {gf.FP64: 1e-12, gf.FP32: 2e-5}


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev_canon(U, torch):
    """numpy canonical complex128 field -> torch float64 CUDA tensor (same layout)."""
    return torch.from_numpy(np.ascontiguousarray(U).view(np.float64).reshape(-1).copy()).to("cuda")


def host_canon(t, dims):
    a = t.detach().cpu().numpy().astype(np.float64, copy=False)
    return a.view(np.complex128).reshape(tuple(dims) + (4, 3, 3)).copy()


def upload(ctx, U, prec, storage):
    torch = ctx.torch
    geom = gf.Geom.make(U.shape[:4], prec, storage)
    canon = dev_canon(U, torch)
    field = ctx.empty_field(geom)
    ctx.pack(geom, canon, field)
    return field, geom


def download(ctx, field, geom):
    torch = ctx.torch
    canon = torch.empty(geom.volume * 4 * 18, dtype=torch.float64, device="cuda")
    ctx.unpack(geom, field, canon)
    torch.cuda.synchronize()
    return host_canon(canon, geom.dims)


def rebuild_row2(U):
    """row 2 = conj(row0 x row1), as for a link stored as its first two rows"""
    V = U.copy()
    V[..., 2, :] = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    return V


def oracle_input(U, prec, storage):
    """The field the GPU kernels see after packing U, as a canonical FP64 field:
    elements rounded to the storage precision, row 2 rebuilt for 12 reals."""
    V = U.astype(np.complex64).astype(np.complex128) if prec == gf.FP32 else U.copy()
    if storage == gf.R12:
        V = rebuild_row2(V)
    return np.ascontiguousarray(V)


def site_parity(dims, s):
    nt, nz, ny, nx = dims
    x = s % nx
    y = (s // nx) % ny
    z = (s // (nx * ny)) % nz
    t = s // (nx * ny * nz)
    return (t + x + y + z) % 2


def sites_links(dims, sites):
    """(site, mu) pairs touched by updating `sites`: forward U_mu(x) and U_mu(x-mu)"""
    nt, nz, ny, nx = dims
    out = []
    for s in sites:
        x = s % nx
        y = (s // nx) % ny
        z = (s // (nx * ny)) % nz
        t = s // (nx * ny * nz)
        c = [t, x, y, z]
        ext = [nt, nx, ny, nz]
        for mu in range(4):
            out.append((s, mu))
            b = list(c)
            b[mu] = (b[mu] - 1) % ext[mu]
            sb = ((b[0] * nz + b[3]) * ny + b[2]) * nx + b[1]
            out.append((sb, mu))
    return out


def back_index(dims):
    """b[s, mu] = canonical index of s - mu (periodic)"""
    nt, nz, ny, nx = dims
    t, z, y, x = np.indices(dims)
    out = np.empty(tuple(dims) + (4,), dtype=np.int64)
    for mu, (dt, dz, dy, dx) in enumerate([(1, 0, 0, 0), (0, 0, 0, 1), (0, 0, 1, 0),
                                           (0, 1, 0, 0)]):
        out[..., mu] = ((((t - dt) % nt) * nz + (z - dz) % nz) * ny + (y - dy) % ny) * nx + \
            (x - dx) % nx
    return out.reshape(-1, 4)


def site_errors(dims, got, ref, parity):
    """(sites of `parity`, max |got - ref| over each site's 8 links)"""
    V = int(np.prod(dims))
    el = np.abs(got.reshape(V, 4, 3, 3) - ref.reshape(V, 4, 3, 3)).max(axis=(2, 3))
    b = back_index(dims)
    t, z, y, x = np.indices(dims)
    sites = np.flatnonzero(((t + z + y + x) % 2).reshape(-1) == parity)
    fw = el[sites].max(axis=1)
    bw = el[b[sites], np.arange(4)[None, :]].max(axis=1)
    return sites, np.maximum(fw, bw)


def eight_links(U, dims, s, b):
    """U_mu(s), mu = 0..3, then U_mu(s - mu): the links a site update moves"""
    V = int(np.prod(dims))
    U4 = U.reshape(V, 4, 3, 3)
    return np.concatenate([U4[s], U4[b[s], np.arange(4)]])


def heatbath_sites_check(dims, U_in, got, ref, gauge, T, seed, sweep, sites, bar, tau, what):
    """Heatbath half-sweep result `got` (GPU) against `ref` (oracle, from U_in)
    at the given sites of one parity. A site within `bar` passes; a site
    beyond it must have a borderline Kennedy-Pendleton trial (margin < tau,
    oracle.heatbath_site_outcomes) and match one of the outcomes that deciding
    such trials either way gives. Returns the number of borderline sites."""
    import oracle as O
    b = back_index(dims)
    border = 0
    worst = 0.0
    for s in sites:
        s = int(s)
        g8 = eight_links(got, dims, s, b)
        e = np.abs(g8 - eight_links(ref, dims, s, b)).max()
        if e <= bar:
            worst = max(worst, e)
            continue
        outs, mm = O.heatbath_site_outcomes(U_in, gauge, T, seed, sweep, s, tau)
        assert len(outs) > 1, (what, "site", s, "has no borderline trial (smallest margin",
                               mm, ") yet differs by", e)
        best = min(np.abs(g8 - o).max() for o in outs)
        assert best <= bar, (what, "site", s, "matches none of", len(outs),
                             "outcomes; closest", best)
        border += 1
    say(what, f"max err at exactly decided sites {worst:.2e};",
        f"borderline sites {border} of {len(sites)}")
    return border
