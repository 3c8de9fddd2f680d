"""Helpers shared by the GPU tests: moving canonical fields to and from the
device through the C ABI, and preparing the oracle's input from the same
generator output (never from the GPU path)."""
import sys

import numpy as np

import paper_1209_4008_amd as gf

TOL = {gf.FP64: 1e-12, gf.FP32: 2e-5}
# sites per tile of the device layout that gf.h documents
LAYOUT_TILE = 2048


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


def site_transform_residual(in8, out8):
    """How far out8 is from in8 transformed by one SU(3) matrix G at the site
    (U_mu(x) -> G U_mu(x), U_mu(x - mu) -> U_mu(x - mu) G^dag, eq. (4)), with
    G read off the first link; includes the unitarity of G."""
    G = out8[0] @ in8[0].conj().T
    r = np.abs(G @ G.conj().T - np.eye(3)).max()
    for mu in range(4):
        r = max(r, np.abs(out8[mu] - G @ in8[mu]).max(),
                np.abs(out8[4 + mu] - in8[4 + mu] @ G.conj().T).max())
    return r


def heatbath_spread(U_in, dims, gauge, T, seed, sweep, s, b, n=16, rng_seed=0):
    """How far the oracle's update of site s moves when each real component of
    its 8 input links is perturbed by a relative N(0, 1) * 2^-23 (the unit
    roundoff of FP32): the largest change of the site's 8 output links over n
    perturbations. An FP32 computation of the same update, rounding at every
    step, can differ from the FP64 result by a multiple of this without any
    mistake."""
    import oracle as O
    V = int(np.prod(dims))
    W = U_in.copy()
    W4 = W.reshape(V, 4, 3, 3)
    pos = [(s, mu) for mu in range(4)] + [(int(b[s, mu]), mu) for mu in range(4)]
    orig = [W4[i, mu].copy() for i, mu in pos]
    ref = W.copy()
    O.heatbath_sites(ref, gauge, T, seed, sweep, [s])
    e0 = eight_links(ref, dims, s, b)
    rng = np.random.default_rng(rng_seed)
    spread = 0.0
    for _ in range(n):
        for (i, mu), o in zip(pos, orig):
            d = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
            W4[i, mu] = o.real * (1 + 2.0 ** -23 * d.real) + 1j * o.imag * (1 + 2.0 ** -23 * d.imag)
        O.heatbath_sites(W, gauge, T, seed, sweep, [s])
        spread = max(spread, np.abs(eight_links(W, dims, s, b) - e0).max())
        for (i, mu), o in zip(pos, orig):
            W4[i, mu] = o
    return spread


def heatbath_sites_check(dims, U_in, got, ref, gauge, T, seed, sweep, sites, bar, tau, what):
    """Heatbath half-sweep result `got` (GPU) against `ref` (oracle, from U_in)
    at the given sites of one parity. A site within `bar` passes. A site
    beyond it must either
      - have a borderline Kennedy-Pendleton trial (margin < tau,
        oracle.heatbath_site_outcomes) and match one of the outcomes that
        deciding such trials either way gives, or
      - be ill-conditioned: its update moves by spread(s) under FP32-level
        perturbations of its inputs (heatbath_spread), and the bar scales
        with that: |got - ref| <= bar * spread(s) / spread0, spread0 the
        median spread of 8 sites that passed; such a site's result must also
        be a transformation of its input by one SU(3) matrix (to 1e-5).
    Returns the number of sites that needed either (each kind bounded by the
    caller)."""
    import oracle as O
    b = back_index(dims)
    border = ill = 0
    worst = 0.0
    passed = []
    spread0 = None
    for s in sites:
        s = int(s)
        g8 = eight_links(got, dims, s, b)
        e = np.abs(g8 - eight_links(ref, dims, s, b)).max()
        if e <= bar:
            worst = max(worst, e)
            passed.append(s)
            continue
        outs, mm = O.heatbath_site_outcomes(U_in, gauge, T, seed, sweep, s, tau)
        if len(outs) > 1:
            best = min(np.abs(g8 - o).max() for o in outs)
            assert best <= bar, (what, "site", s, "matches none of", len(outs),
                                 "outcomes; closest", best)
            border += 1
            continue
        if spread0 is None:
            others = [q for q in passed[:8]] or [int(q) for q in sites[:8] if int(q) != s]
            spread0 = float(np.median([heatbath_spread(U_in, dims, gauge, T, seed, sweep, q, b)
                                       for q in others]))
        sp = heatbath_spread(U_in, dims, gauge, T, seed, sweep, s, b)
        allowed = bar * max(1.0, sp / spread0)
        res = site_transform_residual(eight_links(U_in, dims, s, b), g8)
        say(what, "site", s, "no borderline trial (smallest margin", mm, "); differs by", e,
            "spread", sp, "typical", spread0, "allowed", allowed, "SU(3) residual", res)
        assert e <= allowed and res <= 1e-5, (what, "site", s, "differs by", e, "allowed", allowed,
                                              "residual", res)
        ill += 1
    say(what, f"max err at exactly decided sites {worst:.2e};",
        f"borderline sites {border}, ill-conditioned sites {ill} of {len(sites)}")
    return border + ill
