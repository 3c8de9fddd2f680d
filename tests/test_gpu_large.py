"""The largest lattices one device holds: V = 2^30 sites (the library's limit)
in FP32 and 2^29 sites in FP64, 12-real storage (206 GB each). Their canonical
FP64 form would not fit beside them, so the input is generated straight into
the device layout and only the links around sampled sites are read back. Each
sampled RED site's update is recomputed by the oracle on a 2^4 lattice that
holds the site's 8 links: with extent 2 every neighbour x - mu is x + mu, so
site 0 of that lattice sees exactly the 8 links of the sampled site, and the
oracle's update of site 0 is the update of the sampled site."""
import numpy as np
import pytest

import inputs
import oracle as O
import paper_1209_4008_amd as gf
from gpu_helpers import LAYOUT_TILE, TOL, rebuild_row2, say, site_parity, sites_links

@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = gf.Context()
    yield c
    torch.cuda.synchronize()
    c.close()


def packed_index(dims, nc, s, mu):
    """complex-element indices of link (s, mu) in the tiled device layout
    (rows 0.. of the link, c = 3a + b < nc)"""
    V = int(np.prod(dims))
    W = LAYOUT_TILE
    vp = (V // 2 + W - 1) // W * W
    p = site_parity(dims, s)
    h = s >> 1
    base = p * 4 * nc * vp + (h // W) * W * 4 * nc + mu * nc * W + h % W
    return [base + c * W for c in range(nc)]


def gather(F, dims, prec, nc, links):
    """the listed (site, mu) links of a packed field, as complex128 rows (len(links), nc)"""
    import torch
    ftype = torch.float32 if prec == gf.FP32 else torch.float64
    flat = F.view(ftype)
    idx = np.array([packed_index(dims, nc, s, mu) for s, mu in links], dtype=np.int64)
    t = torch.from_numpy(np.stack([2 * idx, 2 * idx + 1], axis=-1).reshape(-1)).to("cuda")
    v = flat[t].double().cpu().numpy().reshape(len(links), nc, 2)
    return v[..., 0] + 1j * v[..., 1]


def as_links(rows):
    """(n, 6) rows 0, 1 -> (n, 3, 3) with row 2 rebuilt, as the kernels see a 12-real link"""
    U = np.zeros((rows.shape[0], 3, 3), dtype=np.complex128)
    U[:, :2, :] = rows.reshape(-1, 2, 3)
    return rebuild_row2(U)


# site of e_mu on a 2^4 lattice, (t, z, y, x) lexicographic, mu = 0:t 1:x 2:y 3:z
_E = {0: 8, 1: 1, 2: 2, 3: 4}


def oracle_site_update(links8, omega):
    """links8[2 mu] = U_mu(x), links8[2 mu + 1] = U_mu(x - mu) -> the same links
    after the oracle's update of x (Landau)"""
    m = np.zeros((2, 2, 2, 2, 4, 3, 3), dtype=np.complex128)
    m[..., :, :] = np.eye(3)
    flat = m.reshape(16, 4, 3, 3)
    for mu in range(4):
        flat[0, mu] = links8[2 * mu]
        flat[_E[mu], mu] = links8[2 * mu + 1]
    O.update_sites(m, gf.LANDAU, omega, [0])
    flat = m.reshape(16, 4, 3, 3)
    return np.stack([x for mu in range(4) for x in (flat[0, mu], flat[_E[mu], mu])])


def test_mini_lattice_update_is_the_site_update():
    """(CPU) the 2^4 embedding reproduces the oracle's update of a site of a
    full lattice, for sites anywhere including the boundaries"""
    dims = (4, 6, 4, 8)
    U = inputs.config0(dims, 0.6, 3)
    V = int(np.prod(dims))
    sites = [0, V - 1] + [s for s in range(5, V, 97) if site_parity(dims, s) == 0]
    sites = [s for s in sites if site_parity(dims, s) == 0]
    links = sites_links(dims, sites)
    U4 = U.reshape(V, 4, 3, 3)
    before = np.stack([U4[s, mu] for s, mu in links])
    ref = U.copy()
    O.update_sites(ref, gf.LANDAU, 1.7, sites)
    R4 = ref.reshape(V, 4, 3, 3)
    for k, s in enumerate(sites):
        got = oracle_site_update(before[8 * k:8 * k + 8], 1.7)
        want = np.stack([R4[s2, mu] for s2, mu in links[8 * k:8 * k + 8]])
        assert np.abs(got - want).max() < 1e-14


@pytest.mark.gpu
@pytest.mark.parametrize("dims,prec", [((10, 8, 10, 14), gf.FP32), ((10, 8, 10, 14), gf.FP64)])
@pytest.mark.parametrize("nc", [6, 9])
def test_packed_generator_matches_canonical(ctx, dims, prec, nc):
    """the packed-layout generator writes gpu_config0's links (V/2 = 5600: two
    tiles and a ragged third)"""
    import torch
    storage = gf.R12 if nc == 6 else gf.R18
    geom = gf.Geom.make(dims, prec, storage)
    F = ctx.empty_field(geom)
    inputs.gpu_config0_packed(F, dims, 4 if prec == gf.FP32 else 8, nc, 0.3, 5)
    canon = inputs.gpu_config0(dims, 0.3, 5)
    torch.cuda.synchronize()
    U = canon.cpu().numpy().view(np.complex128).reshape(-1, 4, 3, 3)
    if prec == gf.FP32:
        U = U.astype(np.complex64).astype(np.complex128)
    V = int(np.prod(dims))
    links = [(s, mu) for s in range(V) for mu in range(4)]
    got = gather(F, dims, prec, nc, links)
    want = np.stack([U[s, mu].reshape(9)[:nc] for s, mu in links])
    assert np.array_equal(got, want)


@pytest.mark.gpu
@pytest.mark.parametrize("dims,prec", [((128, 128, 256, 256), gf.FP32),
                                       ((128, 128, 128, 256), gf.FP64)])
def test_largest_lattice_sampled_parity(ctx, dims, prec):
    """One RED half-sweep (the built-in variant) at the largest volume the
    device holds; 256 sampled sites against the oracle, and the plaquette
    unchanged."""
    import torch
    geom = gf.Geom.make(dims, prec, gf.R12)
    need = gf.field_bytes(geom)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < need + (8 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} free")
    say("largest lattice", dims, "precision", prec, "field GiB", need / 2**30)
    F = ctx.empty_field(geom)
    try:
        inputs.gpu_config0_packed(F, dims, 4 if prec == gf.FP32 else 8, 6, 0.3, 9)
        V = int(np.prod(dims))
        rng = np.random.default_rng(9)
        cand = rng.choice(V, size=1024, replace=False)
        sites = [int(s) for s in cand if site_parity(dims, s) == 0 and s != V - 1][:255] + [V - 1]
        assert site_parity(dims, V - 1) == 0  # the last RED site: h = V/2 - 1
        links = sites_links(dims, sites)
        before = as_links(gather(F, dims, prec, 6, links))
        P0, P1 = ctx.empty_out(1), ctx.empty_out(1)
        ctx.plaquette(F, geom, P0)
        ctx.sweep(F, geom, gf.LANDAU, 0, 1.7)
        ctx.plaquette(F, geom, P1)
        after = gather(F, dims, prec, 6, links).reshape(-1, 2, 3)
        torch.cuda.synchronize()
        err = 0.0
        for k in range(len(sites)):
            want = oracle_site_update(before[8 * k:8 * k + 8], 1.7)[:, :2, :]
            err = max(err, np.abs(after[8 * k:8 * k + 8] - want).max())
        say("largest lattice max |diff|", err, "plaquette", P0.item(), P1.item())
        assert err <= TOL[prec], err
        assert P1.item() == pytest.approx(P0.item(), abs=1e-12 if prec == gf.FP64 else 1e-5)
    finally:
        del F
        torch.cuda.empty_cache()
