"""Pins of the oracle's maximally Abelian gauge (named in Sec. 1 and the
summary; the functional R = sum_{x,mu} sum_k |U_mu(x)_kk|^2 is the standard
one from the literature, the paper does not write it out)."""
import math

import numpy as np
import pytest

import inputs
import oracle as O

SG = [(0, 1), (0, 2), (1, 2)]


def su2(a):
    return np.array([[a[0] + 1j * a[3], a[2] + 1j * a[1]],
                     [-a[2] + 1j * a[1], a[0] - 1j * a[3]]])


def embed(a, i, j):
    G = np.eye(3, dtype=np.complex128)
    B = su2(a)
    G[i, i], G[i, j], G[j, i], G[j, j] = B[0, 0], B[0, 1], B[1, 0], B[1, 1]
    return G


def quat_of(M):
    return np.array([M[0, 0].real, M[0, 1].imag, M[0, 1].real, M[0, 0].imag])


def coords(dims, s):
    nt, nz, ny, nx = dims
    return [s // (nx * ny * nz), s % nx, (s // nx) % ny, (s // (nx * ny)) % nz]  # t, x, y, z


def back(dims, s, mu):
    nt, nz, ny, nx = dims
    t, x, y, z = coords(dims, s)
    c = [t, x, y, z]
    e = [nt, nx, ny, nz]
    c[mu] = (c[mu] - 1) % e[mu]
    t, x, y, z = c
    return ((t * nz + z) * ny + y) * nx + x


def local_R(U, s, a, i, j):
    """R of the 8 links at s after G = embed(a), with full 3x3 products"""
    dims = U.shape[:4]
    Uf = U.reshape(-1, 4, 3, 3)
    G = embed(a, i, j)
    R = 0.0
    for mu in range(4):
        A = G @ Uf[s, mu]
        B = Uf[back(dims, s, mu), mu] @ G.conj().T
        R += np.sum(np.abs(np.diag(A)) ** 2) + np.sum(np.abs(np.diag(B)) ** 2)
    return R


def test_mag_matrix_is_the_quadratic_form():
    dims = (4, 4, 4, 6)
    U = inputs.config0(dims, 0.6, 81)
    rng = np.random.default_rng(81)
    for s in rng.integers(0, U.size // 36, size=6):
        for sg, (i, j) in enumerate(SG):
            M = O.mag_matrix(U, s, sg)
            assert np.allclose(M, M.T, atol=0)
            C = local_R(U, s, np.zeros(4), i, j)
            for _ in range(5):
                a = rng.normal(size=4) * 2
                assert local_R(U, s, a, i, j) == pytest.approx(a @ M @ a + C, abs=1e-12)
            # the diagonal phases of the subgroup are a symmetry of R
            a = rng.normal(size=4)
            a /= np.linalg.norm(a)
            d = np.array([math.cos(0.7), 0, 0, math.sin(0.7)])
            da = quat_of(su2(d) @ su2(a))
            assert local_R(U, s, da, i, j) == pytest.approx(local_R(U, s, a, i, j), abs=1e-12)
            assert M[0, 3] == pytest.approx(0, abs=1e-12)


def test_mag_local_max_is_the_top_eigenvector_and_beats_sampling():
    dims = (4, 4, 4, 4)
    U = inputs.config0(dims, 0.8, 82)
    rng = np.random.default_rng(82)
    samples = rng.normal(size=(100000, 4))
    samples /= np.linalg.norm(samples, axis=1, keepdims=True)
    for s in (0, 37, 200):
        for sg, (i, j) in enumerate(SG):
            M = O.mag_matrix(U, s, sg)
            a = O.mag_local_max(U, s, sg)
            assert np.linalg.norm(a) == pytest.approx(1, abs=1e-14)
            assert a[3] == 0 and a[0] >= 0
            lam = np.linalg.eigh(M)[0][-1]
            assert a @ M @ a == pytest.approx(lam, rel=1e-12, abs=1e-12)
            best = np.max(np.einsum("nk,kl,nl->n", samples, M, samples))
            assert best <= lam + 1e-12
            assert best >= lam - 0.05 * (abs(lam) + 1)


@pytest.mark.parametrize("psi", [0.0, math.pi / 2, 0.9])
@pytest.mark.parametrize("sg", [0, 1, 2])
def test_mag_single_link_closed_form(sg, psi):
    """Unit field with one link rotated by (cos e, sin e cos psi, sin e sin psi, 0)
    in one subgroup: F = 1 - 2 sin^2(e) / (12 V), theta = 2 sin^2(2e) / (3 V)
    (M_01 or M_02 = -+sin(2e) at the two sites of the link, by hand)."""
    dims = (4, 4, 2, 6)
    V = 4 * 4 * 2 * 6
    e = 0.23
    U = inputs.unit_field(dims)
    i, j = SG[sg]
    U[1, 2, 1, 3, 2] = embed([math.cos(e), math.sin(e) * math.cos(psi),
                              math.sin(e) * math.sin(psi), 0], i, j)
    assert O.mag_functional(U) == pytest.approx(1 - 2 * math.sin(e) ** 2 / (12 * V), rel=1e-15)
    assert O.mag_theta(U) == pytest.approx(2 * math.sin(2 * e) ** 2 / (3 * V), rel=1e-12)
    U = inputs.unit_field(dims)
    assert O.mag_functional(U) == 1.0 and O.mag_theta(U) == 0.0


@pytest.mark.parametrize("omega,form", [(1.0, 0), (1.7, 0), (1.7, 3), (1.9, 2)])
def test_mag_sweep_monotone_and_invariants(omega, form):
    dims = (4, 4, 4, 6)
    U = inputs.config0(dims, 0.6, 83)
    P0 = O.plaquette(U)
    F_prev = O.mag_functional(U)
    for k in range(10):
        O.mag_sweep(U, k % 2, omega, form)
        F = O.mag_functional(U)
        assert F >= F_prev - 1e-14, (k, F - F_prev)
        F_prev = F
    assert abs(O.plaquette(U) - P0) < 1e-13
    M = U.reshape(-1, 3, 3)
    assert np.abs(M @ M.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-13


@pytest.mark.parametrize("seed", [1, 2])
def test_mag_abelian_copy_reaches_global_maximum(seed):
    """A gauge copy of a diagonal field: the maximum F = 1, theta = 0 is known."""
    U = inputs.abelian_gauge((4, 4, 4, 4), seed, eps=0.3)
    assert O.mag_functional(U) < 0.9
    r = O.fix_mag(U, 1.7, 1e-24, 2000, check_every=20)
    assert r["converged"]
    assert abs(r["F"] - 1.0) < 1e-12
    assert np.abs(U[..., [0, 0, 1, 1, 2, 2], [1, 2, 0, 2, 0, 1]]).max() < 1e-10


def test_mag_fixed_point_local_maxima_are_identity():
    dims = (4, 4, 4, 4)
    U = inputs.config0(dims, 0.5, 84)
    r = O.fix_mag(U, 1.7, 1e-26, 3000, check_every=50)
    assert r["converged"]
    for s in (0, 11, 100):
        for sg in range(3):
            a = O.mag_local_max(U, s, sg)
            assert np.abs(a - [1, 0, 0, 0]).max() < 1e-10


def test_mag_argument_errors():
    U = inputs.config0((4, 4, 4, 4), 0.5, 1)
    for bad in [(2, 1.7, 0), (0, 2.0, 0), (0, 1.7, 4)]:
        with pytest.raises(ValueError):
            O.mag_sweep(U, *bad)


def test_mag_site_gaps_first_step_against_eigh():
    """The gap of the first subgroup step is that of the 3x3 block of M at the
    input (numpy eigh); later steps are taken on the updated links."""
    dims = (4, 4, 2, 6)
    U = inputs.config0(dims, 0.6, 77)
    for s in (0, 5, 17, 40):
        g = O.mag_site_gaps(U, s, 1.0)
        ev = np.linalg.eigvalsh(O.mag_matrix(U, s, 0)[:3, :3])
        assert g[0] == pytest.approx((ev[2] - ev[1]) / abs(ev[2]), rel=1e-9, abs=1e-14)
        assert np.all(g >= 0) and np.all(g <= 2)
    # the field is not changed
    V = inputs.config0(dims, 0.6, 77)
    assert np.array_equal(U, V)
