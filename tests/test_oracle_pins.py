"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, brute force on tiny inputs, invariants and
symmetries. They are chosen so that a plausible slip (a dropped term, a wrong
sign or index, a transposed operand, a wrong normalisation) fails at least one.
"""
import math
import os

import numpy as np
import pytest

import inputs
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
L, CLB = O.LANDAU, O.COULOMB


def haar_su2(rng, n):
    a = rng.normal(size=(n, 4))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    return a


def su2_matrix(a):
    """quaternion -> 2x2 matrix [[a0 + i a3, a2 + i a1], [-a2 + i a1, a0 - i a3]]"""
    a = np.atleast_2d(a)
    M = np.empty((a.shape[0], 2, 2), dtype=np.complex128)
    M[:, 0, 0] = a[:, 0] + 1j * a[:, 3]
    M[:, 0, 1] = a[:, 2] + 1j * a[:, 1]
    M[:, 1, 0] = -a[:, 2] + 1j * a[:, 1]
    M[:, 1, 1] = a[:, 0] - 1j * a[:, 3]
    return M


def embed(a, i, j):
    M2 = su2_matrix(a)
    G = np.tile(np.eye(3, dtype=np.complex128), (M2.shape[0], 1, 1))
    G[:, i, i], G[:, i, j], G[:, j, i], G[:, j, j] = M2[:, 0, 0], M2[:, 0, 1], M2[:, 1, 0], M2[:, 1, 1]
    return G


def site_parity(dims, s):
    nt, nz, ny, nx = dims
    x = s % nx
    y = (s // nx) % ny
    z = (s // (nx * ny)) % nz
    t = s // (nx * ny * nz)
    return (t + x + y + z) % 2


# ---------------------------------------------------------------------------
# Philox4x32-10: published known-answer vectors
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    n = 0
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        v = [int(w, 16) for w in line.split()]
        assert O.philox4x32(v[0:4], v[4:6]) == v[6:10]
        n += 1
    assert n == 3


# ---------------------------------------------------------------------------
# eq. (6): SU(2) local maximum, closed form and brute force
# ---------------------------------------------------------------------------

def test_local_solution_closed_form():
    """For a block of K^dag that is rho * SU(2), eq. (6) gives g = K^dag/sqrt(det K^dag)."""
    rng = np.random.default_rng(11)
    for _ in range(50):
        a = haar_su2(rng, 1)[0]
        rho = rng.uniform(0.1, 5.0)
        Kd = np.zeros((3, 3), dtype=np.complex128)
        Kd[np.ix_([0, 2], [0, 2])] = rho * su2_matrix(a)[0]
        Kd[1, 1] = rng.normal() + 1j * rng.normal()
        Kd[0, 1], Kd[1, 2] = rng.normal(), 1j * rng.normal()  # outside the (0,2) block
        q = O.su2_part(Kd, 0, 2)
        B = Kd[np.ix_([0, 2], [0, 2])]
        g_closed = B / np.sqrt(np.linalg.det(B))
        assert np.allclose(su2_matrix(q / np.linalg.norm(q))[0], g_closed, atol=1e-13)


@pytest.mark.parametrize("sg,ij", [(0, (0, 1)), (1, (0, 2)), (2, (1, 2))])
def test_local_maximum_brute_force(sg, ij):
    """On a 2^4 lattice, no sampled SU(2) element of subgroup (i,j) beats the
    normalised quaternion part of K(x)^dag for Re tr[g K(x)]; its value is 2|q|."""
    i, j = ij
    dims = (2, 2, 2, 2)
    U = inputs.config0(dims, 0.9, 5)
    rng = np.random.default_rng(100 + sg)
    H = embed(haar_su2(rng, 100_000), i, j)
    for s in range(0, 16, 3):
        K = O.local_K(U, L, s)
        q = O.su2_part(K.conj().T, i, j)
        G = embed(q / np.linalg.norm(q), i, j)[0]
        best = np.trace(G @ K).real
        assert best == pytest.approx(2 * np.linalg.norm(q) + np.trace(K).real
                                     - (K[i, i] + K[j, j]).real, abs=1e-12)
        sampled = np.einsum("nab,ba->n", H, K).real
        assert sampled.max() <= best + 1e-12
        assert sampled.max() > best - 0.05 * abs(best)  # sampling gets close


def test_relaxation_reaches_subgroup_stationarity():
    """After a relaxation (omega = 1) update of a site, the last subgroup (1,2)
    is at its maximum: the quaternion part of that block of K^dag is along 1."""
    dims = (4, 4, 4, 4)
    U = inputs.config0(dims, 0.5, 7)
    O.sweep(U, L, 0, 1.0)
    for s in range(0, 256, 17):
        if site_parity(dims, s) != 0:
            continue
        q = O.su2_part(O.local_K(U, L, s).conj().T, 1, 2)
        assert abs(q[1]) + abs(q[2]) + abs(q[3]) < 1e-12 * np.linalg.norm(q)
        assert q[0] > 0


# ---------------------------------------------------------------------------
# overrelaxation form g -> g^omega
# ---------------------------------------------------------------------------

def test_overrelax_relaxation_limit_and_norm():
    rng = np.random.default_rng(3)
    for _ in range(200):
        q = rng.normal(size=4) * rng.uniform(0.1, 10)
        s1 = O.overrelax(q, 1.0)
        assert np.array_equal(s1, q * (1.0 / math.sqrt(float(q @ q)))) or np.allclose(
            s1, q / np.linalg.norm(q), atol=1e-15)
        for w in (1.3, 1.7, 1.99):
            s = O.overrelax(q, w)
            assert np.linalg.norm(s) == pytest.approx(1.0, abs=1e-14)
            # never lowers the local functional: s.q >= 1.q = q0
            assert s @ q >= q[0] - 1e-12 * np.linalg.norm(q)
            # same rotation axis as the local maximum
            assert np.allclose(np.cross(s[1:], q[1:]), 0, atol=1e-12 * np.linalg.norm(q))
    assert O.overrelax(np.zeros(4), 1.7) is None


def test_overrelax_angle_closed_form():
    """For q = (cos phi, sin phi n): tan phi' = (1 + (omega-1) cos^2 phi) tan phi,
    hence phi'/phi -> omega as phi -> 0 (first-order overrelaxation)."""
    n = np.array([0.36, -0.48, 0.8])
    for w in (1.0, 1.5, 1.8):
        for phi in (1e-4, 0.01, 0.3, 1.0, 1.4):
            q = 2.5 * np.concatenate([[math.cos(phi)], math.sin(phi) * n])
            s = O.overrelax(q, w)
            phip = math.atan2(np.linalg.norm(s[1:]), s[0])
            assert math.tan(phip) == pytest.approx((1 + (w - 1) * math.cos(phi) ** 2)
                                                   * math.tan(phi), rel=1e-12)
        q = np.concatenate([[math.cos(1e-5)], math.sin(1e-5) * n])
        s = O.overrelax(q, w)
        assert math.atan2(np.linalg.norm(s[1:]), s[0]) / 1e-5 == pytest.approx(w, rel=1e-8)


def quat_of(M):
    """inverse of su2_matrix for one 2x2 matrix"""
    return np.array([M[0, 0].real, M[0, 1].imag, M[0, 1].real, M[0, 0].imag])


@pytest.mark.parametrize("form", [1, 2])
def test_overrelax_series_forms_from_matrix_algebra(form):
    """Forms 1 and 2 (Sec. 2: the power to first or second order): the binomial
    series of (1 + A)^omega, A = G - 1, truncated after the first or second
    order and projected onto SU(2), evaluated here with 2x2 complex matrices."""
    rng = np.random.default_rng(40 + form)
    I2 = np.eye(2)
    for _ in range(300):
        q = rng.normal(size=4) * rng.uniform(0.1, 10)
        w = rng.uniform(1.0, 2.0)
        G = su2_matrix(q / np.linalg.norm(q))[0]
        A = G - I2
        S = I2 + w * A
        if form == 2:
            S = S + 0.5 * w * (w - 1) * (A @ A)
        S = S / np.sqrt(np.linalg.det(S).real)
        assert np.allclose(O.overrelax_form(q, w, form), quat_of(S), atol=1e-13)


def test_overrelax_exact_power():
    """Form 3 is the principal power G^omega of the SU(2) matrix of g = q/|q|:
    the rotation angle times omega about the same axis."""
    from scipy.linalg import fractional_matrix_power
    rng = np.random.default_rng(44)
    for _ in range(200):
        q = rng.normal(size=4) * rng.uniform(0.1, 10)
        if q[0] < -0.95 * np.linalg.norm(q):
            continue  # principal branch ill-conditioned near G = -1
        w = rng.uniform(1.0, 2.0)
        G = su2_matrix(q / np.linalg.norm(q))[0]
        S = fractional_matrix_power(G, w)
        assert np.allclose(O.overrelax_form(q, w, 3), quat_of(S), atol=1e-10)
    n = np.array([0.36, -0.48, 0.8])
    for phi in (1e-6, 0.2, 1.1, 2.5):
        q = 3.0 * np.concatenate([[math.cos(phi)], math.sin(phi) * n])
        s = O.overrelax_form(q, 1.6, 3)
        assert s[0] == pytest.approx(math.cos(1.6 * phi), abs=1e-14)
        assert np.allclose(s[1:], math.sin(1.6 * phi) * n, atol=1e-14)


def test_overrelax_forms_limits_and_monotone():
    rng = np.random.default_rng(45)
    for _ in range(200):
        q = rng.normal(size=4) * rng.uniform(0.1, 10)
        g = q / np.linalg.norm(q)
        assert np.array_equal(O.overrelax_form(q, 1.7, 0), O.overrelax(q, 1.7))
        for form in (1, 2, 3):
            assert np.allclose(O.overrelax_form(q, 1.0, form), g, atol=1e-15)
            for w in (1.3, 1.7, 1.99):
                s = O.overrelax_form(q, w, form)
                assert np.linalg.norm(s) == pytest.approx(1.0, abs=1e-14)
                assert s @ g >= g[0] - 1e-12  # local functional not lowered
                assert np.allclose(np.cross(s[1:], g[1:]), 0, atol=1e-12)
    assert O.overrelax_form(np.zeros(4), 1.7, 2) is None
    assert O.overrelax_form(np.ones(4), 1.7, 4) is None
    assert np.array_equal(O.overrelax_form(np.array([-2.0, 0, 0, 0]), 1.7, 3), [-1.0, 0, 0, 0])


@pytest.mark.parametrize("form", [1, 2, 3])
def test_sweep_forms_monotone_and_pure_gauge(form):
    dims = (4, 4, 4, 6)
    U = inputs.config0(dims, 0.6, 21)
    A = U.copy()
    O.sweep_form(A, L, 0, 1.7, 0)
    B = U.copy()
    O.sweep(B, L, 0, 1.7)
    assert np.array_equal(A, B)
    P0 = O.plaquette(U)
    for gauge in (L, CLB):
        W = U.copy()
        F_prev = O.functional(W, gauge)[1]
        for k in range(10):
            O.sweep_form(W, gauge, k % 2, 1.7, form)
            F = O.functional(W, gauge)[1]
            assert np.all(F >= F_prev - 1e-14), (k, F - F_prev)
            F_prev = F
        assert abs(O.plaquette(W) - P0) < 1e-13
        assert unitarity_dev(W) < 1e-13
    P = inputs.pure_gauge((4, 4, 4, 4), 5)
    r = O.fix(P, L, 1.7, 1e-24, 3000, check_every=20, form=form)
    assert r["converged"] and abs(r["F"] - 1.0) < 1e-12
    with pytest.raises(ValueError):
        O.sweep_form(U.copy(), L, 0, 1.7, 5)


# ---------------------------------------------------------------------------
# sweep invariants
# ---------------------------------------------------------------------------

def unitarity_dev(U):
    M = U.reshape(-1, 3, 3)
    d1 = np.abs(M @ M.conj().transpose(0, 2, 1) - np.eye(3)).max()
    d2 = np.abs(np.linalg.det(M) - 1).max()
    return max(d1, d2)


@pytest.mark.parametrize("omega", [1.0, 1.7])
@pytest.mark.parametrize("gauge", [L, CLB])
def test_functional_monotone_plaquette_unitarity(omega, gauge):
    dims = (4, 4, 4, 6) if gauge == L else (4, 4, 6, 4)
    U = inputs.config0(dims, 0.6, 21)
    P0 = O.plaquette(U)
    F_prev = O.functional(U, gauge)[1]
    for k in range(12):
        O.sweep(U, gauge, k % 2, omega)
        F = O.functional(U, gauge)[1]
        assert np.all(F >= F_prev - 1e-14), (k, F - F_prev)
        F_prev = F
    assert abs(O.plaquette(U) - P0) < 1e-13
    assert unitarity_dev(U) < 1e-13


def test_unit_field_is_fixed_point():
    dims = (4, 2, 4, 2)
    U = inputs.unit_field(dims)
    for p in (0, 1, 0, 1):
        O.sweep(U, L, p, 1.7)
    assert np.array_equal(U, inputs.unit_field(dims))
    assert O.functional(U, L)[0] == 1.0
    assert O.theta_K(U, L)[0] == 0.0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pure_gauge_reaches_global_maximum(seed):
    """U_mu(x) = h(x) h(x+mu)^dag is a gauge transform of U = 1: the maximum
    F = 1 with theta = 0 is known."""
    dims = (4, 4, 4, 4)
    U = inputs.pure_gauge(dims, seed)
    r = O.fix(U, L, 1.7, 1e-24, 3000, check_every=20)
    assert r["converged"], r
    assert abs(r["F"] - 1.0) < 1e-12
    assert O.theta_A(U, L)[0] < 1e-24


def test_pure_gauge_coulomb_every_timeslice():
    dims = (4, 4, 4, 4)
    U = inputs.pure_gauge(dims, 9)
    r = O.fix(U, CLB, 1.7, 1e-24, 3000, check_every=20)
    assert r["converged"]
    F, Ft = O.functional(U, CLB)
    th, tht = O.theta_K(U, CLB)
    assert np.all(np.abs(Ft - 1) < 1e-12) and np.all(tht < 1e-24)


# ---------------------------------------------------------------------------
# F and theta: closed forms and identities
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mu", [0, 1, 2, 3])
def test_single_link_closed_form(mu):
    """One link U = diag(e^{i e}, e^{-i e}, 1) in a unit field:
    A = diag(sin e, -sin e, 0) at both ends with opposite signs, so
    theta = 2 * 2 sin^2(e) / (3 V) and F = 1 - (2 - 2 cos e)/(12 V)."""
    dims = (4, 4, 6, 2)
    nt, nz, ny, nx = dims
    V = nt * nz * ny * nx
    e = 0.37
    U = inputs.unit_field(dims)
    t0, z0, y0, x0 = 1, 2, 3, 1
    U[t0, z0, y0, x0, mu] = np.diag([np.exp(1j * e), np.exp(-1j * e), 1.0])
    thA, thK = O.theta_A(U, L)[0], O.theta_K(U, L)[0]
    want = 4 * math.sin(e) ** 2 / (3 * V)
    assert thA == pytest.approx(want, rel=1e-13)
    assert thK == pytest.approx(want, rel=1e-13)
    assert O.functional(U, L)[0] == pytest.approx(1 - (2 - 2 * math.cos(e)) / (12 * V), rel=1e-15)
    assert O.functional_raw(U, L) == pytest.approx(12 * V - 2 + 2 * math.cos(e), rel=1e-15)
    # Coulomb: only spatial links count, per timeslice
    Vs = V // nt
    thc = O.theta_K(U, CLB)[1]
    Fc = O.functional(U, CLB)[1]
    for t in range(nt):
        if mu != 0 and t == t0:
            assert thc[t] == pytest.approx(4 * math.sin(e) ** 2 / (3 * Vs), rel=1e-13)
            assert Fc[t] == pytest.approx(1 - (2 - 2 * math.cos(e)) / (9 * Vs), rel=1e-15)
        else:
            assert thc[t] == 0.0 and Fc[t] == 1.0


def test_theta_two_formulas_agree():
    for dims, gauge in [((4, 4, 4, 4), L), ((6, 4, 2, 4), L), ((4, 4, 4, 6), CLB)]:
        U = inputs.config0(dims, 0.8, 4)
        a, aa = O.theta_A(U, gauge)
        k, kk = O.theta_K(U, gauge)
        assert a == pytest.approx(k, rel=1e-13)
        assert np.allclose(aa, kk, rtol=1e-13)
        assert a > 0


# ---------------------------------------------------------------------------
# indexing: translation covariance
# ---------------------------------------------------------------------------

def test_shift_covariance():
    dims = (4, 4, 6, 4)
    U = inputs.config0(dims, 0.7, 8)
    axes = {0: 0, 1: 3, 2: 2, 3: 1}  # direction -> array axis (t, x, y, z)
    for mu, ax in axes.items():
        # shift by 2: same sublattice, the sweep commutes bitwise
        A = np.ascontiguousarray(np.roll(U, 2, axis=ax))
        B = U.copy()
        O.sweep(A, L, 0, 1.7)
        O.sweep(B, L, 0, 1.7)
        assert np.array_equal(A, np.roll(B, 2, axis=ax))
        # shift by 1 swaps RED and BLACK
        A = np.ascontiguousarray(np.roll(U, 1, axis=ax))
        B = U.copy()
        O.sweep(A, L, 1, 1.7)
        O.sweep(B, L, 0, 1.7)
        assert np.array_equal(A, np.roll(B, 1, axis=ax))


def test_coulomb_timeslices_are_independent():
    """Coulomb sweeps of timeslice t use spatial links of t only: changing the
    spatial links of another timeslice leaves them unchanged bitwise."""
    dims = (4, 4, 4, 4)
    U = inputs.config0(dims, 0.7, 12)
    W = U.copy()
    W[2, :, :, :, 1:] = inputs.config0(dims, 0.7, 99)[2, :, :, :, 1:]
    for p in (0, 1, 0, 1):
        O.sweep(U, CLB, p, 1.7)
        O.sweep(W, CLB, p, 1.7)
    for t in (0, 1, 3):
        assert np.array_equal(U[t, ..., 1:, :, :], W[t, ..., 1:, :, :])


def test_results_independent_of_thread_count():
    dims = (4, 4, 4, 4)
    U0 = inputs.config0(dims, 0.7, 13)
    out = []
    nthr = O.num_threads()
    for n in (1, max(2, nthr)):
        O.set_num_threads(n)
        U = U0.copy()
        O.sweep(U, L, 0, 1.7)
        O.sweep(U, L, 1, 1.7)
        out.append((U, O.theta_K(U, L)[0], O.functional(U, L)[0]))
    O.set_num_threads(nthr)
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]


# ---------------------------------------------------------------------------
# reunitarisation
# ---------------------------------------------------------------------------

def test_reunitarize():
    U = inputs.config0((2, 2, 2, 2), 0.5, 3)
    V = U.copy()
    O.reunitarize(V)
    assert np.abs(V - U).max() < 1e-14  # SU(3) is (numerically) a fixed point
    rng = np.random.default_rng(5)
    W = U + 1e-3 * (rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape))
    O.reunitarize(W)
    assert unitarity_dev(W) < 1e-14
    assert np.abs(W - U).max() < 1e-2
    # Gram-Schmidt keeps the direction of row 0 and the span of rows 0, 1
    M = (rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3)))
    X = np.zeros((1, 1, 1, 1, 4, 3, 3), dtype=np.complex128)
    X[..., :, :] = M
    O.reunitarize(X)
    R = X.reshape(-1, 3, 3)[0]
    assert np.allclose(R[0], M[0] / np.linalg.norm(M[0]), atol=1e-14)
    r1 = M[1] - (M[0].conj() @ M[1]) / (M[0].conj() @ M[0]) * M[0]
    assert np.allclose(R[1], r1 / np.linalg.norm(r1), atol=1e-13)
    assert abs(np.linalg.det(R) - 1) < 1e-14


def test_gauge_transform_and_plaquette():
    dims = (4, 2, 4, 2)
    U = inputs.config0(dims, 0.7, 14)
    P = O.plaquette(U)
    g = inputs.haar_sites(dims, 77)
    O.gauge_transform(U, g)
    assert O.plaquette(U) == pytest.approx(P, abs=1e-14)
    assert O.plaquette(inputs.unit_field(dims)) == 1.0


# ---------------------------------------------------------------------------
# argument checks
# ---------------------------------------------------------------------------

def test_argument_errors():
    assert O.check_dims((4, 4, 4, 4)) == 0
    for bad in [(3, 4, 4, 4), (4, 4, 4, 5), (0, 4, 4, 4), (4, 4, 1, 4)]:
        assert O.check_dims(bad) == -1
    U = inputs.unit_field((2, 2, 2, 2))
    for w in (0.99, 2.0, float("nan")):
        with pytest.raises(ValueError):
            O.sweep(U, L, 0, w)
    with pytest.raises(ValueError):
        O.sweep(U, L, 2, 1.5)
    with pytest.raises(ValueError):
        O.heatbath_half(U, L, 0, 0.0, 1, 0)
    with pytest.raises(ValueError):
        O.heatbath_half(U, L, 0, -1.0, 1, 0)


def test_vanishing_subgroup_parts_are_skipped():
    """Every link the cyclic permutation P (det 1): K is proportional to P + P^T,
    whose three SU(2) parts vanish, so each subgroup is skipped and the field
    is a stationary point with F = 0 and theta = 0 (not a maximum)."""
    dims = (4, 2, 4, 2)
    P = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], dtype=np.complex128)
    U = np.ascontiguousarray(np.broadcast_to(P, tuple(dims) + (4, 3, 3)))
    for gauge in (L, CLB):
        W = U.copy()
        for p in (0, 1):
            O.sweep(W, gauge, p, 1.7)
        assert np.array_equal(W, U)
        assert O.functional(W, gauge)[0] == 0.0
        assert O.theta_K(W, gauge)[0] == 0.0
    r = O.fix(U.copy(), L, 1.7, 1e-12, 100)
    assert r["converged"] and r["sweeps"] == 0 and r["F"] == 0.0


def test_coulomb_frozen_driver():
    """Coulomb timeslices are independent problems; freezing each one once
    its theta_t is below the target (i) changes nothing while none is frozen,
    (ii) leaves a frozen timeslice's spatial links exactly as they were at
    its freeze, (iii) still yields a gauge transform of the input with every
    theta_t below the target."""
    dims = (6, 4, 4, 6)
    U = inputs.config0(dims, 0.5, 31)
    # (i) target 0: nothing freezes, identical to the plain driver
    A, B = U.copy(), U.copy()
    ra = O.fix_coulomb_frozen(A, 1.7, 0.0, 60, check_every=20)
    rb = O.fix(B, CLB, 1.7, 0.0, 60, check_every=20)
    assert not ra["converged"] and ra["sweeps"] == rb["sweeps"] == 60
    assert np.array_equal(A, B)
    assert np.all(ra["frozen_at"] == -1)
    # (iii) converged run
    target = 1e-12
    C = U.copy()
    rc = O.fix_coulomb_frozen(C, 1.7, target, 4000, check_every=20, reunit_at_check=0)
    assert rc["converged"] and np.all(rc["theta"] < target)
    assert np.all(rc["frozen_at"] >= 0)
    assert len(set(rc["frozen_at"].tolist())) > 1  # timeslices converge at different times
    assert abs(O.plaquette(C) - O.plaquette(U)) < 1e-13
    M = C.reshape(-1, 3, 3)
    assert np.abs(M @ M.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-12
    # (ii) spatial links of each timeslice as at its freeze (no reunitarisation)
    for t in np.unique(rc["frozen_at"]):
        D = U.copy()
        O.fix_coulomb_frozen(D, 1.7, target, int(t), check_every=20, reunit_at_check=0)
        for ts in np.nonzero(rc["frozen_at"] == t)[0]:
            assert np.array_equal(C[ts, :, :, :, 1:], D[ts, :, :, :, 1:])


def test_unitarity_deviation():
    """or_unitarity against closed forms: 0 for SU(3) links (to rounding) and
    for a U(3) phase, 2d + d^2 for a row scaled by 1 + d, |e| for row 1 tilted
    by e times row 0, +inf for a NaN."""
    dims = (2, 2, 2, 4)
    U = inputs.config0(dims, 0.4, 9)
    assert O.unitarity(U) < 1e-14
    V = U.copy()
    V[1, 0, 1, 2, 3] *= np.exp(0.7j)  # a phase keeps U U^dag = 1
    assert O.unitarity(V) < 1e-14
    d = 3e-4
    V = U.copy()
    V[0, 1, 0, 3, 2, 0, :] *= 1 + d
    assert O.unitarity(V) == pytest.approx(2 * d + d * d, rel=1e-9)
    e = 2e-5 - 1e-5j
    V = U.copy()
    link = V[1, 1, 1, 1, 0]
    link[1, :] = link[1, :] + e * link[0, :]
    # (U U^dag)_10 = e <row0, row0> = e; (U U^dag)_11 = 1 + |e|^2
    assert O.unitarity(V) == pytest.approx(abs(e), rel=1e-6)
    V = U.copy()
    V[0, 0, 0, 0, 2, 1, 1] = np.nan
    assert O.unitarity(V) == math.inf
