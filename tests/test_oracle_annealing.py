"""Pins of the oracle's simulated-annealing pieces (heatbath + microcanonical).

The annealing algorithm is not spelled out in the paper (it is named as a
preconditioner in Sec. 1). The reading pinned here: weight exp(Re tr[g K]/T)
per SU(2) subgroup, Kennedy-Pendleton sampling from Philox draws, and
microcanonical reflections g = ghat^2.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import inputs
import oracle as O

L, CLB = O.LANDAU, O.COULOMB


def kp_cdf(alpha, x):
    """CDF of the density ~ sqrt(1 - t^2) exp(alpha (t - 1)) on [-1, 1]."""
    f = lambda t: math.sqrt(max(0.0, 1 - t * t)) * math.exp(alpha * (t - 1))
    tot = integrate.quad(f, -1, 1, limit=200, points=[1 - 1e-3])[0]
    return integrate.quad(f, -1, x, limit=200)[0] / tot


@pytest.mark.parametrize("alpha", [0.5, 2.0, 10.0, 60.0])
def test_kp_mean_and_histogram(alpha):
    n = 20000
    x = np.empty(n)
    for k in range(n):
        v, att = O.kp_draw(alpha, 1234, k, 7, 1)
        assert att > 0
        x[k] = v
    # <X0> = I_2(alpha) / I_1(alpha) for density ~ sqrt(1 - x^2) exp(alpha x)
    mean = special.iv(2, alpha) / special.iv(1, alpha)
    assert abs(x.mean() - mean) < 5 * x.std() / math.sqrt(n)
    # goodness of fit on 20 equiprobable-ish bins
    qs = np.quantile(x, np.linspace(0, 1, 21))
    qs[0], qs[-1] = -1.0, 1.0
    cdf = np.array([kp_cdf(alpha, q) for q in qs])
    expected = np.diff(cdf) * n
    observed = np.histogram(x, bins=qs)[0]
    chi2 = ((observed - expected) ** 2 / expected).sum()
    assert stats.chi2.sf(chi2, df=19) > 1e-4


def test_heatbath_su2_direction_isotropic():
    n = 20000
    X = np.array([O.heatbath_su2(3.0, 99, k, 1, 2)[0] for k in range(n)])
    assert np.allclose(np.linalg.norm(X, axis=1), 1.0, atol=1e-14)
    v = X[:, 1:]
    se = 1.0 / math.sqrt(n)
    assert np.all(np.abs(v.mean(axis=0)) < 5 * se)
    m2 = (v ** 2).mean(axis=0)
    want = (1 - (X[:, 0] ** 2).mean()) / 3
    assert np.all(np.abs(m2 - want) < 0.05 * want)
    # off-diagonal second moments vanish
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs((v[:, a] * v[:, b]).mean()) < 5 * se * math.sqrt(want)


def test_draws_depend_on_every_counter_field():
    base = O.heatbath_su2(2.0, 5, 10, 3, 1)[0]
    for args in [(6, 10, 3, 1), (5, 11, 3, 1), (5, 10, 4, 1), (5, 10, 3, 2),
                 ((1 << 32) + 5, 10, 3, 1)]:
        assert not np.array_equal(O.heatbath_su2(2.0, *args)[0], base)
    assert np.array_equal(O.heatbath_su2(2.0, 5, 10, 3, 1)[0], base)


def test_lattice_heatbath_local_distribution():
    """After a heatbath half-sweep, at each updated site the last subgroup
    (1,2) has q'0/|q'| = X0 distributed with density ~ sqrt(1-x^2) exp(alpha x),
    alpha = 2|q'|/T (|q'| = |q| since the update is unitary): the probability
    integral transform must be uniform."""
    dims = (8, 4, 4, 8)
    U = inputs.config0(dims, 0.6, 31)
    T = 0.9
    O.heatbath_half(U, L, 0, T, seed=17, sweep=3)
    nt, nz, ny, nx = dims
    pit = []
    for s in range(nt * nz * ny * nx):
        x = s % nx
        y = (s // nx) % ny
        z = (s // (nx * ny)) % nz
        t = s // (nx * ny * nz)
        if (t + x + y + z) % 2:
            continue
        q = O.su2_part(O.local_K(U, L, s).conj().T, 1, 2)
        nq = np.linalg.norm(q)
        pit.append(kp_cdf(2 * nq / T, q[0] / nq))
    assert len(pit) == 512
    assert stats.kstest(pit, "uniform").pvalue > 1e-3


@pytest.mark.parametrize("gauge", [L, CLB])
def test_microcanonical_conserves_functional(gauge):
    dims = (4, 4, 4, 4)
    U = inputs.config0(dims, 0.6, 41)
    F0 = O.functional(U, gauge)[1]
    U0 = U.copy()
    for p in (0, 1, 0, 1):
        O.micro_half(U, gauge, p)
    assert np.allclose(O.functional(U, gauge)[1], F0, rtol=0, atol=1e-14)
    assert np.abs(U - U0).max() > 1e-2  # it does move the field
    assert O.plaquette(U) == pytest.approx(O.plaquette(U0), abs=1e-13)


def test_heatbath_cold_limit_is_relaxation():
    """T -> 0: the heatbath draw concentrates on the local maximum (omega = 1)."""
    dims = (4, 4, 4, 4)
    U = inputs.config0(dims, 0.6, 42)
    A, B = U.copy(), U.copy()
    capped = O.heatbath_half(A, L, 0, 1e-9, seed=3, sweep=0)
    O.sweep(B, L, 0, 1.0)
    assert capped == 0
    d = np.abs(A - B).max()
    assert d < 1e-3 and d > 0


def test_heatbath_hot_disorders_unit_field():
    """A hot anneal drives the unit field (F = 1) far from the maximum."""
    dims = (4, 4, 4, 4)
    U = inputs.unit_field(dims)
    capped = 0
    for k in range(10):
        capped += O.anneal_sweep(U, L, 4.0, seed=8, sweep=k, n_micro=1)
    assert capped == 0
    assert O.functional(U, L)[0] < 0.5
    M = U.reshape(-1, 3, 3)
    assert np.abs(M @ M.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-13
    assert O.plaquette(U) == pytest.approx(1.0, abs=1e-13)  # still pure gauge


def test_anneal_resume_is_exact_and_seeded():
    """Draws are keyed by the sweep index, so k sweeps then m more equal k + m."""
    dims = (4, 2, 4, 2)
    U0 = inputs.config0(dims, 0.6, 43)
    A = U0.copy()
    for k in range(4):
        O.anneal_sweep(A, CLB, 1.0 - 0.2 * k, seed=5, sweep=k, n_micro=3)
    B = U0.copy()
    for k in range(2):
        O.anneal_sweep(B, CLB, 1.0 - 0.2 * k, seed=5, sweep=k, n_micro=3)
    B = B.copy()  # "checkpoint"
    for k in range(2, 4):
        O.anneal_sweep(B, CLB, 1.0 - 0.2 * k, seed=5, sweep=k, n_micro=3)
    assert np.array_equal(A, B)
    C = U0.copy()
    for k in range(4):
        O.anneal_sweep(C, CLB, 1.0 - 0.2 * k, seed=6, sweep=k, n_micro=3)
    assert not np.array_equal(A, C)


# ---------------------------------------------------------------------------
# stochastic relaxation (Sec. 1; tuned against overrelaxation in Fig. 2)
# ---------------------------------------------------------------------------

def test_stochastic_relaxation_limits():
    """p = 0 is (over)relaxation and p = 1 the microcanonical step, bit for bit."""
    dims = (4, 4, 6, 4)
    U = inputs.config0(dims, 0.6, 51)
    for gauge in (L, CLB):
        A, B = U.copy(), U.copy()
        O.sweep_sr(A, gauge, 0, 1.7, 0.0, 9, 3)
        O.sweep(B, gauge, 0, 1.7)
        assert np.array_equal(A, B)
        A, B = U.copy(), U.copy()
        O.sweep_sr(A, gauge, 1, 1.3, 1.0, 9, 3)
        O.micro_half(B, gauge, 1)
        assert np.array_equal(A, B)


def test_stochastic_relaxation_monotone_and_mixed():
    """Neither branch lowers the local functional, so F never decreases; an
    intermediate p gives a field different from both limits."""
    dims = (4, 4, 4, 4)
    U = inputs.config0(dims, 0.6, 52)
    F = O.functional(U, L)[0]
    W = U.copy()
    for k in range(10):
        O.sweep_sr(W, L, k % 2, 1.0, 0.3, 5, k // 2)
        F2 = O.functional(W, L)[0]
        assert F2 >= F - 1e-14
        F = F2
    A, B, C = U.copy(), U.copy(), U.copy()
    O.sweep_sr(A, L, 0, 1.0, 0.3, 5, 0)
    O.sweep(B, L, 0, 1.0)
    O.micro_half(C, L, 0)
    assert not np.array_equal(A, B) and not np.array_equal(A, C)
    with pytest.raises(ValueError):
        O.sweep_sr(U.copy(), L, 0, 1.0, 1.5, 5, 0)


def _su3_checks(g, tol=1e-13):
    eye = np.eye(3)
    gg = np.einsum("...ab,...cb->...ac", g, g.conj())
    assert np.abs(gg - eye).max() < tol
    assert np.abs(np.linalg.det(g) - 1).max() < tol


@pytest.mark.parametrize("kind,param", [(O.OR, 0.0), (O.HEATBATH, 0.8), (O.MICRO, 0.0),
                                        (O.SR, 0.5)])
@pytest.mark.parametrize("gauge", [L, CLB])
def test_half_sweep_g_is_the_site_transformation(kind, param, gauge):
    """The g that half_sweep_g reports, applied to the input by eq. (4),
    reproduces the half-sweep; it is in SU(3), and 1 at the other parity."""
    dims = (4, 2, 4, 6)
    U0 = inputs.config0(dims, 0.5, 21)
    for parity in (0, 1):
        U = U0.copy()
        g = O.half_sweep_g(U, gauge, parity, kind, omega=1.6, param=param, seed=3, sweep=11)
        _su3_checks(g)
        t, z, y, x = np.indices(dims)
        other = (t + z + y + x) % 2 != parity
        assert np.array_equal(g[other], np.broadcast_to(np.eye(3), g[other].shape))
        V = U0.copy()
        O.gauge_transform(V, g)
        assert np.abs(V - U).max() < 1e-13
        # the field it leaves is the plain half-sweep's, bit for bit
        W = U0.copy()
        if kind == O.OR:
            O.sweep(W, gauge, parity, 1.6)
        elif kind == O.HEATBATH:
            O.heatbath_half(W, gauge, parity, param, 3, 11)
        elif kind == O.MICRO:
            O.micro_half(W, gauge, parity)
        else:
            O.sweep_sr(W, gauge, parity, 1.6, param, 3, 11)
        assert np.array_equal(W, U)


def _site_links(U, s):
    dims = U.shape[:4]
    t, z, y, x = np.unravel_index(s, dims)
    c = [t, x, y, z]
    ext = [dims[0], dims[3], dims[2], dims[1]]
    f = [U[t, z, y, x, mu] for mu in range(4)]
    b = []
    for mu in range(4):
        d = list(c)
        d[mu] = (d[mu] - 1) % ext[mu]
        b.append(U[d[0], d[3], d[2], d[1], mu])
    return np.array(f + b)


@pytest.mark.parametrize("gauge", [L, CLB])
def test_heatbath_outcomes(gauge):
    """Outcome 0 is the exact update; tau = 0 leaves it alone; every other
    outcome is still a transformation by eq. (4) at the site, with an SU(3)
    factor, and the smallest margin separates one outcome from two."""
    dims = (4, 4, 4, 4)
    U0 = inputs.config0(dims, 0.7, 5)
    T, seed, sweep = 1.1, 17, 4
    many = 0
    for s in range(0, 256, 5):
        if sum(np.unravel_index(s, dims)) % 2:
            continue
        ref = U0.copy()
        O.heatbath_sites(ref, gauge, T, seed, sweep, [s])
        exact = _site_links(ref, s)
        outs, mm = O.heatbath_site_outcomes(U0, gauge, T, seed, sweep, s, 0.0)
        assert len(outs) == 1 and np.array_equal(outs[0], exact)
        assert mm > 0
        outs, _ = O.heatbath_site_outcomes(U0, gauge, T, seed, sweep, s, 0.5, max_out=64)
        assert np.array_equal(outs[0], exact)
        old = _site_links(U0, s)
        for o in outs:
            h = o[0] @ old[0].conj().T
            _su3_checks(h[None], tol=1e-12)
            for mu in range(4):
                assert np.abs(o[mu] - h @ old[mu]).max() < 1e-12
                assert np.abs(o[4 + mu] - old[4 + mu] @ h.conj().T).max() < 1e-12
        many += len(outs) > 1
        if len(outs) > 1:
            n_lo = len(O.heatbath_site_outcomes(U0, gauge, T, seed, sweep, s, mm * 0.999)[0])
            n_hi = len(O.heatbath_site_outcomes(U0, gauge, T, seed, sweep, s, mm * 1.001)[0])
            assert n_lo == 1 and n_hi >= 2
    assert many > 0
