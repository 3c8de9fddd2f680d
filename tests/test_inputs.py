"""Checks of the seeded input generators (host entry points).

The generators make inputs only; these tests check that the fields have the
structure the workloads need (SU(3) links, Haar statistics, heatbath
plaquettes in the strong- and weak-coupling limits).
"""
import math

import numpy as np
import pytest

import inputs
import oracle as O


def unitarity_dev(M):
    M = M.reshape(-1, 3, 3)
    return max(np.abs(M @ M.conj().transpose(0, 2, 1) - np.eye(3)).max(),
               np.abs(np.linalg.det(M) - 1).max())


def test_generator_philox_matches_published_vectors():
    assert inputs.philox4x32([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C,
                                                        0x9B00DBD8]


def test_haar_su3_statistics():
    g = inputs.haar_sites((8, 8, 8, 8), seed=3).reshape(-1, 3, 3)
    n = g.shape[0]
    assert unitarity_dev(g) < 1e-14
    tr = np.trace(g, axis1=1, axis2=2)
    # Haar SU(3): E[tr U] = 0, E[|tr U|^2] = 1, E[|U_ab|^2] = 1/3
    assert abs(tr.mean()) < 5 / math.sqrt(n)
    assert abs((np.abs(tr) ** 2).mean() - 1) < 0.05
    assert np.allclose((np.abs(g) ** 2).mean(axis=0), 1 / 3, atol=0.01)
    # different copies differ, same copy repeats
    assert not np.array_equal(inputs.haar_sites((2, 2, 2, 2), 3, 1), inputs.haar_sites((2, 2, 2, 2), 3, 0))
    assert np.array_equal(inputs.haar_sites((2, 2, 2, 2), 3, 1), inputs.haar_sites((2, 2, 2, 2), 3, 1))


def test_smooth_links_are_exponentials():
    V = inputs.smooth_links((2, 2, 2, 2), 0.3, 1).reshape(-1, 3, 3)
    assert unitarity_dev(V) < 1e-14
    # V = exp(i eps H): the eigenphases of V are eps * eigenvalues of H (traceless)
    ph = np.angle(np.linalg.eigvals(V))
    assert np.allclose(ph.sum(axis=1), 0, atol=1e-12)
    assert np.abs(ph).max() < 0.3 * 6


def test_config0_and_pure_gauge():
    dims = (4, 2, 4, 2)
    U = inputs.config0(dims, 0.3, 1)
    assert unitarity_dev(U) < 1e-14
    # the Haar transform does not change the plaquette of the smooth field
    assert O.plaquette(U) == pytest.approx(O.plaquette(inputs.smooth_links(dims, 0.3, 1)), abs=1e-13)
    P = inputs.pure_gauge(dims, 4)
    assert O.plaquette(P) == pytest.approx(1.0, abs=1e-14)
    W = inputs.smooth_links(dims, 0.3, 1)
    inputs.haar_copy(W, 1, 0)
    assert np.allclose(W, U, atol=1e-14)


def _mean_plaquette(dims, beta, therm, meas, seed):
    U = inputs.heatbath(dims, beta, therm, seed)
    acc = []
    for k in range(meas):
        inputs.heatbath(dims, beta, 1, seed, U=U, first_sweep=therm + k)
        acc.append(O.plaquette(U))
    return float(np.mean(acc)), U


def test_heatbath_strong_coupling():
    """Strong coupling: <P> = beta/18 + beta^2/216 + O(beta^3) for SU(3)."""
    beta = 0.6
    P, U = _mean_plaquette((4, 4, 4, 4), beta, 10, 20, seed=2)
    assert unitarity_dev(U) < 1e-13
    assert P == pytest.approx(beta / 18 + beta ** 2 / 216, abs=0.004)


def test_heatbath_weak_coupling():
    """Weak coupling (equipartition): 1 - <P> = 2/beta + O(1/beta^2) for SU(3)."""
    beta = 40.0
    P, _ = _mean_plaquette((4, 4, 4, 4), beta, 30, 10, seed=3)
    assert (1 - P) * beta / 2 == pytest.approx(1.0, abs=0.1)


def test_argument_errors():
    with pytest.raises(RuntimeError):
        inputs.config0((3, 4, 4, 4))
    with pytest.raises(RuntimeError):
        inputs.heatbath((4, 4, 4, 4), -1.0, 1, 1)
