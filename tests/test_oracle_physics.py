"""Pins of oracle/physics.py: eigenvectors against the flux Jacobian obtained by
complex-step differentiation of the flux functions (eqs. euler1, euler2), L R = I, and the
spectral radius against the Jacobian's eigenvalues."""
import numpy as np
import pytest

from oracle.physics import Equation


def jacobian(eq, U, d, h=1e-30):
    n = len(U)
    J = np.zeros((n, n))
    for j in range(n):
        Uc = U.astype(complex)
        Uc[j] += 1j * h
        J[:, j] = np.imag(eq.flux(Uc, d)) / h
    return J


@pytest.mark.parametrize("dim,d", [(1, 0), (2, 0), (2, 1)])
def test_eigenvectors_diagonalise_flux_jacobian(dim, d):
    eq = Equation("euler", dim)
    rng = np.random.default_rng(11)
    for _ in range(20):
        rho = rng.uniform(0.1, 3.0)
        vel = rng.uniform(-2.0, 2.0, dim)
        p = rng.uniform(0.1, 5.0)
        U = np.concatenate([[rho], rho * vel, [p / 0.4 + 0.5 * rho * np.sum(vel ** 2)]])
        A = jacobian(eq, U, d)
        Lm, Rm = eq.eigen_pair(U, d)
        lam = eq.eigenvalues(U, d)
        assert np.allclose(A @ Rm, Rm @ np.diag(lam), atol=1e-10 * np.abs(A).max())
        assert np.allclose(Lm @ Rm, np.eye(dim + 2), atol=1e-12)
        # spectral radius used for the Lax-Friedrichs speed
        assert np.isclose(eq.spectral_radius(U[:, None], d)[0], np.abs(np.linalg.eigvals(A)).max())


def test_batched_eigenvectors_match_single():
    eq = Equation("euler", 2)
    U = np.array([[1.0, 0.5], [0.2, -0.3], [0.1, 0.4], [2.5, 3.0]])
    Rb = eq.right_eigenvectors(U, 1)
    for k in range(2):
        assert np.array_equal(Rb[k], eq.right_eigenvectors(U[:, k], 1))


def test_scalar_fluxes():
    eq = Equation("burgers", 2)
    u = np.array([[0.3, -2.0]])
    assert np.array_equal(eq.flux(u, 0), 0.5 * u * u)
    eq = Equation("advection", 2, adv=(0.7, -0.2))
    assert np.array_equal(eq.flux(u, 1), -0.2 * u)
    assert np.array_equal(eq.spectral_radius(u, 1), [0.2, 0.2])
