"""Nonlinear weights with artificial linear weights (oracle; test infrastructure).

Section 2.1 Step 1 / Step 2.1 (eqs. p_big, GHYZ, tao5) and Section 2.2 Step 5.1
(eqs. 2dGHYZ, tao4, 99):

  tau        = ( mean_{n>=1} |beta_0 - beta_n| )^2
  wbar_n     = gamma_n (1 + tau / (beta_n + eps))
  omega_n    = wbar_n / sum_l wbar_l
  value      = omega_0 (q_0/gamma_0 - sum_{n>=1} gamma_n/gamma_0 q_n) + sum_{n>=1} omega_n q_n

where q_n is whatever the n-th polynomial delivers (a first moment for the limiter, a
point value for the reconstruction).  All arrays broadcast over cells; axis 0 of
``betas`` and ``qs`` runs over the polynomials n = 0..K.

Pins: omega sums to one; omega = gamma when all beta_n are equal (tau = 0); with omega
forced to gamma the combination returns q_0 for any data (eq. p_big).

The absolute value is written as x * sign(Re x) so that complex-step differentiation
(used by the adjoint checks) differentiates it as sign(x), its derivative for real x != 0,
and as 0 where the real part is exactly 0 (the frozen-flag adjoint's choice there).
"""
import numpy as np


def real_abs(x):
    """|x| for real x; for complex-step arguments x = a + i h the value |a| + i h sign(a)
    with sign(0) = 0, i.e. the first-order expansion of |a + h| away from a = 0."""
    if np.iscomplexobj(x):
        return np.where(x.real < 0, -x, np.where(x.real > 0, x, np.abs(x.real) + 0j))
    return np.abs(x)


def nonlinear_weights(betas, gammas, eps):
    betas = np.asarray(betas)
    K = betas.shape[0] - 1
    diff = sum(real_abs(betas[0] - betas[n]) for n in range(1, K + 1)) / K
    tau = diff * diff
    wbar = np.stack([gammas[n] * (1.0 + tau / (betas[n] + eps)) for n in range(K + 1)])
    return wbar / wbar.sum(axis=0)


def combine(omegas, gammas, qs):
    K = len(gammas) - 1
    g0 = gammas[0]
    lin = qs[0] / g0 - sum(gammas[n] / g0 * qs[n] for n in range(1, K + 1))
    return omegas[0] * lin + sum(omegas[n] * qs[n] for n in range(1, K + 1))
