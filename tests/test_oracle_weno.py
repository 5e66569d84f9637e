"""Pins of the nonlinear weights (oracle/weno.py; eqs. p_big, tao5, tao4, 99)."""
import numpy as np

from oracle.weno import nonlinear_weights, combine


def test_weights_sum_to_one_and_positive():
    rng = np.random.default_rng(0)
    for K in (2, 4):
        g = rng.uniform(0.01, 1.0, K + 1)
        g = g / g.sum()
        betas = rng.uniform(0.0, 10.0, (K + 1, 100)) ** 3
        w = nonlinear_weights(betas, g, 1e-6)
        assert np.allclose(w.sum(0), 1.0, atol=1e-15)
        assert (w > 0).all()


def test_equal_indicators_give_linear_weights():
    g = (0.96, 0.01, 0.01, 0.01, 0.01)
    betas = np.full((5, 3), 0.37)
    w = nonlinear_weights(betas, g, 1e-6)
    assert np.allclose(w, np.array(g)[:, None], atol=1e-16)


def test_linear_weights_reproduce_high_order_value():
    # eq. p_big: the decomposition holds for any gamma with gamma_0 != 0
    rng = np.random.default_rng(1)
    g = (0.5, 0.3, 0.2)
    qs = [rng.normal(size=7) for _ in range(3)]
    out = combine(np.array(g)[:, None] * np.ones((3, 7)), g, qs)
    assert np.allclose(out, qs[0], atol=1e-14)


def test_tau_definition_two_and_four_candidates():
    betas = np.array([[1.0], [3.0], [0.0]])
    # tau = ((|1-3| + |1-0|)/2)^2 = 2.25 ; wbar_n = g_n (1 + 2.25/(b_n + eps))
    g = (0.6, 0.2, 0.2)
    eps = 1e-6
    wbar = np.array([g[0] * (1 + 2.25 / (1 + eps)), g[1] * (1 + 2.25 / (3 + eps)),
                     g[2] * (1 + 2.25 / eps)])
    assert np.allclose(nonlinear_weights(betas, g, eps)[:, 0], wbar / wbar.sum(), rtol=1e-15)
    betas = np.array([[2.0], [1.0], [4.0], [2.0], [0.0]])
    tau = ((1 + 2 + 0 + 2) / 4.0) ** 2
    g = (0.96, 0.01, 0.01, 0.01, 0.01)
    wbar = np.array([gi * (1 + tau / (b + eps)) for gi, b in zip(g, betas[:, 0])])
    assert np.allclose(nonlinear_weights(betas, g, eps)[:, 0], wbar / wbar.sum(), rtol=1e-15)
