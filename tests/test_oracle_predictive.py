"""Pins of the posterior-predictive oracle: a model linear in the sampled
parameters has a closed-form predictive mean and variance; one sample has
zero spread; hand-worked relative L2 errors."""

import numpy as np

from oracle import network as on
from oracle import predictive as op


def test_linear_in_the_samples_closed_form():
    """No hidden layer: F(x) = W x + b is linear in (W, b), so over samples
    the mean prediction is F at the sample mean and the variance is
    z^T Cov z with z = (x, 1) and Cov the empirical covariance."""
    rng = np.random.default_rng(0)
    wa = [3, 1]
    P = on.net_size("mlp", wa)
    fixed = rng.normal(size=P)
    sel = np.array([0, 2, 3])            # W[0][0], W[0][2], b
    S = rng.normal(size=(50, 3))
    x = rng.normal(size=(7, 3))
    mean, var = op.predictive_moments("mlp", wa, None, fixed, sel, S, {"x": x})
    m = S.mean(axis=0)
    C = (S - m).T @ (S - m) / S.shape[0]
    Z = np.column_stack([x[:, 0], x[:, 2], np.ones(7)])
    base = x[:, 1] * fixed[1]
    np.testing.assert_allclose(mean[:, 0], Z @ m + base, rtol=1e-12)
    np.testing.assert_allclose(var[:, 0], np.einsum("ij,jk,ik->i", Z, C, Z), rtol=1e-10)


def test_one_sample_has_no_spread():
    rng = np.random.default_rng(1)
    wa = [2, 5, 2]
    P = on.net_size("mlp", wa)
    fixed = rng.normal(size=P)
    sel = np.arange(0, P, 3)
    s = rng.normal(size=(1, sel.size))
    x = {"x": rng.normal(size=(4, 2))}
    mean, var = op.predictive_moments("mlp", wa, None, fixed, sel, s, x)
    np.testing.assert_allclose(mean, on.predict("mlp", wa, None, op.full_parameters(fixed, sel, s[0]), x), rtol=1e-14)
    assert np.all(var == 0.0)


def test_mean_relative_l2_hand_cases():
    Y = np.array([[3.0, 4.0], [1.0, 0.0]])
    Yp = np.array([[3.0, 4.0], [0.0, 0.0]])      # errors 0 and 1
    assert op.mean_relative_l2(Y, Yp) == 0.5
    assert abs(op.mean_relative_l2(Y, 1.1 * Y) - 0.1) < 1e-15
