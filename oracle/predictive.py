"""Posterior predictive summaries over stored samples, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each stored HMC sample of the selected subset, with every other parameter at
its fixed value, is a parameter vector theta^(s); the network evaluated with
it at new inputs is one draw of the predictive distribution.  The results
sections summarise these draws by their mean (the mean prediction) and
their spread (uncertainty bands of three standard deviations), and score the
mean prediction by the mean relative L2 error over the N test cases,
(1/N) sum ||Y - Y_p||_2 / ||Y||_2 (Sec. 4.2.1).

Reading: the spread is the variance of the empirical distribution of the
draws, (1/S) sum_s (F_s - mean)^2 (no Bessel correction); for a DeepONet a
test case is one input function, the norm runs over its query points.
"""

from __future__ import annotations

import numpy as np

from .network import predict


def full_parameters(theta_fixed, sel, theta_s):
    """The whole parameter vector of one sample."""
    th = np.array(theta_fixed, dtype=np.float64, copy=True)
    th[np.asarray(sel)] = theta_s
    return th


def predictive_moments(kind, widths_a, widths_b, theta_fixed, sel, samples, inputs):
    """Mean and variance over the samples (rows of `samples`) of the network
    output at `inputs` (MLP: rows x outputs; DeepONet: functions x query
    points)."""
    draws = np.stack([predict(kind, widths_a, widths_b, full_parameters(theta_fixed, sel, s), inputs)
                      for s in np.asarray(samples, dtype=np.float64)])
    mean = draws.mean(axis=0)
    var = np.mean((draws - mean) ** 2, axis=0)
    return mean, var


def mean_relative_l2(Y, Yp):
    """(1/N) sum over test cases (rows) of ||Y - Yp||_2 / ||Y||_2."""
    Y, Yp = np.atleast_2d(np.asarray(Y, dtype=np.float64)), np.atleast_2d(np.asarray(Yp, dtype=np.float64))
    return float(np.mean(np.linalg.norm(Y - Yp, axis=1) / np.linalg.norm(Y, axis=1)))
