"""Parameter sensitivities and the sensitive subset, in FP64 (Sec. 3.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Around the VI mean mu, the first-order Taylor expansion of the network in its
parameters (Sec. 3.1, first equation) makes the output variance, for
independent parameters with standard deviations sigma_i, the sum over
parameters of sigma_i^2 (dF_mu/dtheta_i)^2.  The sensitivity of parameter i
is its share, averaged over the N_d training inputs (Sec. 3.1, sensitivity
equation):

    S_i^2 = sigma_i^2 / N_d * sum_j (dF_mu(x_j) / dtheta_i)^2 .

Reading for vector outputs (an MLP with several outputs; a DeepONet, whose
output for the input function u_j is the vector over the query points): the
variances of the output entries add, so the squared derivatives are summed
over the output entries of each input, and averaged over the N_d inputs (MLP
rows; DeepONet input functions, the text puts u_j in place of x_j).

Selection (Sec. 3.1, threshold equation): order the parameters from the most
to the least sensitive and take the largest count N whose cumulative share of
the total sum of S^2 is at most tau; the sensitive subset is those N
parameters.  Reading for ties: equal sensitivities keep their index order (a
stable sort), which makes the subset well defined; a total of zero has no
shares and is rejected.

This is the plain definition: one reverse pass per output entry of one
input, each giving a full row of the Jacobian, squared and summed.  It is
slow and meant for small cases.
"""

from __future__ import annotations

import numpy as np

from .network import _flatten_grads, tower_backward, tower_forward, unflatten


def jacobian_rows(kind, widths_a, widths_b, theta, data):
    """Yields, for every input j and output entry o, the gradient of
    F_{j,o} with respect to the whole flat parameter vector."""
    net = unflatten(kind, widths_a, widths_b, theta)
    if kind == "mlp":
        X = np.asarray(data["x"], dtype=np.float64)
        for j in range(X.shape[0]):
            acts = tower_forward(net["a"], X[j:j + 1])
            d_out = acts[-1].shape[1]
            for o in range(d_out):
                seed = np.zeros((1, d_out))
                seed[0, o] = 1.0
                yield np.concatenate(_flatten_grads(tower_backward(net["a"], acts, seed)))
        return
    U = np.asarray(data["u"], dtype=np.float64)
    acts_t = tower_forward(net["b"], data["yq"])
    T = acts_t[-1]
    for j in range(U.shape[0]):
        acts_b = tower_forward(net["a"], U[j:j + 1])
        B = acts_b[-1]
        for q in range(T.shape[0]):
            # F_{jq} = <B_j, T_q> + b0: dF/dB_j = T_q, dF/dT_q = B_j, dF/db0 = 1
            g_branch = tower_backward(net["a"], acts_b, T[q:q + 1])
            g_trunk = tower_backward(net["b"], [a[q:q + 1] for a in acts_t], B)
            yield np.concatenate(_flatten_grads(g_branch) + _flatten_grads(g_trunk) + [np.array([1.0])])


def jacobian_square_sums(kind, widths_a, widths_b, theta, data):
    """sum over inputs j and output entries o of (dF_{j,o}/dtheta_i)^2, for
    every parameter i, and N_d."""
    acc = None
    for g in jacobian_rows(kind, widths_a, widths_b, theta, data):
        acc = g * g if acc is None else acc + g * g
    n_d = np.asarray(data["x"] if kind == "mlp" else data["u"]).shape[0]
    return acc, n_d


def sensitivities(kind, widths_a, widths_b, mu, sigma, data):
    """S_i^2 = sigma_i^2 / N_d * sum_j sum_o (dF_mu(x_j)_o / dtheta_i)^2."""
    acc, n_d = jacobian_square_sums(kind, widths_a, widths_b, mu, data)
    sigma = np.asarray(sigma, dtype=np.float64)
    return sigma * sigma * acc / n_d


def select_mask(s2, tau):
    """Indices (ascending) of the N most sensitive parameters, N the largest
    count whose cumulative share of sum(S^2), most sensitive first, is at
    most tau."""
    s2 = np.asarray(s2, dtype=np.float64)
    if not 0.0 <= tau <= 1.0:
        raise ValueError("tau must lie in [0, 1]")
    order = np.argsort(-s2, kind="stable")
    cum = np.cumsum(s2[order])
    total = cum[-1]
    if not total > 0.0:
        raise ValueError("the sensitivities sum to zero")
    n = int(np.searchsorted(cum / total, tau, side="right"))
    return np.sort(order[:n])
