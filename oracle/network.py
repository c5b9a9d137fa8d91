"""Networks, potential energy and the masked gradient, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Networks (Sec. 2, App. A): a fully connected tower maps its input through
linear layers, with tanh after every layer except the last, which is linear.
An MLP is one tower.  A DeepONet has a branch tower over the input-function
samples u and a trunk tower over the query coordinates y; its output at
(function a, query q) is the dot product of the two final feature vectors
plus one scalar bias b0 (the odd parameter counts of Sec. 4.2 require that
scalar).

Flat parameter order: tower by tower (branch, then trunk, then b0), layer
by layer, W[out][in] row-major and then b[out].

Potential (Sec. 2.2, Algorithm 2, App. C):
    U(Theta_s) = sum_{rows, outputs} (F - y)^2 / (2 lik_sd^2)
               + sum_{i in s} theta_i^2 / (2 prior_sd^2)
The Gaussian normalising constants and the prior of the fixed entries do not
depend on Theta_s and are dropped; U is the sum over the whole training set
(full batch, temperature one).
"""

from __future__ import annotations

import numpy as np


def layer_shapes(widths):
    """(out, in) of each linear layer of a tower."""
    return [(int(widths[i + 1]), int(widths[i])) for i in range(len(widths) - 1)]


def tower_size(widths) -> int:
    return sum(o * i + o for o, i in layer_shapes(widths))


def net_size(kind, widths_a, widths_b=None) -> int:
    if kind == "mlp":
        return tower_size(widths_a)
    return tower_size(widths_a) + tower_size(widths_b) + 1


def unflatten_tower(theta, widths, start):
    """Views (W, b) of each layer of one tower, starting at flat position ``start``."""
    layers = []
    pos = start
    for out, inn in layer_shapes(widths):
        W = theta[pos:pos + out * inn].reshape(out, inn)
        pos += out * inn
        b = theta[pos:pos + out]
        pos += out
        layers.append((W, b))
    return layers, pos


def unflatten(kind, widths_a, widths_b, theta):
    """Split the flat vector into towers (and b0); asserts that the whole
    vector is consumed."""
    theta = np.asarray(theta, dtype=np.float64)
    a, pos = unflatten_tower(theta, widths_a, 0)
    if kind == "mlp":
        if pos != theta.size:
            raise ValueError(f"parameter vector has {theta.size} entries, network needs {pos}")
        return {"a": a}
    b, pos = unflatten_tower(theta, widths_b, pos)
    if pos + 1 != theta.size:
        raise ValueError(f"parameter vector has {theta.size} entries, network needs {pos + 1}")
    return {"a": a, "b": b, "b0": theta[pos]}


def tower_forward(layers, x):
    """All activations a_0 = x, ..., a_L of a tower (tanh hidden, linear last)."""
    acts = [np.asarray(x, dtype=np.float64)]
    n = len(layers)
    for l, (W, b) in enumerate(layers):
        z = acts[-1] @ W.T + b
        acts.append(np.tanh(z) if l < n - 1 else z)
    return acts


def tower_backward(layers, acts, delta_out):
    """Gradient of a scalar with respect to every (W, b) of a tower, given its
    derivative ``delta_out`` with respect to the tower output (rows x out).
    Plain reverse-mode chain rule; tanh'(z) = 1 - tanh(z)^2."""
    grads = [None] * len(layers)
    d = delta_out
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (d.T @ acts[l], d.sum(axis=0))
        if l > 0:
            d = (d @ W) * (1.0 - acts[l] ** 2)
    return grads


def _flatten_grads(grads):
    out = []
    for gW, gb in grads:
        out.append(gW.ravel())
        out.append(gb)
    return out


def predict(kind, widths_a, widths_b, theta, data):
    """Network output: MLP rows x d_out, DeepONet functions x query points."""
    net = unflatten(kind, widths_a, widths_b, theta)
    if kind == "mlp":
        return tower_forward(net["a"], data["x"])[-1]
    B = tower_forward(net["a"], data["u"])[-1]
    T = tower_forward(net["b"], data["yq"])[-1]
    return B @ T.T + net["b0"]


def likelihood_and_grad(kind, widths_a, widths_b, theta, data, lik_sd):
    """U_lik = sum (F - y)^2 / (2 lik_sd^2) and its dense gradient with respect
    to the full parameter vector."""
    net = unflatten(kind, widths_a, widths_b, theta)
    inv_var = 1.0 / (lik_sd * lik_sd)
    if kind == "mlp":
        acts = tower_forward(net["a"], data["x"])
        r = acts[-1] - data["y"]
        U = 0.5 * inv_var * float(np.sum(r * r))
        grads = tower_backward(net["a"], acts, r * inv_var)
        return U, np.concatenate(_flatten_grads(grads))
    acts_b = tower_forward(net["a"], data["u"])
    acts_t = tower_forward(net["b"], data["yq"])
    B, T = acts_b[-1], acts_t[-1]
    r = B @ T.T + net["b0"] - data["v"]
    U = 0.5 * inv_var * float(np.sum(r * r))
    dG = r * inv_var
    g_branch = tower_backward(net["a"], acts_b, dG @ T)
    g_trunk = tower_backward(net["b"], acts_t, dG.T @ B)
    g = np.concatenate(_flatten_grads(g_branch) + _flatten_grads(g_trunk) + [np.array([dG.sum()])])
    return U, g


class MaskedPosterior:
    """The conditional posterior of Sec. 3.2: Theta_~s fixed at the given
    values, U and its gradient as functions of Theta_s only."""

    def __init__(self, kind, widths_a, widths_b, theta_fixed, sel, data, prior_sd, lik_sd, prior_weight=1.0):
        self.kind = kind
        self.widths_a = list(widths_a)
        self.widths_b = None if widths_b is None else list(widths_b)
        self.theta_fixed = np.array(theta_fixed, dtype=np.float64)
        self.sel = np.asarray(sel, dtype=np.int64)
        if self.sel.size and (np.any(np.diff(self.sel) <= 0) or self.sel[0] < 0
                              or self.sel[-1] >= self.theta_fixed.size):
            raise ValueError("selected indices must be strictly increasing and in range")
        self.data = data
        self.prior_sd = float(prior_sd)
        self.lik_sd = float(lik_sd)
        self.prior_weight = float(prior_weight)   # the share of the prior term this potential carries

    def full(self, theta_s):
        th = self.theta_fixed.copy()
        th[self.sel] = theta_s
        return th

    def potential(self, theta_s):
        return self.potential_and_grad(theta_s)[0]

    def potential_and_grad(self, theta_s):
        theta_s = np.asarray(theta_s, dtype=np.float64)
        U_lik, g_full = likelihood_and_grad(self.kind, self.widths_a, self.widths_b,
                                            self.full(theta_s), self.data, self.lik_sd)
        inv_pv = self.prior_weight / (self.prior_sd * self.prior_sd)
        U = U_lik + 0.5 * inv_pv * float(np.sum(theta_s * theta_s))
        g = g_full[self.sel] + inv_pv * theta_s
        return U, g


def batch_posteriors(post, bounds):
    """The split of a posterior's potential over consecutive data batches used
    by symmetric-splitting HMC (Sec. 4.2.3's full-HMC baseline): batch m holds
    the data rows bounds[m] <= i < bounds[m+1] (MLP rows; DeepONet input
    functions, each with all its query points) and 1/M of the prior term, so
    that the batch potentials add up to U."""
    bounds = [int(b) for b in bounds]
    M = len(bounds) - 1
    if M < 1 or bounds[0] != 0 or any(b1 <= b0 for b0, b1 in zip(bounds, bounds[1:])):
        raise ValueError("bounds must start at 0 and increase strictly")
    keys = ("x", "y") if post.kind == "mlp" else ("u", "v")
    if bounds[-1] != post.data[keys[0]].shape[0]:
        raise ValueError("bounds must end at the number of data rows")
    out = []
    for b0, b1 in zip(bounds, bounds[1:]):
        data = dict(post.data)
        for k in keys:
            data[k] = post.data[k][b0:b1]
        out.append(MaskedPosterior(post.kind, post.widths_a, post.widths_b, post.theta_fixed, post.sel, data,
                                   post.prior_sd, post.lik_sd, prior_weight=post.prior_weight / M))
    return out


def data_from_workload(w):
    """The arrays of a ``workloads.Workload`` as the dict used here."""
    if w.kind == "mlp":
        return {"x": w.x, "y": w.y}
    return {"u": w.u, "yq": w.yq, "v": w.v}


def posterior_for_chain(w, c):
    """MaskedPosterior of chain ``c`` of a workload."""
    return MaskedPosterior(w.kind, w.widths_a, w.widths_b, w.theta0, w.chain_idx(c),
                           data_from_workload(w), w.prior_sd, w.lik_sd)
