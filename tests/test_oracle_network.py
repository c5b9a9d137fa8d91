"""Pins of the oracle's network, potential and masked gradient.

Each check compares the oracle with something it does not compute itself:
the paper's printed parameter counts, the closed-form Bayesian linear
regression posterior, symmetries of tanh networks, Taylor coefficients of
tanh, brute-force loops on tiny DeepONets, and central finite differences.
"""

import json
import os

import numpy as np
import pytest

from oracle import network as on

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Parameter counts printed in the paper pin the layer bookkeeping.

@pytest.mark.parametrize("key", ["case2_bnn", "burgers_deeponet", "cone_deeponet"])
def test_printed_parameter_counts(key):
    spec = json.load(open(os.path.join(GOLDEN, "architecture_counts.json")))[key]
    n = on.net_size(spec["kind"], spec["widths_a"], spec.get("widths_b"))
    assert n == spec["count"]
    # unflatten consumes exactly that many entries
    on.unflatten(spec["kind"], spec["widths_a"], spec.get("widths_b"), np.zeros(n))
    for bad in (n - 1, n + 1):
        with pytest.raises(ValueError):
            on.unflatten(spec["kind"], spec["widths_a"], spec.get("widths_b"), np.zeros(bad))


# --------------------------------------------------------------------------
# Bayesian linear regression: a tower with no hidden layer.

def _design_linear(X, d_out):
    """Design matrix of F_flat[(n, o)] = sum_i W[o][i] X[n][i] + b[o] over the
    flat order W[out][in] row-major then b[out], built entry by entry."""
    N, d_in = X.shape
    P = d_out * d_in + d_out
    Phi = np.zeros((N * d_out, P))
    for n in range(N):
        for o in range(d_out):
            for i in range(d_in):
                Phi[n * d_out + o, o * d_in + i] = X[n, i]
            Phi[n * d_out + o, d_out * d_in + o] = 1.0
    return Phi


def _blr(Phi, yflat, theta_fixed, sel, prior_sd, lik_sd):
    """Textbook posterior precision and mean of the selected coefficients."""
    rest = np.setdiff1d(np.arange(Phi.shape[1]), sel)
    y_shift = yflat - Phi[:, rest] @ theta_fixed[rest]
    Ps = Phi[:, sel]
    Lam = Ps.T @ Ps / lik_sd**2 + np.eye(len(sel)) / prior_sd**2
    m = np.linalg.solve(Lam, Ps.T @ y_shift / lik_sd**2)
    const = y_shift @ y_shift / (2 * lik_sd**2) - 0.5 * m @ Lam @ m
    return Lam, m, const


@pytest.mark.parametrize("d_in,d_out,frac", [(3, 1, 1.0), (4, 2, 0.6), (2, 3, 0.5)])
def test_linear_tower_matches_closed_form_posterior(d_in, d_out, frac):
    rng = np.random.default_rng(1 + d_in + 10 * d_out)
    N = 37
    X = rng.uniform(-1, 1, (N, d_in))
    Y = rng.normal(size=(N, d_out))
    P = d_out * d_in + d_out
    theta_fixed = rng.normal(size=P)
    sel = np.sort(rng.choice(P, max(1, int(frac * P)), replace=False))
    prior_sd, lik_sd = 0.7, 0.3
    post = on.MaskedPosterior("mlp", [d_in, d_out], None, theta_fixed, sel, {"x": X, "y": Y},
                              prior_sd, lik_sd)
    Lam, m, const = _blr(_design_linear(X, d_out), Y.ravel(), theta_fixed, sel, prior_sd, lik_sd)
    for _ in range(3):
        th = m + rng.normal(size=len(sel))
        U, g = post.potential_and_grad(th)
        d = th - m
        np.testing.assert_allclose(U, 0.5 * d @ Lam @ d + const, rtol=1e-12)
        np.testing.assert_allclose(g, Lam @ d, rtol=1e-10, atol=1e-10 * np.abs(Lam @ d).max())
    # the gradient vanishes at the posterior mean
    _, g_m = post.potential_and_grad(m)
    assert np.abs(g_m).max() < 1e-9 * np.abs(Lam).max()


# --------------------------------------------------------------------------
# Structure of tanh networks.

def _rand_mlp(widths, rng, scale=0.7):
    P = on.tower_size(widths)
    return rng.normal(scale=scale, size=P)


def test_hidden_unit_permutation_symmetry():
    rng = np.random.default_rng(5)
    widths = [3, 5, 4, 2]
    th = _rand_mlp(widths, rng)
    X, Y = rng.normal(size=(11, 3)), rng.normal(size=(11, 2))
    perm = np.array([3, 0, 4, 1, 2])
    th2 = th.copy()
    layers, _ = on.unflatten_tower(th2, widths, 0)   # views into th2
    W1, b1 = layers[0]
    W2, _ = layers[1]
    W1[:] = W1[perm]
    b1[:] = b1[perm]
    W2[:] = W2[:, perm]
    F1 = on.predict("mlp", widths, None, th, {"x": X})
    F2 = on.predict("mlp", widths, None, th2, {"x": X})
    np.testing.assert_allclose(F1, F2, rtol=1e-13, atol=1e-13)
    # a permutation of the wrong axis is not a symmetry
    th3 = th.copy()
    l3, _ = on.unflatten_tower(th3, widths, 0)
    l3[0][0][:] = l3[0][0][:, [1, 2, 0]]
    assert np.abs(on.predict("mlp", widths, None, th3, {"x": X}) - F1).max() > 1e-3


def test_tanh_odd_symmetry():
    rng = np.random.default_rng(6)
    widths = [2, 4, 3, 1]
    th = _rand_mlp(widths, rng)
    X = rng.normal(size=(9, 2))
    th2 = th.copy()
    layers, _ = on.unflatten_tower(th2, widths, 0)
    h = 2
    layers[1][0][h, :] *= -1      # incoming weights of unit h of layer 2
    layers[1][1][h] *= -1         # its bias
    layers[2][0][:, h] *= -1      # its outgoing weights
    np.testing.assert_allclose(on.predict("mlp", widths, None, th, {"x": X}),
                               on.predict("mlp", widths, None, th2, {"x": X}), rtol=1e-13, atol=1e-14)


def test_small_weight_taylor_coefficients():
    """F(s) = b2 + W2 tanh(s (A x + beta)) = b2 + s W2 z - s^3 W2 z^3 / 3 + O(s^5):
    pins tanh'(0) = 1, tanh'''(0) = -2 and the wiring of both layers."""
    rng = np.random.default_rng(7)
    d, H, o = 3, 5, 2
    A, beta = rng.normal(size=(H, d)), rng.normal(size=H)
    W2, b2 = rng.normal(size=(o, H)), rng.normal(size=o)
    X = rng.normal(size=(6, d))
    z = X @ A.T + beta
    for s in (1e-2, 5e-3):
        th = np.concatenate([(s * A).ravel(), s * beta, W2.ravel(), b2])
        F = on.predict("mlp", [d, H, o], None, th, {"x": X})
        lin = b2 + s * z @ W2.T
        cub = -(s**3) / 3.0 * (z**3) @ W2.T
        np.testing.assert_allclose(F, lin + cub, rtol=0, atol=10 * s**5 * np.abs(z).max() ** 5 * np.abs(W2).sum())


def test_saturation_gives_sign_features():
    rng = np.random.default_rng(8)
    d, H, o = 2, 4, 1
    A, beta = rng.normal(size=(H, d)), rng.normal(size=H)
    W2, b2 = rng.normal(size=(o, H)), rng.normal(size=o)
    X = rng.normal(size=(7, d))
    s = 1e6
    th = np.concatenate([(s * A).ravel(), s * beta, W2.ravel(), b2])
    F = on.predict("mlp", [d, H, o], None, th, {"x": X})
    np.testing.assert_allclose(F, np.sign(X @ A.T + beta) @ W2.T + b2, rtol=1e-12)


# --------------------------------------------------------------------------
# DeepONet: brute force and the linear special case.

def _deeponet_bruteforce(Ub, Yq, Wb, bb, Wt, bt, b0):
    """G[a][q] = sum_k B[a][k] T[q][k] + b0 with one linear layer per tower."""
    na, m = Ub.shape
    nq, dy = Yq.shape
    p = Wb.shape[0]
    G = np.zeros((na, nq))
    for a in range(na):
        for q in range(nq):
            acc = b0
            for k in range(p):
                Bk = bb[k] + sum(Wb[k, i] * Ub[a, i] for i in range(m))
                Tk = bt[k] + sum(Wt[k, j] * Yq[q, j] for j in range(dy))
                acc += Bk * Tk
            G[a, q] = acc
    return G


def test_deeponet_single_layer_bruteforce():
    rng = np.random.default_rng(9)
    m, dy, p, na, nq = 4, 2, 3, 5, 6
    Wb, bb = rng.normal(size=(p, m)), rng.normal(size=p)
    Wt, bt = rng.normal(size=(p, dy)), rng.normal(size=p)
    b0 = 0.37
    Ub, Yq = rng.normal(size=(na, m)), rng.normal(size=(nq, dy))
    th = np.concatenate([Wb.ravel(), bb, Wt.ravel(), bt, [b0]])
    G = on.predict("deeponet", [m, p], [dy, p], th, {"u": Ub, "yq": Yq})
    np.testing.assert_allclose(G, _deeponet_bruteforce(Ub, Yq, Wb, bb, Wt, bt, b0), rtol=1e-12)


def test_deeponet_branch_posterior_closed_form():
    """Trunk fixed, sampled = branch weights, branch bias and b0: G is linear in
    them, so U is the BLR quadratic with design U[a][m] T[q][k] / T[q][k] / 1."""
    rng = np.random.default_rng(10)
    m, dy, p, na, nq = 3, 2, 4, 7, 5
    Ub, Yq = rng.normal(size=(na, m)), rng.normal(size=(nq, dy))
    V = rng.normal(size=(na, nq))
    P = on.net_size("deeponet", [m, p], [dy, p])
    theta_fixed = rng.normal(size=P)
    nb = p * m + p
    Wt = theta_fixed[nb:nb + p * dy].reshape(p, dy)
    bt = theta_fixed[nb + p * dy:nb + p * dy + p]
    T = np.array([[bt[k] + sum(Wt[k, j] * Yq[q, j] for j in range(dy)) for k in range(p)] for q in range(nq)])
    Phi = np.zeros((na * nq, P))
    for a in range(na):
        for q in range(nq):
            row = a * nq + q
            for k in range(p):
                for i in range(m):
                    Phi[row, k * m + i] = Ub[a, i] * T[q, k]
                Phi[row, p * m + k] = T[q, k]
            Phi[row, P - 1] = 1.0
    sel = np.concatenate([np.arange(nb), [P - 1]])
    prior_sd, lik_sd = 0.8, 0.4
    # the fixed trunk enters through T only: its columns of Phi stay zero
    Lam, mu, const = _blr(Phi, V.ravel(), theta_fixed, sel, prior_sd, lik_sd)
    post = on.MaskedPosterior("deeponet", [m, p], [dy, p], theta_fixed, sel, {"u": Ub, "yq": Yq, "v": V},
                              prior_sd, lik_sd)
    th = mu + rng.normal(size=len(sel))
    U, g = post.potential_and_grad(th)
    d = th - mu
    np.testing.assert_allclose(U, 0.5 * d @ Lam @ d + const, rtol=1e-12)
    np.testing.assert_allclose(g, Lam @ d, rtol=1e-9, atol=1e-9 * np.abs(Lam @ d).max())


def test_deeponet_latent_rescaling_symmetry():
    rng = np.random.default_rng(11)
    wa, wb = [3, 5, 4], [2, 6, 4]
    P = on.net_size("deeponet", wa, wb)
    th = rng.normal(size=P)
    data = {"u": rng.normal(size=(5, 3)), "yq": rng.normal(size=(4, 2))}
    th2 = th.copy()
    net = on.unflatten("deeponet", wa, wb, th2)
    c = np.array([2.0, -0.5, 3.0, 0.25])
    Wb, bb = net["a"][-1]
    Wt, bt = net["b"][-1]
    Wb *= c[:, None]
    bb *= c
    Wt /= c[:, None]
    bt /= c
    np.testing.assert_allclose(on.predict("deeponet", wa, wb, th, data),
                               on.predict("deeponet", wa, wb, th2, data), rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# Finite differences pin the back-propagated gradient against the potential.

def _fd_check(post, th, rng, n_dir=6):
    U, g = post.potential_and_grad(th)
    for _ in range(n_dir):
        d = rng.normal(size=th.size)
        d /= np.linalg.norm(d)
        h = 1e-5
        fd = (post.potential(th + h * d) - post.potential(th - h * d)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * (np.linalg.norm(g) + 1.0), (fd, g @ d)
    # coordinate-wise on the largest entries
    for i in np.argsort(-np.abs(g))[:5]:
        e = np.zeros(th.size)
        h = 1e-6 * max(1.0, abs(th[i]))
        e[i] = h
        fd = (post.potential(th + e) - post.potential(th - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * np.abs(g).max() + 1e-8


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(12)
    widths = [2, 6, 5, 3]
    P = on.tower_size(widths)
    theta_fixed = rng.normal(scale=0.5, size=P)
    sel = np.sort(rng.choice(P, 40, replace=False))
    data = {"x": rng.uniform(-1, 1, (23, 2)), "y": rng.normal(size=(23, 3))}
    post = on.MaskedPosterior("mlp", widths, None, theta_fixed, sel, data, 1.3, 0.6)
    _fd_check(post, theta_fixed[sel] + 0.1 * rng.normal(size=len(sel)), rng)


def test_deeponet_gradient_matches_finite_differences():
    rng = np.random.default_rng(13)
    wa, wb = [4, 5, 6, 3], [2, 4, 3]
    P = on.net_size("deeponet", wa, wb)
    theta_fixed = rng.normal(scale=0.5, size=P)
    sel = np.sort(np.concatenate([rng.choice(P - 1, 30, replace=False), [P - 1]]))
    data = {"u": rng.normal(size=(9, 4)), "yq": rng.uniform(size=(7, 2)), "v": rng.normal(size=(9, 7))}
    post = on.MaskedPosterior("deeponet", wa, wb, theta_fixed, sel, data, 0.9, 0.5)
    _fd_check(post, theta_fixed[sel] + 0.1 * rng.normal(size=len(sel)), rng)


def test_masked_gradient_is_the_selected_part_of_the_full_gradient():
    """Fixing parameters changes nothing but which entries are reported."""
    rng = np.random.default_rng(14)
    widths = [2, 5, 4, 1]
    P = on.tower_size(widths)
    th = rng.normal(size=P)
    data = {"x": rng.normal(size=(13, 2)), "y": rng.normal(size=(13, 1))}
    full = on.MaskedPosterior("mlp", widths, None, th, np.arange(P), data, 1.0, 0.5)
    U_all, g_all = full.potential_and_grad(th)
    sel = np.sort(rng.choice(P, 9, replace=False))
    part = on.MaskedPosterior("mlp", widths, None, th, sel, data, 1.0, 0.5)
    U_s, g_s = part.potential_and_grad(th[sel])
    np.testing.assert_allclose(g_s, g_all[sel], rtol=1e-13)
    rest = np.setdiff1d(np.arange(P), sel)
    np.testing.assert_allclose(U_all - U_s, 0.5 * np.sum(th[rest] ** 2), rtol=1e-12)
