"""Pins of the sensitivity oracle (Sec. 3.1) against facts outside it:
central finite differences of the network output, closed forms of linear
models, a hidden-unit permutation, and hand-worked threshold cases."""

import numpy as np
import pytest

from oracle import network as on
from oracle import sensitivity as os_


def _fd_square_sums(kind, wa, wb, theta, data, h=1e-6):
    """sum_{j,o} (dF_{j,o}/dtheta_i)^2 by central differences of the output."""
    out = np.zeros(theta.size)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        d = (on.predict(kind, wa, wb, tp, data) - on.predict(kind, wa, wb, tm, data)) / (2 * h)
        out[i] = np.sum(d * d)
    return out


def test_mlp_square_sums_match_finite_differences():
    rng = np.random.default_rng(0)
    wa = [3, 4, 5, 2]
    theta = rng.normal(0, 0.7, on.net_size("mlp", wa))
    data = {"x": rng.uniform(-1, 1, (6, 3))}
    acc, n_d = os_.jacobian_square_sums("mlp", wa, None, theta, data)
    assert n_d == 6
    np.testing.assert_allclose(acc, _fd_square_sums("mlp", wa, None, theta, data), rtol=1e-6, atol=1e-10)


def test_deeponet_square_sums_match_finite_differences():
    rng = np.random.default_rng(1)
    wa, wb = [4, 3, 2], [2, 3, 2]
    theta = rng.normal(0, 0.7, on.net_size("deeponet", wa, wb))
    data = {"u": rng.normal(size=(3, 4)), "yq": rng.uniform(0, 1, (5, 2))}
    acc, n_d = os_.jacobian_square_sums("deeponet", wa, wb, theta, data)
    assert n_d == 3
    np.testing.assert_allclose(acc, _fd_square_sums("deeponet", wa, wb, theta, data), rtol=1e-6, atol=1e-10)


def test_linear_model_closed_form():
    """No hidden layer, two outputs: F_o = W[o] x + b[o], so dF_o/dW[o'][k] =
    [o = o'] x_k and dF_o/db[o'] = [o = o']: S^2(W[o][k]) = sigma^2 mean_j
    x_jk^2 and S^2(b[o]) = sigma^2 (each output counted once)."""
    rng = np.random.default_rng(2)
    x = rng.normal(size=(40, 3))
    wa = [3, 2]
    mu = rng.normal(size=on.net_size("mlp", wa))
    sigma = rng.uniform(0.1, 2.0, mu.size)
    s2 = os_.sensitivities("mlp", wa, None, mu, sigma, {"x": x})
    expect = np.concatenate([np.tile(np.mean(x * x, axis=0), 2), np.ones(2)]) * sigma ** 2
    np.testing.assert_allclose(s2, expect, rtol=1e-13)


def test_linear_deeponet_closed_form():
    """One-layer towers: B_j = Wa u_j + ba, T_q = Wb y_q + bb,
    F_jq = <B_j, T_q> + b0.  Then dF/dWa[k][m] = u_jm T_qk, dF/dba[k] = T_qk,
    dF/dWb[k][m] = B_jk y_qm, dF/dbb[k] = B_jk, dF/db0 = 1; sums over q and
    the mean over the n_u functions follow in closed form."""
    rng = np.random.default_rng(3)
    m, d, p = 4, 2, 3
    wa, wb = [m, p], [d, p]
    mu = rng.normal(size=on.net_size("deeponet", wa, wb))
    sigma = np.ones(mu.size)
    u, yq = rng.normal(size=(7, m)), rng.uniform(0, 1, (5, d))
    s2 = os_.sensitivities("deeponet", wa, wb, mu, sigma, {"u": u, "yq": yq})
    net = on.unflatten("deeponet", wa, wb, mu)
    (Wa, ba), = net["a"]
    (Wb, bb), = net["b"]
    B, T = u @ Wa.T + ba, yq @ Wb.T + bb
    nu = u.shape[0]
    tq = np.sum(T * T, axis=0)                        # sum_q T_qk^2
    e_Wa = np.outer(tq, np.sum(u * u, axis=0)) / nu    # [k][m]
    e_ba = tq
    e_Wb = np.outer(np.sum(B * B, axis=0), np.sum(yq * yq, axis=0)) / nu
    e_bb = np.sum(B * B, axis=0) / nu * yq.shape[0]
    e_b0 = np.array([yq.shape[0]], dtype=float)
    expect = np.concatenate([e_Wa.ravel(), e_ba, e_Wb.ravel(), e_bb, e_b0])
    np.testing.assert_allclose(s2, expect, rtol=1e-12)


def test_hidden_unit_permutation_permutes_sensitivities():
    """Relabelling the hidden units of a 2-H-1 network relabels the
    sensitivities of their weights and biases the same way."""
    rng = np.random.default_rng(4)
    wa = [2, 5, 1]
    mu = rng.normal(size=on.net_size("mlp", wa))
    sigma = rng.uniform(0.5, 1.5, mu.size)
    x = {"x": rng.uniform(-1, 1, (9, 2))}
    perm = np.array([3, 0, 4, 1, 2])
    # flat index map: W1 [5][2], b1 [5], W2 [1][5], b2 [1]
    idx = np.arange(mu.size)
    W1, b1 = idx[:10].reshape(5, 2), idx[10:15]
    W2, b2 = idx[15:20].reshape(1, 5), idx[20:]
    new = np.concatenate([W1[perm].ravel(), b1[perm], W2[:, perm].ravel(), b2])
    s = os_.sensitivities("mlp", wa, None, mu, sigma, x)
    sp = os_.sensitivities("mlp", wa, None, mu[new], sigma[new], x)
    np.testing.assert_allclose(sp, s[new], rtol=1e-13)
    # a relabelling that mixes the two weight blocks breaks it
    bad = new.copy()
    bad[[0, 15]] = bad[[15, 0]]
    assert not np.allclose(os_.sensitivities("mlp", wa, None, mu[bad], sigma[bad], x), s[bad])


@pytest.mark.parametrize("s2,tau,expect", [
    ([1.0, 4.0, 2.0, 3.0], 0.7, [1, 3]),        # shares 0.4, 0.7, 0.9, 1.0
    ([1.0, 4.0, 2.0, 3.0], 0.69, [1]),
    ([1.0, 4.0, 2.0, 3.0], 0.39, []),
    ([1.0, 4.0, 2.0, 3.0], 1.0, [0, 1, 2, 3]),
    ([2.0, 2.0, 2.0, 2.0], 0.5, [0, 1]),        # ties keep index order
    ([0.0, 5.0, 0.0, 5.0], 0.5, [1]),
])
def test_threshold_selection_hand_cases(s2, tau, expect):
    assert os_.select_mask(s2, tau).tolist() == expect


def test_threshold_selection_rejects_bad_input():
    with pytest.raises(ValueError):
        os_.select_mask([0.0, 0.0], 0.5)
    with pytest.raises(ValueError):
        os_.select_mask([1.0, 2.0], 1.5)
