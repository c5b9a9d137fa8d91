"""Pins of the oracle's symmetric-splitting integrator and its batch
potentials (the full-HMC baseline integrator of Sec. 4.2.3).

* The batch potentials of a split add up to the full potential and gradient,
  prior included, for an MLP and a DeepONet.
* On the Bayesian linear regression posterior (a one-layer MLP is linear in
  its parameters) the split step is the kick-drift-kick map of the full
  quadratic potential, so it conserves the closed-form shadow energy
  p.p/2 + d.(Lam - eps^2 Lam^2/4) d/2 exactly, for every number of batches.
  An integrator that drifts between batch kicks (the splitting of Neal,
  2011, Sec. 5.1) conserves a different form and fails the same check.
* On a tanh MLP the split trajectory equals the leapfrog trajectory up to
  rounding, is reversible under a momentum flip, and one Metropolis step
  takes the same decision as the leapfrog one.
"""

import math

import numpy as np
import pytest

from oracle import hmc as oh
from oracle import network as on


def _blr(rng, d_in=3, N=41, prior_sd=1.0, lik_sd=0.5):
    X = rng.uniform(-1, 1, (N, d_in))
    Y = rng.normal(size=(N, 1))
    P = d_in + 1
    post = on.MaskedPosterior("mlp", [d_in, 1], None, np.zeros(P), np.arange(P),
                              {"x": X, "y": Y}, prior_sd, lik_sd)
    Phi = np.hstack([X, np.ones((N, 1))])
    Lam = Phi.T @ Phi / lik_sd**2 + np.eye(P) / prior_sd**2
    m = np.linalg.solve(Lam, Phi.T @ Y[:, 0] / lik_sd**2)
    return post, Lam, m


def _bounds(N, M):
    return [round(i * N / M) for i in range(M + 1)]


def _tanh_mlp(rng, N=37):
    widths = [2, 6, 5, 1]
    P = on.net_size("mlp", widths)
    theta = rng.normal(scale=0.6, size=P)
    sel = np.sort(rng.choice(P, 20, replace=False))
    data = {"x": rng.uniform(-1, 1, (N, 2)), "y": rng.normal(size=(N, 1))}
    return on.MaskedPosterior("mlp", widths, None, theta, sel, data, 1.3, 0.4)


def test_batch_potentials_add_up_to_the_potential():
    rng = np.random.default_rng(1)
    mlp = _tanh_mlp(rng)
    wa, wb = [4, 5, 3], [1, 6, 3]
    P = on.net_size("deeponet", wa, wb)
    don = on.MaskedPosterior("deeponet", wa, wb, rng.normal(scale=0.5, size=P),
                             np.sort(rng.choice(P, 25, replace=False)),
                             {"u": rng.normal(size=(9, 4)), "yq": rng.uniform(size=(7, 1)),
                              "v": rng.normal(size=(9, 7))}, 0.8, 0.3)
    for post, N in ((mlp, 37), (don, 9)):
        th = post.theta_fixed[post.sel] + 0.1 * rng.normal(size=post.sel.size)
        U, g = post.potential_and_grad(th)
        for M in (1, 2, 5):
            parts = [b.potential_and_grad(th) for b in on.batch_posteriors(post, _bounds(N, M))]
            assert abs(sum(u for u, _ in parts) - U) <= 1e-12 * abs(U)
            np.testing.assert_allclose(np.sum([gm for _, gm in parts], axis=0), g, rtol=1e-12, atol=1e-12)
    with pytest.raises(ValueError):
        on.batch_posteriors(mlp, [0, 10, 10, 37])
    with pytest.raises(ValueError):
        on.batch_posteriors(mlp, [0, 20])


def _shadow(Lam, m, eps, th, p):
    d = th - m
    return 0.5 * float(p @ p) + 0.5 * float(d @ (Lam - eps * eps * Lam @ Lam / 4) @ d)


@pytest.mark.parametrize("M", [1, 3, 7])
def test_split_step_conserves_the_shadow_energy_of_the_full_potential(M):
    rng = np.random.default_rng(10 + M)
    post, Lam, m = _blr(rng)
    lam_max = np.linalg.eigvalsh(Lam).max()
    eps, L = 1.1 / math.sqrt(lam_max), 23
    th0 = m + rng.normal(size=m.size) / math.sqrt(lam_max)
    p0 = rng.normal(size=m.size)
    batches = [b.potential_and_grad for b in on.batch_posteriors(post, _bounds(41, M))]
    th, p, U, g = oh.split_leapfrog(batches, th0, p0, eps, L)
    s0, s1 = _shadow(Lam, m, eps, th0, p0), _shadow(Lam, m, eps, th, p)
    assert abs(s1 - s0) <= 1e-12 * s0
    # the energy itself moves (the check is not trivially met)
    H0 = post.potential(th0) + 0.5 * p0 @ p0
    assert abs(post.potential(th) + 0.5 * p @ p - H0) > 1e-4
    U_ref, g_ref = post.potential_and_grad(th)
    assert abs(U - U_ref) <= 1e-12 * abs(U_ref)
    np.testing.assert_allclose(g, g_ref, rtol=1e-11, atol=1e-11)


def test_drifts_between_batch_kicks_break_the_shadow_energy():
    """The pin above tells the symmetric split from the data-subset splitting
    that drifts between batch kicks (each batch: half kick, drift eps/M, half
    kick), a different integrator of the same Hamiltonian."""
    rng = np.random.default_rng(30)
    post, Lam, m = _blr(rng)
    lam_max = np.linalg.eigvalsh(Lam).max()
    eps, L, M = 1.1 / math.sqrt(lam_max), 23, 3
    th = m + rng.normal(size=m.size) / math.sqrt(lam_max)
    p = rng.normal(size=m.size)
    s0 = _shadow(Lam, m, eps, th, p)
    batches = [b.potential_and_grad for b in on.batch_posteriors(post, _bounds(41, M))]
    for _ in range(L):
        for f in batches:
            p = p - 0.5 * eps * f(th)[1]
            th = th + eps / M * p
            p = p - 0.5 * eps * f(th)[1]
    assert abs(_shadow(Lam, m, eps, th, p) - s0) > 1e-6 * s0


def test_split_equals_leapfrog_and_is_reversible_on_a_tanh_mlp():
    rng = np.random.default_rng(4)
    post = _tanh_mlp(rng)
    th0 = post.theta_fixed[post.sel].copy()
    p0 = rng.normal(size=th0.size)
    eps, L = 0.02, 15
    batches = [b.potential_and_grad for b in on.batch_posteriors(post, [0, 5, 6, 20, 37])]
    th, p, U, g = oh.split_leapfrog(batches, th0, p0, eps, L)
    th_r, p_r, U_r, g_r = oh.leapfrog(post.potential_and_grad, th0, p0, eps, L)
    assert np.abs(th - th_r).max() <= 1e-12 * np.abs(th_r).max()
    assert np.abs(p - p_r).max() <= 1e-11 * np.abs(p_r).max()
    assert abs(U - U_r) <= 1e-12 * abs(U_r)
    assert np.max(np.abs(th - th0)) > 1e-3          # the trajectory moved
    th_b, p_b, _, _ = oh.split_leapfrog(batches, th, -p, eps, L)
    assert np.abs(th_b - th0).max() <= 1e-11 and np.abs(p_b + p0).max() <= 1e-10


def test_split_transition_takes_the_leapfrog_decision():
    rng = np.random.default_rng(5)
    post = _tanh_mlp(rng)
    th0 = post.theta_fixed[post.sel].copy()
    U0, g0 = post.potential_and_grad(th0)
    batches = [b.potential_and_grad for b in on.batch_posteriors(post, _bounds(37, 4))]
    for it, eps in enumerate((0.01, 0.05, 0.2)):
        p = oh.momentum(9, 0, it, th0.size)
        u = 0.5
        th_s, U_s, _, st_s = oh.split_transition(batches, th0, U0, p, eps, 10, u)
        th_l, U_l, _, st_l = oh.transition(post.potential_and_grad, th0, U0, g0, p, eps, 10, u)
        assert st_s["accepted"] == st_l["accepted"]
        assert abs(st_s["H1"] - st_l["H1"]) <= 1e-10 * abs(st_l["H1"])
        np.testing.assert_allclose(th_s, th_l, rtol=0, atol=1e-11)
