"""Pins of the oracle's integrator and Metropolis step.

On a quadratic potential the kick-drift-kick leapfrog map is linear and has
closed forms: an exactly conserved shadow energy, and an L-step map given by
Chebyshev polynomials of the one-step map.  On any potential it is exactly
reversible under a momentum flip and its energy error is second order in the
step size.  The sampler as a whole must reproduce known posteriors: the
Bayesian linear regression posterior and a one-dimensional nonlinear
conditional obtained by quadrature.
"""

import math

import numpy as np
import pytest

from oracle import hmc as oh
from oracle import network as on


def _blr_problem(rng, d_in=3, N=40, prior_sd=1.0, lik_sd=0.5):
    X = rng.uniform(-1, 1, (N, d_in))
    Y = rng.normal(size=(N, 1))
    P = d_in + 1
    post = on.MaskedPosterior("mlp", [d_in, 1], None, np.zeros(P), np.arange(P),
                              {"x": X, "y": Y}, prior_sd, lik_sd)
    Phi = np.hstack([X, np.ones((N, 1))])
    Lam = Phi.T @ Phi / lik_sd**2 + np.eye(P) / prior_sd**2
    m = np.linalg.solve(Lam, Phi.T @ Y[:, 0] / lik_sd**2)
    return post, Lam, m


def test_shadow_energy_on_quadratic_potential():
    """H~ = p.p/2 + d.(Lam - eps^2 Lam^2 / 4) d / 2 is conserved exactly, so
    dH = eps^2/8 (|Lam d_L|^2 - |Lam d_0|^2)."""
    rng = np.random.default_rng(20)
    post, Lam, m = _blr_problem(rng)
    lam_max = np.linalg.eigvalsh(Lam).max()
    eps, L = 1.2 / math.sqrt(lam_max), 37
    th0 = m + rng.normal(size=m.size) / math.sqrt(lam_max)
    p0 = rng.normal(size=m.size)
    U0, _ = post.potential_and_grad(th0)
    thL, pL, UL, _ = oh.leapfrog(post.potential_and_grad, th0, p0, eps, L)
    dH = (UL + 0.5 * pL @ pL) - (U0 + 0.5 * p0 @ p0)
    d0, dL = th0 - m, thL - m
    expect = eps**2 / 8 * ((Lam @ dL) @ (Lam @ dL) - (Lam @ d0) @ (Lam @ d0))
    assert abs(dH - expect) <= 1e-9 * (abs(expect) + 1e-3)
    assert abs(expect) > 1e-3    # the test is not vacuous


def _chebyshev_map(lam, eps, L):
    """L-th power of the one-step map [[c, eps], [-eps lam (1 - eps^2 lam/4), c]],
    c = 1 - eps^2 lam / 2 = cos(phi), via M^L = S_L M - S_{L-1} I."""
    c = 1 - eps * eps * lam / 2
    phi = math.acos(c)
    M = np.array([[c, eps], [-eps * lam * (1 - eps * eps * lam / 4), c]])
    sL, sL1 = math.sin(L * phi) / math.sin(phi), math.sin((L - 1) * phi) / math.sin(phi)
    return sL * M - sL1 * np.eye(2)


@pytest.mark.parametrize("with_mass", [False, True])
def test_closed_form_trajectory_on_quadratic_potential(with_mass):
    rng = np.random.default_rng(21)
    post, Lam, m = _blr_problem(rng, d_in=4)
    n = m.size
    minv = rng.uniform(0.5, 2.0, n) if with_mass else np.ones(n)
    # in coordinates phi = D^-1/2 theta, ptilde = D^1/2 p the mass is the identity
    Dh = np.sqrt(minv)
    Lt = Dh[:, None] * Lam * Dh[None, :]
    lam, Q = np.linalg.eigh(Lt)
    eps, L = 0.9 / math.sqrt(lam.max()), 23
    th0 = m + rng.normal(size=n) * 0.3
    p0 = rng.normal(size=n)
    thL, pL, _, _ = oh.leapfrog(post.potential_and_grad, th0, p0, eps, L,
                                inv_mass=minv if with_mass else None)
    x0 = Q.T @ ((th0 - m) / Dh)
    v0 = Q.T @ (p0 * Dh)
    xL, vL = np.empty(n), np.empty(n)
    for k in range(n):
        xL[k], vL[k] = _chebyshev_map(lam[k], eps, L) @ np.array([x0[k], v0[k]])
    np.testing.assert_allclose(thL, m + Dh * (Q @ xL), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(pL, (Q @ vL) / Dh, rtol=1e-10, atol=1e-10)


def _small_net_posterior(rng):
    widths = [2, 8, 6, 1]
    P = on.tower_size(widths)
    theta_fixed = rng.normal(scale=0.6, size=P)
    sel = np.sort(rng.choice(P, 35, replace=False))
    X = rng.uniform(-1, 1, (50, 2))
    Y = np.sin(2 * X[:, :1]) + 0.1 * rng.normal(size=(50, 1))
    post = on.MaskedPosterior("mlp", widths, None, theta_fixed, sel, {"x": X, "y": Y}, 1.0, 0.3)
    return post, theta_fixed[sel]


def test_reversibility_under_momentum_flip():
    rng = np.random.default_rng(22)
    post, th0 = _small_net_posterior(rng)
    p0 = rng.normal(size=th0.size)
    eps, L = 2e-3, 40
    th1, p1, _, _ = oh.leapfrog(post.potential_and_grad, th0, p0, eps, L)
    assert np.abs(th1 - th0).max() > 1e-3
    th2, p2, _, _ = oh.leapfrog(post.potential_and_grad, th1, -p1, eps, L)
    np.testing.assert_allclose(th2, th0, rtol=0, atol=1e-12 * L * max(1, np.abs(th0).max()))
    np.testing.assert_allclose(-p2, p0, rtol=0, atol=1e-11 * L * max(1, np.abs(p0).max()))


def test_energy_error_is_second_order():
    rng = np.random.default_rng(23)
    post, th0 = _small_net_posterior(rng)
    p0 = rng.normal(size=th0.size)
    T = 0.08
    errs = []
    eps_list = [4e-3, 2e-3, 1e-3]
    U0, _ = post.potential_and_grad(th0)
    H0 = U0 + 0.5 * p0 @ p0
    for eps in eps_list:
        L = int(round(T / eps))
        th, p, U, _ = oh.leapfrog(post.potential_and_grad, th0, p0, eps, L)
        errs.append(abs(U + 0.5 * p @ p - H0))
    slope = np.polyfit(np.log(eps_list), np.log(errs), 1)[0]
    assert 1.8 <= slope <= 2.2, (slope, errs)


def test_exactly_L_gradient_evaluations_after_the_start():
    rng = np.random.default_rng(24)
    post, th0 = _small_net_posterior(rng)
    calls = []

    def counted(th):
        calls.append(1)
        return post.potential_and_grad(th)

    start = post.potential_and_grad(th0)
    oh.leapfrog(counted, th0, np.ones(th0.size), 1e-3, 7, start=start)
    assert len(calls) == 7


def test_momentum_covariance_is_the_mass_matrix():
    """p ~ N(0, M) with M = diag(1 / inv_mass)."""
    minv = np.array([0.25, 1.0, 4.0, 16.0])
    P = np.stack([oh.momentum(5, 0, it, 4, minv) for it in range(20000)])
    np.testing.assert_allclose(P.var(axis=0), 1.0 / minv, rtol=0.05)
    assert np.all(np.abs(P.mean(axis=0)) < 5 * np.sqrt(1.0 / minv / 20000))


def test_metropolis_decisions():
    assert oh.metropolis_accept(10.0, 9.0, 0.999999)          # energy decreased
    assert not oh.metropolis_accept(10.0, float("inf"), 1e-300)
    assert not oh.metropolis_accept(10.0, float("nan"), 1e-300)
    e = math.exp(-1.0)
    assert oh.metropolis_accept(1.0, 2.0, e * (1 - 1e-12))
    assert not oh.metropolis_accept(1.0, 2.0, e * (1 + 1e-12))


def _ess_1d(x):
    """Effective sample size from the initial positive sequence of autocorrelations."""
    x = x - x.mean()
    n = len(x)
    f = np.fft.rfft(x, 2 * n)
    ac = np.fft.irfft(f * np.conj(f))[:n] / (x @ x)
    s = 0.0
    for k in range(1, n - 1, 2):
        pair = ac[k] + ac[k + 1]
        if pair < 0:
            break
        s += pair
    return n / (1 + 2 * s)


def test_sampler_recovers_linear_regression_posterior():
    rng = np.random.default_rng(25)
    post, Lam, m = _blr_problem(rng, d_in=1, N=30, prior_sd=1.0, lik_sd=0.4)
    cov = np.linalg.inv(Lam)
    lam_max = np.linalg.eigvalsh(Lam).max()
    eps = 0.5 / math.sqrt(lam_max)
    samples, stats = oh.sample_chain(post.potential_and_grad, m + 1.0, eps, 6, 3000, seed=99, chain=0)
    s = samples[300:]
    acc = np.mean([st["accepted"] for st in stats])
    assert acc > 0.8
    for k in range(m.size):
        ess = _ess_1d(s[:, k])
        mcse = math.sqrt(cov[k, k] / ess)
        assert abs(s[:, k].mean() - m[k]) < 5 * mcse, (k, s[:, k].mean(), m[k], mcse)
    np.testing.assert_allclose(np.cov(s.T), cov, rtol=0.2, atol=0.2 * np.abs(cov).max())


def test_sampler_recovers_one_dimensional_nonlinear_conditional():
    """One selected weight of a small tanh network: compare the chain's mean
    and variance with the conditional density exp(-U) integrated on a grid."""
    rng = np.random.default_rng(26)
    widths = [1, 3, 1]
    P = on.tower_size(widths)
    theta_fixed = rng.normal(size=P)
    X = rng.uniform(-2, 2, (15, 1))
    Y = np.tanh(1.5 * X) + 0.2 * rng.normal(size=(15, 1))
    sel = np.array([1])     # W1[1][0]
    post = on.MaskedPosterior("mlp", widths, None, theta_fixed, sel, {"x": X, "y": Y}, 1.0, 0.5)
    grid = np.linspace(-6, 6, 20001)
    Ug = np.array([post.potential(np.array([t])) for t in grid])
    w = np.exp(-(Ug - Ug.min()))
    w /= w.sum()
    mean = (grid * w).sum()
    var = ((grid - mean) ** 2 * w).sum()
    samples, stats = oh.sample_chain(post.potential_and_grad, np.array([theta_fixed[1]]), 0.15, 8, 4000,
                                     seed=7, chain=3)
    s = samples[200:, 0]
    ess = _ess_1d(s)
    assert abs(s.mean() - mean) < 5 * math.sqrt(var / ess), (s.mean(), mean)
    assert abs(s.var() - var) < 0.15 * var


# ---------------------------------------------------------------------------
# Step-size adaptation (dual averaging) and the App. C trajectory length.

def test_dual_averaging_fixed_point():
    """When every trajectory accepts with exactly the target probability the
    running deviation stays zero, every step size equals exp(mu) = 10 eps0,
    and so does the average."""
    st = oh.dual_averaging_start(3e-4)
    for _ in range(50):
        e = oh.dual_averaging_update(st, 0.8, target=0.8)
        assert math.isclose(e, 3e-3, rel_tol=1e-12)
    assert math.isclose(math.exp(st["log_bar"]), 3e-3, rel_tol=1e-12)


@pytest.mark.parametrize("target", [0.65, 0.8, 0.9])
def test_dual_averaging_solves_a_known_acceptance_curve(target):
    """With a deterministic acceptance curve alpha(eps) = exp(-(eps/s)^2) the
    averaged step size must converge to the root s sqrt(-ln target), from
    either side (a sign or scale mistake in the update drifts away)."""
    s = 2e-3
    root = s * math.sqrt(-math.log(target))
    for eps0 in (1e-5, 5e-2):
        st = oh.dual_averaging_start(eps0)
        e = eps0
        for _ in range(20000):
            e = oh.dual_averaging_update(st, math.exp(-(e / s) ** 2), target=target)
        assert abs(math.exp(st["log_bar"]) / root - 1.0) < 0.01


def test_acceptance_probability():
    assert oh.acceptance_probability(1.0, 0.5) == 1.0
    assert math.isclose(oh.acceptance_probability(0.5, 1.0), math.exp(-0.5), rel_tol=1e-15)
    assert oh.acceptance_probability(0.0, math.inf) == 0.0
    assert oh.acceptance_probability(0.0, math.nan) == 0.0


def test_adapted_step_size_gives_the_target_acceptance_on_a_gaussian():
    """Adaptation on a 12-dimensional Gaussian with precisions from 1 to 400
    (L = 12), then the expected acceptance at the adapted step size computed
    without the sampler: per dimension the leapfrog is the linear map of one
    step raised to the power L (a matrix power), applied to exact draws of
    the stationary distribution, with H evaluated in closed form."""
    lam = np.geomspace(1.0, 400.0, 12)
    pg = lambda th: (0.5 * float(th @ (lam * th)), lam * th)
    L = 12
    eps_bar, _, used, _ = oh.adapt_chain(pg, np.zeros(12), 1e-3, L, 1500, seed=5, chain=0, target=0.8)
    assert used[0] > 1e-3 and math.log2(used[0] / 1e-3) % 1 == 0   # moved by the starting heuristic
    rng = np.random.default_rng(0)
    n = 200000
    th = rng.standard_normal((n, 12)) / np.sqrt(lam)
    p = rng.standard_normal((n, 12))
    H0 = 0.5 * (lam * th * th).sum(1) + 0.5 * (p * p).sum(1)
    th1, p1 = np.empty_like(th), np.empty_like(p)
    for i, l in enumerate(lam):
        kick = np.array([[1.0, 0.0], [-0.5 * eps_bar * l, 1.0]])      # (theta, p) -> (theta, p - eps/2 l theta)
        drift = np.array([[1.0, eps_bar], [0.0, 1.0]])
        M = np.linalg.matrix_power(kick @ drift @ kick, L)
        th1[:, i], p1[:, i] = M[0, 0] * th[:, i] + M[0, 1] * p[:, i], M[1, 0] * th[:, i] + M[1, 1] * p[:, i]
    H1 = 0.5 * (lam * th1 * th1).sum(1) + 0.5 * (p1 * p1).sum(1)
    acc = np.minimum(1.0, np.exp(np.minimum(H0 - H1, 0.0))).mean()
    assert abs(acc - 0.8) < 0.03, (eps_bar, acc)


def test_trajectory_length_is_a_quarter_period_on_a_unit_gaussian():
    """For a standard normal target the exact flow over time pi/2 turns
    (theta, p) into (p, -theta); the rule at unit variance picks that time,
    so the leapfrog end point is the quarter turn up to O(eps^2)."""
    for eps in (0.05, 0.01):
        L = oh.trajectory_length([1.0], eps)
        assert abs(L * eps - math.pi / 2) <= eps / 2
        th, p, _, _ = oh.leapfrog(lambda t: (0.5 * float(t @ t), t), np.array([0.7, -1.2]), np.array([0.3, 0.9]),
                                  eps, L)
        assert np.abs(th - np.array([0.3, 0.9])).max() < 2 * eps
        assert np.abs(p - np.array([-0.7, 1.2])).max() < 2 * eps


def test_trajectory_length_of_the_app_c_cases():
    """The App. C table prints the posterior variance and the VI-HMC step
    size of each case; the rule gives the step counts in the fixture (the
    paper prints the rule, not the counts).  Median and largest variance."""
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "appc_trajectory_lengths.json")))
    for case in d["cases"]:
        assert oh.trajectory_length([case["posterior_variance"]], case["step_size"]) == case["L"], case
    v = [0.1, 0.4, 0.2, 0.3]
    assert oh.trajectory_length(v, 0.01, "max") == round(math.pi * 0.4 / 0.02)
    assert oh.trajectory_length(v, 0.01, "median") == round(math.pi * 0.25 / 0.02)
    assert oh.trajectory_length([1e-9], 1.0) == 1


@pytest.mark.parametrize("th0,p0,eps0", [(0.7, -0.3, 1e-6), (1.5, 0.9, 40.0), (-0.2, 2.0, 0.8), (0.0, 0.1, 3.0)])
def test_reasonable_step_size_stops_where_one_step_crosses_one_half(th0, p0, eps0):
    """On a unit Gaussian one kick-drift-kick step changes the energy by
    exactly (e^2/8)(theta_1^2 - theta_0^2), theta_1 = theta_0 (1 - e^2/2) + e p_0
    (the conserved shadow energy).  The heuristic must return eps0 times a
    power of two at which that ratio has crossed 1/2, having stayed on the
    starting side at the step before."""
    def ratio(e):
        t1 = th0 * (1 - e * e / 2) + e * p0
        return math.exp(-(e * e / 8) * (t1 * t1 - th0 * th0))
    pg = lambda t: (0.5 * float(t @ t), t.copy())
    e = oh.reasonable_step_size(pg, np.array([th0]), np.array([p0]), eps0)
    k = math.log2(e / eps0)
    assert abs(k - round(k)) < 1e-12 and round(k) != 0
    up = ratio(eps0) > 0.5
    prev = e / 2 if up else e * 2
    assert (ratio(prev) > 0.5) == up
    assert (ratio(e) > 0.5) != up


def test_calibration_brackets_the_step_size_of_the_target_acceptance():
    """Bisection on batch means for a one-dimensional Gaussian and L = 1,
    where the expected acceptance at step size e has a closed form over the
    stationary draws (the one-step energy change is (e^2/8)(theta_1^2 -
    theta_0^2)): after enough rounds of large batches the expected
    acceptance at the returned step size is the target to 0.02."""
    def expected(e, n=400000):
        r = np.random.default_rng(1)
        th, p = r.standard_normal(n), r.standard_normal(n)
        t1 = th * (1 - e * e / 2) + e * p
        return np.minimum(1.0, np.exp(-(e * e / 8) * (t1 * t1 - th * th))).mean()
    pg = lambda t: (0.5 * float(t @ t), t.copy())
    e, mean, _ = oh.calibrate_chain(pg, np.array([0.3]), 1.0, 1, rounds=9, batch=1500, seed=3, chain=0, target=0.8)
    assert abs(expected(e) - 0.8) < 0.02, (e, expected(e), mean)
