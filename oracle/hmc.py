"""Leapfrog trajectory, Hamiltonian and Metropolis-Hastings step, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Algorithms 1 and 2 of the paper:
  draw p ~ N(0, M); integrate Hamilton's equations (Sec. 2.2) for L steps of
  size eps; accept the end point when the ratio r of exp(-H) values exceeds a
  uniform draw u, else keep the current point; the momentum is discarded.

Readings (the paper leaves these open):
  * kinetic energy K = p^T M^-1 p / 2: the text identifies K with the
    Gaussian log-density of p ~ N(0, M), which carries the one half;
  * the integrator is leapfrog in kick-drift-kick form (the text allows Euler
    or leapfrog; only leapfrog is volume preserving and reversible, which the
    Metropolis correction relies on);
  * r > u is decided as log u < H0 - H1 in FP64, u in the open interval
    (0, 1); a non-finite H1 is a rejected, divergent proposal (Sec. 4.2.3
    reports infinite gradients in full-batch runs);
  * fixed step size, no jitter; M = I unless a diagonal inverse mass is given;
  * symmetric splitting (the integrator the paper's full-HMC baseline takes
    from Cobb and Jalaian, whose algorithm the paper does not restate): the
    potential is a sum of data-batch potentials, each with 1/M of the prior,
    and a step applies their half kicks in batch order, one drift, then
    their half kicks in the mirrored order.  The half kicks on either side of
    the drift act at one position, so in exact arithmetic the step is the
    leapfrog step; only the order in which batch gradients reach p differs.
"""

from __future__ import annotations

import math

import numpy as np

from . import philox


def kinetic(p, inv_mass=None) -> float:
    p = np.asarray(p, dtype=np.float64)
    if inv_mass is None:
        return 0.5 * float(np.dot(p, p))
    return 0.5 * float(np.dot(p * inv_mass, p))


def leapfrog(potential_and_grad, theta, p, eps, L, inv_mass=None, start=None):
    """L kick-drift-kick steps of Hamilton's equations dtheta/dt = M^-1 p,
    dp/dt = -grad U.  Consecutive half kicks are merged, so there are exactly
    L gradient evaluations after the starting one.

    ``start`` = (U, g) at ``theta`` if already known.
    Returns (theta_L, p_L, U_L, g_L)."""
    theta = np.array(theta, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    minv = 1.0 if inv_mass is None else np.asarray(inv_mass, dtype=np.float64)
    U, g = potential_and_grad(theta) if start is None else start
    p = p - 0.5 * eps * g
    for t in range(1, L + 1):
        theta = theta + eps * minv * p
        U, g = potential_and_grad(theta)
        p = p - (eps if t < L else 0.5 * eps) * g
    return theta, p, U, g


def split_leapfrog(batch_potentials, theta, p, eps, L, inv_mass=None):
    """L steps of symmetric-splitting HMC, the integrator of the paper's
    full-HMC baseline (Sec. 4.2.3, after Cobb and Jalaian): with the
    potential split over data batches, U = sum_m U_m, one step of size eps is
    the half kicks -eps/2 grad U_m in batch order m = 1..M, one drift
    eps M^-1 p, then the half kicks in the mirrored order m = M..1.  Every
    batch gradient is evaluated where it is applied, at the position of that
    half step (nothing is cached or merged).

    ``batch_potentials``: the M callables theta -> (U_m, grad U_m).
    Returns (theta_L, p_L, U_L, g_L) with U_L and g_L the sums over the
    batches at theta_L."""
    theta = np.array(theta, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    minv = 1.0 if inv_mass is None else np.asarray(inv_mass, dtype=np.float64)
    for _ in range(L):
        for f in batch_potentials:
            p = p - 0.5 * eps * f(theta)[1]
        theta = theta + eps * minv * p
        for f in reversed(batch_potentials):
            p = p - 0.5 * eps * f(theta)[1]
    parts = [f(theta) for f in batch_potentials]
    U = sum(u for u, _ in parts)
    g = np.sum([gm for _, gm in parts], axis=0)
    return theta, p, U, g


def split_transition(batch_potentials, theta, U, p, eps, L, u, inv_mass=None):
    """One iteration of Algorithm 2 with the symmetric-splitting integrator:
    as ``transition``, the leapfrog replaced by ``split_leapfrog``."""
    H0 = hamiltonian(U, p, inv_mass)
    th1, p1, U1, g1 = split_leapfrog(batch_potentials, theta, p, eps, L, inv_mass)
    H1 = hamiltonian(U1, p1, inv_mass)
    acc = metropolis_accept(H0, H1, u)
    stats = {"H0": H0, "H1": H1, "log_u": math.log(u), "accepted": acc,
             "divergent": not math.isfinite(H1)}
    if acc:
        return th1, U1, g1, stats
    return np.array(theta, dtype=np.float64), U, None, stats


def hamiltonian(U, p, inv_mass=None) -> float:
    return float(U) + kinetic(p, inv_mass)


def metropolis_accept(H0, H1, u) -> bool:
    """Accept iff exp(-H1)/exp(-H0) > u, taken in log space; non-finite H1 rejects."""
    if not math.isfinite(H1):
        return False
    return math.log(u) < H0 - H1


def momentum(seed, chain, iteration, n, inv_mass=None):
    """p ~ N(0, M) for the refresh of (chain, iteration) from the Philox stream."""
    z = philox.normals(seed, chain, iteration, n)
    if inv_mass is None:
        return z
    return z / np.sqrt(np.asarray(inv_mass, dtype=np.float64))


def transition(potential_and_grad, theta, U, g, p, eps, L, u, inv_mass=None):
    """One iteration of the loop of Algorithm 2 from state (theta, U, g) with
    momentum p and uniform u.  Returns the next state and a stats dict."""
    H0 = hamiltonian(U, p, inv_mass)
    th1, p1, U1, g1 = leapfrog(potential_and_grad, theta, p, eps, L, inv_mass, start=(U, g))
    H1 = hamiltonian(U1, p1, inv_mass)
    acc = metropolis_accept(H0, H1, u)
    stats = {"H0": H0, "H1": H1, "log_u": math.log(u), "accepted": acc,
             "divergent": not math.isfinite(H1)}
    if acc:
        return th1, U1, g1, stats
    return np.array(theta, dtype=np.float64), U, g, stats


def sample_chain(potential_and_grad, theta_init, eps, L, n, seed, chain,
                 inv_mass=None, start_iter=0):
    """n iterations of Algorithm 2 for one chain.  Momentum and uniform come
    from the Philox streams keyed by (seed, chain) at iteration
    start_iter + i.  Returns (samples [n, n_s], list of stats)."""
    theta = np.array(theta_init, dtype=np.float64)
    U, g = potential_and_grad(theta)
    out = np.empty((n, theta.size))
    stats = []
    for i in range(n):
        it = start_iter + i
        p = momentum(seed, chain, it, theta.size, inv_mass)
        u = philox.metropolis_uniform(seed, chain, it)
        theta, U, g, st = transition(potential_and_grad, theta, U, g, p, eps, L, u, inv_mass)
        out[i] = theta
        stats.append(st)
    return out, stats


# ---------------------------------------------------------------------------
# Step-size adaptation (Sec. 4.2.3: step sizes for an 80% acceptance rate by
# the dual-averaging scheme of Hoffman and Gelman, 2014) and the trajectory
# length rule of App. C.

DA_GAMMA, DA_T0, DA_KAPPA = 0.05, 10.0, 0.75


def dual_averaging_start(eps0):
    """State of the dual-averaging iteration before the first trajectory:
    no iterations yet, H-bar = 0, log eps-bar = 0, and the shrinkage point
    mu = log(10 eps0)."""
    return {"m": 0, "hbar": 0.0, "log_bar": 0.0, "mu": math.log(10.0 * eps0)}


def dual_averaging_update(state, alpha, target=0.8, gamma=DA_GAMMA, t0=DA_T0, kappa=DA_KAPPA):
    """One update after a trajectory whose acceptance statistic is alpha.
    The iteration drives the running average H-bar of (target - alpha) to
    zero: H-bar_m is the (m + t0)-weighted mean of the deviations, the next
    log step size sits sqrt(m)/gamma * H-bar_m below mu, and the returned
    averaged log step size weighs iterate m by m^-kappa.  Returns the step
    size of the next trajectory (the averaged one is state["log_bar"])."""
    m = state["m"] + 1
    w = 1.0 / (m + t0)
    hbar = (1.0 - w) * state["hbar"] + w * (target - alpha)
    log_eps = state["mu"] - math.sqrt(m) / gamma * hbar
    eta = m ** (-kappa)
    state.update(m=m, hbar=hbar, log_bar=eta * log_eps + (1.0 - eta) * state["log_bar"])
    return math.exp(log_eps)


def acceptance_probability(H0, H1) -> float:
    """Metropolis acceptance probability min(1, exp(H0 - H1)); 0 for a
    non-finite H1 (a divergent trajectory)."""
    if not math.isfinite(H1):
        return 0.0
    return min(1.0, math.exp(min(H0 - H1, 0.0)))


def reasonable_step_size(potential_and_grad, theta, p, eps, inv_mass=None, max_probes=60):
    """Starting step size of the adaptation (the heuristic Hoffman and Gelman
    start dual averaging from): the acceptance ratio exp(H0 - H1) of one
    leapfrog step from (theta, p) decides a direction, up if it exceeds 1/2,
    down otherwise; the step size then doubles (or halves) as long as the
    ratio stays on that side, and the first step size where it crosses is
    returned.  A non-finite H1 counts as ratio 0."""
    U, g = potential_and_grad(np.asarray(theta, dtype=np.float64))
    H0 = hamiltonian(U, p, inv_mass)

    def above(e):
        _, p1, U1, _ = leapfrog(potential_and_grad, theta, p, e, 1, inv_mass, start=(U, g))
        H1 = hamiltonian(U1, p1, inv_mass)
        return math.isfinite(H1) and H0 - H1 > -math.log(2.0)

    up = above(eps)
    for _ in range(max_probes):
        e = 2.0 * eps if up else 0.5 * eps
        eps = e
        if above(e) != up:
            break
    return eps


def adapt_chain(potential_and_grad, theta_init, eps0, L, n, seed, chain, target=0.8,
                inv_mass=None, start_iter=0):
    """n iterations of Algorithm 2 for one chain (the Philox streams of
    sample_chain) whose step size is updated by dual averaging after every
    Metropolis step, starting from the reasonable step size found from eps0
    with the momentum of the first iteration.  Returns (averaged step size
    eps-bar, final theta, the step sizes used, list of stats)."""
    theta = np.array(theta_init, dtype=np.float64)
    U, g = potential_and_grad(theta)
    eps1 = reasonable_step_size(potential_and_grad, theta,
                                momentum(seed, chain, start_iter, theta.size, inv_mass), eps0, inv_mass)
    st_da = dual_averaging_start(eps1)
    eps, used, stats = eps1, [], []
    for i in range(n):
        it = start_iter + i
        p = momentum(seed, chain, it, theta.size, inv_mass)
        u = philox.metropolis_uniform(seed, chain, it)
        used.append(eps)
        theta, U, g, st = transition(potential_and_grad, theta, U, g, p, eps, L, u, inv_mass)
        stats.append(st)
        eps = dual_averaging_update(st_da, acceptance_probability(st["H0"], st["H1"]), target)
    return math.exp(st_da["log_bar"]), theta, used, stats


def trajectory_length(var, eps, mode="median") -> int:
    """Number of leapfrog steps of App. C: pi times the posterior variance
    over twice the step size, rounded to the nearest integer (at least one).
    The posterior variance is the largest ("max") or the median ("median")
    of the given per-parameter variances."""
    v = np.asarray(var, dtype=np.float64).ravel()
    pv = float(v.max()) if mode == "max" else float(np.median(v))
    return max(1, int(round(math.pi * pv / (2.0 * eps))))


def calibrate_chain(potential_and_grad, theta_init, eps0, L, rounds, batch, seed, chain, target=0.8,
                    inv_mass=None, start_iter=0):
    """Bisection of one chain's step size in log eps on the batch mean of
    the acceptance probability: each round runs `batch` iterations of
    Algorithm 2 at the current step size; a mean above the target makes it
    a lower bound, otherwise an upper bound, and the next step size is the
    midpoint of the bounds in log eps (a factor 1.25 up or down while one
    bound is missing).  Returns (final midpoint, last batch mean, theta)."""
    theta = np.array(theta_init, dtype=np.float64)
    U, g = potential_and_grad(theta)
    lo, hi, lx, it, mean = -math.inf, math.inf, math.log(eps0), start_iter, 0.0
    for _ in range(rounds):
        eps, s = math.exp(lx), 0.0
        for _ in range(batch):
            p = momentum(seed, chain, it, theta.size, inv_mass)
            u = philox.metropolis_uniform(seed, chain, it)
            theta, U, g, st = transition(potential_and_grad, theta, U, g, p, eps, L, u, inv_mass)
            s += acceptance_probability(st["H0"], st["H1"])
            it += 1
        mean = s / batch
        if mean > target:
            lo = lx
        else:
            hi = lx
        if math.isfinite(lo) and math.isfinite(hi):
            lx = 0.5 * (lo + hi)
        else:
            lx += math.log(1.25) if math.isfinite(lo) else -math.log(1.25)
    return math.exp(lx), mean, theta
