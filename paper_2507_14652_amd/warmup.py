"""Warm-up controllers that drive the engine between sampling runs.

Step-size adaptation follows the dual-averaging scheme of Hoffman and Gelman
(2014, Algorithm 5), the method the paper uses to find the step size that
gives 80% acceptance (Sec. 4.3).  Each chain adapts its own step size from
its own Metropolis acceptance probabilities; the engine takes one step size
per chain, so chains with masks of different sizes settle independently.
"""

from __future__ import annotations

import numpy as np


def adapt_step_size(sampler, eps0, L, n_adapt=200, target=0.8, gamma=0.05, t0=10.0, kappa=0.75):
    """Runs n_adapt iterations of the sampler (they move the chains) and
    returns the adapted per-chain step sizes (the dual-averaging iterates)."""
    C = sampler.n_chains
    eps = np.broadcast_to(np.asarray(eps0, dtype=np.float64), (C,)).copy()
    mu = np.log(10.0 * eps)
    hbar = np.zeros(C)
    log_bar = np.zeros(C)
    for m in range(1, n_adapt + 1):
        _, st = sampler.sample(1, eps, L)
        dh = st["H0"][0] - st["H1"][0]
        alpha = np.where(np.isfinite(dh), np.minimum(1.0, np.exp(np.minimum(0.0, np.nan_to_num(dh)))), 0.0)
        w = 1.0 / (m + t0)
        hbar = (1.0 - w) * hbar + w * (target - alpha)
        log_eps = mu - np.sqrt(m) / gamma * hbar
        eta = m ** (-kappa)
        log_bar = eta * log_eps + (1.0 - eta) * log_bar
        eps = np.exp(log_eps)
    return np.exp(log_bar)
