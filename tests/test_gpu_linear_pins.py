"""Closed-form pins of the GPU path at the workloads' real shapes, with no
oracle involved.

With only the last layer of an MLP sampled (or part of the last branch layer
and b0 of a DeepONet, the trunk fixed), the network output is linear in the
sampled parameters, F = F_fixed + Phi theta, so the conditional posterior of
Sec. 3.2 is the Bayesian linear regression posterior (textbook, e.g. Bishop,
PRML Sec. 3.3): precision Lam = Phi^T Phi / lik_sd^2 + I / prior_sd^2, mean
m = Lam^-1 Phi^T (y - F_fixed) / lik_sd^2, and
    U(theta) = (theta - m)^T Lam (theta - m) / 2 + |y - F_fixed|^2 / (2 lik_sd^2) - m^T Lam m / 2,
    grad U = Lam (theta - m).
Leapfrog on this quadratic U conserves p.p/2 + d.(Lam - eps^2 Lam^2 / 4) d / 2
exactly (d = theta - m), so H1 - H0 = eps^2/8 (|Lam d_L|^2 - |Lam d_0|^2).
The features Phi come from a plain NumPy forward pass of the fixed layers.

Near the mode the gradient is a small difference of large sums, so its
error is measured against the magnitude of what is summed,
S = | |Phi|^T |F - y| / lik_sd^2 + |theta| / prior_sd^2 | (the gradient
itself is about 1e-3 S at posterior draws): FP64 engines within 1e-12 S,
FP32 engines within 4e-5 S (FP32 rounding of sums over N rows grows like
sqrt(N) eps_32, 8e-6 at N = 16384; measured 2.3e-6 S at N = 4096, 1.0e-5 S
at N = 16384, 3e-7 S on the DeepONet).
U: FP64 1e-10 relative, FP32 1e-5.  Positions after a trajectory: FP64
1e-10, FP32 1e-5 of the largest entry.  H1 - H0 against the shadow-energy
identity: FP64 within 1e-7 of it; FP32 engines take U from FP32 products,
whose error is a few 1e-7 of U itself (measured up to 1.7e-6 of H0 on the
256-wide MLP), so within 1e-3 of it plus 5e-6 of H0."""

import math

import numpy as np
import pytest
import torch


pytestmark = pytest.mark.gpu


from linear_cases import CASES, engine, gaussian as _gaussian


TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_gradient_and_potential_are_the_gaussian_closed_form(label, make, prec):
    desc, Lam, m, const, n, Phi, r0 = make(np.random.default_rng(11))
    s = engine(prec, desc)
    U, g = s.grad()
    th = s.get_state()[0].double().cpu().numpy()
    g = g.double().cpu().numpy()
    absPhi = np.abs(Phi)
    for c in range(len(desc["offs"]) - 1):
        sl = slice(c * n, (c + 1) * n)
        d = th[sl] - m
        g_ref = Lam @ d
        U_ref = 0.5 * d @ Lam @ d + const
        S = np.linalg.norm(absPhi.T @ np.abs(Phi @ th[sl] - r0) / desc["lik_sd"] ** 2
                           + np.abs(th[sl]) / desc["prior_sd"] ** 2)
        eg = np.linalg.norm(g[sl] - g_ref) / S
        eU = abs(U[c] - U_ref) / abs(U_ref)
        print(f"{label} {prec} chain {c}: g err / S {eg:.2e} (|g| / S {np.linalg.norm(g_ref) / S:.1e}), "
              f"U rel {eU:.2e}")
        assert eg <= {"fp64": 1e-12, "fp32": 4e-5}[prec]
        assert eU <= TOL[prec]
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_trajectory_and_shadow_energy_closed_form(label, make, prec):
    """Positions after L steps against the leapfrog map with the closed-form
    gradient, and H1 - H0 against the shadow-energy identity, at a step size
    near the stability limit (eps sqrt(lam_max) = 1.2) so that dH is O(1)."""
    rng = np.random.default_rng(12)
    desc, Lam, m, const, n, _, _ = make(rng)
    s = engine(prec, desc)
    C = len(desc["offs"]) - 1
    eps, L = 1.2 / math.sqrt(np.linalg.eigvalsh(Lam).max()), 25
    dt = np.float64 if prec == "fp64" else np.float32
    p0 = rng.standard_normal(C * n).astype(dt)
    th0 = s.get_state()[0].double().cpu().numpy()
    thL, pL, H0, H1 = s.trajectory(p0, eps, L)
    thL = thL.double().cpu().numpy()
    for c in range(C):
        sl = slice(c * n, (c + 1) * n)
        d, p = th0[sl] - m, p0[sl].astype(np.float64)
        d0 = d.copy()
        for _ in range(L):                          # kick-drift-kick with grad U = Lam d
            p = p - 0.5 * eps * (Lam @ d)
            d = d + eps * p
            p = p - 0.5 * eps * (Lam @ d)
        eth = np.abs(thL[sl] - (d + m)).max() / np.abs(d + m).max()
        shadow = eps**2 / 8 * ((Lam @ d) @ (Lam @ d) - (Lam @ d0) @ (Lam @ d0))
        dH = H1[c] - H0[c]
        print(f"{label} {prec} chain {c}: theta {eth:.2e}, dH {dH:.6f} shadow {shadow:.6f}")
        assert abs(shadow) > 1e-2                   # the check is not vacuous
        assert eth <= TOL[prec]
        if prec == "fp64":
            assert abs(dH - shadow) <= 1e-7 * abs(shadow) + 1e-12 * abs(H0[c])
        else:
            assert abs(dH - shadow) <= 1e-3 * abs(shadow) + 5e-6 * abs(H0[c])
    s.close()


def test_sampler_draws_the_gaussian_posterior():
    """Algorithm 2 on the GPU (FP64, no hidden layer: Bayesian linear
    regression, all parameters sampled), 8 chains: the sample mean of every
    coordinate is within 4 Monte Carlo standard errors of m (batch means) and
    the sample covariance matches Lam^-1 (variances within 15%, correlations
    within 0.1)."""
    from paper_2507_14652_amd import Sampler
    rng = np.random.default_rng(13)
    N, d_in, C, n_iter, burn = 200, 3, 8, 1600, 100
    x = rng.uniform(-1, 1, (N, d_in))
    y = (x @ np.array([0.5, -1.0, 0.3]) + 0.2 + 0.3 * rng.standard_normal(N))[:, None]
    prior_sd, lik_sd = 1.0, 0.3
    P = d_in + 1
    Phi = np.hstack([x, np.ones((N, 1))])
    Lam, m, _ = _gaussian(Phi, y[:, 0], prior_sd, lik_sd)
    S = np.linalg.inv(Lam)
    ev = np.linalg.eigvalsh(Lam)
    eps = 0.5 / math.sqrt(ev.max())
    L = int(math.ceil(1.5 / (eps * math.sqrt(ev.min()))))
    s = Sampler(kind="mlp", widths_a=[d_in, 1], theta0=np.zeros(P), prior_sd=prior_sd, lik_sd=lik_sd,
                precision="fp64", offs=np.arange(C + 1) * P, idx=np.tile(np.arange(P), C),
                theta_init=np.tile(m, C) + 0.1 * rng.standard_normal(C * P), x=x, y=y, seed=31)
    out = torch.empty((n_iter, C * P), dtype=torch.float64, device="cuda")
    _, stats = s.sample(n_iter, eps, L, out=out)
    s.close()
    draws = out.cpu().numpy()[burn:].reshape(n_iter - burn, C, P)
    acc = stats["accepted"].mean()
    flat = draws.reshape(-1, P)
    mean, cov = flat.mean(axis=0), np.cov(flat.T)
    batches = draws.reshape(30, (n_iter - burn) // 30, C, P).mean(axis=1).reshape(-1, P)
    mcse = batches.std(axis=0, ddof=1) / math.sqrt(batches.shape[0])
    sd = np.sqrt(np.diag(S))
    corr = cov / np.sqrt(np.outer(np.diag(cov), np.diag(cov)))
    corr_ref = S / np.outer(sd, sd)
    print(f"acceptance {acc:.3f}, eps {eps:.3e}, L {L}; |mean - m| / mcse {np.abs(mean - m) / mcse}; "
          f"var ratio {np.diag(cov) / np.diag(S)}; max corr err {np.abs(corr - corr_ref).max():.3f}")
    assert 0.5 < acc <= 1.0
    assert np.all(np.abs(mean - m) <= 4 * mcse)
    assert np.all(np.abs(np.diag(cov) / np.diag(S) - 1) <= 0.15)
    assert np.abs(corr - corr_ref).max() <= 0.1
