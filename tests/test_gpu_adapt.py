"""Step-size adaptation on the device (hmc_adapt: dual averaging after each
Metropolis step, inside the trajectory graph) against the oracle's
adaptation loop, and the acceptance rate it reaches on Gaussian targets
whose chains sample subsets of different sizes."""

import math

import numpy as np
import pytest
import torch

import workloads
from oracle import hmc as oh
from oracle import network as on

pytestmark = pytest.mark.gpu


def _Sampler():
    from paper_2507_14652_amd import Sampler
    return Sampler


def test_fp64_adaptation_matches_the_oracle():
    """Three chains with masks of 5, 40 and 120 entries of a 2-16-16-1 tanh
    MLP, FP64: the adapted step sizes and the end positions equal the
    oracle's adaptation loop on the same Philox streams."""
    rng = np.random.default_rng(4)
    widths = [2, 16, 16, 1]
    P = on.tower_size(widths)
    th0 = rng.normal(scale=0.5, size=P)
    X = rng.uniform(-1, 1, (200, 2))
    Y = np.sin(2 * X[:, :1]) + 0.1 * rng.normal(size=(200, 1))
    sels = [np.sort(rng.choice(P, k, replace=False)) for k in (5, 40, 120)]
    offs = np.concatenate([[0], np.cumsum([len(s) for s in sels])])
    seed, n, L = 31, 30, 8
    eps0 = np.array([1e-3, 3e-4, 5e-2])
    s = _Sampler()(kind="mlp", widths_a=widths, theta0=th0, prior_sd=1.0, lik_sd=0.1, precision="fp64",
                   offs=offs, idx=np.concatenate(sels), x=X, y=Y, seed=seed)
    eps_bar = s.adapt(n, eps0, L)
    th = s.get_state()[0].cpu().numpy()
    s.close()
    for c, sel in enumerate(sels):
        post = on.MaskedPosterior("mlp", widths, None, th0, sel, {"x": X, "y": Y}, 1.0, 0.1)
        e_ref, th_ref, used, st = oh.adapt_chain(post.potential_and_grad, th0[sel], eps0[c], L, n, seed, c)
        acc = np.mean([x["accepted"] for x in st])
        print(f"chain {c}: {len(sel)} entries, eps {eps0[c]:.1e} -> {eps_bar[c]:.6e} (oracle {e_ref:.6e}), "
              f"acceptance during adaptation {acc:.2f}")
        assert abs(eps_bar[c] / e_ref - 1) < 1e-6     # device and host exp, log and pow differ in the last bits
        np.testing.assert_allclose(th[offs[c]:offs[c + 1]], th_ref, rtol=1e-6, atol=1e-6 * np.abs(th_ref).max())


def _blr_subsets(rng, sizes, N=400, d=60, lik_sd=0.5):
    """Bayesian linear regression through the engine (an MLP with no hidden
    layer, 60 standard-normal inputs, 400 rows): chain c samples its own
    subset of the 61 parameters with the others fixed at theta0, so its
    conditional posterior is Gaussian with precision Lam_c; each chain
    starts from a draw of it.  The precisions spread over about a factor of
    five, so the acceptance rate falls smoothly with the step size (a
    posterior dominated by one stiff direction makes it oscillate with the
    step size at fixed L, and no step size is then well defined)."""
    X = rng.standard_normal((N, d))
    y = rng.normal(size=(N, 1))
    theta0 = 0.1 * rng.standard_normal(d + 1)
    Phi_all = np.hstack([X, np.ones((N, 1))])
    sels, starts, lams = [], [], []
    for k in sizes:
        sel = np.sort(rng.choice(d + 1, k, replace=False))
        fixed = np.setdiff1d(np.arange(d + 1), sel)
        r = y[:, 0] - Phi_all[:, fixed] @ theta0[fixed]
        Lam = Phi_all[:, sel].T @ Phi_all[:, sel] / lik_sd**2 + np.eye(k)
        m = np.linalg.solve(Lam, Phi_all[:, sel].T @ r / lik_sd**2)
        ev, Q = np.linalg.eigh(Lam)
        sels.append(sel)
        starts.append(m + Q @ (rng.standard_normal(k) / np.sqrt(ev)))
        lams.append(ev)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    desc = dict(kind="mlp", widths_a=[d, 1], theta0=theta0, prior_sd=1.0, lik_sd=lik_sd, offs=offs,
                idx=np.concatenate(sels), theta_init=np.concatenate(starts), x=X, y=y)
    return desc, lams


def _expected_acceptance(lam, eps, L, n=100000):
    """E[min(1, exp(H0 - H1))] of L leapfrog steps of size eps from exact
    draws of a Gaussian with precision eigenvalues lam: per eigen-direction
    the L-step map is a 2 x 2 matrix power, and H is evaluated exactly."""
    r = np.random.default_rng(0)
    th = r.standard_normal((n, lam.size)) / np.sqrt(lam)
    p = r.standard_normal((n, lam.size))
    dH = np.zeros(n)
    for i, l in enumerate(lam):
        kick = np.array([[1.0, 0.0], [-0.5 * eps * l, 1.0]])
        drift = np.array([[1.0, eps], [0.0, 1.0]])
        M = np.linalg.matrix_power(kick @ drift @ kick, L)
        t1, p1 = M[0, 0] * th[:, i] + M[0, 1] * p[:, i], M[1, 0] * th[:, i] + M[1, 1] * p[:, i]
        dH += 0.5 * l * (t1 * t1 - th[:, i] ** 2) + 0.5 * (p1 * p1 - p[:, i] ** 2)
    return float(np.minimum(1.0, np.exp(-np.maximum(dH, 0.0))).mean())


@pytest.mark.parametrize("target", [0.8, 0.65])
def test_adapted_acceptance_on_gaussian_targets_with_uneven_masks(target):
    """Dual averaging from a step size far too small (1e-6), then bisection
    on batch means (8 rounds of 400 iterations): every chain's expected
    acceptance at its final step size (exact, from the closed-form leapfrog
    map) is the target within 0.04 (about two standard errors of the last
    batch means), and
    the acceptance probability averaged over the next 800 iterations of all
    chains within 0.02, for chains whose subsets (20 to 61 of 61 entries)
    differ in size and conditioning.  Dual averaging alone is reported too:
    it settles somewhat above its target."""
    rng = np.random.default_rng(9)
    sizes = [20, 30, 41, 50, 61, 25]
    desc, lams = _blr_subsets(rng, sizes)
    s = _Sampler()(precision="fp32", seed=5, **desc)
    L = 10
    eps_da = s.adapt(800, 1e-6, L, target=target)
    eps, acc_last = s.calibrate(8, 400, eps_da, L, target=target)
    _, st = s.sample(800, eps, L)
    s.close()
    dh = st["H0"] - st["H1"]
    alpha = np.where(np.isfinite(dh), np.minimum(1.0, np.exp(np.minimum(dh, 0.0))), 0.0)
    exp_da = [_expected_acceptance(l, e, L) for l, e in zip(lams, eps_da)]
    exp_cal = [_expected_acceptance(l, e, L) for l, e in zip(lams, eps)]
    print(f"target {target}: dual averaging {np.round(exp_da, 3)}; after bisection {np.round(exp_cal, 3)} "
          f"(last batches {np.round(acc_last, 3)}); sampled per chain {np.round(alpha.mean(axis=0), 3)}, "
          f"all {alpha.mean():.4f}")
    assert len(set(np.round(eps, 12))) == len(sizes)           # each chain has its own step size
    assert np.all(np.abs(np.array(exp_cal) - target) <= 0.04)
    assert abs(alpha.mean() - target) <= 0.02


def test_fp64_calibration_matches_the_oracle():
    """Bisection rounds on the device (sums of the acceptance probability in
    k_traj_end) against the oracle's calibration loop, FP64, two chains."""
    rng = np.random.default_rng(2)
    desc, _ = _blr_subsets(rng, [12, 33], N=120, d=40)
    seed, L = 13, 6
    s = _Sampler()(precision="fp64", seed=seed, **desc)
    eps_in = np.array([0.02, 0.005])
    eps, acc = s.calibrate(3, 7, eps_in, L, target=0.75)
    s.close()
    offs = desc["offs"]
    X, y = desc["x"], desc["y"]
    for c in range(2):
        sel = desc["idx"][offs[c]:offs[c + 1]]
        post = on.MaskedPosterior("mlp", [40, 1], None, desc["theta0"], sel, {"x": X, "y": y}, 1.0, 0.5)
        e_ref, a_ref, _ = oh.calibrate_chain(post.potential_and_grad, desc["theta_init"][offs[c]:offs[c + 1]],
                                             eps_in[c], L, 3, 7, seed, c, target=0.75)
        print(f"chain {c}: eps {eps[c]:.6e} (oracle {e_ref:.6e}), last batch {acc[c]:.4f} ({a_ref:.4f})")
        assert abs(eps[c] / e_ref - 1) < 1e-12 and abs(acc[c] - a_ref) < 1e-9


def test_adapt_leaves_sampling_unchanged_afterwards():
    """The adaptation flag is off after hmc_adapt: a later hmc_sample with
    fixed step sizes gives the same draws as on an engine that never
    adapted but was set to the same state and iteration counters."""
    w = workloads.make("regress2d_fp32", n_rows=500, n_chains=2)
    S = _Sampler()
    a = S.from_workload(w, seed=8)
    a.adapt(5, w.eps, 4)
    th, _, it = a.get_state()
    b = S.from_workload(w, seed=8)
    b.set_state(th, it)
    out_a = torch.empty((3, w.nnz), device="cuda")
    out_b = torch.empty((3, w.nnz), device="cuda")
    a.sample(3, w.eps, 4, out=out_a)
    b.sample(3, w.eps, 4, out=out_b)
    assert torch.equal(out_a, out_b)
    a.close(); b.close()
