"""Synced trajectories of every precision against the exact leapfrog,
500 per mode, at the real workload shapes.  The engines sample only the last
layer (the 256-wide MLP of the uneven-chains workload, 16,384 rows) or 200
last-branch-layer entries and b0 (the full-size antiderivative DeepONet), so
the exact trajectory is the leapfrog map with the closed-form gradient
Lam (theta - m) of the Gaussian posterior, in FP64 NumPy.  Every trajectory
starts from the engine's state (a posterior draw) with a fresh momentum, at
a step size giving about 80% acceptance; per trajectory we record
|theta_L - theta_L,ref|_inf / |theta_L,ref|_inf, |dH - dH_ref| and the two
Metropolis decisions for one shared uniform u.

BF16 and split BF16 are parity unpinned; the bounds are the measured values
with margin.  They show what the product precision buys on posteriors of
different stiffness: on the DeepONet split BF16 decides like exact HMC
(0.2% of the decisions differ, acceptance 0.810 against 0.808) where BF16
differs in 57%; the last-layer posterior of the 16,384-row MLP is far
stiffer (largest precision eigenvalue 2.3e8, and near the mode the gradient
is about 1e-3 of the sums it is made of), so the gradient error of split
BF16 products already moves the energy by tens (61% of the decisions
differ) and only FP32 keeps the acceptance rate within 1 point there (0.6%
of the decisions differ, with the output layer and residual in FP64).
"""

import math

import numpy as np
import pytest

from linear_cases import CASES

pytestmark = pytest.mark.gpu

N_TRAJ = 500


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16"])
@pytest.mark.parametrize("label,make", CASES[1:], ids=[c[0] for c in CASES[1:]])
def test_synced_trajectories_against_the_exact_leapfrog(label, make, prec):
    from paper_2507_14652_amd import Sampler
    rng = np.random.default_rng(41)
    desc, Lam, m, const, n, _, _ = make(rng)
    s = Sampler(precision=prec, **desc)
    C = len(desc["offs"]) - 1
    ev = np.linalg.eigvalsh(Lam)
    eps, L = 1.5 / math.sqrt(ev.max()), 20      # about 80% acceptance
    th0 = s.get_state()[0].double().cpu().numpy()
    eth, edh, dis, acc, acc_ref = [], [], [], [], []
    for k in range(N_TRAJ // C):
        p0 = rng.standard_normal(C * n).astype(np.float64 if prec == "fp64" else np.float32)
        thL, _, H0, H1 = s.trajectory(p0, eps, L)
        thL = thL.double().cpu().numpy()
        for c in range(C):
            sl = slice(c * n, (c + 1) * n)
            d, p = th0[sl] - m, p0[sl].astype(np.float64)
            H0r = 0.5 * d @ Lam @ d + 0.5 * p @ p
            for _ in range(L):
                p = p - 0.5 * eps * (Lam @ d)
                d = d + eps * p
                p = p - 0.5 * eps * (Lam @ d)
            dHr = 0.5 * d @ Lam @ d + 0.5 * p @ p - H0r
            dH = H1[c] - H0[c]
            log_u = math.log(rng.uniform(1e-300, 1.0))
            a, b = log_u < -dH, log_u < -dHr
            eth.append(np.abs(thL[sl] - (d + m)).max() / np.abs(d + m).max())
            edh.append(abs(dH - dHr))
            dis.append(a != b)
            acc.append(a)
            acc_ref.append(b)
    s.close()
    eth, edh = np.array(eth), np.array(edh)
    d_rate, a_gpu, a_ref = float(np.mean(dis)), float(np.mean(acc)), float(np.mean(acc_ref))
    print(f"{label} {prec}: {len(dis)} trajectories, eps {eps:.2e}, L {L}: theta err max {eth.max():.2e} "
          f"p99 {np.quantile(eth, 0.99):.2e}; |dH - dH_ref| max {edh.max():.3e} p99 {np.quantile(edh, 0.99):.3e}; "
          f"decisions differ {d_rate:.4f}; acceptance {a_gpu:.3f} vs {a_ref:.3f}")
    assert 0.2 < a_ref < 0.98                         # the decision test is not vacuous
    deep = "DeepONet" in label
    # (p99 of the position error, fraction of differing decisions, acceptance
    # difference): the 1% acceptance target where a precision meets it, and
    # measured values with a margin as regression bounds where it does not
    # (BF16 everywhere: 57% and 83% of the decisions differ; split BF16 on
    # the stiff MLP posterior: 61%)
    bounds = {
        "fp64": (1e-12, 0.002, 0.002),
        "fp32": (1e-5, 0.01 if deep else 0.015, 0.01),
        "bf16x3": (1e-4, 0.01, 0.01) if deep else (1e-5, 0.75, 0.70),
        "bf16": (0.05, 0.70, 0.65) if deep else (0.05, 0.95, 0.90),
    }[prec]
    assert np.quantile(eth, 0.99) <= bounds[0]
    assert d_rate <= bounds[1] and abs(a_gpu - a_ref) <= bounds[2]
