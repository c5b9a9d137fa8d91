"""Synced trajectories of every precision against the exact leapfrog,
500 per mode, at the real workload shapes.  The engines sample only the last
layer (the 256-wide MLP of the uneven-chains workload, 16,384 rows) or 200
last-branch-layer entries and b0 (the full-size antiderivative and surface
DeepONets, the latter with its FP64 energies), so the exact trajectory is
the leapfrog map with the closed-form gradient
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
of the decisions differ, with the output layer and residual in FP64).  The
surface operator (2048 x 512 rows, likelihood sd 5e-3) is stiffer still:
largest precision eigenvalue 6.3e12, so the posterior sd in that direction
(4e-7) is below the FP32 spacing of the mean's entries (up to 37), and near
the mode the gradient is 1.5e-6 of the sums it is made of while FP32
rounding of those 1M-row sums is 1.1e-6 of them.  There FP32 products (with
FP64 energies) differ from exact HMC in 81% of the decisions and split BF16
in 84%; FP64 tiles of the 512-wide towers do not fit in LDS, so no
precision this engine runs at that width meets the 1% target there.
"""

import math

import numpy as np
import pytest

from linear_cases import CASES, engine

pytestmark = pytest.mark.gpu

N_TRAJ = 500


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16"])
@pytest.mark.parametrize("label,make", CASES[1:], ids=[c[0] for c in CASES[1:]])
def test_synced_trajectories_against_the_exact_leapfrog(label, make, prec):
    rng = np.random.default_rng(41)
    desc, Lam, m, const, n, _, _ = make(rng)
    s = engine(prec, desc)
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
    case = "surface" if "surface" in label else "antideriv" if "DeepONet" in label else "mlp"
    # (p99 of the position error, fraction of differing decisions, acceptance
    # difference, p99 of |dH - dH_ref|): the 1% acceptance target where a
    # precision meets it, and measured values with a margin as regression
    # bounds where it does not (BF16 everywhere: 57% and 83% of the decisions
    # differ; split BF16 on the stiff MLP posterior: 61%; every precision
    # that fits on the surface operator: 81-84%, where the energy error
    # bound is what the test guards)
    bounds = {
        "mlp": {"fp64": (1e-12, 0.002, 0.002, 1e-6), "fp32": (1e-5, 0.015, 0.01, 0.3),
                "bf16x3": (1e-5, 0.75, 0.70, 100.0), "bf16": (0.05, 0.95, 0.90, 1e7)},
        "antideriv": {"fp64": (1e-12, 0.002, 0.002, 1e-10), "fp32": (1e-5, 0.01, 0.01, 1e-3),
                      "bf16x3": (1e-4, 0.01, 0.01, 0.03), "bf16": (0.05, 0.70, 0.65, 30.0)},
        "surface": {"fp32": (1e-5, 0.95, 0.95, 150.0), "bf16x3": (1e-5, 0.95, 0.95, 1e6),
                    "bf16": (3e-3, 0.95, 0.95, 5e11)},
    }[case][prec]
    assert np.quantile(eth, 0.99) <= bounds[0]
    assert d_rate <= bounds[1] and abs(a_gpu - a_ref) <= bounds[2]
    assert np.quantile(edh, 0.99) <= bounds[3]
