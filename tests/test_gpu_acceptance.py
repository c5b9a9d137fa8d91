"""Metropolis decisions of the product precisions against an exact reference
at the real workload masks: the antiderivative DeepONet (1000 functions x
100 points, 5% of 112,257 parameters per chain) and the uneven-chains MLP
(4-256x4-1 over 16,384 rows, masks of 1% to 20% per chain, 32 of its
chains), both at full size.  The reference engine (FP64) adapts the step
sizes to 80% acceptance (dual averaging, then bisection on batch means);
then, 512 times, every engine integrates a trajectory from the same state
with the same momentum, and the two Metropolis decisions for one shared
uniform are compared (as the mean of |alpha - alpha_ref|, the probability
that they differ, and as a count); the reference chain then takes its own
decision.

Parity unpinned: the bounds are the acceptance target of this build
(decisions differ in at most 1% of the trajectories, acceptance rates
within 1 point) for the precision each workload samples in (split BF16 on
the DeepONet, FP32 on the MLP), and measured regression bounds for the
others: plain BF16, whose gradient error moves the energy by far more than
the energy differences that decide acceptance, and split BF16 on the
stiffer MLP."""

import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _synced(name, n_chains, rounds, cands, adapt, calib, seed=7):
    from paper_2507_14652_amd import Sampler
    w = workloads.make(name, n_chains=n_chains)
    ref = Sampler.from_workload(w, precision="fp64", seed=1)
    eng = {p: Sampler.from_workload(w, precision=p, seed=1) for p in cands}
    eps = ref.adapt(adapt, w.eps, w.L)
    eps, _ = ref.calibrate(calib[0], calib[1], eps, w.L)
    rng = np.random.default_rng(seed)
    dec_ref, dec = [], {p: [] for p in cands}
    al_ref, al = [], {p: [] for p in cands}   # acceptance probabilities min(1, exp(H0 - H1))
    prob = lambda h0, h1: np.where(np.isfinite(h1), np.minimum(1.0, np.exp(np.minimum(h0 - h1, 0.0))), 0.0)
    for _ in range(rounds):
        th = ref.get_state()[0]
        p0 = rng.standard_normal(w.nnz)
        logu = np.log(rng.uniform(size=n_chains))
        thL, _, H0, H1 = ref.trajectory(p0, eps, w.L)
        d_ref = logu < H0 - H1
        dec_ref.append(d_ref)
        al_ref.append(prob(H0, H1))
        for p, s in eng.items():
            s.set_state(th.float())
            _, _, h0, h1 = s.trajectory(p0.astype(np.float32), eps, w.L)
            dec[p].append(logu < h0 - h1)
            al[p].append(prob(h0, h1))
        new = th.clone()
        for c in range(n_chains):
            if d_ref[c]:
                new[w.offs[c]:w.offs[c + 1]] = thL[w.offs[c]:w.offs[c + 1]]
        ref.set_state(new)
    for s in [ref, *eng.values()]:
        s.close()
    A, AR = np.concatenate(dec_ref), np.concatenate(al_ref)
    out = {}
    for p in cands:
        D, AP = np.concatenate(dec[p]), np.concatenate(al[p])
        # with one shared uniform the two decisions differ with probability
        # |alpha - alpha_ref|: its mean is the disagreement rate, estimated
        # with far less noise than by counting the differing decisions
        out[p] = (float(np.mean(np.abs(AP - AR))), float(AP.mean()), float(AR.mean()), float(np.mean(D != A)))
        print(f"{name} {p}: {D.size} trajectories at eps median {np.median(eps):.3e}: disagreement "
              f"{out[p][0]:.4f} (decisions that differed {out[p][3]:.4f}), acceptance {out[p][1]:.4f} vs "
              f"{out[p][2]:.4f} (FP64)")
    return out


def test_antiderivative_deeponet_decisions():
    r = _synced("antideriv_deeponet_bf16", 64, 8, ["bf16x3", "bf16"], adapt=40, calib=(4, 10))
    differ, acc, acc_ref, _ = r["bf16x3"]
    assert 0.5 < acc_ref < 0.97                       # the decision test is not vacuous
    assert differ <= 0.01 and abs(acc - acc_ref) <= 0.01
    assert r["bf16"][0] <= 0.85                       # measured 0.58 to 0.72 (decisions)


def test_uneven_mlp_decisions():
    """The 256-wide MLP is stiffer: split BF16 (about 16 significant bits per
    product) misses the 1% target there (measured disagreement 0.023 at
    0.62 acceptance), FP32 meets it; the uneven-chains workload therefore
    samples in FP32 when decisions must match exact HMC."""
    r = _synced("uneven_mlp_bf16", 32, 16, ["fp32", "bf16x3"], adapt=15, calib=(3, 5))
    differ, acc, acc_ref, _ = r["fp32"]
    assert 0.5 < acc_ref < 0.99
    assert differ <= 0.01 and abs(acc - acc_ref) <= 0.01
    assert r["bf16x3"][0] <= 0.05                     # measured 0.023
