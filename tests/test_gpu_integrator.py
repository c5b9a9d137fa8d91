"""Properties of the GPU leapfrog that hold on any potential, checked on the
tanh networks of the workloads: exact reversibility under a momentum flip
(L steps, flip p, L steps return to (theta_0, -p_0); FP64 within 1e-12 L
relative, FP32 within 1e-5) and a second-order energy error (|dH| at a fixed
integration time T = L eps for eps, eps/2, eps/4 has log-log slope 2 +- 0.2,
FP64)."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

CASES = [
    ("regress2d_fp32", dict(n_rows=1000, n_chains=3), 2e-4),
    ("antideriv_deeponet_bf16", dict(n_u=120, n_q=29, n_chains=2), 1e-3),
]


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,kw,eps", CASES)
def test_reversibility_under_momentum_flip(name, kw, eps, prec):
    from paper_2507_14652_amd import Sampler
    w = workloads.make(name, **kw)
    s = Sampler.from_workload(w, precision=prec)
    L = 20
    dt = np.float64 if prec == "fp64" else np.float32
    p0 = np.random.default_rng(21).standard_normal(w.nnz).astype(dt)
    th0 = s.get_state()[0].double().cpu().numpy()
    thL, pL, _, _ = s.trajectory(p0, eps, L)
    s.set_state(thL)
    thR, pR, _, _ = s.trajectory(-pL, eps, L)
    eth, ep = _rel(thR.double().cpu().numpy(), th0), _rel(-pR.double().cpu().numpy(), p0.astype(np.float64))
    moved = _rel(thL.double().cpu().numpy(), th0)
    print(f"{name} {prec}: theta back {eth:.2e}, p back {ep:.2e} (the forward leg moved theta by {moved:.2e})")
    tol = 1e-12 * L if prec == "fp64" else 1e-5
    assert moved > 1e3 * tol                       # the trajectory went somewhere
    assert eth <= tol and ep <= tol
    s.close()


@pytest.mark.parametrize("name,kw,eps", CASES)
def test_energy_error_is_second_order(name, kw, eps):
    from paper_2507_14652_amd import Sampler
    w = workloads.make(name, **kw)
    s = Sampler.from_workload(w, precision="fp64")
    p0 = np.random.default_rng(22).standard_normal(w.nnz)
    dh = []
    for k in range(3):
        _, _, H0, H1 = s.trajectory(p0, eps / 2**k, 20 * 2**k)
        dh.append(np.mean(np.abs(H1 - H0)))
    slope = np.polyfit(np.log([1.0, 0.5, 0.25]), np.log(dh), 1)[0]
    print(f"{name}: mean |dH| {dh}, slope {slope:.3f}")
    assert dh[-1] > 1e-6                              # far above FP64 rounding of H
    assert abs(slope - 2.0) <= 0.2
    s.close()
