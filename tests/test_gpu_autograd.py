"""The engine's adjoint behind torch.autograd: checked by finite differences
(torch's gradcheck on an FP64 engine) and against the oracle's gradient."""

import numpy as np
import pytest
import torch

import workloads
from oracle import network as on

pytestmark = pytest.mark.gpu


def test_gradcheck_fp64_engine():
    from paper_2507_14652_amd import Sampler
    from paper_2507_14652_amd.autograd import MaskedPotential
    w = workloads.make("regress2d_fp32", n_rows=40, n_chains=2, widths_a=[2, 8, 8, 1], mask_frac=0.4)
    s = Sampler.from_workload(w, precision="fp64")
    theta = torch.tensor(np.concatenate([w.chain_theta(c) for c in range(2)]), dtype=torch.float64,
                         device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: MaskedPotential.apply(t, s), (theta,), eps=1e-6, atol=1e-6,
                                    rtol=1e-5, nondet_tol=0.0)
    s.close()


@pytest.mark.parametrize("name,kw,prec,tol", [
    ("regress2d_fp32", dict(n_rows=500, n_chains=3), "fp32", 1e-5),
    ("antideriv_deeponet_bf16", dict(n_u=60, n_q=13, n_chains=2), "fp32", 1e-5),
    ("antideriv_deeponet_bf16", dict(n_u=60, n_q=13, n_chains=2), "bf16", 3e-2),
])
def test_backward_matches_oracle_gradient(name, kw, prec, tol):
    """(w . U).backward() gives w_c * grad U_c on chain c's entries."""
    from paper_2507_14652_amd import Sampler
    from paper_2507_14652_amd.autograd import masked_potential
    w = workloads.make(name, **kw)
    s = Sampler.from_workload(w, precision=prec)
    rng = np.random.default_rng(4)
    th = np.concatenate([w.chain_theta(c) for c in range(w.n_chains)]) + 0.01 * rng.standard_normal(w.nnz)
    dt = torch.float64 if prec == "fp64" else torch.float32
    theta = torch.tensor(th, dtype=dt, device="cuda", requires_grad=True)
    U = masked_potential(theta, s)
    weights = torch.arange(1, w.n_chains + 1, dtype=torch.float64, device="cuda")
    (weights * U).sum().backward()
    g = theta.grad.double().cpu().numpy()
    thr = theta.detach().double().cpu().numpy()
    for c in range(w.n_chains):
        sl = slice(w.offs[c], w.offs[c + 1])
        Ur, gr = on.posterior_for_chain(w, c).potential_and_grad(thr[sl])
        e = np.linalg.norm(g[sl] - (c + 1) * gr) / np.linalg.norm((c + 1) * gr)
        print(f"{name} {prec} chain {c}: U rel {abs(U[c].item() - Ur) / abs(Ur):.2e}, grad rel {e:.2e}")
        assert e <= tol
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-3), ("bf16", 3e-2)])
def test_directional_finite_differences(prec, tol):
    """Central differences of U along random directions against the autograd
    gradient, on FP32 and BF16 engines.  The displaced points are rounded to
    the state type and the derivative is taken along the rounded step.
    FP32: U and the gradient come from the same products, so the only gap is
    roundoff over the step.  BF16: U comes from the FP32 energy pass and the
    gradient from the BF16 products, so backward is the derivative of
    forward only to the BF16 gradient error (bounded by tol)."""
    from paper_2507_14652_amd import Sampler
    from paper_2507_14652_amd.autograd import masked_potential
    w = workloads.make("regress2d_fp32", n_rows=600, n_chains=2)
    s = Sampler.from_workload(w, precision=prec)
    rng = np.random.default_rng(6)
    th = np.concatenate([w.chain_theta(c) for c in range(2)]).astype(np.float32)
    theta = torch.tensor(th, device="cuda", requires_grad=True)
    U = masked_potential(theta, s)
    U.sum().backward()
    g = theta.grad.double().cpu().numpy()
    worst = 0.0
    for k in range(4):
        v = rng.standard_normal(w.nnz)
        v /= np.linalg.norm(v)
        h = 2e-3
        tp = (th + h * v).astype(np.float32)
        tm = (th - h * v).astype(np.float32)
        Up = masked_potential(torch.tensor(tp, device="cuda"), s).cpu().numpy()
        Um = masked_potential(torch.tensor(tm, device="cuda"), s).cpu().numpy()
        for c in range(2):
            sl = slice(w.offs[c], w.offs[c + 1])
            d = tp[sl].astype(np.float64) - tm[sl].astype(np.float64)
            fd = Up[c] - Um[c]
            an = float(g[sl] @ d)
            rel = abs(fd - an) / (np.linalg.norm(g[sl]) * np.linalg.norm(d))
            worst = max(worst, rel)
            print(f"{prec} direction {k} chain {c}: dU {fd:.6e}, g.d {an:.6e}, gap / (|g| |d|) {rel:.2e}")
    assert worst <= tol
    s.close()
