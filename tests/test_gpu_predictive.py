"""GPU posterior predictive moments against the FP64 oracle, through the C
ABI, on samples the sampler itself drew.  FP64 engines are held to 1e-10
relative; FP32 engines (and BF16 engines, which predict through their FP32
weight shadow) to 1e-5 in the mean and, for the variance (a small spread
around a large mean), 1e-3 relative plus 1e-7 of the largest squared
mean."""

import numpy as np
import pytest
import torch

import workloads
from oracle import predictive as op

pytestmark = pytest.mark.gpu


def _run(name, kw, prec, n, chain, n_new, seed=3):
    from paper_2507_14652_amd import Sampler
    w = workloads.make(name, **kw)
    s = Sampler.from_workload(w, precision=prec, seed=seed)
    out = torch.empty((n, w.nnz), dtype=s.state_dtype, device="cuda")
    s.sample(n, w.eps, w.L, out=out)
    rng = np.random.default_rng(9)
    lo, hi = w.x.min(axis=0), w.x.max(axis=0)
    x_new = rng.uniform(lo, hi, (n_new, w.x.shape[1]))
    return w, s, out, x_new, chain


def _ref(w, out, x_new, chain):
    sl = slice(w.offs[chain], w.offs[chain + 1])
    S = out.double().cpu().numpy()[:, sl]
    return op.predictive_moments("mlp", w.widths_a, None, w.theta0, w.chain_idx(chain), S, {"x": x_new})


@pytest.mark.parametrize("name,kw,prec,n,chain,n_new", [
    ("sine1d_fp64", {}, "fp64", 20, 0, 50),
    ("regress2d_fp32", dict(n_rows=500, n_chains=2), "fp32", 10, 1, 333),
    ("uneven_mlp_bf16", dict(n_rows=200, n_chains=2), "bf16", 6, 1, 70),
])
def test_predictive_moments_match_oracle(name, kw, prec, n, chain, n_new):
    w, s, out, x_new, c = _run(name, kw, prec, n, chain, n_new)
    mean, var = s.predict(out, x_new, chain=c)
    m_ref, v_ref = _ref(w, out, x_new, c)
    em = np.linalg.norm(mean - m_ref) / np.linalg.norm(m_ref)
    print(f"{name} {prec}: mean rel {em:.2e}, var max {v_ref.max():.3e}, "
          f"var err {np.abs(var - v_ref).max():.2e}")
    if prec == "fp64":
        np.testing.assert_allclose(mean, m_ref, rtol=1e-10, atol=1e-12 * np.abs(m_ref).max())
        np.testing.assert_allclose(var, v_ref, rtol=1e-6, atol=1e-12 * np.max(m_ref ** 2))
    else:
        assert em <= 1e-5
        np.testing.assert_allclose(var, v_ref, rtol=1e-3, atol=1e-7 * np.max(m_ref ** 2))
    assert np.all(var >= 0.0)
    s.close()


def test_predict_leaves_the_sampler_state_and_accepts_host_samples():
    w, s, out, x_new, c = _run("regress2d_fp32", dict(n_rows=300, n_chains=3), "fp32", 5, 2, 40)
    th0, U0, it0 = s.get_state()
    g0 = s.grad()[1].clone()
    mean_d, var_d = s.predict(out, x_new, chain=c)
    mean_h, var_h = s.predict(out.cpu().numpy(), x_new, chain=c)
    np.testing.assert_array_equal(mean_d, mean_h)
    np.testing.assert_array_equal(var_d, var_h)
    th1, U1, it1 = s.get_state()
    assert torch.equal(th0, th1) and np.array_equal(U0, U1) and np.array_equal(it0, it1)
    assert torch.equal(g0, s.grad()[1])
    # one sample: zero spread, the mean is that sample's prediction
    m1, v1 = s.predict(out[:1], x_new, chain=c)
    assert np.all(v1 == 0.0)
    s.close()


@pytest.mark.parametrize("prec,n", [("fp32", 5), ("bf16", 4), ("fp64", 3)])
def test_deeponet_predictive_moments_match_oracle(prec, n):
    """New functions and query points (ragged tiles in both towers); the
    combination G = <B_j, T_q> + b0 over the samples."""
    from paper_2507_14652_amd import Sampler
    w = workloads.make("antideriv_deeponet_bf16", n_u=50, n_q=11, n_chains=2)
    s = Sampler.from_workload(w, precision=prec, seed=4)
    out = torch.empty((n, w.nnz), dtype=s.state_dtype, device="cuda")
    s.sample(n, 1e-4, 10, out=out)
    rng = np.random.default_rng(2)
    u_new, yq_new = rng.normal(0, 1, (37, w.u.shape[1])), rng.uniform(0, 1, (19, 1))
    mean, var = s.predict(out, u=u_new, yq=yq_new, chain=1)
    sl = slice(w.offs[1], w.offs[2])
    m_ref, v_ref = op.predictive_moments("deeponet", w.widths_a, w.widths_b, w.theta0, w.chain_idx(1),
                                         out.double().cpu().numpy()[:, sl], {"u": u_new, "yq": yq_new})
    em = np.linalg.norm(mean - m_ref) / np.linalg.norm(m_ref)
    print(f"deeponet {prec}: mean rel {em:.2e}, var err {np.abs(var - v_ref).max():.2e} (max {v_ref.max():.2e})")
    if prec == "fp64":
        np.testing.assert_allclose(mean, m_ref, rtol=1e-10, atol=1e-12 * np.abs(m_ref).max())
        np.testing.assert_allclose(var, v_ref, rtol=1e-6, atol=1e-12 * np.max(m_ref ** 2))
    else:
        assert em <= 1e-5
        np.testing.assert_allclose(var, v_ref, rtol=1e-3, atol=1e-7 * np.max(m_ref ** 2))
    s.close()
