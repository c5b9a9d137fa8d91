"""hmc_predict_noalloc (the posterior predictive with the library's fixed
device scratch instead of per-call allocations) against hmc_predict, through
the C ABI: two calls in a row on one engine, the second with fewer new
inputs, for an MLP and a DeepONet engine; and a request larger than the
fixed region is refused before any device work."""

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _sampler(name, kw, prec, n):
    from paper_2507_14652_amd import Sampler
    w = workloads.make(name, **kw)
    s = Sampler.from_workload(w, precision=prec, seed=4)
    out = torch.empty((n, w.nnz), dtype=s.state_dtype, device="cuda")
    s.sample(n, w.eps, 5, out=out)
    return w, s, out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_mlp_noalloc_matches_predict_twice(prec):
    w, s, out = _sampler("regress2d_fp32", dict(n_rows=400, n_chains=2), prec, 12)
    rng = np.random.default_rng(1)
    for n_new, chain in ((3000, 1), (700, 0)):
        x_new = rng.uniform(-1, 1, (n_new, 2))
        m_ref, v_ref = s.predict(out, x_new, chain=chain)
        m, v = s.predict(out, x_new, chain=chain, no_alloc=True)
        print(f"MLP {prec} rows {n_new}: mean max diff {np.abs(m - m_ref).max():.1e}")
        np.testing.assert_array_equal(m, m_ref)
        np.testing.assert_array_equal(v, v_ref)
    s.close()


def test_deeponet_noalloc_matches_predict_twice():
    w, s, out = _sampler("antideriv_deeponet_bf16", dict(n_u=60, n_q=25, n_chains=2), "bf16", 6)
    rng = np.random.default_rng(2)
    for n_u, n_q, chain in ((90, 40, 1), (13, 7, 1)):
        u = rng.normal(size=(n_u, w.u.shape[1]))
        yq = rng.uniform(0, 1, (n_q, 1))
        m_ref, v_ref = s.predict(out, chain=chain, u=u, yq=yq)
        m, v = s.predict(out, chain=chain, u=u, yq=yq, no_alloc=True)
        print(f"DeepONet {n_u}x{n_q}: mean max diff {np.abs(m - m_ref).max():.1e}")
        np.testing.assert_array_equal(m, m_ref)
        np.testing.assert_array_equal(v, v_ref)
    s.close()


def test_noalloc_refuses_a_request_beyond_the_fixed_region():
    from paper_2507_14652_amd.binding import HMCError, HMC_EUNSUPPORTED
    w, s, out = _sampler("regress2d_fp32", dict(n_rows=300, n_chains=1), "fp32", 2)
    x_new = np.zeros((1_000_000, 2))            # 88 bytes per row: more than 64 MiB
    th0 = s.get_state()[0].clone()
    with pytest.raises(HMCError) as e:
        s.predict(out, x_new, no_alloc=True)
    assert e.value.status == HMC_EUNSUPPORTED and "scratch" in str(e.value)
    assert torch.equal(s.get_state()[0], th0)
    # a small call still works afterwards
    m_ref, _ = s.predict(out, x_new[:50])
    m, _ = s.predict(out, x_new[:50], no_alloc=True)
    np.testing.assert_array_equal(m, m_ref)
    s.close()
