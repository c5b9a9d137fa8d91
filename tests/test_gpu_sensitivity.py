"""GPU sensitivities (Sec. 3.1) against the FP64 oracle, through the C ABI.

FP64 networks are held to 1e-10 relative; FP32 (and BF16 networks, which the
library evaluates in FP32) to 1e-5 norm-wise and, entry by entry, 1e-4
relative plus 1e-7 of the largest entry.  The sensitive subsets chosen from
the GPU values must equal the oracle's, except for entries whose cumulative
share lies within the rounding of the threshold."""

import numpy as np
import pytest

import workloads
from oracle import sensitivity as osen

pytestmark = pytest.mark.gpu


def _gpu(widths, mu, sigma, x, precision):
    from paper_2507_14652_amd import sensitivities
    return sensitivities(widths_a=widths, theta0=mu, sigma=sigma, x=x, precision=precision)


def _check(got, ref, prec):
    if prec == "fp64":
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-14 * ref.max())
        return
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= 1e-5, rel
    np.testing.assert_allclose(got, ref, rtol=1e-4, atol=1e-7 * ref.max())


def _same_selection(s_gpu, s_ref, tau):
    """Equal subsets, or differences confined to entries whose cumulative
    share (in the oracle's order) is within 1e-6 of tau."""
    a, b = set(osen.select_mask(s_gpu, tau).tolist()), set(osen.select_mask(s_ref, tau).tolist())
    if a == b:
        return True
    order = np.argsort(-s_ref, kind="stable")
    share = np.cumsum(s_ref[order]) / s_ref.sum()
    pos = {int(k): share[i] for i, k in enumerate(order)}
    return all(abs(pos[k] - tau) < 1e-6 for k in a ^ b)


@pytest.mark.parametrize("name,kw,prec", [
    ("sine1d_fp64", {}, "fp64"),
    ("regress2d_fp32", dict(n_rows=300), "fp32"),
    ("regress2d_fp32", dict(n_rows=300), "fp64"),
    ("uneven_mlp_bf16", dict(n_rows=130, n_chains=1), "bf16"),
])
def test_sensitivities_match_oracle(name, kw, prec):
    w = workloads.make(name, **kw)
    rng = np.random.default_rng(7)
    sigma = rng.uniform(0.05, 0.3, w.n_params)
    got = _gpu(w.widths_a, w.theta0, sigma, w.x, prec)
    ref = osen.sensitivities("mlp", w.widths_a, None, w.theta0, sigma, {"x": w.x})
    print(f"{name} {prec}: rel {np.linalg.norm(got - ref) / np.linalg.norm(ref):.2e}")
    _check(got, ref, prec)
    for tau in (0.3, 0.9):
        assert _same_selection(got, ref, tau)


@pytest.mark.parametrize("rows", [1, 15, 16, 17, 65, 129])
def test_multi_output_and_ragged_rows(rows):
    """Three outputs (one pass per output, summed), row counts around the
    tile height."""
    rng = np.random.default_rng(rows)
    widths = [3, 24, 40, 3]
    from oracle import network as on
    P = on.net_size("mlp", widths)
    mu = rng.normal(0, 0.4, P)
    sigma = rng.uniform(0.1, 1.0, P)
    x = rng.uniform(-1, 1, (rows, 3))
    got = _gpu(widths, mu, sigma, x, "fp32")
    ref = osen.sensitivities("mlp", widths, None, mu, sigma, {"x": x})
    _check(got, ref, "fp32")


@pytest.mark.parametrize("name,kw,prec", [
    ("antideriv_deeponet_bf16", dict(n_u=40, n_q=9, n_chains=1), "fp32"),
    ("antideriv_deeponet_bf16", dict(n_u=70, n_q=23, n_chains=1), "fp64"),
    ("antideriv_deeponet_bf16", dict(n_u=33, n_q=17, n_chains=1), "bf16"),
])
def test_deeponet_sensitivities_match_oracle(name, kw, prec):
    """Branch passes seeded with the trunk features of each query point,
    trunk passes with the branch features of each function, b0 in closed
    form; ragged tiles in both towers."""
    from paper_2507_14652_amd import sensitivities
    w = workloads.make(name, **kw)
    rng = np.random.default_rng(8)
    sigma = rng.uniform(0.05, 0.3, w.n_params)
    got = sensitivities(kind="deeponet", widths_a=w.widths_a, widths_b=w.widths_b, theta0=w.theta0, sigma=sigma,
                        u=w.u, yq=w.yq, precision=prec)
    ref = osen.sensitivities("deeponet", w.widths_a, w.widths_b, w.theta0, sigma, {"u": w.u, "yq": w.yq})
    print(f"{name} {prec}: rel {np.linalg.norm(got - ref) / np.linalg.norm(ref):.2e}")
    _check(got, ref, "fp64" if prec == "fp64" else "fp32")
    for tau in (0.3, 0.9):
        assert _same_selection(got, ref, tau)


def test_zero_sigma_gives_zero_sensitivity():
    w = workloads.make("regress2d_fp32", n_rows=64)
    sigma = np.full(w.n_params, 0.1)
    sigma[::7] = 0.0
    got = _gpu(w.widths_a, w.theta0, sigma, w.x, "fp32")
    assert np.all(got[::7] == 0.0) and np.all(got[1::7] > 0.0)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_deeponet_gram_seeded_passes_match_oracle(prec):
    """More functions and query points than latent features (40 and 30
    against p = 16): both towers' passes are seeded with the factor of the
    feature Gram matrix instead of one pass per row; the sums must not
    change."""
    from oracle import network as on
    from paper_2507_14652_amd import sensitivities
    rng = np.random.default_rng(12)
    wa, wb = [20, 32, 16], [1, 24, 16]
    P = on.net_size("deeponet", wa, wb)
    mu = rng.normal(0, 0.3, P)
    sigma = rng.uniform(0.05, 0.3, P)
    u = rng.normal(0, 1, (40, 20))
    yq = rng.uniform(0, 1, (30, 1))
    got = sensitivities(kind="deeponet", widths_a=wa, widths_b=wb, theta0=mu, sigma=sigma, u=u, yq=yq, precision=prec)
    ref = osen.sensitivities("deeponet", wa, wb, mu, sigma, {"u": u, "yq": yq})
    print(f"gram-seeded deeponet {prec}: rel {np.linalg.norm(got - ref) / np.linalg.norm(ref):.2e}")
    _check(got, ref, prec)
