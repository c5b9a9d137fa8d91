"""Split-BF16 engines (float operands, three bf16 MFMAs per product) against
the FP64 oracle.  Each product carries about 16 significant bits, so this
mode has no exact reference either; the asserted bounds are measured
values with margin: gradients 1e-4 norm-wise relative, U 1e-5 (it comes
from the FP32 energy pass), trajectory positions 1e-4 of the largest entry."""

import numpy as np
import pytest

import workloads
from oracle import hmc as oh
from oracle import network as on

pytestmark = pytest.mark.gpu

GRAD_BOUND = 1e-4
THETA_BOUND = 1e-4


def _state0(w, c):
    return w.chain_theta(c).astype(np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dw", ["auto", "dense", "gather"])
@pytest.mark.parametrize("name,kw", [
    ("regress2d_fp32", dict(n_rows=1000, n_chains=3)),
    ("uneven_mlp_bf16", dict(n_rows=200, n_chains=4)),
    ("antideriv_deeponet_bf16", dict(n_u=150, n_q=37, n_chains=2)),
    ("surface_deeponet_bf16", dict(n_u=40, n_q=50, n_chains=2)),
])
def test_split_bf16_gradient_matches_oracle(name, kw, dw, monkeypatch):
    from paper_2507_14652_amd import HMCError, Sampler
    from paper_2507_14652_amd.binding import HMC_EUNSUPPORTED
    if dw != "auto":
        monkeypatch.setenv("HMC_DW", dw)
    w = workloads.make(name, **kw)
    try:
        s = Sampler.from_workload(w, precision="bf16x3")
    except HMCError as e:
        if e.status == HMC_EUNSUPPORTED and "LDS" in str(e):
            pytest.skip(str(e))
        raise
    U, g = s.grad()
    g = g.double().cpu().numpy()
    for c in range(w.n_chains):
        Ur, gr = on.posterior_for_chain(w, c).potential_and_grad(_state0(w, c))
        sl = slice(w.offs[c], w.offs[c + 1])
        eU, eg = abs(U[c] - Ur) / abs(Ur), _rel(g[sl], gr)
        print(f"bf16x3 {dw} {name} chain {c}: U rel {eU:.2e}  g rel {eg:.2e}")
        assert eU <= 1e-5 and eg <= GRAD_BOUND
    s.close()


@pytest.mark.parametrize("name,kw,eps,L", [
    ("regress2d_fp32", dict(n_rows=1000, n_chains=3), 5e-4, 50),
    ("antideriv_deeponet_bf16", dict(n_u=150, n_q=37, n_chains=2), 2e-4, 20),
])
def test_split_bf16_trajectory_matches_oracle(name, kw, eps, L):
    from paper_2507_14652_amd import Sampler
    w = workloads.make(name, **kw)
    s = Sampler.from_workload(w, precision="bf16x3")
    p0 = np.random.default_rng(3).standard_normal(w.nnz).astype(np.float32)
    th, p, H0, H1 = s.trajectory(p0, eps, L)
    th = th.double().cpu().numpy()
    for c in range(w.n_chains):
        post = on.posterior_for_chain(w, c)
        sl = slice(w.offs[c], w.offs[c + 1])
        t0 = _state0(w, c)
        tr, pr, Ur, _ = oh.leapfrog(post.potential_and_grad, t0, p0[sl].astype(np.float64), eps, L)
        H1r = Ur + oh.kinetic(pr)
        eth = np.abs(th[sl] - tr).max() / np.abs(tr).max()
        print(f"bf16x3 {name} chain {c}: theta {eth:.2e}  H1 rel {abs(H1[c] - H1r) / abs(H1r):.2e}")
        assert eth <= THETA_BOUND
        assert abs(H1[c] - H1r) <= 1e-5 * abs(H1r)
    s.close()


def test_split_bf16_is_closer_to_the_oracle_than_bf16():
    """The point of the mode: on the same states, split-BF16 gradients are
    at least 50 times closer to the FP64 gradient than BF16 ones."""
    from paper_2507_14652_amd import Sampler
    w = workloads.make("antideriv_deeponet_bf16", n_u=150, n_q=37, n_chains=2)
    err = {}
    for prec in ("bf16", "bf16x3"):
        s = Sampler.from_workload(w, precision=prec)
        g = s.grad()[1].double().cpu().numpy()
        s.close()
        ref = np.concatenate([on.posterior_for_chain(w, c).potential_and_grad(_state0(w, c))[1]
                              for c in range(w.n_chains)])
        err[prec] = _rel(g, ref)
    print(err)
    assert err["bf16x3"] * 50 <= err["bf16"]


@pytest.mark.parametrize("name,kw", [
    ("uneven_mlp_bf16", dict(n_rows=200, n_chains=3)),
    ("antideriv_deeponet_bf16", dict(n_u=150, n_q=37, n_chains=2)),
])
def test_split_bf16_weight_gradient_paths_agree(name, kw, monkeypatch):
    """The dense tile product (three bf16 MFMAs per term) and the per-entry
    FP32 sums read the same split operands: they agree to FP32 rounding,
    and differ, so both really ran."""
    from paper_2507_14652_amd import Sampler
    out = {}
    monkeypatch.setenv("HMC_ROWS_A", "32")   # the dense product needs tiles of a multiple of 32 rows
    monkeypatch.setenv("HMC_ROWS_B", "32")
    for path in ("dense", "gather"):
        monkeypatch.setenv("HMC_DW", path)
        w = workloads.make(name, **kw)
        s = Sampler.from_workload(w, precision="bf16x3")
        out[path] = s.grad()[1].double().cpu().numpy()
        s.close()
    e = _rel(out["dense"], out["gather"])
    print(f"bf16x3 {name}: dense vs gather {e:.2e}")
    assert 0 < e <= 1e-5
