"""The trajectory graph with staggered chain halves (the two halves of the
chains as two graph branches, one gradient evaluation apart, so that one
half's k_update runs beside the other half's gradient kernel) gives bitwise
the samples and Metropolis records of the single-branch graph: the chains
are independent and each chain's arithmetic is unchanged.  HMC_HALVES forces
either form on grids small enough to test; MLP and DeepONet, even and odd
chain counts."""

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


CASES = [("uneven_mlp_bf16", dict(n_rows=700)), ("antideriv_deeponet_bf16", dict(n_u=150, n_q=37))]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("chains", [4, 3])
@pytest.mark.parametrize("name,kw", CASES)
def test_halves_match_single_branch_bitwise(name, kw, prec, chains, monkeypatch):
    from paper_2507_14652_amd import Sampler
    w = workloads.make(name, n_chains=chains, **kw)
    res = {}
    for halves in ("0", "1"):
        monkeypatch.setenv("HMC_HALVES", halves)
        s = Sampler.from_workload(w, precision=prec, seed=11)
        out = torch.empty((4, w.nnz), dtype=torch.float32, device="cuda")
        _, st = s.sample(4, np.full(chains, w.eps), 7, out=out)
        th, U, it = s.get_state()
        res[halves] = (out.cpu().numpy(), st, th.cpu().numpy(), U, it)
        s.close()
    a, b = res["0"], res["1"]
    print(f"{name} {prec}, {chains} chains: acceptance {a[1]['accepted'].mean():.2f}")
    assert 0 < a[1]["accepted"].mean()
    np.testing.assert_array_equal(a[0], b[0])
    for f in ("H0", "H1", "log_u", "accepted", "divergent"):
        np.testing.assert_array_equal(a[1][f], b[1][f])
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_array_equal(a[3], b[3])
    np.testing.assert_array_equal(a[4], b[4])


@pytest.mark.parametrize("name,eps", [("uneven_mlp_bf16", None), ("surface_deeponet_bf16", 2e-7)])
def test_halves_at_full_size_match_single_branch_bitwise(name, eps, monkeypatch):
    """The two workloads whose engines stagger the halves by themselves, at
    full size in the launch configuration the bench times (the products
    they sample in, 16-row tiles): the 256-chain, 16,384-row MLP and the
    32-chain 512-wide DeepONet (FP64 energies; a step size near the one its
    adaptation reaches, though from the unadapted start its proposals are
    rejected).  One Metropolis iteration of three leapfrog steps, bitwise
    against the single-branch graph: the end-point energies H1 carry the
    whole trajectory whether or not the proposal is accepted."""
    import dataclasses
    from paper_2507_14652_amd import Sampler
    w = workloads.make(name)
    w = dataclasses.replace(w, precision=w.sample_precision or w.precision)
    e = np.full(w.n_chains, eps or w.eps)
    res = {}
    for halves in ("0", None):
        if halves is None:
            monkeypatch.delenv("HMC_HALVES", raising=False)
        else:
            monkeypatch.setenv("HMC_HALVES", halves)
        s = Sampler.from_workload(w, seed=5)
        assert s.info["rows_per_tile_a"] == 16
        assert s.info["chain_halves"] == (0 if halves == "0" else 1)   # the engine's own choice at full size
        out = torch.empty((1, w.nnz), dtype=s.state_dtype, device="cuda")
        _, st = s.sample(1, e, 3, out=out)
        res[halves] = (out.cpu().numpy(), st)
        s.close()
    a, b = res["0"], res[None]
    print(f"{name} full size: acceptance {a[1]['accepted'].mean():.2f}")
    np.testing.assert_array_equal(a[0], b[0])
    for f in ("H0", "H1", "log_u", "accepted"):
        np.testing.assert_array_equal(a[1][f], b[1][f])
