"""Symmetric-splitting HMC on the GPU (hmc_set_split) against the oracle's
split integrator (Sec. 4.2.3's full-HMC baseline).

* Trajectories of the split engine match oracle.hmc.split_leapfrog over the
  same data batches (FP64 1e-11, FP32 1e-5 relative), with a ragged last
  batch and a ragged last row tile, and several batch sizes.
* The FP64 Algorithm 2 loop with the split integrator takes the oracle's
  decisions and positions (oracle.hmc.split_transition).
* Turning the split off gives back the plain leapfrog engine bitwise, and
  the split trajectory equals the plain one up to rounding.
* Argument errors: a DeepONet, a batch size that is not a multiple of the
  row tile, too many batches, a negative size.
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import hmc as oh
from oracle import network as on
from oracle import philox
from paper_2507_14652_amd.binding import HMCError, HMC_EINVAL, HMC_EUNSUPPORTED

pytestmark = pytest.mark.gpu

REL = {"fp64": 1e-11, "fp32": 1e-5}


def _sampler(w, **kw):
    from paper_2507_14652_amd import Sampler
    return Sampler.from_workload(w, **kw)


def _state0(w, c, precision):
    t = w.chain_theta(c)
    return t if precision == "fp64" else t.astype(np.float32).astype(np.float64)


def _bounds(n_rows, batch_rows):
    b = list(range(0, n_rows, batch_rows)) + [n_rows]
    return b


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n_rows,batches", [(1000, 7), (1000, 16), (777, 1)])
def test_split_trajectory_matches_oracle(prec, n_rows, batches):
    w = workloads.make("regress2d_fp32", n_rows=n_rows, n_chains=3)
    s = _sampler(w, precision=prec, seed=3)
    R, tiles = s.info["rows_per_tile_a"], s.info["tiles_a"]
    batch_rows = -(-tiles // batches) * R      # at most `batches` batches of whole tiles
    s.set_split(batch_rows)
    bounds = _bounds(n_rows, batch_rows)
    dt = np.float64 if prec == "fp64" else np.float32
    p0 = np.random.default_rng(8).standard_normal(w.nnz).astype(dt)
    eps, L = 2e-4, 12
    th, p, H0, H1 = s.trajectory(p0, eps, L)
    th, p = th.double().cpu().numpy(), p.double().cpu().numpy()
    print(f"{prec}: {n_rows} rows, tiles of {R}, {len(bounds) - 1} batches of {batch_rows} rows")
    for c in range(w.n_chains):
        post = on.posterior_for_chain(w, c)
        batches = [b.potential_and_grad for b in on.batch_posteriors(post, bounds)]
        sl = slice(w.offs[c], w.offs[c + 1])
        t0 = _state0(w, c, prec)
        U0 = post.potential(t0)
        pc = p0[sl].astype(np.float64)
        tr, pr, Ur, _ = oh.split_leapfrog(batches, t0, pc, eps, L)
        H0r, H1r = U0 + oh.kinetic(pc), Ur + oh.kinetic(pr)
        eth = np.abs(th[sl] - tr).max() / np.abs(tr).max()
        ep = np.abs(p[sl] - pr).max() / np.abs(pr).max()
        moved = np.abs(tr - t0).max() / np.abs(tr).max()
        print(f"  chain {c}: theta {eth:.2e} p {ep:.2e} (moved {moved:.2e}) dH gpu {H1[c] - H0[c]:.6e} "
              f"ref {H1r - H0r:.6e}")
        assert moved > 1e2 * REL[prec]
        assert eth <= REL[prec] and ep <= 10 * REL[prec]
        assert abs(H0[c] - H0r) <= REL[prec] * abs(H0r)
        assert abs(H1[c] - H1r) <= REL[prec] * abs(H1r) + 1e-9
    s.close()


@pytest.mark.parametrize("L", [1, 2])
def test_short_split_trajectories_match_oracle(L):
    """The kick modes at a trajectory's ends: L = 1 goes from the first batch
    kicks straight to the closing ones, L = 2 has one interior step (the
    last drift)."""
    w = workloads.make("regress2d_fp32", n_rows=500, n_chains=2)
    s = _sampler(w, precision="fp64", seed=3)
    R, tiles = s.info["rows_per_tile_a"], s.info["tiles_a"]
    batch_rows = -(-tiles // 3) * R
    s.set_split(batch_rows)
    p0 = np.random.default_rng(12).standard_normal(w.nnz)
    th, p, H0, H1 = s.trajectory(p0, 3e-4, L)
    th, p = th.double().cpu().numpy(), p.double().cpu().numpy()
    s.close()
    for c in range(w.n_chains):
        post = on.posterior_for_chain(w, c)
        batches = [b.potential_and_grad for b in on.batch_posteriors(post, _bounds(500, batch_rows))]
        sl = slice(w.offs[c], w.offs[c + 1])
        tr, pr, Ur, _ = oh.split_leapfrog(batches, w.chain_theta(c), p0[sl], 3e-4, L)
        assert np.abs(th[sl] - tr).max() <= 1e-11 * np.abs(tr).max()
        assert np.abs(p[sl] - pr).max() <= 1e-10 * np.abs(pr).max()
        assert abs(H1[c] - (Ur + oh.kinetic(pr))) <= 1e-11 * abs(H1[c])


def test_split_refused_with_tile_groups(monkeypatch):
    monkeypatch.setenv("HMC_ROWS_A", "32")
    monkeypatch.setenv("HMC_TILE_GROUP", "4")
    w = workloads.make("uneven_mlp_bf16", n_rows=900, n_chains=2)
    s = _sampler(w, precision="fp32")
    assert s.info["rows_per_tile_a"] == 32
    with pytest.raises(HMCError) as e:
        s.set_split(32 * 8)
    assert e.value.status == HMC_EUNSUPPORTED and "tile groups" in str(e.value)
    s.close()


def test_split_off_is_plain_leapfrog_and_split_equals_it_to_rounding():
    w = workloads.make("regress2d_fp32", n_rows=1000, n_chains=2)
    p0 = np.random.default_rng(9).standard_normal(w.nnz)
    plain = _sampler(w, precision="fp64", seed=3)
    ref = [x.double().cpu().numpy() if torch.is_tensor(x) else x for x in plain.trajectory(p0, 2e-4, 10)]
    plain.close()
    s = _sampler(w, precision="fp64", seed=3)
    s.set_split(-(-s.info["tiles_a"] // 4) * s.info["rows_per_tile_a"])   # four batches
    split = [x.double().cpu().numpy() if torch.is_tensor(x) else x for x in s.trajectory(p0, 2e-4, 10)]
    s.set_split(0)
    back = [x.double().cpu().numpy() if torch.is_tensor(x) else x for x in s.trajectory(p0, 2e-4, 10)]
    s.close()
    for a, b in zip(back, ref):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(split, ref):
        assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max()
    assert not all(np.array_equal(a, b) for a, b in zip(split, ref))   # a different summation order


def test_fp64_split_chain_matches_oracle_chain():
    w = workloads.make("sine1d_fp64", n_rows=256)
    n, eps, L, seed = 20, w.eps, w.L, 77
    s = _sampler(w, seed=seed)
    R = s.info["rows_per_tile_a"]
    batch_rows = 3 * R
    s.set_split(batch_rows)
    out = torch.empty((n, w.nnz), dtype=torch.float64, device="cuda")
    _, stats = s.sample(n, eps, L, out=out)
    got = out.cpu().numpy()
    s.close()
    post = on.posterior_for_chain(w, 0)
    batches = [b.potential_and_grad for b in on.batch_posteriors(post, _bounds(256, batch_rows))]
    theta = w.chain_theta(0).astype(np.float64)
    U = post.potential(theta)
    acc, ref = [], []
    for it in range(n):
        p = oh.momentum(seed, 0, it, theta.size)
        u = philox.metropolis_uniform(seed, 0, it)
        theta, U, _, st = oh.split_transition(batches, theta, U, p, eps, L, u)
        acc.append(st["accepted"])
        ref.append(theta)
    ref = np.array(ref)
    print("acceptance", np.mean(acc), "gpu", stats["accepted"][:, 0].mean())
    assert any(acc)
    np.testing.assert_array_equal(stats["accepted"][:, 0].astype(bool), np.array(acc))
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_split_argument_errors():
    w = workloads.make("regress2d_fp32", n_rows=2000, n_chains=2)
    s = _sampler(w, precision="fp32")
    R = s.info["rows_per_tile_a"]
    for rows, status in ((R + 1, HMC_EINVAL), (-R, HMC_EINVAL), (R, HMC_EINVAL)):   # 2000 / R > 16 batches
        with pytest.raises(HMCError) as e:
            s.set_split(rows)
        assert e.value.status == status
    s.set_split(0)
    s.close()
    d = workloads.make("antideriv_deeponet_bf16", n_u=64, n_q=29, n_chains=2)
    s = _sampler(d, precision="fp32")
    with pytest.raises(HMCError) as e:
        s.set_split(s.info["rows_per_tile_a"])
    assert e.value.status == HMC_EUNSUPPORTED
    s.close()
