"""Edge cases and engine behaviour through the C ABI: ragged and tiny row
counts, odd widths, degenerate masks, unsupported shapes, divergent
trajectories, determinism, checkpoint/resume, graph replay against direct
launches, chain subsets, a diagonal mass matrix, and the BF16 Metropolis
decision bound."""

import math

import numpy as np
import pytest
import torch

import workloads
from oracle import hmc as oh
from oracle import network as on

pytestmark = pytest.mark.gpu


def _Sampler():
    from paper_2507_14652_amd import Sampler
    return Sampler


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _mlp_engine(widths, N, sel_per_chain, prec, seed=0, theta0=None, inv_mass=None, rng_seed=1):
    rng = np.random.default_rng(rng_seed)
    P = on.tower_size(widths)
    th0 = rng.normal(scale=0.5, size=P) if theta0 is None else theta0
    X = rng.uniform(-1, 1, (N, widths[0]))
    Y = rng.normal(size=(N, widths[-1]))
    offs = np.concatenate([[0], np.cumsum([len(s) for s in sel_per_chain])])
    idx = np.concatenate(sel_per_chain)
    S = _Sampler()(kind="mlp", widths_a=widths, theta0=th0, prior_sd=0.9, lik_sd=0.4, precision=prec,
                   offs=offs, idx=idx, x=X, y=Y, seed=seed, inv_mass=inv_mass)
    posts = [on.MaskedPosterior("mlp", widths, None, th0, s, {"x": X, "y": Y}, 0.9, 0.4) for s in sel_per_chain]
    return S, posts, th0, offs


def _check(S, posts, th0, offs, prec):
    U, g = S.grad()
    g = g.double().cpu().numpy()
    tol = 1e-11 if prec == "fp64" else 1e-5
    for c, post in enumerate(posts):
        t = th0[post.sel]
        if prec != "fp64":
            t = t.astype(np.float32).astype(np.float64)
        Ur, gr = post.potential_and_grad(t)
        assert abs(U[c] - Ur) <= tol * abs(Ur)
        assert _rel(g[offs[c]:offs[c + 1]], gr) <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N,rows", [(1, None), (15, None), (16, None), (17, None), (63, "64"), (64, "64"),
                                    (65, "64"), (129, "32")])
def test_ragged_and_tiny_row_counts(N, rows, prec, monkeypatch):
    if rows:
        monkeypatch.setenv("HMC_ROWS_A", rows)
    widths = [3, 17, 5, 2]   # odd widths, two outputs
    P = on.tower_size(widths)
    rng = np.random.default_rng(N)
    sels = [np.sort(rng.choice(P, 60, replace=False)) for _ in range(2)]
    S, posts, th0, offs = _mlp_engine(widths, N, sels, prec)
    _check(S, posts, th0, offs, prec)
    S.close()


def test_degenerate_masks():
    widths = [2, 8, 8, 1]
    P = on.tower_size(widths)
    first_layer_w = np.arange(16)
    biases = np.concatenate([np.arange(16, 24), np.arange(88, 96), [104]])
    masks = [
        np.array([0]),                      # one weight of the first layer
        np.array([P - 1]),                  # only the output bias
        biases,                             # only biases
        first_layer_w,                      # only first-layer weights
        np.arange(96, 105),                 # only the output layer
        np.arange(P),                       # everything
    ]
    S, posts, th0, offs = _mlp_engine(widths, 40, masks, "fp64")
    _check(S, posts, th0, offs, "fp64")
    S.close()


def test_deeponet_degenerate_masks():
    wa, wb = [6, 9, 5], [2, 7, 5]
    P = on.net_size("deeponet", wa, wb)
    nbr = on.tower_size(wa)
    rng = np.random.default_rng(3)
    th0 = rng.normal(scale=0.5, size=P)
    u, yq, v = rng.normal(size=(5, 6)), rng.uniform(size=(3, 2)), rng.normal(size=(5, 3))
    masks = [np.array([P - 1]), np.arange(nbr, P - 1), np.arange(0, nbr), np.array([0, nbr, P - 1])]
    offs = np.concatenate([[0], np.cumsum([len(m) for m in masks])])
    S = _Sampler()(kind="deeponet", widths_a=wa, widths_b=wb, theta0=th0, prior_sd=1.1, lik_sd=0.3,
                   precision="fp64", offs=offs, idx=np.concatenate(masks), u=u, yq=yq, v=v)
    U, g = S.grad()
    g = g.cpu().numpy()
    for c, m in enumerate(masks):
        post = on.MaskedPosterior("deeponet", wa, wb, th0, m, {"u": u, "yq": yq, "v": v}, 1.1, 0.3)
        Ur, gr = post.potential_and_grad(th0[m])
        assert abs(U[c] - Ur) <= 1e-11 * abs(Ur)
        assert _rel(g[offs[c]:offs[c + 1]], gr) <= 1e-11
    S.close()


def test_unsupported_shape_is_an_error_not_a_fault():
    from paper_2507_14652_amd.binding import HMCError, HMC_EUNSUPPORTED
    widths = [2, 4096, 4096, 1]
    P = on.tower_size(widths)
    with pytest.raises(HMCError) as e:
        _mlp_engine(widths, 8, [np.array([0, 5])], "bf16", theta0=np.zeros(P))
    assert e.value.status == HMC_EUNSUPPORTED
    assert "LDS" in str(e.value)


def test_divergent_trajectory_is_rejected():
    w = workloads.make("regress2d_fp32", n_rows=300, n_chains=2)
    S = _Sampler().from_workload(w)
    th_before = S.get_state()[0].clone()
    st = S.leapfrog(1e8, 10)
    assert np.all(st["divergent"] == 1) and np.all(st["accepted"] == 0)
    assert torch.equal(S.get_state()[0], th_before)
    acc, div = S.counters()
    assert list(div) == [1, 1] and list(acc) == [0, 0]
    # the chain goes on normally afterwards
    st = S.leapfrog(1e-6, 3)
    assert np.all(st["divergent"] == 0)
    S.close()


def _run(w, n, seed=9, eps=2e-4, L=7):
    S = _Sampler().from_workload(w, seed=seed)
    out = torch.empty((n, w.nnz), dtype=torch.float32, device="cuda")
    _, st = S.sample(n, eps, L, out=out)
    return S, out, st


def test_runs_are_bitwise_reproducible():
    w = workloads.make("regress2d_fp32", n_rows=700, n_chains=3)
    S1, a, st1 = _run(w, 6)
    S2, b, st2 = _run(w, 6)
    assert torch.equal(a, b)
    np.testing.assert_array_equal(st1, st2)
    assert st1["accepted"].sum() > 0
    S1.close(); S2.close()


def test_checkpoint_resume_is_identical():
    w = workloads.make("regress2d_fp32", n_rows=700, n_chains=3)
    S1, full, _ = _run(w, 7)
    S2, head, _ = _run(w, 4)
    th, U, it = S2.get_state()
    assert list(it) == [4, 4, 4]
    S3 = _Sampler().from_workload(w, seed=9)
    S3.set_state(th, it)
    tail = torch.empty((3, w.nnz), dtype=torch.float32, device="cuda")
    S3.sample(3, 2e-4, 7, out=tail)
    assert torch.equal(full[4:], tail)
    assert torch.equal(full[:4], head)
    for s in (S1, S2, S3):
        s.close()


def test_graph_replay_equals_direct_launches():
    w = workloads.make("antideriv_deeponet_bf16", n_u=90, n_q=21, n_chains=3)
    S1 = _Sampler().from_workload(w, seed=4, precision="fp32")
    out = torch.empty((4, w.nnz), dtype=torch.float32, device="cuda")
    _, st1 = S1.sample(4, 3e-4, 5, out=out)
    S2 = _Sampler().from_workload(w, seed=4, precision="fp32")
    rows, st2 = [], []
    for _ in range(4):
        st2.append(S2.leapfrog(3e-4, 5))
        rows.append(S2.get_state()[0].clone())
    assert torch.equal(out, torch.stack(rows))
    np.testing.assert_array_equal(st1, np.stack(st2))
    S1.close(); S2.close()


def test_chain_subset_leaves_other_chains_alone():
    w = workloads.make("regress2d_fp32", n_rows=300, n_chains=3)
    S = _Sampler().from_workload(w, seed=2)
    th0, U0, it0 = S.get_state()
    st = S.leapfrog([1e-5], 4, chains=[1])
    th1, U1, it1 = S.get_state()
    o = w.offs
    assert torch.equal(th1[o[0]:o[1]], th0[o[0]:o[1]]) and torch.equal(th1[o[2]:o[3]], th0[o[2]:o[3]])
    assert list(it1) == [0, 1, 0]
    if st["accepted"][0]:
        assert not torch.equal(th1[o[1]:o[2]], th0[o[1]:o[2]])
    S.close()


def test_diagonal_mass_trajectory_matches_oracle():
    widths = [2, 9, 1]
    P = on.tower_size(widths)
    rng = np.random.default_rng(8)
    minv = rng.uniform(0.3, 3.0, P)
    sel = [np.sort(rng.choice(P, 25, replace=False))]
    S, posts, th0, offs = _mlp_engine(widths, 50, sel, "fp64", inv_mass=minv)
    p0 = rng.normal(size=25)
    th, p, H0, H1 = S.trajectory(p0, 2e-3, 15)
    tr, pr, Ur, _ = oh.leapfrog(posts[0].potential_and_grad, th0[sel[0]], p0, 2e-3, 15, inv_mass=minv[sel[0]])
    np.testing.assert_allclose(th.cpu().numpy(), tr, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(H1[0], Ur + oh.kinetic(pr, minv[sel[0]]), rtol=1e-11)
    # the refresh draws p ~ N(0, M): p * sqrt(minv) is the standard normal stream
    z = S.momentum(3).cpu().numpy() * np.sqrt(minv[sel[0]])
    np.testing.assert_allclose(z, oh.momentum(0, 0, 3, 25), rtol=1e-13)
    S.close()


# FP32 mode meets a 1% bound with a wide margin (measured 2.4e-5).  BF16 mode
# is parity unpinned: its energies come from the FP32 pass, so every decision
# is the exact Metropolis test of the trajectory it integrated, but BF16
# gradients move the end point; near the mode, where the gradient is small
# and BF16 rounding is not, the measured disagreement is 0.17 and the
# acceptance 0.06 lower than FP64 HMC.  The asserted bound is that
# measurement with margin.
@pytest.mark.parametrize("prec,bound,acc_bound", [("bf16", 0.25, 0.10), ("bf16x3", 0.01, 0.01),
                                                  ("fp32", 1e-3, 1e-3)])
def test_metropolis_decisions_agree_with_fp64(prec, bound, acc_bound):
    """From the same states and momenta, the probability that a BF16 (or
    FP32) trajectory and the FP64 oracle trajectory take different Metropolis
    decisions, E|min(1, e^-dH) - min(1, e^-dH_ref)|, is within the bound,
    and so is the difference in acceptance rate.  The chains start at
    their conditional modes (found on the oracle) and the step size is the
    first of a ladder at which the engine accepts between 40% and 95%."""
    from scipy.optimize import minimize
    w = workloads.make("antideriv_deeponet_bf16", n_u=150, n_q=37, n_chains=4)
    posts = [on.posterior_for_chain(w, c) for c in range(w.n_chains)]
    modes = [minimize(p.potential_and_grad, w.chain_theta(c), jac=True, method="L-BFGS-B",
                      options={"maxiter": 400}).x for c, p in enumerate(posts)]
    S = _Sampler().from_workload(w, precision=prec)
    S.set_state(np.concatenate(modes).astype(np.float32))
    start = S.get_state()[0].double().cpu().numpy()
    L = 20
    rng = np.random.default_rng(5)
    eps = None
    for e in (4e-2, 2e-2, 1e-2, 5e-3, 2.5e-3, 1.2e-3, 6e-4):
        acc = []
        for _ in range(4):
            _, _, H0, H1 = S.trajectory(rng.standard_normal(w.nnz).astype(np.float32), e, L)
            acc += [min(1.0, math.exp(min(0.0, h0 - h1))) for h0, h1 in zip(H0, H1)]
        if 0.4 < np.mean(acc) < 0.95:
            eps = e
            break
    assert eps is not None
    dis, acc, acc_ref = [], [], []
    for k in range(20):
        p0 = rng.standard_normal(w.nnz).astype(np.float32)
        _, _, H0, H1 = S.trajectory(p0, eps, L)
        for c in range(w.n_chains):
            sl = slice(w.offs[c], w.offs[c + 1])
            t0 = start[sl]
            U0, g0 = posts[c].potential_and_grad(t0)
            pp = p0[sl].astype(np.float64)
            _, pr, Ur, _ = oh.leapfrog(posts[c].potential_and_grad, t0, pp, eps, L, start=(U0, g0))
            dh_ref = (Ur + oh.kinetic(pr)) - (U0 + oh.kinetic(pp))
            dh = H1[c] - H0[c]
            a = min(1.0, math.exp(min(0.0, -dh))) if math.isfinite(dh) else 0.0
            b = min(1.0, math.exp(min(0.0, -dh_ref))) if math.isfinite(dh_ref) else 0.0
            dis.append(abs(a - b))
            acc.append(a)
            acc_ref.append(b)
    d = float(np.mean(dis))
    print(f"{prec}: eps {eps}, expected decision disagreement {d:.2e}, acceptance {np.mean(acc):.3f} "
          f"vs {np.mean(acc_ref):.3f} over {len(dis)} trajectories")
    assert 0.05 < np.mean(acc_ref) < 0.98     # the test is not vacuous
    assert d <= bound and abs(np.mean(acc) - np.mean(acc_ref)) <= acc_bound
    S.close()


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("L", [1, 2, 3, 6])
@pytest.mark.parametrize("name,kw", [("uneven_mlp_bf16", dict(n_rows=150, n_chains=2)),
                                     ("antideriv_deeponet_bf16", dict(n_u=45, n_q=17, n_chains=2))])
def test_energy_copy_holds_the_end_positions(name, kw, L, prec):
    """BF16 and split-BF16 engines take U in the Hamiltonian from an FP32
    weight copy that only the first and the last drift of a trajectory
    write.  H1 - K(p_L) must equal the U that a fresh state set to theta_L
    gives (every copy rewritten, same energy kernels), for short trajectories
    too (L = 1: the first drift is the last; L = 2: the last kick-drift is
    step 1)."""
    w = workloads.make(name, **kw)
    s = _Sampler().from_workload(w, precision=prec)
    p0 = np.random.default_rng(L).standard_normal(w.nnz).astype(np.float32)
    thL, pL, H0, H1 = s.trajectory(p0, w.eps, L)
    s.set_state(thL)
    _, U, _ = s.get_state()
    p = pL.double().cpu().numpy()
    for c in range(w.n_chains):
        K = 0.5 * float(p[w.offs[c]:w.offs[c + 1]] @ p[w.offs[c]:w.offs[c + 1]])
        print(f"{name} {prec} L={L} chain {c}: H1 {H1[c]:.12e}, U(theta_L) + K {U[c] + K:.12e}")
        assert abs(H1[c] - (U[c] + K)) <= 1e-12 * abs(H1[c])
    s.close()


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("name,kw", [("uneven_mlp_bf16", dict(n_rows=150, n_chains=2)),
                                     ("antideriv_deeponet_bf16", dict(n_u=45, n_q=17, n_chains=2))])
def test_kernel_timing_leaves_the_state_alone(name, kw, prec):
    """hmc_time_kernels after a rejected trajectory: BF16 and split-BF16
    engines define U by the FP32 energy pass, whose partials then hold the
    rejected end point; the hook must leave positions, gradient and U of
    every chain exactly as they were, and the next trajectory's H0 must use
    that U."""
    w = workloads.make(name, **kw)
    s = _Sampler().from_workload(w, precision=prec, seed=3)
    s.sample(2, w.eps, 5)
    st = s.leapfrog(1e3, 4)                              # far too large: rejected
    assert np.all(st["accepted"] == 0)
    th0, U0, _ = s.get_state()
    th0 = th0.clone()
    s.time_kernels(3)
    th1, U1, _ = s.get_state()
    assert torch.equal(th0, th1)
    np.testing.assert_array_equal(U0, U1)
    # H0 of the next trajectory starts from that U
    p0 = np.zeros(w.nnz, dtype=np.float32)
    _, _, H0, _ = s.trajectory(p0, w.eps, 1)
    np.testing.assert_array_equal(H0, U0)
    s.close()
