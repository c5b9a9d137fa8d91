"""The launch-shape autotuner: it returns a shape from its candidate set, and
engines built with explicit shapes (every tile height, both workgroup sizes,
both masked-dW forms) give the oracle's gradient to the tolerance of their
precision (FP32: 1e-5 relative, BF16: 3e-2, as for the default engine)."""

import numpy as np
import pytest

import workloads
from oracle import network as on

pytestmark = pytest.mark.gpu


def _tuned(w, prec, tuning):
    """An engine with explicit launch shapes; a tile height that does not
    fit in LDS is reported as unsupported and skipped."""
    from paper_2507_14652_amd import HMCError, Sampler
    from paper_2507_14652_amd.binding import HMC_EUNSUPPORTED
    try:
        return Sampler.from_workload(w, precision=prec, tuning=tuning)
    except HMCError as e:
        if e.status == HMC_EUNSUPPORTED and "LDS" in str(e):
            pytest.skip(f"{tuning}: {e}")
        raise


def _grad_error(w, s):
    U, g = s.grad()
    g = g.double().cpu().numpy()
    worst = 0.0
    for c in range(w.n_chains):
        sl = slice(w.offs[c], w.offs[c + 1])
        th = w.chain_theta(c).astype(np.float32).astype(np.float64)   # as the FP32 state holds it
        _, gr = on.posterior_for_chain(w, c).potential_and_grad(th)
        worst = max(worst, np.linalg.norm(g[sl] - gr) / np.linalg.norm(gr))
    return worst


def test_autotune_returns_a_candidate_shape_mlp():
    from paper_2507_14652_amd import Sampler, autotune_workload
    w = workloads.make("regress2d_fp32", n_rows=700, n_chains=2)
    best, ms = autotune_workload(w, reps=3)
    print("mlp", best, f"{ms:.4f} ms")
    assert best["rows_a"] in (16, 32, 64) and best["rows_b"] == 0
    assert best["threads"] in (256, 512) and best["dw"] in (1, 2)
    assert ms > 0.0
    s = Sampler.from_workload(w, tuning=best)
    assert s.info["rows_per_tile_a"] == best["rows_a"] and s.info["threads_a"] == best["threads"]
    assert _grad_error(w, s) <= 1e-5
    s.close()


def test_autotune_returns_a_candidate_shape_deeponet():
    from paper_2507_14652_amd import Sampler, autotune_workload
    w = workloads.make("antideriv_deeponet_bf16", n_u=70, n_q=21, n_chains=2)
    best, ms = autotune_workload(w, precision="fp32", reps=3)
    print("deeponet", best, f"{ms:.4f} ms")
    assert best["rows_a"] in (16, 32, 64) and best["rows_b"] in (16, 32, 64)
    s = Sampler.from_workload(w, precision="fp32", tuning=best)
    assert s.info["rows_per_tile_b"] == best["rows_b"]
    assert _grad_error(w, s) <= 1e-5
    s.close()


@pytest.mark.parametrize("rows", [16, 32, 64])
@pytest.mark.parametrize("threads", [256, 512])
@pytest.mark.parametrize("dw", [1, 2])
def test_forced_shapes_give_the_oracle_gradient_mlp(rows, threads, dw):
    w = workloads.make("uneven_mlp_bf16", n_rows=150, n_chains=2)
    s = _tuned(w, "bf16", dict(rows_a=rows, threads=threads, dw=dw))
    assert s.info["rows_per_tile_a"] == rows and s.info["threads_a"] == threads
    e = _grad_error(w, s)
    print(rows, threads, dw, f"{e:.2e}")
    assert e <= 3e-2
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-2), ("bf16x3", 1e-4)])
@pytest.mark.parametrize("rows_a,rows_b,threads,dw", [(16, 64, 256, 1), (64, 16, 512, 2), (32, 32, 256, 2)])
def test_forced_shapes_give_the_oracle_gradient_deeponet(prec, tol, rows_a, rows_b, threads, dw):
    w = workloads.make("antideriv_deeponet_bf16", n_u=45, n_q=17, n_chains=2)
    s = _tuned(w, prec, dict(rows_a=rows_a, rows_b=rows_b, threads=threads, dw=dw))
    assert s.info["rows_per_tile_a"] == rows_a and s.info["rows_per_tile_b"] == rows_b
    e = _grad_error(w, s)
    print(prec, rows_a, rows_b, threads, dw, f"{e:.2e}")
    assert e <= tol
    s.close()
