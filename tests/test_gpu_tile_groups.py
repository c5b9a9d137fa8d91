"""The tile-group instance of the FP32 MLP gradient kernel, which sums the
weight-gradient terms of several consecutive row tiles of a chain into one
partial slot (the engine takes it for large grids; HMC_TILE_GROUP forces a
group size here, on a grid small enough for the oracle).

With 32-row tiles of the 256-wide MLP over 900 rows (29 tiles: the last
group of eight holds five, the last tile is ragged) and 1024 rows, groups
of 1, 2, 4 and 8
give the same potential bitwise (the likelihood partials stay per tile) and
gradients equal up to FP32 rounding of the reordered sums (1e-6 relative);
every group size matches the FP64 oracle to 1e-5, and trajectories of 10
leapfrog steps agree to 1e-6 of the largest position.  Summing in a fixed
order, each group size repeats its own result bitwise.
"""

import numpy as np
import pytest

import workloads
from oracle import network as on

pytestmark = pytest.mark.gpu


def _engine(w, group, rows, monkeypatch):
    from paper_2507_14652_amd import Sampler
    monkeypatch.setenv("HMC_ROWS_A", str(rows))
    monkeypatch.setenv("HMC_TILE_GROUP", str(group))
    return Sampler.from_workload(w, precision="fp32", seed=7)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("rows", [32])
@pytest.mark.parametrize("n_rows", [900, 1024])
def test_tile_groups_match_single_tiles_and_the_oracle(n_rows, rows, monkeypatch):
    w = workloads.make("uneven_mlp_bf16", n_rows=n_rows, n_chains=4)
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(w.nnz).astype(np.float32)
    res = {}
    for group in (1, 2, 4, 8):
        s = _engine(w, group, rows, monkeypatch)
        assert s.info["rows_per_tile_a"] == rows
        U, g = s.grad()
        U2, g2 = s.grad()
        g, g2 = g.double().cpu().numpy(), g2.double().cpu().numpy()
        assert np.array_equal(g, g2) and np.array_equal(U, U2)     # fixed summation order
        th, _, H0, H1 = s.trajectory(p0, 5e-5, 10)
        res[group] = (U, g, th.double().cpu().numpy(), H1 - H0)
        s.close()
    U1, g1, th1, dh1 = res[1]
    for group in (2, 4, 8):
        U, g, th, dh = res[group]
        eg = _rel(g, g1)
        eth = np.abs(th - th1).max() / np.abs(th1).max()
        print(f"{n_rows} rows in tiles of {rows}, groups of {group}: U equal {np.array_equal(U, U1)}, g rel {eg:.2e}, "
              f"positions {eth:.2e}, dH {np.abs(dh - dh1).max():.2e}")
        assert np.array_equal(U, U1)
        assert eg <= 1e-6
        assert eth <= 1e-6
    for group, (U, g, _, _) in res.items():
        for c in range(w.n_chains):
            post = on.posterior_for_chain(w, c)
            Ur, gr = post.potential_and_grad(w.chain_theta(c).astype(np.float32).astype(np.float64))
            sl = slice(w.offs[c], w.offs[c + 1])
            assert abs(U[c] - Ur) <= 1e-5 * abs(Ur)
            assert _rel(g[sl], gr) <= 1e-5, (group, c, _rel(g[sl], gr))
