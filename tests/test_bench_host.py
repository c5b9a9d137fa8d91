"""Host-side pieces of the benchmark: the effective-sample-size estimator
against chains with known ESS, the algorithmic flop count against a hand
count, and the traffic record's source-hash guard."""

import json
import os

import numpy as np

import bench
import workloads


def test_bulk_ess_of_independent_draws():
    x = np.random.default_rng(0).normal(size=(2000, 4, 5))
    ess = bench.bulk_ess(x)
    assert np.all(np.abs(ess / 8000 - 1) < 0.15)


def test_bulk_ess_of_ar1_chains():
    rng = np.random.default_rng(1)
    phi, N = 0.8, 6000
    x = np.zeros((N, 2, 4))
    for t in range(1, N):
        x[t] = phi * x[t - 1] + rng.normal(size=(2, 4))
    expect = 2 * N * (1 - phi) / (1 + phi)
    assert np.all(np.abs(bench.bulk_ess(x) / expect - 1) < 0.2)


def test_bulk_ess_sees_chains_that_disagree():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1000, 4, 2))
    x[:, 0, :] += 5.0          # one chain stuck elsewhere
    assert np.all(bench.bulk_ess(x) < 400)


def test_algorithmic_flops_hand_count():
    w = workloads.make("regress2d_fp32", n_rows=10, n_chains=1, mask_frac=1.0)
    mm = 2 * 64 + 64 * 64 + 64 * 64 + 64
    # forward, adjoint above the first layer, one product per selected entry
    expect = 2 * 10 * mm + 2 * 10 * (mm - 2 * 64) + 2 * 10 * w.n_params
    assert bench.algorithmic_flops(w) == expect


def test_recorded_traffic_requires_matching_kernel_source(tmp_path, monkeypatch):
    rec = os.path.join(bench.ROOT, "profiles", "k_mlp_grad_regress2d_fp32_traffic.json")
    d = json.load(open(rec))
    fake = tmp_path / "profiles"
    fake.mkdir()
    d["kernel_source_sha256"] = "0" * 64
    (fake / "k_mlp_grad_regress2d_fp32_traffic.json").write_text(json.dumps(d))
    csrc = tmp_path / "paper_2507_14652_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "hmc_kernels.hip").write_text("changed")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("k_mlp_grad", "regress2d_fp32") is None


def test_split_ess_sees_a_drift_inside_one_chain():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(4000, 3))
    assert np.all(np.abs(bench.split_ess(x) / 4000 - 1) < 0.15)
    x += np.linspace(0.0, 6.0, 4000)[:, None]     # a trend the chain has not left
    assert np.all(bench.split_ess(x) < 100)


def test_energy_pass_instances_are_told_apart():
    assert bench.energy_pass("void (anonymous namespace)::k_mlp_grad<1, 32, true, false>(GradArgs)")
    assert bench.energy_pass("void (anonymous namespace)::k_branch_grad<1, 64, true>(GradArgs)")
    assert not bench.energy_pass("void (anonymous namespace)::k_mlp_grad<1, 32, false, true>(GradArgs)")
    assert not bench.energy_pass("void (anonymous namespace)::k_branch_grad<3, 32, false>(GradArgs)")
    assert not bench.energy_pass("void (anonymous namespace)::k_update<1>(StateArgs, int, int)")
