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


def _write_trace(path, rows):
    cols = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id", "Kernel_Name",
            "Correlation_Id", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    with open(path, "w") as f:
        f.write(",".join(cols) + "\n")
        for i, (q, name, t0, t1, grid) in enumerate(rows):
            f.write(f"KERNEL_DISPATCH,1,{q},{q},1,{i + 1},1,\"{name}\",{i + 1},{t0},{t1},{grid},1,1\n")


def test_trajectory_gaps_take_the_union_over_queues(tmp_path):
    """Two branches on two queues: idle time is where no kernel of either
    queue runs inside a trajectory's span, and the summed kernel time shows
    the overlap."""
    g, u = "k_mlp_grad<1, 16, false, false>(GradArgs)", "k_update<1>(StateArgs, int, int)"
    rows = [(1, "k_traj_begin<1>(StateArgs)", 0, 1000, 8),
            (1, g, 1000, 11000, 64), (2, g, 6000, 16000, 64),   # overlap 6000..11000
            (1, u, 11000, 12000, 8), (2, u, 16500, 17000, 8),    # idle 16000..16500
            (1, "k_traj_end<1>(StateArgs, int)", 17000, 18000, 8)]
    p = tmp_path / "trace.csv"
    _write_trace(p, rows)
    line = bench.trajectory_gaps(str(p))[0]
    assert "over 1 trajectories (6 kernel dispatches)" in line
    assert "kernels cover 0.018 ms" in line           # 18000 - 500 ns covered
    assert "idle 0.001 ms" in line                    # 500 ns
    assert "1.343x the covered time" in line          # 23500 / 17500


def test_timed_dispatches_are_the_last_full_grid_launches():
    """The launches bench.py times are the last reps + 1 of each kernel's
    largest grid; half-grid launches of the trajectory graphs and earlier
    full-grid ones are left out."""
    k = "k_mlp_grad<1, 16, false, false>(GradArgs)"
    rows = []
    did = 0
    for grid in (64, 128, 128, 64, 64, 128, 128, 128):
        did += 1
        rows.append({"Kernel_Name": k, "Grid_Size": str(grid), "Dispatch_Id": str(did), "Counter_Value": str(did)})
    got = bench.timed_dispatches(rows, 2)
    assert [r["Dispatch_Id"] for r in got] == ["6", "7", "8"]
