"""Throughput of masked full-batch HMC on one MI355X.

One step = one iteration of the sampler for every chain: momentum refresh,
L leapfrog steps (each a full-batch forward pass, adjoint pass and masked
weight gradient), Hamiltonian and Metropolis test, and the copy of the new
positions into a device-resident sample buffer.  The metric is leapfrog
gradient evaluations per second summed over chains.

Prints one JSON line.  The default workload is the largest single-GPU
configuration, the batched uneven chains: 256 chains on the MLP
4-256-256-256-256-1 tanh over 16,384 rows, each chain sampling its own 1% to
20% of the parameters, L = 50, per-chain step sizes adapted on the device
toward 80% acceptance before the timed region.  Each workload samples in the
product precision whose Metropolis decisions match FP64 ones on it (FP32
here; the line names it); --config selects another named workload and
--precision another precision.  The line also carries the roofline of the
dominant kernel, the FP64 oracle timed on the host cores, and the ESS/s
comparison with plain single-chain FP32 HMC on the DeepONet workload.
"""

from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X dense peaks; a split-BF16 product is three BF16 MFMAs, so its peak is a third of BF16's
    "f64": 78.6, "f32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0 / 3,
}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16": "bf16", "bf16x3": "bf16x3"}


def algorithmic_flops(w, part=None):
    """Flops one gradient evaluation of every chain must do: forward products,
    adjoint products down to the lowest layer holding a selected entry, and
    2 * rows per selected entry (the masked weight gradient).  DeepONet adds
    the combination G = B T^T and its two adjoint products dB = dG T and
    dT = dG^T B.  part: None for the whole gradient; for DeepONet "branch"
    (branch tower, G and dB: the branch kernel's work) or "trunk" (trunk
    tower and dT)."""
    total = 0.0
    for c in range(w.n_chains):
        idx = w.chain_idx(c)
        if w.kind == "mlp":
            towers = [(w.widths_a, w.x.shape[0], 0, "branch")]
        else:
            nb = sum(w.widths_a[i] * w.widths_a[i + 1] + w.widths_a[i + 1] for i in range(len(w.widths_a) - 1))
            towers = [(w.widths_a, w.u.shape[0], 0, "branch"), (w.widths_b, w.yq.shape[0], nb, "trunk")]
        for widths, rows, flat0, name in towers:
            if part is not None and name != part:
                continue
            starts, pos = [], flat0
            for i in range(len(widths) - 1):
                starts.append(pos)
                pos += widths[i] * widths[i + 1] + widths[i + 1]
            mm = [widths[i] * widths[i + 1] for i in range(len(widths) - 1)]
            sel = [(np.sum((idx >= starts[i]) & (idx < (starts[i + 1] if i + 1 < len(starts) else pos))))
                   for i in range(len(mm))]
            lowest = next((i for i, s in enumerate(sel) if s > 0), len(mm))
            total += 2.0 * rows * sum(mm)                                  # forward
            total += 2.0 * rows * sum(mm[i] for i in range(lowest + 1, len(mm)))   # adjoint products
            total += 2.0 * rows * sum(sel)                                  # masked weight gradient
        if w.kind == "deeponet":
            nu, nq, p = w.u.shape[0], w.yq.shape[0], w.widths_a[-1]
            ncomb = {None: 3, "branch": 2, "trunk": 1}[part]
            total += ncomb * 2.0 * nu * nq * p
    return total


def recorded_traffic(kernel, workload, instance=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (calibrated against a plain copy), or None
    when the kernel source has changed since the counters were taken or they
    were taken on another instance (instance: the prefix of its name, up to
    the tile height)."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_sha256") != _kernel_sha() or (instance and not d.get("instance", "").startswith(instance)):
        return None
    return d["traffic_bytes_per_launch"]


KERNEL_OF = {"mlp": "k_mlp_grad", "deeponet": "k_branch_grad"}
PMC_TIMING_REPS = 5      # --timing-reps of the counter runs below
TRACE_TIMING_REPS = 50   # bench.py's default --timing-reps (the trace run)
PROFILE_CMDS = {
    "trace": "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/trace_{w} -o bench -- "
             "python bench.py --config {w} --steps 5 --warmup 1 --adapt 5 --no-cpu-baseline --no-ess",
    "trace_sens": "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/trace_sens_{w} -o bench -- "
                  "python bench.py --config {w} --sensitivity --steps 3 --no-cpu-baseline",
    "FETCH_SIZE": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_FETCH_SIZE_{w} -o bench -- "
                  "python bench.py --config {w} --steps 2 --warmup 1 --adapt 2 --no-cpu-baseline --no-ess --timing-reps 5",
    "WRITE_SIZE": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_WRITE_SIZE_{w} -o bench -- "
                  "python bench.py --config {w} --steps 2 --warmup 1 --adapt 2 --no-cpu-baseline --no-ess --timing-reps 5",
    "copy": "rocprofv3 --pmc {c} --output-format csv -d gpurun_out/pmc_copy_{c} -o copy -- python -c \"import torch; "
            "a=torch.ones(64*2**20, device='cuda'); b=torch.empty_like(a); torch.cuda.synchronize(); b.copy_(a); "
            "torch.cuda.synchronize()\"",
}
COPY_BYTES = 64 * 2 ** 20 * 4


PRECISION_INDEX = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}


def main_kernel(w):
    """The name prefix of the gradient kernel a workload's sampler runs, as
    rocprofv3 prints it: its product precision, not the energy pass's."""
    return f"{KERNEL_OF[w.kind]}<{PRECISION_INDEX[w.sample_precision or w.precision]}, "


def _kernel_sha():
    src = os.path.join(ROOT, "paper_2507_14652_amd", "csrc", "hmc_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def energy_pass(kernel_name):
    """Whether a gradient-kernel instance, as rocprofv3 names it, is the
    forward-only energy pass (its third template argument, FWD, true)."""
    if "<" not in kernel_name:
        return False
    args = kernel_name[kernel_name.index("<") + 1:].split(">")[0].split(",")
    return len(args) >= 3 and args[2].strip() == "true"


def _grid(r):
    if "Grid_Size" in r:
        return int(r["Grid_Size"])
    return int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])


def timed_dispatches(rows, reps):
    """The rows (rocprofv3 trace or counter records) of the launches that
    bench.py times with HIP events (Sampler.time_kernels: one warm-up launch
    and `reps` timed ones, over the full grid with every chain active, the
    last launches of each kernel in the process): per kernel instance, the
    last reps + 1 dispatches of its largest grid.  The trajectory graphs
    before them may launch a gradient kernel over half of the chains at a
    time (staggered chain halves), and the step-size search with chains
    inactive; neither is the launch the roofline prices."""
    top, by = {}, {}
    for r in rows:
        top[r["Kernel_Name"]] = max(top.get(r["Kernel_Name"], 0), _grid(r))
    for r in rows:
        if _grid(r) == top[r["Kernel_Name"]]:
            by.setdefault(r["Kernel_Name"], {}).setdefault(int(r["Dispatch_Id"]), []).append(r)
    out = []
    for d in by.values():
        for k in sorted(d)[-(reps + 1):]:
            out += d[k]
    return out


def _pmc_mean(csv_path, counter, name_part):
    """Mean per timed dispatch (timed_dispatches) of `counter` over the
    kernels whose name contains name_part (KiB for FETCH_SIZE / WRITE_SIZE), and the dispatch
    count.  Gradient kernels count only in their gradient form, not as the
    forward-only energy pass."""
    import csv
    vals, names = [], set()
    with open(csv_path) as f:
        rows = [r for r in csv.DictReader(f) if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]
                and not energy_pass(r["Kernel_Name"])]
    for r in timed_dispatches(rows, PMC_TIMING_REPS):
        vals.append(float(r["Counter_Value"]))
        names.add(r["Kernel_Name"].replace("void (anonymous namespace)::", ""))
    if not vals:
        raise SystemExit(f"no {counter} rows for {name_part} in {csv_path}")
    if len(names) != 1:
        raise SystemExit(f"{counter}: several instances match {name_part}: {sorted(names)}")
    return sum(vals) / len(vals), len(vals), names.pop()


def record_traffic(workload, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """Writes profiles/<kernel>_<workload>_traffic.json: the dominant kernel's
    HBM bytes per launch from FETCH_SIZE and WRITE_SIZE, each scaled by what
    the counter reads for a plain device copy of known size."""
    import glob
    import workloads
    w = workloads.make(workload, n_chains=1)
    kern = KERNEL_OF[w.kind]
    main = main_kernel(w)
    one = lambda d: glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
    fk, nd, inst = _pmc_mean(one(fetch_dir), "FETCH_SIZE", main)
    wk, _, inst_w = _pmc_mean(one(write_dir), "WRITE_SIZE", main)
    assert inst == inst_w, (inst, inst_w)
    cf, _, _ = _pmc_mean(one(copy_fetch_dir), "FETCH_SIZE", "copy")
    cw, _, _ = _pmc_mean(one(copy_write_dir), "WRITE_SIZE", "copy")
    ff, wf = COPY_BYTES / 1024 / cf, COPY_BYTES / 1024 / cw
    out = {
        "kernel": kern, "template": main, "instance": inst, "workload": workload,
        "kernel_source_sha256": _kernel_sha(),
        "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk, "dispatches": nd,
        "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": cf, "write_kib": cw,
                             "fetch_factor": ff, "write_factor": wf},
        "traffic_bytes_per_launch": (fk * ff + wk * wf) * 1024,
        "commands": ["export TMPDIR=/tmp",
                     PROFILE_CMDS["FETCH_SIZE"].format(w=workload), PROFILE_CMDS["WRITE_SIZE"].format(w=workload),
                     PROFILE_CMDS["copy"].format(c="FETCH_SIZE"), PROFILE_CMDS["copy"].format(c="WRITE_SIZE")],
    }
    path = os.path.join(ROOT, "profiles", f"{kern}_{workload}_traffic.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path, out["traffic_bytes_per_launch"])


MFMA_COUNTERS = ("SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU_MFMA_MOPS_F32",
                 "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F64")
PROFILE_CMDS["mfma"] = ("rocprofv3 --pmc " + " ".join(MFMA_COUNTERS) + " --output-format csv -d gpurun_out/pmc_mfma_{w} "
                        "-o bench -- python bench.py --config {w} --steps 2 --warmup 1 --adapt 2 --no-cpu-baseline "
                        "--no-ess --timing-reps 5")
N_SIMD = 256 * 4   # MI355X: 256 compute units of 4 SIMDs
N_XCD = 8          # the per-dispatch GRBM_GUI_ACTIVE value is summed over the 8 XCDs


def record_mfma(workload, pmc_dir):
    """Writes profiles/<kernel>_<workload>_mfma.txt: per tile kernel, the
    MFMA busy fraction (SQ_VALU_MFMA_BUSY_CYCLES over the active cycles of one
    XCD times the SIMD count, as rocprof's MfmaUtil, which takes the maximum
    of GRBM_GUI_ACTIVE over XCDs where the per-dispatch value sums them) and
    the MFMA flops the hardware executed (MOPS x 512) against the
    algorithmic flops."""
    import csv
    import glob
    import workloads
    w = workloads.make(workload)
    rows = timed_dispatches(list(csv.DictReader(open(glob.glob(os.path.join(pmc_dir, "*counter_collection.csv"))[0]))),
                            PMC_TIMING_REPS)
    names = ["k_mlp_grad<", "k_trunk_fwd<", "k_branch_grad<", "k_trunk_bwd<", "k_update<"]
    parts = {"k_mlp_grad<": None, "k_branch_grad<": "branch", "k_trunk_fwd<": None, "k_trunk_bwd<": None}
    main = main_kernel(w)
    lines = [f"MFMA counters per dispatch: masked full-batch HMC, workload {workload} "
             f"({(w.sample_precision or w.precision).upper()} products, {w.n_chains} chains, L={w.L})",
             f"Device: one MI355X (gfx950).  Kernel source sha256 (hmc_kernels.hip): {_kernel_sha()}",
             "", "Command (repo root on the GPU box):", "  export TMPDIR=/tmp",
             "  " + PROFILE_CMDS["mfma"].format(w=workload), "",
             "busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs * 1024 SIMDs); "
             "executed = MOPS * 512 flops (padding to the MFMA tiles included); over the launches bench.py times "
             "(full grid, every chain active)",
             f"{'kernel':<42}{'dispatches':>11}{'busy %':>9}{'executed GFLOP':>16}{'algorithmic GFLOP':>19}"]
    for n in names:
        # one row per template instance (the gradient form and, where the
        # energies take another precision, the forward-only energy pass)
        for kname in sorted({r["Kernel_Name"] for r in rows if n in r["Kernel_Name"]}):
            sel = [r for r in rows if r["Kernel_Name"] == kname]
            per = {}
            for r in sel:
                per.setdefault(r["Dispatch_Id"], {})[r["Counter_Name"]] = float(r["Counter_Value"])
            full = [d for d in per.values() if all(c in d for c in MFMA_COUNTERS)]
            if not full:
                continue
            mean = {c: sum(d[c] for d in full) / len(full) for c in MFMA_COUNTERS}
            busy = 100.0 * mean["SQ_VALU_MFMA_BUSY_CYCLES"] / max(mean["GRBM_GUI_ACTIVE"] / N_XCD * N_SIMD, 1.0)
            ex = 512.0 * (mean["SQ_INSTS_VALU_MFMA_MOPS_F32"] + mean["SQ_INSTS_VALU_MFMA_MOPS_BF16"] +
                          mean["SQ_INSTS_VALU_MFMA_MOPS_F64"]) / 1e9
            short = kname.replace("void (anonymous namespace)::", "")
            alg = ""
            if n in ("k_mlp_grad<", "k_branch_grad<") and main in kname and not energy_pass(kname):
                alg = f"{algorithmic_flops(w, parts[n]) / 1e9:.3f}"
            lines.append(f"{short[:41]:<42}{len(full):>11}{busy:>9.2f}{ex:>16.3f}{alg:>19}")
    path = os.path.join(ROOT, "profiles", f"{KERNEL_OF[w.kind]}_{workload}_mfma.txt")
    open(path, "w").write("\n".join(lines) + "\n")
    print(path)
    print("\n".join(lines[-6:]))


def record_trace(workload, trace_dir, bench_json=None, sens=False):
    """Writes profiles/<kernel>_<workload>_kernel_trace.txt from the
    rocprofv3 --stats summary of the benchmark command (sens: of the
    sensitivity-pass command)."""
    import csv
    import glob
    import workloads
    w = workloads.make(workload)
    kern = "k_mlp_sens" if sens else KERNEL_OF[w.kind]
    stats = open(glob.glob(os.path.join(trace_dir, "*kernel_stats.csv"))[0]).read().strip()
    net = (f"MLP {'-'.join(map(str, w.widths_a))}" if w.kind == "mlp" else
           f"DeepONet branch {'-'.join(map(str, w.widths_a))}, trunk {'-'.join(map(str, w.widths_b))}")
    if sens:
        head = [f"Kernel-trace summary: parameter sensitivity pass (Sec. 3.1), workload {workload}",
                f"({net} tanh, {w.n_rows()} rows, all {w.n_params} parameters, "
                f"{'FP64' if w.precision == 'fp64' else 'FP32'}; one pass per output)"]
    else:
        head = [f"Kernel-trace summary: masked full-batch HMC, workload {workload}",
                f"({net} tanh, {w.n_rows()} rows, {w.n_chains} chains, {w.nnz // w.n_chains} of {w.n_params} "
                f"parameters sampled per chain on average, {(w.sample_precision or w.precision).upper()} "
                f"products, L={w.L})"]
    lines = head + [f"Device: one MI355X (gfx950).  Kernel source sha256 (hmc_kernels.hip): {_kernel_sha()}",
             "", "Command (repo root on the GPU box):", "  export TMPDIR=/tmp",
             "  " + PROFILE_CMDS["trace_sens" if sens else "trace"].format(w=workload), "",
             "bench_kernel_stats.csv:", stats, ""]
    if bench_json and sens:
        b = json.loads([ln for ln in open(bench_json).read().splitlines() if ln.startswith("{")][-1])
        lines.append(f"The same run's bench line: {json.dumps(b)}")
    elif bench_json:
        b = json.loads([ln for ln in open(bench_json).read().splitlines() if ln.startswith("{")][-1])
        main = main_kernel(w)
        trace = list(csv.DictReader(open(glob.glob(os.path.join(trace_dir, "*kernel_trace.csv"))[0])))
        sel = [r for r in trace if main in r["Kernel_Name"] and not energy_pass(r["Kernel_Name"])]
        full = timed_dispatches(sel, TRACE_TIMING_REPS)
        dur = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in full]
        inst = full[0]["Kernel_Name"].replace("void (anonymous namespace)::", "")
        if min(_grid(r) for r in sel) < _grid(full[0]):
            lines.append(f"The trajectory graphs launched {inst} over half of the chains at a time "
                         f"(grid {min(_grid(r) for r in sel)} against {_grid(full[0])}), so the statistics "
                         f"above mix those dispatches with the full-grid ones that bench.py times.")
        lines.append(f"The {len(full)} launches of {inst} that bench.py times (the last full-grid ones): mean "
                     f"{sum(dur) / len(dur) / 1e6:.4f} ms.")
        lines.append(f"HIP-event mean of {kern} measured inside bench.py in the same run: "
                     f"{b['kernel_ms']['grad_main']:.4f} ms (kernel_ms.grad_main).")
    if not sens:
        lines += ["", *trajectory_gaps(glob.glob(os.path.join(trace_dir, "*kernel_trace.csv"))[0])]
    path = os.path.join(ROOT, "profiles", f"{kern}_{workload}_kernel_trace.txt")
    open(path, "w").write("\n".join(lines) + "\n")
    print(path)


TRAJ_KERNELS = ("k_traj_begin<", "k_mlp_grad<", "k_branch_grad<", "k_trunk_fwd<", "k_trunk_bwd<",
                "k_update<", "k_traj_end<")


def trajectory_gaps(trace_csv):
    """Idle time of the device inside the trajectory graphs, from the
    rocprofv3 kernel trace: over each trajectory's span (the start of its
    k_traj_begin to the end of its k_traj_end) the union of the trajectory
    kernels' intervals on every queue (the graph may run two branches on two
    queues at once), the idle time the span minus that union, and the gaps
    between the union's stretches."""
    import csv
    rows = [r for r in csv.DictReader(open(trace_csv)) if any(k in r["Kernel_Name"] for k in TRAJ_KERNELS)]
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in rows)
    spans, t_open = [], None
    for t0, t1, name in iv:
        if "k_traj_begin<" in name:
            t_open = t0
        elif "k_traj_end<" in name and t_open is not None:
            spans.append((t_open, t1))
            t_open = None
    if not spans:
        return ["Trajectory gaps: no complete trajectory in the trace."]
    covered = idle = kernel_time = dispatches = 0
    gaps = []
    for a, b in spans:
        inside = [(max(t0, a), min(t1, b)) for t0, t1, _ in iv if t1 > a and t0 < b]
        dispatches += len(inside)
        kernel_time += sum(t1 - t0 for t0, t1 in inside)
        end = a
        for i, (t0, t1) in enumerate(inside):   # sorted by start
            if i:
                gaps.append(max(t0 - end, 0))
            if t0 > end:
                idle += t0 - end
            end = max(end, t1)
        idle += max(b - end, 0)
        covered += (b - a)
    covered -= idle
    g = np.array(gaps or [0]) / 1e3
    return [f"Trajectory gaps over {len(spans)} trajectories ({dispatches} kernel dispatches): kernels cover "
            f"{covered / 1e6:.3f} ms of the trajectories' span, the device is idle {idle / 1e6:.3f} ms between "
            f"them ({100 * idle / (covered + idle):.3f}%); gap per dispatch median {np.median(g):.2f} us, p90 "
            f"{np.quantile(g, 0.9):.2f} us, max {g.max():.2f} us; kernel time summed over queues "
            f"{kernel_time / 1e6:.3f} ms, {kernel_time / max(covered, 1):.3f}x the covered time "
            f"(above 1 where kernels on different queues ran at once)."]


def sensitivity_flops(widths, rows):
    """Algorithmic flops of one output's sensitivity pass: forward, the data
    adjoint above the first layer, and the squared weight-gradient product of
    every weight (2 * rows per weight), over all rows."""
    mm = [widths[i] * widths[i + 1] for i in range(len(widths) - 1)]
    return 2.0 * rows * (sum(mm) + sum(mm[1:]) + sum(mm))


def sensitivity_bench(config, reps, cpu_budget):
    """Times hmc_sensitivity (the whole call: engine set-up, one pass per
    output, reduction, copy back) on a workload's full data, and the oracle
    on a bounded row sample; prints one JSON line."""
    import workloads
    from paper_2507_14652_amd import sensitivities
    w = workloads.make(config, n_chains=1)
    sigma = np.full(w.n_params, 0.1)
    prec = "fp64" if w.precision == "fp64" else "fp32"
    sensitivities(widths_a=w.widths_a, theta0=w.theta0, sigma=sigma, x=w.x, precision=prec)   # warm-up
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        sensitivities(widths_a=w.widths_a, theta0=w.theta0, sigma=sigma, x=w.x, precision=prec)
        t.append(time.perf_counter() - t0)
    dt = float(np.median(t))
    rows = w.x.shape[0]
    flops = sensitivity_flops(w.widths_a, rows) * w.widths_a[-1]
    line = {"metric": "sensitivity pass (rows x parameters)/s", "value": rows * w.n_params / dt,
            "unit": "row-params/s", "ms_per_call": dt * 1e3, "config": {"workload": config, "rows": rows,
            "params": w.n_params, "outputs": w.widths_a[-1], "dtype": DTYPE[prec]},
            "algorithmic_tflops_whole_call": flops / dt / 1e12}
    if cpu_budget > 0:
        from oracle import sensitivity as osen
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < cpu_budget and n < rows:
            k = min(8, rows - n)
            osen.jacobian_square_sums("mlp", w.widths_a, None, w.theta0, {"x": w.x[n:n + k]})
            n += k
        el = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": n * w.n_params / el, "unit": "row-params/s", "kind": "oracle",
                                "sample": f"{n} of {rows} rows"}
    print(json.dumps(line))


def predict_bench(config, n_samples, n_new, cpu_budget):
    """Times hmc_predict (posterior predictive mean and variance of a chain
    over n_samples stored samples at n_new new inputs, engine set-up
    excluded) and the oracle on a bounded sample count; prints one JSON
    line.  The samples are stand-ins drawn around the chain's start."""
    import torch
    import workloads
    from paper_2507_14652_amd import Sampler
    w = workloads.make(config, n_chains=1)
    s = Sampler.from_workload(w, seed=5)
    # stand-in samples around the chain's start (the cost does not depend on
    # the values; drawing them with the sampler would dominate the run)
    g = torch.Generator(device="cuda").manual_seed(11)
    start = torch.as_tensor(w.chain_theta(0), dtype=s.state_dtype, device="cuda")
    out = start + 0.01 * torch.randn((n_samples, w.nnz), generator=g, dtype=s.state_dtype, device="cuda")
    x_new = np.random.default_rng(3).uniform(w.x.min(axis=0), w.x.max(axis=0), (n_new, w.x.shape[1]))
    s.predict(out[:2], x_new)                                       # warm-up
    t0 = time.perf_counter()
    s.predict(out, x_new)
    dt = time.perf_counter() - t0
    mm = [w.widths_a[i] * w.widths_a[i + 1] for i in range(len(w.widths_a) - 1)]
    flops = 2.0 * n_new * sum(mm) * n_samples
    line = {"metric": "posterior predictive (samples x rows)/s", "value": n_samples * n_new / dt,
            "unit": "sample-rows/s", "ms_per_call": dt * 1e3,
            "config": {"workload": config, "samples": n_samples, "new_rows": n_new, "dtype": DTYPE[w.precision]},
            "algorithmic_tflops": flops / dt / 1e12}
    if cpu_budget > 0:
        from oracle import predictive as opr
        S = out.double().cpu().numpy()[:, w.offs[0]:w.offs[1]]
        k, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < cpu_budget and k < n_samples:
            opr.predictive_moments("mlp", w.widths_a, None, w.theta0, w.chain_idx(0), S[k:k + 1], {"x": x_new})
            k += 1
        line["cpu_baseline"] = {"value": k * n_new / (time.perf_counter() - t0), "unit": "sample-rows/s",
                                "kind": "oracle", "sample": f"{k} of {n_samples} samples"}
    s.close()
    print(json.dumps(line))


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_grad_rate(w, budget_s):
    """Leapfrog gradient evaluations of the FP64 oracle along trajectories
    that cycle over the workload's chains, each evaluation timed as it runs
    and the loop stopped at the budget (large workloads finish only part of
    a trajectory).  Returns (evaluations/s, evaluations, seconds)."""
    from oracle import hmc as oh
    from oracle import network as on

    evals, t0, traj = 0, time.perf_counter(), 0
    while time.perf_counter() - t0 < budget_s:
        c = traj % w.n_chains
        post = on.posterior_for_chain(w, c)
        th = w.chain_theta(c)
        p = oh.momentum(1, c, traj // w.n_chains, th.size)
        U, g = post.potential_and_grad(th)
        evals += 1
        p = p - 0.5 * w.eps * g
        for t in range(1, w.L + 1):
            if time.perf_counter() - t0 >= budget_s:
                break
            th = th + w.eps * p
            U, g = post.potential_and_grad(th)
            evals += 1
            p = p - (w.eps if t < w.L else 0.5 * w.eps) * g
        traj += 1
    dt = time.perf_counter() - t0
    return evals / dt, evals, dt


def cpu_baseline(w, budget_s):
    """The FP64 oracle on the host cores, gradient evaluations per second on
    a bounded sample of the workload: once with every core BLAS offers and
    once on one thread (half the budget each).  value / cores: the all-core
    run and the threads it used."""
    from threadpoolctl import threadpool_info, threadpool_limits

    half = 0.5 * budget_s
    v_all, n_all, t_all = _oracle_grad_rate(w, half)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    with threadpool_limits(limits=1):
        v_one, n_one, t_one = _oracle_grad_rate(w, half)
    return {"value": v_all, "unit": "grad-evals/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n_all} leapfrog gradient evaluations (trajectories of L={w.L} cycling over the "
                      f"{w.n_chains} chains, stopped at the budget), FP64 NumPy, {t_all:.1f} s",
            "single_thread": {"value": v_one, "unit": "grad-evals/s", "cores": 1,
                              "sample": f"{n_one} gradient evaluations, {t_one:.1f} s"},
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


# ---------------------------------------------------------------------------
# Effective sample size and the plain single-chain FP32 HMC comparison.

def bulk_ess(draws):
    """Rank-normalised bulk effective sample size (Vehtari, Gelman, Simpson,
    Carpenter and Buerkner, 2021) of every coordinate of draws [N, M, D]
    (N iterations, M chains), with Geyer's initial monotone sequence."""
    from scipy.special import ndtri
    from scipy.stats import rankdata
    N, M, D = draws.shape
    flat = draws.reshape(N * M, D)
    r = rankdata(flat, axis=0, method="average")
    z = ndtri((r - 0.375) / (N * M + 0.25)).reshape(N, M, D)
    mean_c = z.mean(axis=0)
    W = z.var(axis=0, ddof=1).mean(axis=0)
    B_N = mean_c.var(axis=0, ddof=1) if M > 1 else np.zeros(D)
    var_plus = (N - 1) / N * W + B_N
    zc = z - mean_c
    f = np.fft.rfft(zc, n=2 * N, axis=0)
    acov = np.fft.irfft(f * np.conj(f), n=2 * N, axis=0)[:N] / N
    rho = 1.0 - (W - acov.mean(axis=1)) / var_plus
    rho[0] = 1.0
    # Geyer: sums of consecutive pairs up to the first negative one, each
    # clipped to the smallest before it
    K = N // 2
    pairs = rho[0:2 * K:2] + rho[1:2 * K:2]
    keep = np.cumprod(pairs >= 0, axis=0).astype(bool)
    s = np.where(keep, np.minimum.accumulate(pairs, axis=0), 0.0).sum(axis=0)
    tau = np.maximum(-1.0 + 2.0 * s, 1.0 / np.log10(max(N * M, 10)))
    return N * M / tau


def split_ess(draws):
    """Within-chain bulk ESS of every coordinate of one chain's draws [N, D]:
    the chain split into halves (two "chains" of N/2), so that a drift inside
    the run lowers the estimate as disagreement between chains does."""
    h = draws.shape[0] // 2
    return bulk_ess(np.stack([draws[:h], draws[h:2 * h]], axis=1))


def plain_torch_hmc(w, theta_s, eps, L, n_iter, seed, budget_s):
    """Plain single-chain HMC in PyTorch eager FP32 (TF32 off), chain 0: the
    full autograd backward over every parameter, then the selected entries
    taken from it.  Same potential (Eq. 3 with the Gaussian prior and
    likelihood of Sec. 2.2), leapfrog integrator and Metropolis rule as the
    engine, for the MLP and the DeepONet.  Stops after n_iter iterations or
    budget_s seconds.  Returns the draws [n, D], the potential of every draw,
    the Metropolis acceptance probability of every trajectory and the
    seconds taken."""
    import torch
    torch.backends.cuda.matmul.allow_tf32 = False
    dev = "cuda"
    f32 = torch.float32
    base = torch.tensor(w.theta0, dtype=f32, device=dev)
    idx = torch.tensor(w.chain_idx(0), dtype=torch.long, device=dev)
    t = lambda a: torch.tensor(a, dtype=f32, device=dev)
    if w.kind == "mlp":
        X, Y = t(w.x), t(w.y)
    else:
        Ub, Yq, V = t(w.u), t(w.yq), t(w.v)
    ivl, ivp = 1.0 / w.lik_sd ** 2, 1.0 / w.prior_sd ** 2

    def tower(full, pos, widths, a):
        n = len(widths) - 1
        for l in range(n):
            o, i = widths[l + 1], widths[l]
            Wm = full[pos:pos + o * i].view(o, i)
            pos += o * i
            a = a @ Wm.t() + full[pos:pos + o]
            pos += o
            if l < n - 1:
                a = torch.tanh(a)
        return a, pos

    def U_and_grad(ts):
        full = base.clone()
        full[idx] = ts
        full.requires_grad_(True)
        if w.kind == "mlp":
            r = tower(full, 0, w.widths_a, X)[0] - Y
        else:
            B, pos = tower(full, 0, w.widths_a, Ub)
            T, pos = tower(full, pos, w.widths_b, Yq)
            r = B @ T.t() + full[pos] - V
        sel = full[idx]
        U = 0.5 * ivl * (r * r).sum() + 0.5 * ivp * (sel * sel).sum()
        (g,) = torch.autograd.grad(U, full)
        return U.detach(), g[idx]

    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    th = torch.tensor(theta_s, dtype=f32, device=dev)
    U, g = U_and_grad(th)
    out, us, alphas, acc = [], [], [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(n_iter):
        p = torch.randn(th.shape, generator=gen, device=dev, dtype=f32)
        H0 = U + 0.5 * (p * p).sum()
        x, pp, gg = th, p - 0.5 * eps * g, g
        for k in range(1, L + 1):
            x = x + eps * pp
            U1, gg = U_and_grad(x)
            pp = pp - (eps if k < L else 0.5 * eps) * gg
        H1 = U1 + 0.5 * (pp * pp).sum()
        u = torch.rand((), generator=gen, device=dev, dtype=torch.float64)
        dH = float(H0 - H1)
        alphas.append(float(np.exp(min(dH, 0.0))) if np.isfinite(dH) else 0.0)
        if np.isfinite(dH) and np.log(float(u)) < dH:
            th, U, g = x, U1, gg
            acc += 1
        out.append(th)
        us.append(U)
        if time.perf_counter() - t0 > budget_s:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return torch.stack(out).cpu().numpy(), torch.stack(us).double().cpu().numpy(), np.array(alphas), dt


ESS_COORDS = 256
ESS_LEGS = {  # workload: engine iterations (adapt, burn-in, calibration rounds x batch, sampled)
    "antideriv_deeponet_bf16": dict(adapt=200, burn=300, rounds=5, batch=120, n=2000),
    "regress2d_fp32": dict(adapt=500, burn=2000, rounds=8, batch=300, n=4000),
}
ESS_DEFAULT = ("antideriv_deeponet_bf16",)


def ess_leg(name, seed, budget_s, adapt, burn, rounds, batch, n, progress=lambda m: None):
    """ESS/s of the batched engine against plain single-chain FP32 HMC at
    matched acceptance (Sec. 4.2.3's fixed-acceptance comparison, 80%).

    Engine, untimed: per-chain dual averaging (the step size and the chains
    move toward the typical set together), a burn-in at the adapted step
    sizes, then bisection of every chain's step size on its batch-mean
    acceptance.  Timed: n iterations of every chain.  The plain sampler runs
    the same potential, integrator, L and chain 0's calibrated step size from
    chain 0's last draw, for budget_s seconds; both acceptance rates are
    measured and reported.

    ESS is the rank-normalised bulk ESS of each coordinate within each chain
    (split halves, so a drift shows), and of the potential U.  The engine's
    ESS is the sum over its chains (each chain samples the same conditional
    posterior from its own start); the multi-chain estimate, which also
    counts disagreement between chains, is reported beside it."""
    import torch
    import workloads
    from paper_2507_14652_amd import Sampler
    w = workloads.make(name)
    w = dataclasses.replace(w, precision=w.sample_precision or w.precision)
    s = Sampler.from_workload(w, seed=seed)
    C, L = w.n_chains, w.L
    t0 = time.perf_counter()
    eps_c = s.adapt(adapt, w.eps, L)
    s.sample(burn, eps_c, L, want_stats=False)
    eps_c, _ = s.calibrate(rounds, batch, eps_c, L)
    progress(f"ESS leg {name}: engine prepared in {time.perf_counter() - t0:.1f} s")
    out = torch.empty((n, w.nnz), dtype=s.state_dtype, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = s.sample(n, eps_c, L, out=out)
    torch.cuda.synchronize()
    t_eng = time.perf_counter() - t0
    flat = out.double().cpu().numpy()
    # ESS of a seeded random subset of each chain's coordinates (all of them
    # up to ESS_COORDS), median and minimum over it
    pick = np.random.default_rng(seed).permutation(int(w.offs[1] - w.offs[0]))[:ESS_COORDS]
    ess_c = [split_ess(flat[:, w.offs[c]:w.offs[c + 1]][:, np.sort(pick[pick < w.offs[c + 1] - w.offs[c]])])
             for c in range(C)]
    med_c = np.array([np.median(e) for e in ess_c])
    same = all(np.array_equal(w.chain_idx(c), w.chain_idx(0)) for c in range(C))
    combined = bulk_ess(flat.reshape(n, C, -1)[:, :, np.sort(pick)]) if same else None
    # the potential of every draw of every chain (untimed)
    U_eng = np.empty((n, C))
    for k in range(n):
        s.set_state(out[k])
        U_eng[k] = s.grad()[0]
    ess_u = np.array([split_ess(U_eng[:, c:c + 1])[0] for c in range(C)])
    dh = st["H0"] - st["H1"]
    alpha = np.where(np.isfinite(dh), np.exp(np.minimum(np.nan_to_num(dh, nan=-np.inf), 0.0)), 0.0)
    s.close()
    progress(f"ESS leg {name}: engine {n} iterations x {C} chains in {t_eng:.2f} s, "
             f"median within-chain ESS {np.median(med_c):.1f}")

    base, U_base, alpha_b, t_base = plain_torch_hmc(w, flat[-1, w.offs[0]:w.offs[1]], float(eps_c[0]), L,
                                                    10 ** 9, seed + 1, budget_s)
    ess_b = split_ess(base[:, np.sort(pick)])
    ess_bu = split_ess(U_base[:, None])[0]
    progress(f"ESS leg {name}: plain FP32 {base.shape[0]} iterations in {t_base:.1f} s, "
             f"median ESS {np.median(ess_b):.1f}")
    eng_tot = float(med_c.sum())
    a0, ab = float(alpha[:, 0].mean()), float(alpha_b.mean())
    r = {
        "workload": name, "products": w.precision, "chains": C, "L": L,
        "coordinates_per_chain": int(min(ESS_COORDS, w.offs[1] - w.offs[0])),
        "eps_chain0": float(eps_c[0]), "eps_median": float(np.median(eps_c)),
        # mean Metropolis acceptance probability, with its Monte Carlo standard error
        "acceptance_engine": float(alpha.mean()),
        "acceptance_engine_chain0": a0, "acceptance_engine_chain0_mcse": batch_mcse(alpha[:, 0]),
        "acceptance_plain": ab, "acceptance_plain_mcse": batch_mcse(alpha_b),
        "matched": bool(abs(a0 - 0.8) <= 0.02 and abs(ab - 0.8) <= 0.02),
        "engine": {"iterations": n, "seconds": t_eng,
                   "ess_median_per_chain": float(np.median(med_c)),
                   "ess_min_per_chain": float(min(e.min() for e in ess_c)),
                   "ess_median_sum_over_chains": eng_tot,
                   "ess_u_sum_over_chains": float(ess_u.sum()),
                   "ess_median_multichain": None if combined is None else float(np.median(combined)),
                   "ess_per_s": eng_tot / t_eng,
                   "ess_per_s_chain0": float(med_c[0]) / t_eng},
        "plain_fp32_torch": {"iterations": int(base.shape[0]), "seconds": t_base,
                             "ess_median": float(np.median(ess_b)), "ess_min": float(ess_b.min()),
                             "ess_u": float(ess_bu), "ess_per_s": float(np.median(ess_b)) / t_base},
    }
    r["ratio"] = r["engine"]["ess_per_s"] / max(r["plain_fp32_torch"]["ess_per_s"], 1e-300)
    r["ratio_one_chain"] = r["engine"]["ess_per_s_chain0"] / max(r["plain_fp32_torch"]["ess_per_s"], 1e-300)
    return r


def batch_mcse(x, batches=20):
    """Monte Carlo standard error of the mean of a chain's values by batch means."""
    x = np.asarray(x, dtype=np.float64)
    k = len(x) // batches
    if k < 2:
        return None
    m = x[:k * batches].reshape(batches, k).mean(axis=1)
    return float(m.std(ddof=1) / np.sqrt(batches))


def ess_comparison(seed, budget_s, progress=lambda m: None, legs=ESS_DEFAULT):
    """The ESS/s comparison on the named workloads (by default the DeepONet;
    the 2-D regression MLP's conditional posterior mixes too slowly at L = 50
    for an ESS estimate within minutes: about 2 per chain in 4000
    iterations)."""
    return [ess_leg(name, seed, budget_s, progress=progress, **ESS_LEGS[name]) for name in legs]


def selected_per_chain(w):
    """Entries each chain samples: the count, or its spread when the masks differ."""
    n = np.diff(w.offs)
    if np.all(n == n[0]):
        return int(n[0])
    return {"min": int(n.min()), "median": float(np.median(n)), "max": int(n.max()), "mean": float(n.mean())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="uneven_mlp_bf16")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-reps", type=int, default=50)
    ap.add_argument("--calibrate", nargs=2, type=int, metavar=("ROUNDS", "BATCH"),
                    help="after adaptation, bisect the step sizes on batch-mean acceptance (untimed)")
    ap.add_argument("--adapt", type=int, default=20,
                    help="untimed step-size adaptation iterations before the warm-up (0: the workload's eps)")
    ap.add_argument("--precision", choices=("fp64", "fp32", "bf16", "bf16x3"),
                    help="run --config's workload at another precision (a comparison, not the headline line)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch shapes with the library's autotuner (untimed) instead of its heuristic")
    ap.add_argument("--split-rows", type=int, default=0, metavar="ROWS",
                    help="symmetric-splitting HMC over data batches of ROWS rows (MLP workloads; "
                         "a multiple of the rows per tile), for adaptation and the timed run")
    ap.add_argument("--no-ess", action="store_true", help="skip the ESS/s comparison with plain FP32 HMC")
    ap.add_argument("--ess-budget", type=float, default=130.0, help="seconds of plain FP32 HMC per ESS leg")
    ap.add_argument("--ess-only", nargs="*", metavar="WORKLOAD",
                    help="run only the ESS/s comparison (on the named legs, default all) and print it")
    ap.add_argument("--predict", action="store_true",
                    help="time the posterior predictive (200 samples of chain 0 at 4096 new inputs) on --config")
    ap.add_argument("--sensitivity", action="store_true",
                    help="time the sensitivity pass (Sec. 3.1) on --config's data instead of the sampler")
    ap.add_argument("--record-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write the profiles/ traffic summary for --config from rocprofv3 counter runs and exit")
    ap.add_argument("--record-mfma", metavar="PMC_DIR",
                    help="write the profiles/ MFMA-counter summary for --config and exit")
    ap.add_argument("--record-trace", nargs="+", metavar="TRACE_DIR [BENCH_LOG]",
                    help="write the profiles/ kernel-trace summary for --config and exit")
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(args.config, *args.record_traffic)
        return
    if args.record_mfma:
        record_mfma(args.config, args.record_mfma)
        return
    if args.record_trace:
        record_trace(args.config, *args.record_trace[:2], sens=args.sensitivity)
        return
    if args.predict:
        predict_bench(args.config, 200, 4096, 0.0 if args.no_cpu_baseline else 10.0)
        return
    if args.sensitivity:
        sensitivity_bench(args.config, args.steps if args.steps != 20 else 5, 0.0 if args.no_cpu_baseline else 10.0)
        return
    if args.ess_only is not None:
        prog = lambda m: print(f"[bench {time.strftime('%H:%M:%S')}] {m}", file=sys.stderr, flush=True)
        print(json.dumps({"ess": ess_comparison(2507, args.ess_budget, prog, args.ess_only or ESS_DEFAULT)}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); chains are independent and would "
              "shard across GPUs with no per-step exchange, which this build does not run.", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_2507_14652_amd import Sampler, autotune_workload

    def progress(msg):
        print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)

    w = workloads.make(args.config)
    # the products this workload samples in (the precision whose Metropolis
    # decisions match FP64 ones within 1% there), unless --precision asks
    w = dataclasses.replace(w, precision=args.precision or w.sample_precision or w.precision)
    progress(f"{w.name}: {w.precision}, {w.n_chains} chains, L={w.L}")
    tuning = autotune_workload(w, reps=10)[0] if args.autotune else None
    s = Sampler.from_workload(w, seed=2507, tuning=tuning)
    progress(f"engine ready ({s.info['device_bytes'] / 2**30:.2f} GiB on the device)")
    C, L = w.n_chains, w.L
    integrator = {"kind": "leapfrog", "grad_evals_per_trajectory": L}
    if args.split_rows:
        s.set_split(args.split_rows)
        integrator = {"kind": "symmetric split", "batch_rows": args.split_rows,
                      "batches": -(-w.n_rows() // args.split_rows), "grad_evals_per_trajectory": L + 1}
        progress(f"symmetric splitting over {integrator['batches']} batches of {args.split_rows} rows")
    st_dtype = torch.float64 if w.precision == "fp64" else torch.float32
    out = torch.empty((args.steps, w.nnz), dtype=st_dtype, device="cuda")
    warm = torch.empty((max(args.warmup, 1), w.nnz), dtype=st_dtype, device="cuda")
    # untimed: per-chain step sizes by dual averaging to 80% acceptance, then
    # the warm-up iterations at those step sizes
    eps_c = s.adapt(args.adapt, w.eps, L) if args.adapt else np.full(C, w.eps)
    progress(f"step sizes adapted over {args.adapt} iterations: median {np.median(eps_c):.3e}")
    if args.calibrate:
        eps_c, _ = s.calibrate(args.calibrate[0], args.calibrate[1], eps_c, L)
        progress(f"step sizes calibrated: median {np.median(eps_c):.3e}")
    if args.warmup:
        s.sample(args.warmup, eps_c, L, out=warm)
    torch.cuda.synchronize()
    progress(f"{args.warmup} warm-up iterations done; timing {args.steps}")
    t0 = time.perf_counter()
    _, stats = s.sample(args.steps, eps_c, L, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # dominant kernel, timed alone with HIP events on the engine's stream
    ms = s.time_kernels(args.timing_reps)
    flops = algorithmic_flops(w, None if w.kind == "mlp" else "branch")
    dom_ms = ms[0]
    achieved = flops / (dom_ms * 1e-3) / 1e12
    peak = PEAK[DTYPE[w.precision]]
    kname = KERNEL_OF[w.kind]
    traffic = recorded_traffic(kname, w.name, f"{kname}<{PRECISION_INDEX[w.precision]}, {s.info['rows_per_tile_a']}, ")
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic, "kernel": kname, "kernel_ms": dom_ms, "flops_per_launch": flops,
            "hbm_gbps": traffic / (dom_ms * 1e-3) / 1e9 if traffic else None}
    # the whole gradient evaluation: every tile kernel plus the partial sums
    grad_ms = sum(ms)
    grad_tf = algorithmic_flops(w) / (grad_ms * 1e-3) / 1e12
    gradient = {"kernels_ms": grad_ms, "achieved": grad_tf, "unit": "TFLOP/s", "frac": grad_tf / peak}

    acc = float(stats["accepted"].mean())
    line = {
        "metric": "leapfrog grad-evals/s x chains",
        "value": C * L * args.steps / dt,
        "unit": "grad-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "us_per_leapfrog_step": dt / args.steps / L * 1e6,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[w.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "net": w.kind, "widths_a": w.widths_a, "widths_b": w.widths_b,
                   "rows": w.n_rows(), "chains": C, "selected_per_chain": selected_per_chain(w), "L": L,
                   "products": w.precision, "energy": w.energy, "integrator": integrator,
                   "eps_start": w.eps, "eps_adapt_iters": args.adapt,
                   "eps_calibration": args.calibrate,
                   "eps_median": float(np.median(eps_c)), "eps_min": float(np.min(eps_c)),
                   "eps_max": float(np.max(eps_c)),
                   "launch": {"autotuned": bool(args.autotune), "dw": (tuning or {}).get("dw", 0),
                              **{k: s.info[k] for k in ("rows_per_tile_a", "rows_per_tile_b", "threads_a",
                                                        "threads_b", "chain_halves")}}},
        "acceptance": acc,
        "kernel_ms": {"grad_main": ms[0], "trunk_fwd": ms[1], "trunk_bwd": ms[2], "reduce": ms[3]},
        "roofline": roof,
        "gradient_roofline": gradient,
    }
    s.close()
    progress(f"timed: {line['value']:.1f} {line['unit']}, acceptance {acc:.3f}")
    if not args.no_ess:
        line["ess"] = ess_comparison(2507, args.ess_budget, progress)
        progress("ESS comparison done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
        progress("CPU baseline done")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
