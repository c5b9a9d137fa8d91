"""Throughput of masked full-batch HMC on one MI355X.

One step = one iteration of the sampler for every chain: momentum refresh,
L leapfrog steps (each a full-batch forward pass, adjoint pass and masked
weight gradient), Hamiltonian and Metropolis test, and the copy of the new
positions into a device-resident sample buffer.  The metric is leapfrog
gradient evaluations per second summed over chains.

Prints one JSON line.  The default workload is the FP32 MLP regression
(2-64-64-64-1 tanh, 4096 rows, 10% of the parameters sampled, 8 chains,
L = 50, eps = 5e-4); --config selects another named workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X dense peaks
    "f64": 78.6, "f32": 157.3, "bf16": 2500.0,
}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}


def algorithmic_flops(w, offs=None):
    """Flops one gradient evaluation of every chain must do: forward products,
    adjoint products down to the lowest layer holding a selected entry, and
    2 * rows per selected entry (the masked weight gradient).  DeepONet adds
    the combination G = B T^T and its two adjoint products."""
    total = 0.0
    for c in range(w.n_chains):
        idx = w.chain_idx(c)
        if w.kind == "mlp":
            towers = [(w.widths_a, w.x.shape[0], 0)]
        else:
            nb = sum(w.widths_a[i] * w.widths_a[i + 1] + w.widths_a[i + 1] for i in range(len(w.widths_a) - 1))
            towers = [(w.widths_a, w.u.shape[0], 0), (w.widths_b, w.yq.shape[0], nb)]
        for widths, rows, flat0 in towers:
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
            total += 3 * 2.0 * nu * nq * p
    return total


def recorded_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (calibrated against a plain copy), or None
    when the kernel source has changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    src = os.path.join(ROOT, "paper_2507_14652_amd", "csrc", "hmc_kernels.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    return d["traffic_bytes_per_launch"] if d.get("kernel_source_sha256") == h else None


def cpu_baseline(w, budget_s):
    """The FP64 oracle on the host cores: gradient evaluations per second,
    summed over the chains it ran, on a bounded sample of the workload."""
    from threadpoolctl import threadpool_info

    from oracle import hmc as oh
    from oracle import network as on

    evals, trajs, t0 = 0, 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        c = trajs % w.n_chains
        post = on.posterior_for_chain(w, c)
        th = w.chain_theta(c)
        p = oh.momentum(1, c, trajs // w.n_chains, th.size)
        start = post.potential_and_grad(th)
        oh.leapfrog(post.potential_and_grad, th, p, w.eps, w.L, start=start)
        evals += w.L + 1
        trajs += 1
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": evals / dt, "unit": "grad-evals/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{trajs} trajectories of L={w.L} (+1 start evaluation each) cycling over the "
                      f"{w.n_chains} chains of the same workload, FP64 NumPy, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="regress2d_fp32")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-reps", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); chains are independent and would "
              "shard across GPUs with no per-step exchange, which this build does not run.", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_2507_14652_amd import Sampler

    w = workloads.make(args.config)
    s = Sampler.from_workload(w, seed=2507)
    C, L = w.n_chains, w.L
    st_dtype = torch.float64 if w.precision == "fp64" else torch.float32
    out = torch.empty((args.steps, w.nnz), dtype=st_dtype, device="cuda")
    warm = torch.empty((max(args.warmup, 1), w.nnz), dtype=st_dtype, device="cuda")
    if args.warmup:
        s.sample(args.warmup, w.eps, L, out=warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats = s.sample(args.steps, w.eps, L, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # dominant kernel, timed alone with HIP events on the engine's stream
    ms = s.time_kernels(args.timing_reps)
    flops = algorithmic_flops(w)
    dom_ms = ms[0]
    achieved = flops / (dom_ms * 1e-3) / 1e12
    peak = PEAK[DTYPE[w.precision]]
    kname = "k_mlp_grad" if w.kind == "mlp" else "k_branch_grad"
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": recorded_traffic(kname, w.name), "kernel": kname,
            "kernel_ms": dom_ms, "flops_per_launch": flops}

    acc = float(stats["accepted"].mean())
    line = {
        "metric": "leapfrog grad-evals/s x chains",
        "value": C * L * args.steps / dt,
        "unit": "grad-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[w.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "net": w.kind, "widths_a": w.widths_a, "widths_b": w.widths_b,
                   "rows": w.n_rows(), "chains": C, "selected_per_chain": int(w.nnz // C), "L": L,
                   "eps": w.eps},
        "acceptance": acc,
        "kernel_ms": {"grad_main": ms[0], "trunk_fwd": ms[1], "trunk_bwd": ms[2], "reduce": ms[3]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    s.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
