"""Throughput of masked full-batch HMC on one MI355X.

One step = one iteration of the sampler for every chain: momentum refresh,
L leapfrog steps (each a full-batch forward pass, adjoint pass and masked
weight gradient), Hamiltonian and Metropolis test, and the copy of the new
positions into a device-resident sample buffer.  The metric is leapfrog
gradient evaluations per second summed over chains.

Prints one JSON line.  The default workload is the FP32 MLP regression
(2-64-64-64-1 tanh, 4096 rows, 10% of the parameters sampled, 8 chains,
L = 50, per-chain step sizes adapted from 5e-4 to 80% acceptance before the
timed region); --config selects another named workload.
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


# ---------------------------------------------------------------------------
# Effective sample size and the plain single-chain FP32 HMC comparison.

def bulk_ess(draws):
    """Rank-normalised bulk effective sample size (Vehtari, Gelman, Simpson,
    Carpenter and Buerkner, 2021) of every coordinate of draws [N, M, D]
    (N iterations, M chains), with Geyer's initial monotone sequence."""
    from scipy.stats import norm, rankdata
    N, M, D = draws.shape
    flat = draws.reshape(N * M, D)
    r = rankdata(flat, axis=0, method="average")
    z = norm.ppf((r - 0.375) / (N * M + 0.25)).reshape(N, M, D)
    mean_c = z.mean(axis=0)
    W = z.var(axis=0, ddof=1).mean(axis=0)
    B_N = mean_c.var(axis=0, ddof=1) if M > 1 else np.zeros(D)
    var_plus = (N - 1) / N * W + B_N
    zc = z - mean_c
    f = np.fft.rfft(zc, n=2 * N, axis=0)
    acov = np.fft.irfft(f * np.conj(f), n=2 * N, axis=0)[:N] / N
    rho = 1.0 - (W - acov.mean(axis=1)) / var_plus
    rho[0] = 1.0
    ess = np.empty(D)
    for d in range(D):
        s, prev = 0.0, np.inf
        for k in range(0, N - 1, 2):
            pk = rho[k, d] + rho[k + 1, d]
            if pk < 0:
                break
            pk = min(pk, prev)
            prev = pk
            s += pk
        tau = max(-1.0 + 2.0 * s, 1.0 / np.log10(max(N * M, 10)))
        ess[d] = N * M / tau
    return ess


def plain_torch_hmc(w, theta_s, eps, L, n_iter, seed, budget_s):
    """Plain single-chain HMC in PyTorch eager FP32 (TF32 off), chain 0: the
    full autograd backward over every parameter, then the selected entries
    taken from it.  Same potential, integrator and Metropolis rule as the
    engine.  Stops after n_iter iterations or budget_s seconds."""
    import torch
    torch.backends.cuda.matmul.allow_tf32 = False
    dev = "cuda"
    f32 = torch.float32
    base = torch.tensor(w.theta0, dtype=f32, device=dev)
    idx = torch.tensor(w.chain_idx(0), dtype=torch.long, device=dev)
    X = torch.tensor(w.x, dtype=f32, device=dev)
    Y = torch.tensor(w.y, dtype=f32, device=dev)
    shapes = [(w.widths_a[i + 1], w.widths_a[i]) for i in range(len(w.widths_a) - 1)]
    ivl, ivp = 1.0 / w.lik_sd ** 2, 1.0 / w.prior_sd ** 2

    def U_and_grad(ts):
        full = base.clone()
        full[idx] = ts
        full.requires_grad_(True)
        a, pos = X, 0
        for l, (o, i) in enumerate(shapes):
            Wm = full[pos:pos + o * i].view(o, i)
            pos += o * i
            b = full[pos:pos + o]
            pos += o
            a = a @ Wm.t() + b
            if l < len(shapes) - 1:
                a = torch.tanh(a)
        r = a - Y
        sel = full[idx]
        U = 0.5 * ivl * (r * r).sum() + 0.5 * ivp * (sel * sel).sum()
        (g,) = torch.autograd.grad(U, full)
        return U.detach(), g[idx]

    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    th = torch.tensor(theta_s, dtype=f32, device=dev)
    U, g = U_and_grad(th)
    out, acc = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(n_iter):
        p = torch.randn(th.shape, generator=gen, device=dev, dtype=f32)
        H0 = U + 0.5 * (p * p).sum()
        x, pp, gg = th, p - 0.5 * eps * g, g
        for t in range(1, L + 1):
            x = x + eps * pp
            U1, gg = U_and_grad(x)
            pp = pp - (eps if t < L else 0.5 * eps) * gg
        H1 = U1 + 0.5 * (pp * pp).sum()
        u = torch.rand((), generator=gen, device=dev, dtype=torch.float64)
        dH = float(H0 - H1)
        if np.isfinite(dH) and np.log(float(u)) < dH:
            th, U, g = x, U1, gg
            acc += 1
        out.append(th)
        if time.perf_counter() - t0 > budget_s:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return torch.stack(out).cpu().numpy(), acc / len(out), dt


def ess_comparison(w, seed, budget_s=20.0):
    """ESS/s of the batched engine against plain single-chain FP32 HMC, both
    at the same step size and L, the step size adapted to 80% acceptance
    (Sec. 4.3) by dual averaging.  Untimed preparation: Adam on the engine's
    own gradient toward the conditional mode of every chain, adaptation,
    burn-in.  The plain sampler starts where the engine's chain 0 ended and
    uses chain 0's step size."""
    import torch
    from paper_2507_14652_amd import Sampler
    from paper_2507_14652_amd.warmup import adapt_step_size
    s = Sampler.from_workload(w, seed=seed)
    C, L = w.n_chains, w.L
    th = s.get_state()[0].double().cpu().numpy()
    m, v = np.zeros_like(th), np.zeros_like(th)
    lr, b1, b2 = 1e-3, 0.9, 0.999
    for k in range(1, 1501):
        s.set_state(th.astype(np.float32))
        _, g = s.grad()
        g = g.double().cpu().numpy()
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        th = th - lr * (m / (1 - b1 ** k)) / (np.sqrt(v / (1 - b2 ** k)) + 1e-8)
    s.set_state(th.astype(np.float32))
    eps_c = adapt_step_size(s, w.eps, L, n_adapt=300)
    s.sample(50, eps_c, L)
    n = 400
    out = torch.empty((n, w.nnz), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = s.sample(n, eps_c, L, out=out)
    torch.cuda.synchronize()
    t_eng = time.perf_counter() - t0
    ns = w.nnz // C
    draws = out.cpu().numpy().reshape(n, C, ns)
    ess_eng = bulk_ess(draws)
    acc_eng = float(st["accepted"].mean())
    start0 = draws[-1, 0]
    eps = float(eps_c[0])
    base, acc_base, t_base = plain_torch_hmc(w, start0, eps, L, n, seed + 1, budget_s)
    ess_base = bulk_ess(base[:, None, :])
    s.close()
    r = {
        "eps_chain0": eps, "eps_median": float(np.median(eps_c)), "L": L,
        "acceptance_engine": acc_eng, "acceptance_plain": acc_base,
        "engine": {"chains": C, "iterations": n, "seconds": t_eng,
                   "ess_median": float(np.median(ess_eng)), "ess_min": float(ess_eng.min()),
                   "ess_per_s_median": float(np.median(ess_eng)) / t_eng,
                   "ess_per_s_min": float(ess_eng.min()) / t_eng},
        "plain_fp32_torch": {"chains": 1, "iterations": int(base.shape[0]), "seconds": t_base,
                             "ess_median": float(np.median(ess_base)), "ess_min": float(ess_base.min()),
                             "ess_per_s_median": float(np.median(ess_base)) / t_base,
                             "ess_per_s_min": float(ess_base.min()) / t_base},
    }
    r["ratio_median"] = r["engine"]["ess_per_s_median"] / max(r["plain_fp32_torch"]["ess_per_s_median"], 1e-300)
    r["ratio_min"] = r["engine"]["ess_per_s_min"] / max(r["plain_fp32_torch"]["ess_per_s_min"], 1e-300)
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="regress2d_fp32")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-reps", type=int, default=50)
    ap.add_argument("--adapt", type=int, default=150,
                    help="untimed step-size adaptation iterations before the warm-up (0: the workload's eps)")
    ap.add_argument("--no-ess", action="store_true", help="skip the ESS/s comparison with plain FP32 HMC")
    ap.add_argument("--ess-budget", type=float, default=20.0, help="seconds for the plain FP32 HMC leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); chains are independent and would "
              "shard across GPUs with no per-step exchange, which this build does not run.", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_2507_14652_amd import Sampler
    from paper_2507_14652_amd.warmup import adapt_step_size

    w = workloads.make(args.config)
    s = Sampler.from_workload(w, seed=2507)
    C, L = w.n_chains, w.L
    st_dtype = torch.float64 if w.precision == "fp64" else torch.float32
    out = torch.empty((args.steps, w.nnz), dtype=st_dtype, device="cuda")
    warm = torch.empty((max(args.warmup, 1), w.nnz), dtype=st_dtype, device="cuda")
    # untimed: per-chain step sizes by dual averaging to 80% acceptance, then
    # the warm-up iterations at those step sizes
    eps_c = adapt_step_size(s, w.eps, L, n_adapt=args.adapt) if args.adapt else np.full(C, w.eps)
    if args.warmup:
        s.sample(args.warmup, eps_c, L, out=warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats = s.sample(args.steps, eps_c, L, out=out)
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
                   "eps_start": w.eps, "eps_adapt_iters": args.adapt,
                   "eps_median": float(np.median(eps_c)), "eps_min": float(np.min(eps_c)),
                   "eps_max": float(np.max(eps_c))},
        "acceptance": acc,
        "kernel_ms": {"grad_main": ms[0], "trunk_fwd": ms[1], "trunk_bwd": ms[2], "reduce": ms[3]},
        "roofline": roof,
    }
    s.close()
    if not args.no_ess and w.kind == "mlp":
        line["ess"] = ess_comparison(w, seed=2507, budget_s=args.ess_budget)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
