"""Workload-shaped engines whose network output is linear in the sampled
parameters (only the last MLP layer, or entries of the last DeepONet branch
layer and b0, are sampled), with the Gaussian posterior they target
(Bayesian linear regression: precision Lam, mean m, and the constant of U).
Features come from a plain NumPy forward pass of the fixed layers.  Shared by
the closed-form GPU tests; draws numbers only."""

import numpy as np
import pytest

import workloads


def engine(prec, desc):
    """The engine for a case at a product precision; skips the test where
    that precision's tiles of the case's widths do not fit in LDS."""
    from paper_2507_14652_amd import Sampler
    from paper_2507_14652_amd.binding import HMC_EUNSUPPORTED, HMCError
    try:
        return Sampler(precision=prec, **desc)
    except HMCError as e:
        if e.status == HMC_EUNSUPPORTED and "LDS" in str(e):
            pytest.skip(f"{prec}: {e}")
        raise


def _tower(theta, widths, pos):
    """(W, b) of each layer, flat layout: layer by layer, W[out][in] row-major, then b."""
    layers = []
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        W = theta[pos:pos + n_in * n_out].reshape(n_out, n_in)
        pos += n_in * n_out
        b = theta[pos:pos + n_out]
        pos += n_out
        layers.append((W, b))
    return layers, pos


def _hidden(layers, x):
    """Activations entering the last layer (tanh after every other layer)."""
    h = np.asarray(x, dtype=np.float64)
    for W, b in layers[:-1]:
        h = np.tanh(h @ W.T + b)
    return h


def gaussian(Phi, r, prior_sd, lik_sd):
    """Lam, m and the constant of U for F = F_fixed + Phi theta, r = y - F_fixed."""
    Lam = Phi.T @ Phi / lik_sd**2 + np.eye(Phi.shape[1]) / prior_sd**2
    m = np.linalg.solve(Lam, Phi.T @ r / lik_sd**2)
    const = r @ r / (2 * lik_sd**2) - 0.5 * m @ Lam @ m
    return Lam, m, const


def _mlp_last_layer(name, n_chains, rng):
    """An engine description sampling the last layer (weights and bias) of
    every chain of the workload's MLP, and the Gaussian it targets."""
    w = workloads.make(name, n_chains=1)
    theta0 = w.theta0
    layers, P = _tower(theta0, w.widths_a, 0)
    assert P == theta0.size and w.widths_a[-1] == 1
    h = _hidden(layers, w.x)
    H = w.widths_a[-2]
    sel = np.arange(P - H - 1, P)               # W_L[0][0..H-1], then b_L
    Phi = np.hstack([h, np.ones((h.shape[0], 1))])
    Lam, m, const = gaussian(Phi, w.y[:, 0], w.prior_sd, w.lik_sd)
    ev, Q = np.linalg.eigh(Lam)
    # chain starts: posterior draws
    starts = [m + Q @ (rng.standard_normal(m.size) / np.sqrt(ev)) for _ in range(n_chains)]
    desc = dict(kind="mlp", widths_a=w.widths_a, theta0=theta0, prior_sd=w.prior_sd, lik_sd=w.lik_sd,
                offs=np.arange(n_chains + 1) * sel.size, idx=np.tile(sel, n_chains),
                theta_init=np.concatenate(starts), x=w.x, y=w.y)
    return desc, Lam, m, const, sel.size, Phi, w.y[:, 0]


def _deeponet_partial_branch(name, n_sel, n_chains, rng):
    """A DeepONet workload at its full size (the antiderivative operator:
    1000 functions x 100 query points; the surface operator: 2048 conditions
    x 512 points): n_sel random entries of the last branch layer plus b0
    sampled, everything else (the trunk included) fixed.  The engine
    description carries the workload's energy setting."""
    w = workloads.make(name, n_chains=1)
    theta0 = w.theta0.copy()
    br, pos = _tower(theta0, w.widths_a, 0)
    tr, pos = _tower(theta0, w.widths_b, pos)
    assert pos + 1 == theta0.size
    p_out, hid = w.widths_a[-1], w.widths_a[-2]
    last0 = sum(a * b + b for a, b in zip(w.widths_a[:-2], w.widths_a[1:-1]))   # flat start of the last branch layer
    cand = np.arange(last0, last0 + p_out * hid + p_out)
    sel = np.sort(np.concatenate([rng.choice(cand, n_sel, replace=False), [theta0.size - 1]]))
    h = _hidden(br, w.u)                                    # [n_u][hid]
    T = _hidden(tr, w.yq) @ tr[-1][0].T + tr[-1][1]         # [n_q][p]
    fixed = theta0.copy()
    fixed[sel] = 0.0
    brf, _ = _tower(fixed, w.widths_a, 0)
    Bf = h @ brf[-1][0].T + brf[-1][1]
    F_fixed = Bf @ T.T                                      # b0 is sampled
    n_u, n_q = h.shape[0], T.shape[0]
    cols = []
    for k in sel:
        if k == theta0.size - 1:                            # b0
            cols.append(np.ones(n_u * n_q))
            continue
        off = k - last0
        if off < p_out * hid:                               # W_L[kk][i]: h[j][i] T[q][kk]
            kk, i = divmod(off, hid)
            cols.append(np.outer(h[:, i], T[:, kk]).ravel())
        else:                                               # b_L[kk]: T[q][kk]
            cols.append(np.tile(T[:, off - p_out * hid], n_u))
    Phi = np.stack(cols, axis=1)
    Lam, m, const = gaussian(Phi, (w.v - F_fixed).ravel(), w.prior_sd, w.lik_sd)
    ev, Q = np.linalg.eigh(Lam)
    starts = [m + Q @ (rng.standard_normal(m.size) / np.sqrt(ev)) for _ in range(n_chains)]
    desc = dict(kind="deeponet", widths_a=w.widths_a, widths_b=w.widths_b, theta0=theta0, prior_sd=w.prior_sd,
                lik_sd=w.lik_sd, offs=np.arange(n_chains + 1) * sel.size, idx=np.tile(sel, n_chains),
                theta_init=np.concatenate(starts), u=w.u, yq=w.yq, v=w.v, energy=w.energy)
    return desc, Lam, m, const, sel.size, Phi, (w.v - F_fixed).ravel()


CASES = [
    ("regress2d_fp32 last layer", lambda rng: _mlp_last_layer("regress2d_fp32", 3, rng)),
    ("uneven_mlp_bf16 shape, last layer", lambda rng: _mlp_last_layer("uneven_mlp_bf16", 2, rng)),
    ("antideriv DeepONet, 200 last-layer branch entries + b0",
     lambda rng: _deeponet_partial_branch("antideriv_deeponet_bf16", 200, 2, rng)),
    ("surface DeepONet, 200 last-layer branch entries + b0",
     lambda rng: _deeponet_partial_branch("surface_deeponet_bf16", 200, 2, rng)),
]
