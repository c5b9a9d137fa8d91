"""Seeded synthetic stand-ins for the paper's workloads.

The paper's data sets (sinusoid regression of Sec. 4.1, the Burgers operator
data of Sec. 4.2.1 and the hypersonic-cone data of Sec. 4.2.2) are not
available, and the VI means that fix the non-sampled parameters come from
training runs that are out of scope.  Every array here is drawn from a
counter-based generator keyed by (master seed, stream[, chain]):

    master seed = 14652 + workload index
    stream 0: inputs, 1: observation noise, 2: parameter vector,
    3: masks, 4: per-chain starting points

Parameter vectors use the canonical flat order: for each tower, layer by
layer, the weight matrix W[out][in] row-major followed by the bias b[out];
a DeepONet stores the branch tower, then the trunk tower, then the scalar
output bias b0.  (App. B describes each layer as an n x m matrix with m
inputs and n outputs; the ordering across layers is a convention of this
code.)
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

CONFIG_NAMES = (
    "sine1d_fp64",
    "regress2d_fp32",
    "antideriv_deeponet_bf16",
    "uneven_mlp_bf16",
    "surface_deeponet_bf16",
)


def tower_param_count(widths) -> int:
    """Number of weights and biases of a fully connected tower."""
    return int(sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1)))


def n_params(kind: str, widths_a, widths_b=None) -> int:
    if kind == "mlp":
        return tower_param_count(widths_a)
    if kind == "deeponet":
        return tower_param_count(widths_a) + tower_param_count(widths_b) + 1
    raise ValueError(kind)


@dataclasses.dataclass
class Workload:
    name: str
    kind: str                 # "mlp" or "deeponet"
    widths_a: list            # MLP widths, or branch widths [m, ..., p]
    widths_b: Optional[list]  # trunk widths [d_y, ..., p] (DeepONet only)
    precision: str            # "fp64", "fp32" or "bf16"
    prior_sd: float
    lik_sd: float
    eps: float
    L: int
    n_chains: int
    n_samples: int
    theta0: np.ndarray        # [P] float64: fixed values and the centre of the chain starts
    offs: np.ndarray          # [C+1] int64 CSR offsets of the selected subsets
    idx: np.ndarray           # [nnz] int64 sorted selected flat indices per chain
    theta_init: np.ndarray    # [nnz] float64 per-chain starting values of the selected entries
    x: Optional[np.ndarray] = None    # MLP inputs  [N, d_in]
    y: Optional[np.ndarray] = None    # MLP targets [N, d_out]
    u: Optional[np.ndarray] = None    # DeepONet branch inputs [n_u, m]
    yq: Optional[np.ndarray] = None   # DeepONet trunk inputs  [n_q, d_y]
    v: Optional[np.ndarray] = None    # DeepONet targets [n_u, n_q]
    note: str = ""
    energy: str = "default"   # forward pass behind U in the Hamiltonian: "default" or "fp64"
    sample_precision: str = ""  # products whose Metropolis decisions match FP64 ones within 1% on this
                                # workload (measured): what it samples in; "" = precision

    @property
    def n_params(self) -> int:
        return n_params(self.kind, self.widths_a, self.widths_b)

    @property
    def nnz(self) -> int:
        return int(self.offs[-1])

    def chain_idx(self, c: int) -> np.ndarray:
        return self.idx[self.offs[c]:self.offs[c + 1]]

    def chain_theta(self, c: int) -> np.ndarray:
        return self.theta_init[self.offs[c]:self.offs[c + 1]]

    def n_rows(self) -> int:
        return int(self.x.shape[0]) if self.kind == "mlp" else int(self.u.shape[0] * self.yq.shape[0])


def _rng(master: int, stream: int, chain: Optional[int] = None) -> np.random.Generator:
    words = [master, stream] if chain is None else [master, stream, chain]
    return np.random.Generator(np.random.Philox(np.random.SeedSequence(words)))


def _subset(rng: np.random.Generator, P: int, count: int) -> np.ndarray:
    count = max(1, min(P, count))
    return np.sort(rng.choice(P, size=count, replace=False)).astype(np.int64)


def _chains(master, theta0, masks, jitter):
    """CSR of per-chain masks and starting points theta0[idx] + jitter * xi_c."""
    offs = np.zeros(len(masks) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(m) for m in masks])
    idx = np.concatenate(masks).astype(np.int64)
    starts = []
    for c, m in enumerate(masks):
        xi = _rng(master, 4, c).standard_normal(len(m))
        starts.append(theta0[m] + jitter * xi)
    return offs, idx, np.concatenate(starts)


def _grf_rows(rng, sensors, length, n_fun):
    """Zero-mean Gaussian random fields with an RBF covariance at the sensors."""
    d = sensors[:, None] - sensors[None, :]
    K = np.exp(-(d * d) / (2.0 * length * length))
    lam, V = np.linalg.eigh(K)
    lam = np.clip(lam, 1e-12, None)
    z = rng.standard_normal((n_fun, len(sensors)))
    return z @ (V * np.sqrt(lam)).T


def _antiderivative(u, s):
    """Cumulative trapezoid from s[0], starting at zero."""
    out = np.zeros_like(u)
    out[:, 1:] = np.cumsum(0.5 * (u[:, 1:] + u[:, :-1]) * np.diff(s)[None, :], axis=1)
    return out


def make(name: str, *, n_rows: Optional[int] = None, n_u: Optional[int] = None,
         n_q: Optional[int] = None, n_chains: Optional[int] = None,
         precision: Optional[str] = None, mask_frac: Optional[float] = None,
         widths_a=None, widths_b=None) -> Workload:
    """Build one of the named workloads.  Keyword overrides shrink it for tests
    (fewer rows, functions, query points or chains) without changing the
    recipe."""
    if name not in CONFIG_NAMES:
        raise KeyError(name)
    master = 14652 + CONFIG_NAMES.index(name)

    if name == "sine1d_fp64":
        # MLP 1-16-16-1 tanh, plain HMC over all parameters.
        wa = list(widths_a or [1, 16, 16, 1])
        N = n_rows or 256
        x = _rng(master, 0).uniform(-3.0, 3.0, size=(N, wa[0]))
        y = np.sin(x[:, :1]) + 0.1 * _rng(master, 1).standard_normal((N, 1))
        P = tower_param_count(wa)
        theta0 = 0.1 * _rng(master, 2).standard_normal(P)
        C = n_chains or 1
        if mask_frac is None:
            masks = [np.arange(P, dtype=np.int64) for _ in range(C)]
        else:
            m = _subset(_rng(master, 3), P, int(np.rint(mask_frac * P)))
            masks = [m for _ in range(C)]
        offs, idx, th = _chains(master, theta0, masks, 0.01)
        return Workload(name, "mlp", wa, None, precision or "fp64", 1.0, 0.1, 1e-3, 20, C, 200,
                        theta0, offs, idx, th, x=x, y=y,
                        note="x~U(-3,3), y=sin x + N(0,0.1^2)")

    if name == "regress2d_fp32":
        wa = list(widths_a or [2, 64, 64, 64, 1])
        N = n_rows or 4096
        x = _rng(master, 0).uniform(-1.0, 1.0, size=(N, wa[0]))
        y = (np.sin(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1]))[:, None]
        y = y + 0.05 * _rng(master, 1).standard_normal((N, 1))
        P = tower_param_count(wa)
        theta0 = 0.1 * _rng(master, 2).standard_normal(P)
        frac = 0.10 if mask_frac is None else mask_frac
        m = _subset(_rng(master, 3), P, int(np.rint(frac * P)))
        C = n_chains or 8
        offs, idx, th = _chains(master, theta0, [m] * C, 0.01)
        return Workload(name, "mlp", wa, None, precision or "fp32", 1.0, 0.05, 5e-4, 50, C, 200,
                        theta0, offs, idx, th, x=x, y=y,
                        note="x~U(-1,1)^2, y=sin(pi x1)cos(pi x2)+N(0,0.05^2)")

    if name == "antideriv_deeponet_bf16":
        wa = list(widths_a or [100, 128, 128, 128, 128])
        wb = list(widths_b or [1, 128, 128, 128, 128])
        nu = n_u or 1000
        s = np.linspace(0.0, 1.0, wa[0])
        u = _grf_rows(_rng(master, 0), s, 0.2, nu)
        v_full = _antiderivative(u, s)
        nq = n_q or wa[0]
        # Query points: the same grid for every function (aligned layout);
        # a smaller n_q keeps an evenly spaced subset of the sensor grid.
        qi = np.unique(np.rint(np.linspace(0, wa[0] - 1, nq)).astype(int)) if nq < wa[0] else np.arange(wa[0])
        yq = s[qi][:, None]
        v = v_full[:, qi]
        P = n_params("deeponet", wa, wb)
        theta0 = 0.1 * _rng(master, 2).standard_normal(P)
        frac = 0.05 if mask_frac is None else mask_frac
        m = _subset(_rng(master, 3), P, int(np.rint(frac * P)))
        C = n_chains or 64
        offs, idx, th = _chains(master, theta0, [m] * C, 0.01)
        return Workload(name, "deeponet", wa, wb, precision or "bf16", 0.1, 1.0, 2e-4, 50, C, 100,
                        theta0, offs, idx, th, u=u, yq=yq, v=v,
                        note="GRF inputs (RBF length 0.2) at equispaced sensors; target = antiderivative",
                        sample_precision="bf16x3")

    if name == "uneven_mlp_bf16":
        wa = list(widths_a or [4, 256, 256, 256, 256, 1])
        N = n_rows or 16384
        x = _rng(master, 0).uniform(-1.0, 1.0, size=(N, wa[0]))
        y = (np.sin(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1]) + 0.5 * np.tanh(x[:, 2] - x[:, 3] ** 2))[:, None]
        y = y + 0.05 * _rng(master, 1).standard_normal((N, 1))
        P = tower_param_count(wa)
        theta0 = 0.1 * _rng(master, 2).standard_normal(P)
        C = n_chains or 256
        masks = []
        for c in range(C):
            f = 0.01 + 0.19 * (c / (C - 1) if C > 1 else 0.0)
            if mask_frac is not None:
                f = mask_frac
            masks.append(_subset(_rng(master, 3, c), P, int(np.rint(f * P))))
        offs, idx, th = _chains(master, theta0, masks, 0.01)
        return Workload(name, "mlp", wa, None, precision or "bf16", 1.0, 0.05, 1e-4, 50, C, 20,
                        theta0, offs, idx, th, x=x, y=y,
                        note="x~U(-1,1)^4, smooth target + N(0,0.05^2); per-chain masks 1%..20%",
                        sample_precision="fp32")

    # surface_deeponet_bf16
    wa = list(widths_a or [8, 512, 512, 512, 512, 256])
    wb = list(widths_b or [2, 512, 512, 512, 512, 256])
    nu = n_u or 2048
    c_in = _rng(master, 0).uniform(0.0, 1.0, size=(nu, wa[0]))
    nx, ny = 32, 16
    xi, eta = np.meshgrid(np.linspace(0, 1, nx), np.linspace(0, 1, ny), indexing="ij")
    pts = np.stack([xi.ravel(), eta.ravel()], axis=1)
    if n_q is not None and n_q < len(pts):
        pts = pts[np.rint(np.linspace(0, len(pts) - 1, n_q)).astype(int)]
    yq = pts
    v = np.zeros((nu, len(pts)))
    K = wa[0]
    for k in range(1, K + 1):
        ck = c_in[:, k - 1][:, None]
        cph = c_in[:, k % K][:, None]
        v += ck * np.sin(k * np.pi * pts[None, :, 0] + np.pi * cph * pts[None, :, 1]) / k
    P = n_params("deeponet", wa, wb)
    theta0 = 0.1 * _rng(master, 2).standard_normal(P)
    frac = 0.02 if mask_frac is None else mask_frac
    m = _subset(_rng(master, 3), P, int(np.rint(frac * P)))
    C = n_chains or 32
    offs, idx, th = _chains(master, theta0, [m] * C, 0.01)
    return Workload(name, "deeponet", wa, wb, precision or "bf16", 0.01, 5e-3, 1e-5, 50, C, 20,
                    theta0, offs, idx, th, u=c_in, yq=yq, v=v,
                    note="8 upstream scalars ~U(0,1), 32x16 surface grid, smooth synthetic field",
                    energy="fp64", sample_precision="fp32")
