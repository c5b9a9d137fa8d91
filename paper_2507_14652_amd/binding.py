"""Python binding of libhmc.so (include/hmc.h): argument marshalling only.

Every step of the sampler runs in the HIP library; this module converts
NumPy arrays and torch tensors into the plain pointers and sizes of the C
ABI and back.  torch is imported first so that the library binds to the HIP
runtime that torch has already loaded (one runtime per process).  There is
no fallback: a missing library raises.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_uint64, c_void_p

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhmc.so")

HMC_OK, HMC_EINVAL, HMC_ENOMEM, HMC_EDEVICE, HMC_ESTATE, HMC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}
ENERGY = {"default": 0, "fp64": 1}
KIND = {"mlp": 0, "deeponet": 1}

ABI_FUNCTIONS = (
    "hmc_init", "hmc_leapfrog", "hmc_sample", "hmc_grad", "hmc_trajectory", "hmc_momentum",
    "hmc_get_state", "hmc_set_state", "hmc_counters", "hmc_get_info", "hmc_time_kernels",
    "hmc_sync", "hmc_last_error", "hmc_destroy", "hmc_sensitivity", "hmc_select_mask",
    "hmc_predict", "hmc_init_tuned", "hmc_autotune", "hmc_adapt", "hmc_trajectory_length", "hmc_predict_noalloc",
    "hmc_calibrate", "hmc_set_split",
)


class HMCError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"hmc status {status}: {message}")
        self.status = status


class NetDesc(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("n_widths_a", c_int32), ("widths_a", POINTER(c_int32)),
                ("n_widths_b", c_int32), ("widths_b", POINTER(c_int32)), ("theta0", POINTER(c_double)),
                ("n_params", c_int64), ("prior_sd", c_double), ("lik_sd", c_double),
                ("precision", c_int32), ("inv_mass_diag", POINTER(c_double)), ("energy", c_int32)]


class MaskDesc(ctypes.Structure):
    _fields_ = [("n_chains", c_int32), ("offs", POINTER(c_int64)), ("idx", POINTER(c_int64)),
                ("theta_init", POINTER(c_double))]


class DataDesc(ctypes.Structure):
    _fields_ = [("x", POINTER(c_double)), ("y", POINTER(c_double)), ("n_rows", c_int64),
                ("u", POINTER(c_double)), ("yq", POINTER(c_double)), ("v", POINTER(c_double)),
                ("n_u", c_int64), ("n_q", c_int64)]


class TrajStat(ctypes.Structure):
    _fields_ = [("H0", c_double), ("H1", c_double), ("log_u", c_double),
                ("accepted", c_int32), ("divergent", c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("rows_a", c_int32), ("rows_b", c_int32), ("threads", c_int32), ("dw", c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_params", c_int64), ("nnz", c_int64), ("n_chains", c_int32), ("precision", c_int32),
                ("kind", c_int32), ("rows_per_tile_a", c_int32), ("rows_per_tile_b", c_int32),
                ("tiles_a", c_int32), ("tiles_b", c_int32), ("device_bytes", c_int64),
                ("threads_a", c_int32), ("threads_b", c_int32), ("energy_precision", c_int32),
                ("chain_halves", c_int32)]


STAT_DTYPE = np.dtype([("H0", "f8"), ("H1", "f8"), ("log_u", "f8"), ("accepted", "i4"), ("divergent", "i4")])

_lib = None


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "hmc_init": [POINTER(c_void_p), POINTER(NetDesc), POINTER(MaskDesc), POINTER(DataDesc), c_uint64, P],
        "hmc_leapfrog": [P, c_int32, POINTER(c_int32), POINTER(c_double), c_int32, POINTER(TrajStat)],
        "hmc_sample": [P, c_int64, POINTER(c_double), c_int32, P, POINTER(TrajStat)],
        "hmc_grad": [P, POINTER(c_double), P],
        "hmc_trajectory": [P, P, POINTER(c_double), c_int32, P, P, POINTER(c_double), POINTER(c_double)],
        "hmc_momentum": [P, c_uint64, P],
        "hmc_get_state": [P, P, POINTER(c_double), POINTER(c_uint64)],
        "hmc_set_state": [P, P, POINTER(c_uint64)],
        "hmc_set_split": [P, c_int64],
        "hmc_counters": [P, POINTER(c_int64), POINTER(c_int64)],
        "hmc_get_info": [P, POINTER(Info)],
        "hmc_time_kernels": [P, c_int32, POINTER(c_double)],
        "hmc_sync": [P],
        "hmc_sensitivity": [POINTER(NetDesc), POINTER(DataDesc), POINTER(c_double), POINTER(c_double), P],
        "hmc_select_mask": [POINTER(c_double), c_int64, c_double, POINTER(c_int64), POINTER(c_int64)],
        "hmc_predict": [P, c_int32, P, c_int64, POINTER(DataDesc), POINTER(c_double), POINTER(c_double)],
        "hmc_predict_noalloc": [P, c_int32, P, c_int64, POINTER(DataDesc), POINTER(c_double), POINTER(c_double)],
        "hmc_init_tuned": [POINTER(c_void_p), POINTER(NetDesc), POINTER(MaskDesc), POINTER(DataDesc), c_uint64, P,
                           POINTER(Tuning)],
        "hmc_autotune": [POINTER(NetDesc), POINTER(MaskDesc), POINTER(DataDesc), c_int32, POINTER(Tuning),
                         POINTER(c_double)],
        "hmc_adapt": [P, c_int64, POINTER(c_double), c_int32, c_double, POINTER(c_double)],
        "hmc_calibrate": [P, c_int32, c_int64, POINTER(c_double), c_int32, c_double, POINTER(c_double),
                          POINTER(c_double)],
        "hmc_trajectory_length": [POINTER(c_double), c_int64, c_int32, c_double, POINTER(c_int32)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c_int32
    lib.hmc_last_error.argtypes = [P]
    lib.hmc_last_error.restype = ctypes.c_char_p
    lib.hmc_destroy.argtypes = [P]
    lib.hmc_destroy.restype = None
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr_of(buf):
    """Address of a torch tensor (host or device) or a NumPy array."""
    if isinstance(buf, torch.Tensor):
        if not buf.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return c_void_p(buf.data_ptr())
    return c_void_p(buf.ctypes.data)


def sensitivities(*, widths_a, theta0, sigma, x=None, kind="mlp", widths_b=None, u=None, yq=None,
                  precision="fp32", stream=None):
    """S_i^2 of every parameter around theta0 with standard deviations sigma
    (hmc_sensitivity; FP64 array): an MLP over the rows of x, or a DeepONet
    over the functions u and query points yq."""
    lib = load()
    wa = np.ascontiguousarray(widths_a, dtype=np.int32)
    wb = np.ascontiguousarray(widths_b if widths_b is not None else [0], dtype=np.int32)
    th0, sg = _f64(theta0), _f64(sigma)
    if sg.shape != th0.shape:
        raise ValueError("sigma must have one entry per parameter")
    net = NetDesc(KIND[kind], len(wa), wa.ctypes.data_as(POINTER(c_int32)),
                  len(wb) if widths_b is not None else 0, wb.ctypes.data_as(POINTER(c_int32)),
                  _dptr(th0), th0.size, 1.0, 1.0, PRECISION[precision], None)
    if kind == "mlp":
        xa = _f64(x)
        keep = [xa]
        data = DataDesc(_dptr(xa), None, xa.shape[0], None, None, None, 0, 0)
    else:
        ua, qa = _f64(u), _f64(yq)
        keep = [ua, qa]
        data = DataDesc(None, None, 0, _dptr(ua), _dptr(qa), None, ua.shape[0], qa.shape[0])
    if stream is None and torch.cuda.is_available():
        stream = torch.cuda.current_stream().cuda_stream
    out = np.empty(th0.size, dtype=np.float64)
    st = lib.hmc_sensitivity(ctypes.byref(net), ctypes.byref(data), _dptr(sg), _dptr(out), c_void_p(stream or None))
    del keep
    if st != HMC_OK:
        raise HMCError(st, lib.hmc_last_error(None).decode())
    return out


def trajectory_length(var, eps, mode="median"):
    """Leapfrog steps L = round(pi * v / (2 eps)) of App. C (hmc_trajectory_length),
    v the median ("median") or largest ("max") of the posterior variances var."""
    lib = load()
    v = _f64(np.atleast_1d(var))
    out = c_int32(0)
    st = lib.hmc_trajectory_length(_dptr(v), v.size, {"max": 0, "median": 1}[mode], float(eps), ctypes.byref(out))
    if st != HMC_OK:
        raise HMCError(st, lib.hmc_last_error(None).decode())
    return int(out.value)


def select_mask(s2, tau):
    """Indices (increasing) of the sensitive subset for threshold tau
    (hmc_select_mask)."""
    lib = load()
    s2 = _f64(s2)
    idx = np.empty(s2.size, dtype=np.int64)
    n = c_int64(0)
    st = lib.hmc_select_mask(_dptr(s2), s2.size, float(tau), idx.ctypes.data_as(POINTER(c_int64)), ctypes.byref(n))
    if st != HMC_OK:
        raise HMCError(st, lib.hmc_last_error(None).decode())
    return idx[:n.value].copy()


def _descs(*, kind, widths_a, widths_b, theta0, prior_sd, lik_sd, precision, offs, idx, theta_init=None,
           inv_mass=None, x=None, y=None, u=None, yq=None, v=None, energy="default"):
    """The C descriptors of a network, its masks and its data, and the arrays
    they point into (keep them alive while the descriptors are used)."""
    wa = np.ascontiguousarray(widths_a, dtype=np.int32)
    wb = np.ascontiguousarray(widths_b if widths_b is not None else [0], dtype=np.int32)
    th0 = _f64(theta0)
    minv = _f64(inv_mass)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    tinit = _f64(theta_init)
    net = NetDesc(KIND[kind], len(wa), wa.ctypes.data_as(POINTER(c_int32)),
                  len(wb) if widths_b is not None else 0, wb.ctypes.data_as(POINTER(c_int32)),
                  _dptr(th0), th0.size, float(prior_sd), float(lik_sd), PRECISION[precision],
                  _dptr(minv) if minv is not None else None, ENERGY[energy])
    mask = MaskDesc(len(offs) - 1, offs.ctypes.data_as(POINTER(c_int64)),
                    idx.ctypes.data_as(POINTER(c_int64)), _dptr(tinit) if tinit is not None else None)
    keep = [wa, wb, offs, idx, th0, minv, tinit]
    if kind == "mlp":
        xa, ya = _f64(x), _f64(y)
        keep += [xa, ya]
        data = DataDesc(_dptr(xa), _dptr(ya), xa.shape[0], None, None, None, 0, 0)
    else:
        ua, qa, va = _f64(u), _f64(yq), _f64(v)
        keep += [ua, qa, va]
        data = DataDesc(None, None, 0, _dptr(ua), _dptr(qa), _dptr(va), ua.shape[0], qa.shape[0])
    return net, mask, data, keep


def _workload_kwargs(w, precision=None, energy=None):
    kw = dict(kind=w.kind, widths_a=w.widths_a, widths_b=w.widths_b, theta0=w.theta0,
              prior_sd=w.prior_sd, lik_sd=w.lik_sd, precision=precision or w.precision,
              offs=w.offs, idx=w.idx, theta_init=w.theta_init, energy=energy or w.energy)
    if w.kind == "mlp":
        kw.update(x=w.x, y=w.y)
    else:
        kw.update(u=w.u, yq=w.yq, v=w.v)
    return kw


def autotune(*, reps=10, **kw):
    """The fastest launch shape for an engine with these arguments (as for
    Sampler) and its gradient-evaluation milliseconds (hmc_autotune)."""
    lib = load()
    net, mask, data, keep = _descs(**kw)
    best = Tuning()
    ms = c_double(0.0)
    st = lib.hmc_autotune(ctypes.byref(net), ctypes.byref(mask), ctypes.byref(data), int(reps), ctypes.byref(best),
                          ctypes.byref(ms))
    del keep
    if st != HMC_OK:
        raise HMCError(st, lib.hmc_last_error(None).decode())
    return {k: getattr(best, k) for k, _ in Tuning._fields_}, ms.value


def autotune_workload(w, precision=None, reps=10):
    """autotune() for a ``workloads.Workload``."""
    return autotune(reps=reps, **_workload_kwargs(w, precision))


class Sampler:
    """One engine (hmc_ctx): a network, per-chain masks, data and chain state
    on the current GPU."""

    def __init__(self, *, kind, widths_a, widths_b=None, theta0, prior_sd, lik_sd, precision,
                 offs, idx, theta_init=None, inv_mass=None, x=None, y=None, u=None, yq=None, v=None,
                 seed=0, stream=None, tuning=None, energy="default"):
        self._lib = load()
        self._ctx = c_void_p()
        self.kind = kind
        self._widths_a = list(widths_a)
        self.precision = precision
        self.state_dtype = torch.float64 if precision == "fp64" else torch.float32
        self._np_state = np.float64 if precision == "fp64" else np.float32
        net, mask, data, keep = _descs(kind=kind, widths_a=widths_a, widths_b=widths_b, theta0=theta0,
                                       prior_sd=prior_sd, lik_sd=lik_sd, precision=precision, offs=offs, idx=idx,
                                       theta_init=theta_init, inv_mass=inv_mass, x=x, y=y, u=u, yq=yq, v=v,
                                       energy=energy)
        self.offs = keep[2]
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        if tuning is None:
            st = self._lib.hmc_init(ctypes.byref(self._ctx), ctypes.byref(net), ctypes.byref(mask),
                                    ctypes.byref(data), c_uint64(seed), c_void_p(stream or None))
        else:
            tn = Tuning(**{k: int(tuning.get(k, 0)) for k, _ in Tuning._fields_})
            st = self._lib.hmc_init_tuned(ctypes.byref(self._ctx), ctypes.byref(net), ctypes.byref(mask),
                                          ctypes.byref(data), c_uint64(seed), c_void_p(stream or None),
                                          ctypes.byref(tn))
        if st != HMC_OK:
            raise HMCError(st, self._lib.hmc_last_error(None).decode())
        info = Info()
        self._check(self._lib.hmc_get_info(self._ctx, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in Info._fields_}
        self.nnz = int(info.nnz)
        self.n_chains = int(info.n_chains)

    @classmethod
    def from_workload(cls, w, *, seed=0, precision=None, stream=None, inv_mass=None, tuning=None, energy=None):
        kw = _workload_kwargs(w, precision, energy)
        kw.update(inv_mass=inv_mass, seed=seed, stream=stream, tuning=tuning)
        return cls(**kw)

    # ------------------------------------------------------------------
    def _check(self, st):
        if st != HMC_OK:
            raise HMCError(st, self._lib.hmc_last_error(self._ctx).decode())

    def _state_tensor(self, n=None):
        return torch.empty(self.nnz if n is None else (n, self.nnz), dtype=self.state_dtype, device="cuda")

    def _eps_array(self, eps, n):
        e = np.broadcast_to(np.asarray(eps, dtype=np.float64), (n,)).copy()
        return e

    def _as_state(self, a):
        if isinstance(a, torch.Tensor):
            return a.to(device="cuda", dtype=self.state_dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a, dtype=self._np_state)).cuda()

    # ------------------------------------------------------------------
    def grad(self):
        """(U [C] float64 numpy, g [nnz] device tensor) at the current positions."""
        U = np.empty(self.n_chains)
        g = self._state_tensor()
        torch.cuda.synchronize()
        self._check(self._lib.hmc_grad(self._ctx, _dptr(U), _ptr_of(g)))
        return U, g

    def trajectory(self, p0, eps, L):
        """Leapfrog without Metropolis from the current state; the state is unchanged."""
        p = self._as_state(p0)
        e = self._eps_array(eps, self.n_chains)
        th, po = self._state_tensor(), self._state_tensor()
        H0, H1 = np.empty(self.n_chains), np.empty(self.n_chains)
        torch.cuda.synchronize()
        self._check(self._lib.hmc_trajectory(self._ctx, _ptr_of(p), _dptr(e), int(L), _ptr_of(th),
                                             _ptr_of(po), _dptr(H0), _dptr(H1)))
        return th, po, H0, H1

    def set_split(self, batch_rows):
        """Symmetric-splitting HMC over data batches of batch_rows rows
        (hmc_set_split); 0 returns to plain leapfrog."""
        self._check(self._lib.hmc_set_split(self._ctx, int(batch_rows)))

    def momentum(self, iteration):
        out = self._state_tensor()
        torch.cuda.synchronize()
        self._check(self._lib.hmc_momentum(self._ctx, c_uint64(iteration), _ptr_of(out)))
        return out

    def leapfrog(self, eps, L, chains=None):
        """One Metropolis-adjusted trajectory for the given chains (all by default)."""
        ids = np.arange(self.n_chains, dtype=np.int32) if chains is None else np.ascontiguousarray(chains, np.int32)
        e = self._eps_array(eps, len(ids))
        stats = (TrajStat * len(ids))()
        self._check(self._lib.hmc_leapfrog(self._ctx, len(ids), ids.ctypes.data_as(POINTER(c_int32)), _dptr(e),
                                           int(L), stats))
        return np.frombuffer(bytes(stats), dtype=STAT_DTYPE)

    def sample(self, n, eps, L, out=None, want_stats=True):
        """n iterations for every chain; returns (samples [n, nnz] or out, stats [n, C] or None)."""
        e = self._eps_array(eps, self.n_chains)
        stats = (TrajStat * (n * self.n_chains))() if want_stats else None
        torch.cuda.synchronize()
        self._check(self._lib.hmc_sample(self._ctx, int(n), _dptr(e), int(L),
                                         _ptr_of(out) if out is not None else None, stats))
        st = np.frombuffer(bytes(stats), dtype=STAT_DTYPE).reshape(n, self.n_chains) if want_stats else None
        return out, st

    def adapt(self, n, eps0, L, target=0.8):
        """n iterations of step-size adaptation on the device (hmc_adapt): each
        chain's step size by dual averaging toward the target acceptance rate;
        returns the per-chain averaged step sizes (float64 numpy).  The
        chains move."""
        e = self._eps_array(eps0, self.n_chains)
        out = np.empty(self.n_chains)
        torch.cuda.synchronize()
        self._check(self._lib.hmc_adapt(self._ctx, int(n), _dptr(e), int(L), float(target), _dptr(out)))
        return out

    def calibrate(self, rounds, batch, eps, L, target=0.8):
        """Bisection of every chain's step size on the batch-mean acceptance
        probability (hmc_calibrate); returns (step sizes, last batch means)."""
        e = self._eps_array(eps, self.n_chains)
        out, acc = np.empty(self.n_chains), np.empty(self.n_chains)
        torch.cuda.synchronize()
        self._check(self._lib.hmc_calibrate(self._ctx, int(rounds), int(batch), _dptr(e), int(L), float(target),
                                            _dptr(out), _dptr(acc)))
        return out, acc

    def get_state(self):
        th = self._state_tensor()
        U = np.empty(self.n_chains)
        it = np.empty(self.n_chains, dtype=np.uint64)
        torch.cuda.synchronize()
        self._check(self._lib.hmc_get_state(self._ctx, _ptr_of(th), _dptr(U), it.ctypes.data_as(POINTER(c_uint64))))
        return th, U, it

    def set_state(self, theta_s, iteration=None):
        th = self._as_state(theta_s)
        it = None if iteration is None else np.ascontiguousarray(iteration, dtype=np.uint64)
        torch.cuda.synchronize()
        self._check(self._lib.hmc_set_state(self._ctx, _ptr_of(th),
                                            it.ctypes.data_as(POINTER(c_uint64)) if it is not None else None))

    def counters(self):
        a = np.empty(self.n_chains, dtype=np.int64)
        d = np.empty(self.n_chains, dtype=np.int64)
        self._check(self._lib.hmc_counters(self._ctx, a.ctypes.data_as(POINTER(c_int64)),
                                           d.ctypes.data_as(POINTER(c_int64))))
        return a, d

    def predict(self, samples, x=None, chain=0, u=None, yq=None, no_alloc=False):
        """Mean and variance (FP64 arrays) of the network output over stored
        samples ([n][nnz], as sample() writes them; torch tensor or NumPy
        array) of one chain: an MLP at the rows of x ([rows][d_out]), a
        DeepONet at functions u and query points yq ([n_u][n_q]).
        no_alloc: hmc_predict_noalloc (the library's fixed device scratch)."""
        if isinstance(samples, torch.Tensor):
            if samples.dtype != self.state_dtype or samples.dim() != 2 or samples.shape[1] != self.nnz:
                raise ValueError("samples must be [n][nnz] in the state dtype")
        else:
            samples = np.ascontiguousarray(samples, dtype=self._np_state)
            if samples.ndim != 2 or samples.shape[1] != self.nnz:
                raise ValueError("samples must be [n][nnz]")
        if self.kind == "mlp":
            xa = _f64(x)
            keep = [xa]
            shape = (xa.shape[0], int(self._widths_a[-1]))
            data = DataDesc(_dptr(xa), None, xa.shape[0], None, None, None, 0, 0)
        else:
            ua, qa = _f64(u), _f64(yq)
            keep = [ua, qa]
            shape = (ua.shape[0], qa.shape[0])
            data = DataDesc(None, None, 0, _dptr(ua), _dptr(qa), None, ua.shape[0], qa.shape[0])
        mean = np.empty(shape)
        var = np.empty(shape)
        torch.cuda.synchronize()
        fn = self._lib.hmc_predict_noalloc if no_alloc else self._lib.hmc_predict
        self._check(fn(self._ctx, int(chain), _ptr_of(samples), int(samples.shape[0]), ctypes.byref(data),
                       _dptr(mean), _dptr(var)))
        del keep
        return mean, var

    def time_kernels(self, reps=20):
        ms = np.zeros(4)
        self._check(self._lib.hmc_time_kernels(self._ctx, int(reps), _dptr(ms)))
        return ms

    def sync(self):
        self._check(self._lib.hmc_sync(self._ctx))

    def close(self):
        if self._ctx:
            self._lib.hmc_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
