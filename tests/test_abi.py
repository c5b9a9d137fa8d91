"""The C-ABI library loads, exports every function that include/hmc.h
declares, and rejects invalid arguments on the host before any device work
(these calls never reach the GPU)."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hmc.h")

binding = pytest.importorskip("paper_2507_14652_amd.binding")

needs_lib = pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="libhmc.so not built")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:hmc_status|const char\*|void)\s+(hmc_\w+)\s*\(", text, re.M)))


def test_header_declares_the_binding_functions():
    assert declared_functions() == sorted(binding.ABI_FUNCTIONS)


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def _init(**over):
    """Calls hmc_init with a valid small MLP description, with overrides."""
    lib = binding.load()
    B = binding
    wa = np.array(over.pop("widths_a", [2, 3, 1]), dtype=np.int32)
    P = int(sum(wa[i] * wa[i + 1] + wa[i + 1] for i in range(len(wa) - 1)))
    n_params = over.pop("n_params", P)
    theta0 = np.zeros(max(P, 1))
    offs = np.array(over.pop("offs", [0, 3]), dtype=np.int64)
    idx = np.array(over.pop("idx", [0, 4, 7]), dtype=np.int64)
    x = np.zeros((5, int(wa[0])))
    y = np.zeros((5, int(wa[-1])))
    net = B.NetDesc(over.pop("kind", 0), len(wa), wa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 0, None,
                    theta0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n_params,
                    over.pop("prior_sd", 1.0), over.pop("lik_sd", 1.0), over.pop("precision", 1), None)
    mask = B.MaskDesc(len(offs) - 1, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None)
    n_rows = over.pop("n_rows", 5)
    data = B.DataDesc(x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if not over.pop("no_y", False) else None,
                      n_rows, None, None, None, 0, 0)
    assert not over
    ctx = ctypes.c_void_p()
    st = lib.hmc_init(ctypes.byref(ctx), ctypes.byref(net), ctypes.byref(mask), ctypes.byref(data), 0, None)
    return st, ctx, lib.hmc_last_error(None).decode()


@needs_lib
@pytest.mark.parametrize("over,needle", [
    (dict(n_params=12), "n_params"),
    (dict(idx=[0, 7, 4]), "strictly increasing"),
    (dict(idx=[0, 4, 13]), "out of range"),
    (dict(idx=[-1, 4, 7]), "out of range"),
    (dict(offs=[0, 0], idx=[]), "selects no entry"),
    (dict(offs=[1, 3]), "offs[0]"),
    (dict(widths_a=[2]), "widths"),
    (dict(widths_a=[2, 0, 1]), "widths"),
    (dict(widths_a=[2, 5000, 1]), "widths"),
    (dict(prior_sd=0.0), "prior_sd"),
    (dict(lik_sd=float("nan")), "lik_sd"),
    (dict(precision=7), "precision"),
    (dict(kind=4), "kind"),
    (dict(n_rows=0), "n_rows"),
    (dict(no_y=True), "x and y"),
])
def test_invalid_arguments_are_rejected_on_the_host(over, needle):
    st, ctx, msg = _init(**over)
    assert st == binding.HMC_EINVAL
    assert not ctx.value
    assert needle in msg, msg


@needs_lib
def test_null_descriptors_are_rejected():
    lib = binding.load()
    ctx = ctypes.c_void_p()
    assert lib.hmc_init(ctypes.byref(ctx), None, None, None, 0, None) == binding.HMC_EINVAL
    assert lib.hmc_init(None, None, None, None, 0, None) == binding.HMC_EINVAL


@needs_lib
def test_calls_on_a_null_engine_are_rejected():
    lib = binding.load()
    assert lib.hmc_sync(None) == binding.HMC_EINVAL
    assert lib.hmc_grad(None, None, None) == binding.HMC_EINVAL
    assert lib.hmc_adapt(None, 1, None, 1, 0.8, None) == binding.HMC_EINVAL
    lib.hmc_destroy(None)


@needs_lib
@pytest.mark.parametrize("seed,n,tau", [(0, 1, 0.5), (1, 50, 0.9), (2, 1000, 0.3), (3, 1000, 1.0), (4, 7, 0.0)])
def test_select_mask_matches_the_oracle(seed, n, tau):
    """The library's threshold selection (host code) against the oracle's,
    including ties (values drawn from a small set)."""
    from oracle import sensitivity as osen
    rng = np.random.default_rng(seed)
    s2 = rng.choice([0.0, 0.5, 1.0, 2.0, 3.5], size=n) * (1 + (seed % 2) * rng.random(n))
    s2[0] = max(s2[0], 1.0)
    got = binding.select_mask(s2, tau)
    np.testing.assert_array_equal(got, osen.select_mask(s2, tau))


@needs_lib
@pytest.mark.parametrize("s2,tau", [([0.0, 0.0], 0.5), ([1.0, -1.0], 0.5), ([1.0, float("nan")], 0.5),
                                   ([1.0, 2.0], 1.5), ([1.0, 2.0], -0.1)])
def test_select_mask_rejects_bad_input(s2, tau):
    with pytest.raises(binding.HMCError) as e:
        binding.select_mask(np.array(s2), tau)
    assert e.value.status == binding.HMC_EINVAL


@needs_lib
def test_sensitivity_rejects_bad_input_on_the_host():
    lib = binding.load()
    B = binding
    wa = np.array([2, 3, 1], dtype=np.int32)
    theta0 = np.zeros(13)
    x = np.zeros((5, 2))
    out = np.zeros(13)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    data = B.DataDesc(dp(x), None, 5, None, None, None, 0, 0)

    def call(kind=0, sigma=np.ones(13), s2=out):
        net = B.NetDesc(kind, len(wa), wa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 0, None, dp(theta0), 13,
                        1.0, 1.0, 1, None)
        return lib.hmc_sensitivity(ctypes.byref(net), ctypes.byref(data), dp(sigma) if sigma is not None else None,
                                   dp(s2) if s2 is not None else None, None)
    assert call(sigma=None) == B.HMC_EINVAL
    assert call(s2=None) == B.HMC_EINVAL
    assert call(sigma=-np.ones(13)) == B.HMC_EINVAL
    assert call(sigma=np.full(13, np.inf)) == B.HMC_EINVAL
    assert call(kind=4) == B.HMC_EINVAL
    assert "kind" in lib.hmc_last_error(None).decode()


@needs_lib
@pytest.mark.parametrize("tune,needle", [
    ((7, 0, 0, 0), "rows"), ((16, 8, 0, 0), "rows"), ((16, 0, 128, 0), "threads"), ((16, 0, 256, 3), "dw"),
])
def test_tuned_init_rejects_bad_launch_shapes(tune, needle):
    """A tuning record outside the allowed shapes is refused before the
    engine is built."""
    lib = binding.load()
    w = workloads.make("regress2d_fp32", n_rows=20, n_chains=1)
    net, mask, data, keep = binding._descs(**binding._workload_kwargs(w))
    ctx = ctypes.c_void_p()
    t = binding.Tuning(*tune)
    st = lib.hmc_init_tuned(ctypes.byref(ctx), ctypes.byref(net), ctypes.byref(mask), ctypes.byref(data), 0, None,
                            ctypes.byref(t))
    assert st == binding.HMC_EINVAL and not ctx.value
    assert needle in lib.hmc_last_error(None).decode()


@needs_lib
def test_autotune_rejects_bad_arguments_on_the_host():
    lib = binding.load()
    w = workloads.make("regress2d_fp32", n_rows=20, n_chains=1)
    net, mask, data, keep = binding._descs(**binding._workload_kwargs(w))
    best = binding.Tuning()
    assert lib.hmc_autotune(ctypes.byref(net), ctypes.byref(mask), ctypes.byref(data), 0, ctypes.byref(best),
                            None) == binding.HMC_EINVAL
    net.lik_sd = -1.0
    assert lib.hmc_autotune(ctypes.byref(net), ctypes.byref(mask), ctypes.byref(data), 3, ctypes.byref(best),
                            None) == binding.HMC_EINVAL
    assert "lik_sd" in lib.hmc_last_error(None).decode()


@needs_lib
def test_trajectory_length_matches_the_oracle():
    """hmc_trajectory_length (host code in the library) against the oracle's
    rule on the App. C cases and on vectors of variances, both modes."""
    import json
    from oracle import hmc as oh
    from paper_2507_14652_amd import trajectory_length
    d = json.load(open(os.path.join(ROOT, "tests", "golden", "appc_trajectory_lengths.json")))
    for case in d["cases"]:
        assert trajectory_length([case["posterior_variance"]], case["step_size"]) == case["L"]
    rng = np.random.default_rng(2)
    for _ in range(50):
        v = rng.uniform(0, 1, rng.integers(1, 9)) ** 3
        e = 10 ** rng.uniform(-4, -1)
        for mode in ("max", "median"):
            if math.pi * (v.max() if mode == "max" else np.median(v)) / (2 * e) > 1e6:
                continue
            assert trajectory_length(v, e, mode) == oh.trajectory_length(v, e, mode)


@needs_lib
@pytest.mark.parametrize("var,eps,mode", [([], 1e-3, 1), ([0.1], 0.0, 1), ([0.1], 1e-3, 2), ([-0.1], 1e-3, 0),
                                          ([float("nan")], 1e-3, 0), ([1e6], 1e-6, 0)])
def test_trajectory_length_rejects_bad_input(var, eps, mode):
    lib = binding.load()
    v = np.array(var if var else [0.0], dtype=np.float64)
    L = ctypes.c_int32(-7)
    st = lib.hmc_trajectory_length(v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(var), mode, eps,
                                   ctypes.byref(L))
    assert st == binding.HMC_EINVAL and L.value == -7
    assert lib.hmc_last_error(None)
