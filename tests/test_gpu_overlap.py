"""The adjoint pass with each layer's weight-gradient terms beside its
adjoint product's multiplies (the product's epilogue after a barrier) does
the same arithmetic in the same order as the two one after the other
(HMC_OVERLAP=0): U and the gradient agree bitwise, for the MLP and both
DeepONet towers, in every product precision, with per-entry sums and with
the dense weight-gradient product."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("name,kw,dw", [
    ("uneven_mlp_bf16", dict(n_rows=300, n_chains=3), "gather"),
    ("uneven_mlp_bf16", dict(n_rows=300, n_chains=3), "dense"),
    ("regress2d_fp32", dict(n_rows=700, n_chains=2), "gather"),
    ("antideriv_deeponet_bf16", dict(n_u=150, n_q=37, n_chains=2), "gather"),
    ("antideriv_deeponet_bf16", dict(n_u=150, n_q=37, n_chains=2), "dense"),
])
def test_overlapped_adjoint_layers_are_bitwise_sequential(name, kw, dw, prec, monkeypatch):
    from paper_2507_14652_amd import Sampler
    from paper_2507_14652_amd.binding import HMC_EUNSUPPORTED, HMCError
    w = workloads.make(name, **kw)
    monkeypatch.setenv("HMC_DW", dw)
    if dw == "dense":
        monkeypatch.setenv("HMC_ROWS_A", "32")   # the dense product needs tiles of whole K chunks
        monkeypatch.setenv("HMC_ROWS_B", "32")
    out = {}
    for ov in ("0", "1"):
        monkeypatch.setenv("HMC_OVERLAP", ov)
        try:
            s = Sampler.from_workload(w, precision=prec, seed=3)
        except HMCError as e:
            if e.status == HMC_EUNSUPPORTED:
                pytest.skip(str(e))
            raise
        U, g = s.grad()
        out[ov] = (U, g.cpu().numpy())
        s.close()
    np.testing.assert_array_equal(out["0"][0], out["1"][0])
    np.testing.assert_array_equal(out["0"][1], out["1"][1])
