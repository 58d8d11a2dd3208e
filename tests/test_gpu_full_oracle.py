"""Whole-grid parity against the direct O(N^2) oracle (every cell compared).

128 x 128 x 32 cubic cells (random state, forward field) and the
512 x 128 x 4 thin-film strip (forward field and the adjoint, i.e. the
transposed operator, applied to a seeded cotangent), in FP32 and FP64.  The
oracle fields come from tests/golden/full_oracle.py (cached; computed there
when the cache is missing, which takes minutes of host time).
Bar: relative max-norm 1e-5 (FP32) and 1e-12 (FP64)."""
import os
import sys

import numpy as np
import pytest
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import full_oracle  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]
TOL = {torch.float32: 1e-5, torch.float64: 1e-12}


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_random_128x128x32_whole_field(dtype):
    from paper_1204_4302_amd import Plan
    w = full_oracle.WORKLOADS["random_128x128x32"]
    ref = full_oracle.load("random_128x128x32")
    plan = Plan(w["shape"], w["cell"], dtype)
    H = plan.field(torch.from_numpy(ref["m"]).to("cuda", dtype), w["Ms"]).double().cpu().numpy()
    err = _rel(H, ref["H"])
    print(f"128x128x32 {dtype}: whole-field rel. max-norm {err:.2e}")
    assert err <= TOL[dtype]
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_strip_512x128x4_whole_field_and_adjoint(dtype):
    from paper_1204_4302_amd import Plan
    w = full_oracle.WORKLOADS["strip_512x128x4"]
    ref = full_oracle.load("strip_512x128x4")
    plan = Plan(w["shape"], w["cell"], dtype)
    H = plan.field(torch.from_numpy(ref["m"]).to("cuda", dtype), w["Ms"]).double().cpu().numpy()
    gm = plan.adjoint(torch.from_numpy(ref["g"]).to("cuda", dtype), w["Ms"]).double().cpu().numpy()
    err, errT = _rel(H, ref["H"]), _rel(gm, ref["HT"])
    print(f"strip {dtype}: forward {err:.2e}, adjoint {errT:.2e}")
    assert err <= TOL[dtype]
    assert errT <= TOL[dtype]
    plan.close()
