"""Radix schedules of the register FFT (the autotuner's search space): every
schedule of the padded lengths that have more than one (128, 256, 1024 and
2048; 128 as 8.8.2, 8.2.8 and 8.4.4) on every axis, forced through the
"radix_schedule" option, against the oracle (field and adjoint; FP64 1e-12,
FP32 1e-5); the autotuner's choice is reported by demag_plan_describe."""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu

CELL, MS = (2e-9, 2e-9, 3e-9), 8e5
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
# padded (Px, Py, Pz): (128, 4, 128), (256, 256, 4), (1024, 4, 4), (4, 2048, 4), (4, 4, 1024), (4, 4, 2048)
SHAPES = [(64, 2, 64), (128, 128, 2), (512, 2, 2), (2, 1024, 2), (2, 2, 512), (2, 2, 1024)]
_ORACLES = {}


def _oracle(shape):
    if shape not in _ORACLES:
        _ORACLES[shape] = oracle.Oracle(shape, CELL)
    return _ORACLES[shape]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_every_radix_schedule_vs_oracle(shape, dtype):
    from paper_1204_4302_amd import Plan
    plan = Plan(shape, CELL, dtype)
    m = inputs.random_unit(shape, 21)
    g = np.random.default_rng(22).standard_normal(m.shape)
    if dtype == torch.float32:
        m, g = (a.astype(np.float32).astype(np.float64) for a in (m, g))
    o = _oracle(shape)
    ref, refT = o.field(m, MS), o.field_T(g, MS)
    seen = set()
    for S in (0, 1, 2):
        plan.set_option("radix_schedule", S)
        desc = plan.describe()
        H = plan.field(torch.from_numpy(m).to("cuda", dtype), MS).double().cpu().numpy()
        gm = plan.adjoint(torch.from_numpy(g).to("cuda", dtype), MS).double().cpu().numpy()
        err = float(np.abs(H - ref).max() / np.abs(ref).max())
        errT = float(np.abs(gm - refT).max() / np.abs(refT).max())
        print(f"{shape} {dtype} S={S}: {desc}\n    field {err:.2e}, adjoint {errT:.2e}")
        assert err <= TOL[dtype] and errT <= TOL[dtype]
        seen.add(desc)
    assert len(seen) >= 2  # the lengths of these grids have more than one schedule
    plan.close()


def test_describe_names_the_radix_schedule():
    from paper_1204_4302_amd import Plan
    plan = Plan((64, 2, 64), CELL, torch.float32)  # padded z 128
    plan.set_option("radix_schedule", 2)
    assert "z_conv:pow2" in plan.describe() and "radix=8.4.4" in plan.describe()
    plan.set_option("radix_schedule", 1)
    assert "radix=8.2.8" in plan.describe()
    plan.set_option("radix_schedule", 0)
    assert "radix=8.8.2" in plan.describe()
    plan.close()


def test_sp_field_with_each_schedule_agrees():
    """The scalar-potential Z pass takes the schedule of the fused Z pass at
    preparation: each schedule's SP field equals the default's to FP32
    rounding."""
    from paper_1204_4302_amd import Plan
    shape = (64, 2, 64)
    m = torch.from_numpy(inputs.random_unit(shape, 23)).to("cuda", torch.float32)
    out = []
    for S in (0, 1, 2):
        plan = Plan(shape, CELL, torch.float32)
        plan.set_option("radix_schedule", S)
        plan.sp_prepare()
        out.append(plan.sp_field(m, MS).double().cpu().numpy())
        plan.close()
    for H in out[1:]:
        assert np.abs(H - out[0]).max() <= 3e-6 * np.abs(out[0]).max()
