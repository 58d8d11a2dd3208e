"""FP32 against FP64 on 128 x 128 x 32 cells of 2.5 nm cubes, Ms = 8e5 A/m,
forward field, for the three states of that workload: i.i.d. random unit
vectors (seed 2), the vortex m = (-y, x, exp(-r^2/r0^2)) normalised with
r0 = 10 nm, and the flower m = (x, y, L) normalised with L the half-width.
Both precisions against the FP64 oracle at sampled cells (seeded random
cells, the 8 corners, the central column), and FP32 against the FP64 GPU
field on the whole grid; the FP32 errors are printed."""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu

SHAPE = (128, 128, 32)
CELL = (2.5e-9, 2.5e-9, 2.5e-9)
MS = 8e5
STATES = {
    "random": lambda: inputs.random_unit(SHAPE, 2),
    "vortex": lambda: inputs.gaussian_vortex(SHAPE, CELL, 10e-9),
    "flower": lambda: inputs.flower_xyl(SHAPE, CELL),
}


@pytest.fixture(scope="module")
def setup():
    from paper_1204_4302_amd import Plan
    return (oracle.Oracle(SHAPE, CELL), Plan(SHAPE, CELL, torch.float32), Plan(SHAPE, CELL, torch.float64),
            inputs.sample_targets(SHAPE, 384, 22))


@pytest.mark.parametrize("state", list(STATES))
def test_fp32_and_fp64_vs_oracle(setup, state):
    o, p32, p64, t = setup
    m = STATES[state]()
    m32 = m.astype(np.float32).astype(np.float64)
    H32 = p32.field(torch.from_numpy(np.ascontiguousarray(m)).to("cuda", torch.float32), MS).double().cpu().numpy()
    H64 = p64.field(torch.from_numpy(np.ascontiguousarray(m)).to("cuda", torch.float64), MS).cpu().numpy()
    ref32 = o.field_targets(m32, MS, t)
    ref64 = o.field_targets(m, MS, t)
    e32 = float(np.abs(H32.reshape(3, -1)[:, t] - ref32).max() / np.abs(ref32).max())
    e64 = float(np.abs(H64.reshape(3, -1)[:, t] - ref64).max() / np.abs(ref64).max())
    whole = float(np.abs(H32 - H64).max() / np.abs(H64).max())
    print(f"{state}: FP32 vs oracle {e32:.2e}, FP64 vs oracle {e64:.2e}, FP32 vs FP64 GPU (whole grid) {whole:.2e}")
    assert e32 <= 1e-5 and e64 <= 1e-12 and whole <= 1e-5
