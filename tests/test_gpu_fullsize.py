"""Full-size parity at 256 x 256 x 64 (2 x 2 x 3 nm cells, Ms = 1.4e6 A/m),
with the plan in the launch shapes bench.py times.

The oracle computes sampled cells one by one (seeded random cells, the 8
corners and the central column); properties that hold at any size check the
whole grid: for a uniform state the body-averaged field equals -Ms D m with
D the cuboid demagnetizing factors of the whole body (closed form).
"""
import os

import numpy as np
import pytest
import torch

import oracle
from closed_forms import body_factors
from paper_1204_4302_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SHAPE = (256, 256, 64)
CELL = (2e-9, 2e-9, 3e-9)
MS = 1.4e6
CACHE = os.environ.get("DEMAG_ORACLE_CACHE", "/tmp/demag_oracle_cache")


@pytest.fixture(scope="module")
def ora():
    return oracle.Oracle(SHAPE, CELL, cache_dir=CACHE)


@pytest.fixture(scope="module")
def plans():
    """Tuned as bench.py tunes them before timing."""
    from paper_1204_4302_amd import Plan
    out = {torch.float32: Plan(SHAPE, CELL, torch.float32), torch.float64: Plan(SHAPE, CELL, torch.float64)}
    for p in out.values():
        p.autotune()
    return out


def _gpu(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


@pytest.mark.parametrize("state", ["random", "vortex"])
def test_sampled_field_vs_oracle(ora, plans, state):
    m = inputs.random_unit(SHAPE, 3) if state == "random" else inputs.gaussian_vortex(SHAPE, CELL, 10e-9)
    t = inputs.sample_targets(SHAPE, 384, 11)
    for dtype, tol in [(torch.float64, 1e-12), (torch.float32, 1e-5)]:
        mq = m.astype(np.float32).astype(np.float64) if dtype == torch.float32 else m
        ref = ora.field_targets(mq, MS, t)
        H = plans[dtype].field(_gpu(m, dtype), MS).double().cpu().numpy().reshape(3, -1)[:, t]
        err = np.max(np.abs(H - ref)) / np.max(np.abs(ref))
        print(f"{state} {dtype}: {t.size} cells, rel err {err:.3e}")
        assert err <= tol


def test_sampled_adjoint_vs_oracle(ora, plans):
    nx, ny, nz = SHAPE
    g = np.random.default_rng(33).standard_normal((3, nz, ny, nx))
    t = inputs.sample_targets(SHAPE, 128, 12)
    for dtype, tol in [(torch.float64, 1e-12), (torch.float32, 1e-5)]:
        gq = g.astype(np.float32).astype(np.float64) if dtype == torch.float32 else g
        ref = ora.field_T_targets(gq, MS, t)
        got = plans[dtype].adjoint(_gpu(g, dtype), MS).double().cpu().numpy().reshape(3, -1)[:, t]
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"adjoint {dtype}: rel err {err:.3e}")
        assert err <= tol


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
def test_uniform_body_average_whole_grid(plans, dtype, tol):
    direction = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    m = inputs.uniform(SHAPE, direction)
    H = plans[dtype].field(_gpu(m, dtype), MS).double()
    mean = H.reshape(3, -1).mean(dim=1).cpu().numpy()
    D = np.array(body_factors(*(SHAPE[k] * CELL[k] for k in range(3))))
    ref = -MS * D * direction
    err = np.max(np.abs(mean - ref)) / np.max(np.abs(ref))
    print(f"{dtype}: body-average rel err {err:.3e}")
    assert err <= tol


def test_energy_fp32_vs_fp64_and_positive(plans):
    for m in [inputs.random_unit(SHAPE, 3), inputs.gaussian_vortex(SHAPE, CELL, 10e-9)]:
        _, e32 = plans[torch.float32].field_energy(_gpu(m, torch.float32), MS, with_field=False)
        _, e64 = plans[torch.float64].field_energy(_gpu(m, torch.float64), MS, with_field=False)
        e32, e64 = float(e32), float(e64)
        print(f"E f32 {e32:.9e} f64 {e64:.9e} rel {abs(e32 - e64) / e64:.2e}")
        assert e64 > 0 and abs(e32 - e64) <= 1e-5 * e64
