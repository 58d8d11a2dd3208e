"""LLG driver (Sec. 2) on the GPU: Heun steps through the C ABI against the
same steps of the reference (oracle/llg.py, DM oracle field), and a single
cubic cell against the closed-form precession/damping."""
import numpy as np
import pytest
import torch

import oracle
from oracle import llg
from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu
GAMMA = 2.2128e5


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)], ids=["f64", "f32"])
def test_llg_heun_vs_reference(dtype, tol):
    from paper_1204_4302_amd import Plan
    shape, cell, Ms = (16, 8, 2), (1.95e-9, 1.95e-9, 0.75e-9), 8e5
    alpha, dt, steps, hext = 0.5, 2e-14, 20, (0.0, 2e4, 5e4)
    m0 = inputs.noisy_strip(shape, 6)
    if dtype == torch.float32:
        m0 = m0.astype(np.float32).astype(np.float64)
    plan = Plan(shape, cell, dtype)
    m = torch.from_numpy(m0).to("cuda", dtype)
    plan.llg_heun(m, Ms, alpha, dt, steps, H_ext=hext)
    o = oracle.Oracle(shape, cell)
    ref = llg.heun(lambda x: o.field(x, Ms), m0, alpha, GAMMA, hext, dt, steps)
    got = m.double().cpu().numpy()
    moved = np.abs(ref - m0).max()
    err = np.abs(got - ref).max()
    print(f"{dtype}: moved {moved:.3e}, max |m_gpu - m_ref| {err:.3e}")
    assert moved > 1e-3  # the test exercises real motion
    assert err <= tol
    assert np.abs(np.sqrt((got ** 2).sum(0)) - 1).max() < (1e-14 if dtype == torch.float64 else 1e-6)


def test_llg_single_cell_closed_form():
    from paper_1204_4302_amd import Plan
    plan = Plan((1, 1, 1), (2e-9,) * 3, torch.float64)
    theta0, phi0, alpha, H = 1.0, 0.3, 0.1, 8e4
    g = GAMMA / (1 + alpha ** 2)
    T, steps = 3.0 / (g * H), 400
    m = torch.tensor([np.sin(theta0) * np.cos(phi0), np.sin(theta0) * np.sin(phi0), np.cos(theta0)],
                     dtype=torch.float64, device="cuda").reshape(3, 1, 1, 1).contiguous()
    plan.llg_heun(m, 8e5, alpha, T / steps, steps, H_ext=(0, 0, H))
    theta = 2 * np.arctan(np.tan(theta0 / 2) * np.exp(-alpha * g * H * T))
    phi = phi0 + g * H * T
    ref = np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
    assert np.abs(m.cpu().numpy().reshape(3) - ref).max() < 2e-5


def test_llg_rejects_bad_arguments():
    from paper_1204_4302_amd import Plan
    from paper_1204_4302_amd._lib import DemagError
    plan = Plan((4, 4, 2), (2e-9,) * 3, torch.float32)
    m = torch.from_numpy(inputs.random_unit((4, 4, 2), 1)).to("cuda", torch.float32)
    with pytest.raises(DemagError):
        plan.llg_heun(m, 8e5, -0.1, 1e-13, 1)
    with pytest.raises(DemagError):
        plan.llg_heun(m, 8e5, 0.1, 0.0, 1)
    with pytest.raises(ValueError):
        plan.llg_heun(m, 8e5, 0.1, 1e-13, 1, work=torch.empty(10, device="cuda"))
    before = m.clone()
    plan.llg_heun(m, 8e5, 0.1, 1e-13, 0)  # zero steps: unchanged
    assert torch.equal(m, before)
