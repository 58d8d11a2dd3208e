"""The README's Python quick start, at a small size: every call runs and the
methods agree with each other where they compute the same quantity (SP and
TG evaluate the same potential; the low-rank path on the compressed state
reproduces the dense TG field of that state)."""
import numpy as np
import pytest
import torch

from oracle import lowrank as olr

pytestmark = pytest.mark.gpu


def test_quickstart_calls():
    from paper_1204_4302_amd import DemagEnergy, Plan, TUCKER, inputs
    shape, cell, Ms = (32, 32, 8), (2e-9, 2e-9, 3e-9), 1.4e6
    plan = Plan(shape, cell, torch.float32)
    plan.autotune()
    m = torch.from_numpy(inputs.random_unit(shape, 3)).cuda().float()
    H = plan.field(m, Ms)
    H2, E = plan.field_energy(m, Ms)
    assert torch.equal(H, H2) and float(E) > 0
    mg = m.clone().requires_grad_(True)
    DemagEnergy.apply(mg, plan, Ms).backward()
    V = np.prod(cell)
    assert torch.allclose(mg.grad, -4e-7 * np.pi * Ms * V * H, rtol=1e-5, atol=0)
    plan.sp_prepare()
    Hsp = plan.sp_field(m, Ms)
    plan.tg_prepare()
    Htg = plan.tg_field(m, Ms)
    scale = Hsp.abs().max()
    assert float((Hsp - Htg).abs().max() / scale) < 1e-5
    plan.tg_lowrank_prepare()
    vort = torch.from_numpy(inputs.gaussian_vortex(shape, cell, 10e-9)).cuda().float()
    _, init = inputs.lowrank(shape, TUCKER, 6, seed=0)
    init = [torch.from_numpy(f).cuda().float() for f in init]
    core, factors, relerr = plan.lowrank_compress(vort, TUCKER, 6, 4, init)
    assert 0 <= relerr < 0.1
    FG, H_lr, E_lr = plan.tg_lowrank_field(TUCKER, core, factors, Ms, dense=True)
    m_lr = olr.magnetization(TUCKER, core.double().cpu().numpy(), [f.double().cpu().numpy() for f in factors])
    Hd, Ed = plan.tg_field_energy(torch.from_numpy(np.ascontiguousarray(m_lr)).cuda().float(), Ms)
    assert float((H_lr - Hd).abs().max() / Hd.abs().max()) < 2e-5
    assert abs(float(E_lr) / float(Ed) - 1) < 2e-5
