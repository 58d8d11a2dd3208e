"""Tensor-grid method (TG dense, Sec. 3.2 eq. (sumpot)) on the GPU.

TG evaluates the same potential as SP -- the exact cell-centre potential of
the cell-wise constant magnetization (eq. (scpot)) -- through the Sinc
quadrature of eq. (transform) and Gaussian mode products, and the same
finite-difference field, so its oracle is the SP oracle.  Tolerances follow
from the quadrature: the kernel 1/r^3 is reproduced to 2e-7 (FP32 step) and
6.5e-13 (FP64 step) relative over all distances (pinned on the host), so
FP64 is held to 1e-10 and FP32 to 1e-5 (relative max-norm).
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 1e-5}
CACHE = os.environ.get("DEMAG_ORACLE_CACHE", "/tmp/demag_oracle_cache")


def rel_err(a, b):
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / scale) if scale > 0 else float(np.abs(a).max())


def _gpu(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def _quantised(m, dtype):
    return m.astype(np.float32).astype(np.float64) if dtype == torch.float32 else m


SHAPES = [
    ((8, 8, 8), (2e-9, 2e-9, 2e-9), 8e5),
    ((1, 1, 1), (2e-9, 2e-9, 3e-9), 1.4e6),
    ((5, 1, 1), (2e-9, 2e-9, 2e-9), 8e5),
    ((2, 3, 4), (2e-9, 2e-9, 2e-9), 8e5),
    ((13, 7, 5), (2e-9, 2e-9, 3e-9), 1.4e6),       # no FFT: any n
    ((24, 17, 3), (1.95e-9, 1.95e-9, 0.75e-9), 8e5),
    ((47, 11, 23), (2e-9, 2e-9, 3e-9), 1.4e6),
    ((64, 32, 8), (2e-9, 2e-9, 3e-9), 1.4e6),
]


@pytest.mark.parametrize("shape,cell,Ms", SHAPES, ids=lambda v: str(v))
@pytest.mark.parametrize("dtype,mode12", [(torch.float64, 0), (torch.float32, 0), (torch.float32, 1)],
                         ids=["f64", "f32", "f32-fused"])
def test_tg_field_vs_oracle(shape, cell, Ms, dtype, mode12):
    from paper_1204_4302_amd import Plan
    plan = Plan(shape, cell, dtype)
    plan.set_option("tg_mode12", mode12)
    plan.tg_prepare()
    assert plan.tg_path()["fused"] == bool(mode12)
    m = inputs.random_unit(shape, 1)
    H = plan.tg_field(_gpu(m, dtype), Ms).double().cpu().numpy()
    ref = oracle.SPOracle(shape, cell).field(_quantised(m, dtype), Ms)
    err = rel_err(H, ref)
    print(f"shape={shape} dtype={dtype} nodes={plan.tg_info()['nodes']} rel_err={err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_tg_energy_and_sp_agree(dtype):
    """Energy vs the oracle, and TG against the FFT-based SP path on one grid."""
    from paper_1204_4302_amd import Plan
    shape, cell, Ms = (32, 16, 8), (2e-9, 2e-9, 3e-9), 1.4e6
    plan = Plan(shape, cell, dtype)
    plan.tg_prepare()
    plan.sp_prepare()
    m = inputs.gaussian_vortex(shape, cell, 10e-9)
    mg = _gpu(m, dtype)
    H, E = plan.tg_field_energy(mg, Ms)
    so = oracle.SPOracle(shape, cell)
    mq = _quantised(m, dtype)
    ref = so.energy(mq, so.field(mq, Ms), Ms)
    assert abs(float(E) / ref - 1) <= TOL[dtype]
    Hsp = plan.sp_field(mg, Ms)
    assert rel_err(H.double().cpu().numpy(), Hsp.double().cpu().numpy()) <= TOL[dtype]


def test_tg_unprepared_and_repeat():
    from paper_1204_4302_amd import Plan
    from paper_1204_4302_amd._lib import DemagError
    shape, cell = (16, 8, 4), (2e-9,) * 3
    plan = Plan(shape, cell, torch.float32)
    m = _gpu(inputs.random_unit(shape, 2), torch.float32)
    with pytest.raises(DemagError):
        plan.tg_field(m, 8e5)
    plan.tg_prepare()
    plan.tg_prepare()
    assert plan.tg_path()["fused"]  # FP32: the fused mode-1/2 kernel by default
    a = plan.tg_field(m, 8e5)
    b = plan.tg_field(m, 8e5)
    assert torch.equal(a, b)
    h1 = plan.field(m, 8e5)  # the DM path of the same plan is unaffected
    plan.tg_field(m, 8e5)
    assert torch.equal(h1, plan.field(m, 8e5))


@pytest.mark.slow
@pytest.mark.parametrize("mode12", [0, 1], ids=["library", "fused"])
def test_tg_full_size_sampled(mode12):
    """256 x 256 x 64, 2 x 2 x 3 nm, Ms = 1.4e6, FP32 (the size bench.py times)."""
    from paper_1204_4302_amd import Plan
    shape, cell, Ms = (256, 256, 64), (2e-9, 2e-9, 3e-9), 1.4e6
    so = oracle.SPOracle(shape, cell, cache_dir=CACHE)
    m = inputs.random_unit(shape, 3)
    t = inputs.sample_targets(shape, 64, 19)
    plan = Plan(shape, cell, torch.float32)
    plan.set_option("tg_mode12", mode12)
    plan.tg_prepare()
    assert plan.tg_path()["fused"] == bool(mode12)
    H = plan.tg_field(_gpu(m, torch.float32), Ms).double().cpu().numpy().reshape(3, -1)[:, t]
    ref = so.field_targets(_quantised(m, torch.float32), Ms, t)
    err = rel_err(H, ref)
    print(f"float32: {t.size} cells, {plan.tg_info()}, rel err {err:.3e}")
    assert err <= TOL[torch.float32]


FUSED_SHAPES = [
    ((130, 72, 6), (2e-9, 2e-9, 3e-9), 1.4e6),    # three row blocks, ragged, 16-byte loads
    ((67, 45, 4), (2e-9, 2e-9, 2e-9), 8e5),       # lengths not multiples of 4: element loads
    ((40, 300, 2), (2e-9, 2e-9, 3e-9), 1.4e6),    # two passes of column tiles per wave
    ((16, 512, 1), (2e-9, 2e-9, 2e-9), 8e5),      # the widest ny (132 KB of LDS), one plane
]


@pytest.mark.parametrize("shape,cell,Ms", FUSED_SHAPES, ids=lambda v: str(v))
def test_tg_fused_vs_library_and_oracle(shape, cell, Ms):
    """FP32: the fused mode-1/2 kernel and the library GEMM chain against the oracle and each other."""
    from paper_1204_4302_amd import Plan
    m = inputs.random_unit(shape, 7)
    ref = oracle.SPOracle(shape, cell).field(_quantised(m, torch.float32), Ms)
    out = {}
    for mode in (1, 0):
        plan = Plan(shape, cell, torch.float32)
        plan.set_option("tg_mode12", mode)
        plan.tg_prepare()
        path = plan.tg_path()
        assert path["fused"] == bool(mode)
        info = plan.tg_info()
        assert 0 < path["flops_issued"] <= info["flops_per_eval"]
        if not mode:
            assert path["flops_issued"] == info["flops_per_eval"]
        H, E = plan.tg_field_energy(_gpu(m, torch.float32), Ms)
        out[mode] = (H.double().cpu().numpy(), float(E))
        err = rel_err(out[mode][0], ref)
        print(f"shape={shape} tg_mode12={mode} {path} rel_err={err:.3e}")
        assert err <= TOL[torch.float32]
    assert rel_err(out[1][0], out[0][0]) <= 2e-6
    assert abs(out[1][1] / out[0][1] - 1) <= 2e-6


def test_tg_fused_skips_zero_blocks_and_switches():
    """The banded Gaussian matrices of a long axis: fewer flops issued, same field; the option rebuilds."""
    from paper_1204_4302_amd import Plan
    shape, cell, Ms = (256, 128, 4), (2e-9, 2e-9, 2e-9), 8e5
    plan = Plan(shape, cell, torch.float32)
    plan.set_option("tg_mode12", 1)
    plan.tg_prepare()
    fused = plan.tg_path()
    assert fused["fused"] and fused["flops_issued"] < plan.tg_info()["flops_per_eval"]
    m = _gpu(inputs.random_unit(shape, 8), torch.float32)
    a = plan.tg_field(m, Ms)
    assert torch.equal(a, plan.tg_field(m, Ms))        # deterministic
    plan.set_option("tg_mode12", 0)                    # rebuilt on the library path
    assert not plan.tg_path()["fused"]
    b = plan.tg_field(m, Ms)
    plan.set_option("tg_mode12", 1)
    assert plan.tg_path()["fused"]
    # rebuilt: the mode-3 GEMM's rocBLAS solution is chosen by timing again, so the
    # sums may run in another order
    c = plan.tg_field(m, Ms)
    assert rel_err(c.double().cpu().numpy(), a.double().cpu().numpy()) <= 1e-6
    assert rel_err(a.double().cpu().numpy(), b.double().cpu().numpy()) <= 2e-6


def test_tg_wide_y_takes_library_path():
    """ny above the fused kernel's LDS limit (512): the fused option falls back to the library GEMMs."""
    from paper_1204_4302_amd import Plan
    shape, cell, Ms = (3, 520, 1), (2e-9, 2e-9, 2e-9), 8e5
    plan = Plan(shape, cell, torch.float32)
    plan.set_option("tg_mode12", 1)
    plan.tg_prepare()
    assert not plan.tg_path()["fused"]
    m = inputs.random_unit(shape, 9)
    H = plan.tg_field(_gpu(m, torch.float32), Ms).double().cpu().numpy()
    ref = oracle.SPOracle(shape, cell).field(_quantised(m, torch.float32), Ms)
    assert rel_err(H, ref) <= TOL[torch.float32]
