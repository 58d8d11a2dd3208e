"""A large grid, 768 x 512 x 512 (201 M cells, 1.6 G padded points), against
the oracle.  With the magnetization zero outside a 10 x 9 x 8 region, the field
inside the region and the energy are those of the region alone, which the
oracle computes on the region's own grid: an exact identity at any grid size.
The region is placed at the origin corner and at the far corner, so that the
highest addresses of every buffer are used.

What the size exercises: the tensor set-up kernels run over more elements than
one launch holds (they are issued in pieces); in FP64 each spectrum component
(6.45 GB) exceeds the 32-bit buffer range of the register Z pass, so the plan
takes the generic Z pass with 64-bit addresses; in FP32 (3.2 GB) the register
Z pass runs close to that range; the X and Y passes address 10-20 GB buffers.
About 100 GB of device memory at the peak (tensor set-up).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu

SHAPE = (768, 512, 512)
CELL = (2e-9, 2e-9, 3e-9)
MS = 8e5
REGION = (10, 9, 8)
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_large_grid_region_vs_oracle(dtype):
    from paper_1204_4302_amd import Plan
    nx, ny, nz = SHAPE
    rx, ry, rz = REGION
    print(f"plan {SHAPE} {dtype}", flush=True)
    plan = Plan(SHAPE, CELL, dtype)
    info = plan.info()
    print(f"padded {info['Px']}x{info['Py']}x{info['Pz']}", flush=True)
    o = oracle.Oracle(REGION, CELL)
    m = torch.zeros((3, nz, ny, nx), dtype=dtype, device="cuda")
    for seed, (x0, y0, z0) in ((21, (0, 0, 0)), (22, (nx - rx, ny - ry, nz - rz))):
        mr = inputs.random_unit(REGION, seed)
        mq = mr.astype(np.float32).astype(np.float64) if dtype == torch.float32 else mr
        m.zero_()
        m[:, z0:z0 + rz, y0:y0 + ry, x0:x0 + rx] = torch.from_numpy(np.ascontiguousarray(mr)).to("cuda", dtype)
        H, E = plan.field_energy(m, MS)
        Hr = H[:, z0:z0 + rz, y0:y0 + ry, x0:x0 + rx].double().cpu().numpy()
        del H
        ref = o.field(mq, MS)
        Eref = o.energy(mq, ref, MS)
        err = float(np.abs(Hr - ref).max() / np.abs(ref).max())
        eerr = abs(float(E.cpu()) - Eref) / abs(Eref)
        print(f"region at {(x0, y0, z0)}: field rel err {err:.2e}, energy rel err {eerr:.2e}", flush=True)
        assert err <= TOL[dtype] and eerr <= TOL[dtype]
    del m
    del plan
    torch.cuda.empty_cache()
