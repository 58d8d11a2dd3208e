"""The largest padded lengths the library takes: 2L = 4096 along x and y (the
X and Y passes hold one pencil per thread group).  Along z the register
kernel holds a pencil and its mirror in one workgroup up to 2048 and one
pencil per workgroup (the split form) at 4096, and takes 3 * 2^a up to 3072
in FP32; the LDS kernel takes lengths whose six pencils fit a workgroup
(6 P <= 8192 values, within its LDS); other z lengths are refused at plan
creation.  Each case is a thin grid so that the oracle's direct sum stays
small: the whole field against the oracle, FP64 and FP32, forward and
adjoint."""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
CELL = (2e-9, 2e-9, 3e-9)
# (the padded z lengths 640, 720 and 1200 run on the generic Z pass in both
# precisions; padded z 3072 has a fused pass in FP32 only and is refused in FP64)
RUNS = [((2048, 2, 2), None), ((2, 2048, 2), None), ((1536, 3, 2), None), ((2, 2, 1024), None),
        ((2, 2, 2048), None), ((3, 3, 2039), None), ((3, 2, 1536), torch.float32),
        ((2, 2, 320), None), ((2, 2, 341), None), ((2, 2, 600), None)]


@pytest.mark.parametrize("shape,only", RUNS, ids=lambda v: str(v))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_max_padded_length(shape, only, dtype):
    from paper_1204_4302_amd import Plan
    if only is not None and dtype != only:
        pytest.skip("refused in this precision at plan creation (test_z_lengths_without_a_fused_pass_are_refused)")
    plan = Plan(shape, CELL, dtype)
    info = plan.info()
    m = inputs.random_unit(shape, 11)
    mq = m.astype(np.float32).astype(np.float64) if dtype == torch.float32 else m
    mg = torch.from_numpy(np.ascontiguousarray(m)).to("cuda", dtype)
    H = plan.field(mg, 8e5).double().cpu().numpy()
    gm = plan.adjoint(mg, 8e5).double().cpu().numpy()
    o = oracle.Oracle(shape, CELL)
    ref = o.field(mq, 8e5)
    err = float(np.abs(H - ref).max() / np.abs(ref).max())
    errT = float(np.abs(gm - ref).max() / np.abs(ref).max())  # A = A^T: the adjoint of m is the field of m
    print(f"{shape} {dtype}: padded {info['Px']}x{info['Py']}x{info['Pz']}, field {err:.2e}, adjoint {errT:.2e}")
    assert err <= TOL[dtype] and errT <= TOL[dtype]


@pytest.mark.parametrize("shape,dtype", [((2, 2, 1000), torch.float32), ((2, 2, 1000), torch.float64),
                                         ((3, 2, 1536), torch.float64), ((2, 2, 700), torch.float64)],
                         ids=lambda v: str(v))
def test_z_lengths_without_a_fused_pass_are_refused(shape, dtype):
    """Refused at plan creation (a host-side check; nothing is launched)."""
    from paper_1204_4302_amd import Plan
    from paper_1204_4302_amd._lib import DemagError
    with pytest.raises(DemagError, match="EUNSUPPORTED"):
        Plan(shape, CELL, dtype)


def test_generic_kernels_refused_where_their_z_pass_does_not_fit():
    from paper_1204_4302_amd import Plan
    from paper_1204_4302_amd._lib import DemagError
    plan = Plan((2, 2, 1024), CELL, torch.float64)  # padded z 2048: register kernel only
    with pytest.raises(DemagError, match="EUNSUPPORTED"):
        plan.set_option("generic_kernels", 1)
    plan.set_option("generic_kernels", 0)


def test_plan_beyond_device_memory_is_enomem():
    """2048 x 2048 x 512 cells in FP64 need about 310 GB for the two spectrum
    buffers alone (B1 103 GB, B2 206 GB), more than the device holds: plan
    creation reports DEMAG_ENOMEM (an allocation failure, nothing is
    launched), and the device stays usable."""
    from paper_1204_4302_amd import Plan
    from paper_1204_4302_amd._lib import DemagError
    with pytest.raises(DemagError, match="ENOMEM"):
        Plan((2048, 2048, 512), CELL, torch.float64)
    plan = Plan((8, 8, 8), CELL, torch.float64)  # the next plan works
    m = torch.from_numpy(inputs.random_unit((8, 8, 8), 3)).to("cuda", torch.float64)
    H = plan.field(m, 8e5).cpu().numpy()
    ref = oracle.Oracle((8, 8, 8), CELL).field(inputs.random_unit((8, 8, 8), 3), 8e5)
    assert np.abs(H - ref).max() <= 1e-12 * np.abs(ref).max()
