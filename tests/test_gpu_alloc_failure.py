"""Every device allocation of plan creation, of the scalar-potential set-up
and of the autotuner failing in turn, forced from the host by the library's
test hook (while DEMAG_FAIL_ALLOC_AT=k is set, the k-th allocation since the
value last changed fails as out of memory; no kernel is launched on a failed
buffer): each failure is DEMAG_ENOMEM, the plan is left as it was (or not
created), and the device stays usable -- a plan made afterwards matches the
oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu

SHAPE, CELL, MS = (12, 10, 6), (2e-9, 2e-9, 3e-9), 8e5


def _field_ok(plan, dtype):
    m = inputs.random_unit(SHAPE, 31)
    mq = m.astype(np.float32).astype(np.float64) if dtype == torch.float32 else m
    H = plan.field(torch.from_numpy(m).to("cuda", dtype), MS).double().cpu().numpy()
    ref = oracle.Oracle(SHAPE, CELL).field(mq, MS)
    return float(np.abs(H - ref).max() / np.abs(ref).max()) <= (1e-12 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_each_plan_creation_allocation_failure_is_enomem(monkeypatch, dtype):
    from paper_1204_4302_amd import Plan
    from paper_1204_4302_amd._lib import DemagError
    failed = 0
    for k in range(1, 64):
        monkeypatch.setenv("DEMAG_FAIL_ALLOC_AT", str(k))
        try:
            plan = Plan(SHAPE, CELL, dtype)
        except DemagError as e:
            assert "ENOMEM" in str(e), str(e)
            failed += 1
            continue
        plan.close()  # k is past the last allocation of plan creation
        break
    else:
        pytest.fail("plan creation never succeeded")
    monkeypatch.delenv("DEMAG_FAIL_ALLOC_AT")
    print(f"{dtype}: {failed} allocations of plan creation failed in turn")
    assert failed >= 5  # B1, B2, the tensor spectrum, the partials, the energy scalar, set-up scratch
    plan = Plan(SHAPE, CELL, dtype)
    assert _field_ok(plan, dtype)
    plan.close()


def test_sp_prepare_and_autotune_allocation_failures_leave_the_plan_usable(monkeypatch):
    from paper_1204_4302_amd import Plan
    from paper_1204_4302_amd._lib import DemagError
    dtype = torch.float32
    plan = Plan(SHAPE, CELL, dtype)
    before = plan.describe()
    for k in (1, 2):  # the autotuner's two scratch vectors
        monkeypatch.setenv("DEMAG_FAIL_ALLOC_AT", str(k))
        with pytest.raises(DemagError, match="ENOMEM"):
            plan.autotune()
        assert plan.describe() == before  # the launch shapes it had
    sp_failed = 0
    for k in range(1, 64):  # (the value differs from the last one set: counting restarts)
        monkeypatch.setenv("DEMAG_FAIL_ALLOC_AT", str(k))
        try:
            plan.sp_prepare()
        except DemagError as e:
            assert "ENOMEM" in str(e), str(e)
            sp_failed += 1
            continue
        break
    monkeypatch.delenv("DEMAG_FAIL_ALLOC_AT")
    assert sp_failed >= 1
    assert _field_ok(plan, dtype)
    m = torch.from_numpy(inputs.random_unit(SHAPE, 32)).to("cuda", dtype)
    plan.sp_prepare()
    H = plan.sp_field(m, MS)
    assert torch.isfinite(H).all()
    plan.close()
