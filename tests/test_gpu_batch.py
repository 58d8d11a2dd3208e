"""Batched evaluation: many grids of uneven shapes recorded into one HIP graph.

The workload mirrors a batch of 96 independent magnetizations whose grid
sizes are drawn (seeded) from {32^3, 64x64x16, 96x48x8, 128x128x4, 48^3},
2 nm cubic cells, FP32.  Each grid of the batch must equal its single-grid
call bit for bit (same kernels, same launch shapes), replays must be
repeatable, and a sample of grids is checked against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu

SIZES = [(32, 32, 32), (64, 64, 16), (96, 48, 8), (128, 128, 4), (48, 48, 48)]
CELL = (2e-9, 2e-9, 2e-9)
MS = 8e5


def batch_shapes(count, seed=4):
    rng = np.random.default_rng(seed)
    return [SIZES[i] for i in rng.integers(0, len(SIZES), size=count)]


def build(count, dtype=torch.float32):
    from paper_1204_4302_amd import Plan
    shapes = batch_shapes(count)
    plans = [Plan(s, CELL, dtype) for s in shapes]
    ms = [torch.from_numpy(inputs.random_unit(s, 4000 + g)).to("cuda", dtype) for g, s in enumerate(shapes)]
    hs = [torch.empty_like(m) for m in ms]
    return shapes, plans, ms, hs


def test_batch_equals_single_calls_and_replays_repeat():
    from paper_1204_4302_amd import Batch
    shapes, plans, ms, hs = build(24)
    batch = Batch(plans, ms, hs, MS)
    info = batch.info()
    groups = len(set(shapes))
    assert info["members"] == 24 and info["groups"] == groups and 1 <= info["streams"] <= groups
    batch.launch()
    torch.cuda.synchronize()
    first = [h.clone() for h in hs]
    for p, m, h in zip(plans, ms, first):
        single = p.field(m, MS)
        assert torch.equal(single, h)
    for _ in range(5):
        for h in hs:
            h.zero_()
        batch.launch()
        torch.cuda.synchronize()
        for a, b in zip(first, hs):
            assert torch.equal(a, b)
    batch.close()


def test_batch_of_96_members_equal_single_calls():
    """The 96-grid workload itself (seeded sizes, m seeds 4000 + g): every
    member of one graph replay equals its single-grid call bit for bit, and
    one member of each shape matches the oracle at sampled cells (FP32 bar
    1e-5)."""
    from paper_1204_4302_amd import Batch
    shapes, plans, ms, hs = build(96)
    assert len(set(shapes)) == len(SIZES)
    batch = Batch(plans, ms, hs, MS)
    for h in hs:
        h.fill_(float("nan"))
    batch.launch()
    torch.cuda.synchronize()
    for p, m, h in zip(plans, ms, hs):
        assert torch.equal(p.field(m, MS), h)
    checked = set()
    for g, s in enumerate(shapes):
        if s in checked:
            continue
        checked.add(s)
        t = inputs.sample_targets(s, 256, 5)
        ref = oracle.Oracle(s, CELL).field_targets(ms[g].double().cpu().numpy(), MS, t)
        got = hs[g].double().cpu().numpy().reshape(3, -1)[:, t]
        err = float(np.abs(got - ref).max() / np.abs(ref).max())
        print(f"grid {g} {s}: {err:.2e}")
        assert err <= 1e-5
    batch.close()
    for p in plans:
        p.close()


def test_batch_autotune_keeps_results():
    """Group-tuned launch shapes may swap kernel families (rounding differs),
    so members are checked against single calls to FP32 rounding; replays of
    the re-recorded graph stay bitwise repeatable."""
    from paper_1204_4302_amd import Batch
    shapes, plans, ms, hs = build(24)
    batch = Batch(plans, ms, hs, MS)
    batch.autotune()
    for h in hs:
        h.fill_(float("nan"))
    batch.launch()
    torch.cuda.synchronize()
    first = [h.clone() for h in hs]
    for p, m, h in zip(plans, ms, first):
        single = p.field(m, MS)
        err = float((single - h).abs().max() / single.abs().max())
        assert err <= 2e-6, err
    for _ in range(3):
        for h in hs:
            h.zero_()
        batch.launch()
        torch.cuda.synchronize()
        for a, b in zip(first, hs):
            assert torch.equal(a, b)
    batch.close()


def test_batch_members_vs_oracle():
    from paper_1204_4302_amd import Batch
    shapes, plans, ms, hs = build(10)
    batch = Batch(plans, ms, hs, MS)
    batch.launch()
    torch.cuda.synchronize()
    seen = set()
    for s, m, h in zip(shapes, ms, hs):
        if s in seen:
            continue
        seen.add(s)
        o = oracle.Oracle(s, CELL)
        t = inputs.sample_targets(s, 128, 3)
        mq = m.double().cpu().numpy()
        ref = o.field_targets(mq, MS, t)
        got = h.double().cpu().numpy().reshape(3, -1)[:, t]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"{s}: {err:.2e}")
        assert err <= 1e-5
    batch.close()


def test_batch_rejects_bad_arguments():
    from paper_1204_4302_amd import Batch, Plan
    from paper_1204_4302_amd._lib import DemagError
    p = Plan((8, 8, 8), CELL, torch.float32)
    q = Plan((8, 8, 8), CELL, torch.float64)
    m = torch.zeros(3, 8, 8, 8, device="cuda")
    h = torch.zeros_like(m)
    with pytest.raises(DemagError):
        Batch([p, p], [m, m], [h, h], MS)  # one plan twice: shared scratch
    m64 = m.double()
    with pytest.raises(DemagError):
        Batch([p, q], [m, m64], [h, m64.clone()], MS)  # mixed precisions


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_batch_with_split_z_pass(dtype):
    """Grids padded to 4096 along z run the fused Z pass in its split form (one
    ky row per workgroup); in a batch its tiles go through the batch's per-grid
    tile ranges.  Three such grids and one ordinary grid: every member equals
    its single-grid call bit for bit, and one is checked against the oracle."""
    from paper_1204_4302_amd import Batch, Plan
    shapes = [(2, 2, 2048), (2, 2, 2048), (3, 2, 2040), (8, 8, 8)]
    plans = [Plan(s, CELL, dtype) for s in shapes]
    ms = [torch.from_numpy(inputs.random_unit(s, 4100 + g)).to("cuda", dtype) for g, s in enumerate(shapes)]
    hs = [torch.empty_like(m) for m in ms]
    batch = Batch(plans, ms, hs, MS)
    batch.launch()
    torch.cuda.synchronize()
    for p, m, h in zip(plans, ms, hs):
        assert torch.equal(p.field(m, MS), h)
    o = oracle.Oracle(shapes[2], CELL)
    m2 = inputs.random_unit(shapes[2], 4102)
    mq = m2.astype(np.float32).astype(np.float64) if dtype == torch.float32 else m2
    ref = o.field(mq, MS)
    err = float(np.abs(hs[2].double().cpu().numpy() - ref).max() / np.abs(ref).max())
    print(f"{dtype}: split-Z member vs oracle {err:.2e}")
    assert err <= (1e-12 if dtype == torch.float64 else 1e-5)
    batch.close()


def test_batch_with_generic_lengths():
    """Grids whose padded lengths are neither 2^a nor 3 * 2^a (80, 50, 20, 10)
    run every pass on the generic kernels; in a batch those take the per-grid
    pointer lists too.  Members equal single calls bit for bit; one against
    the oracle."""
    from paper_1204_4302_amd import Batch, Plan
    shapes = [(40, 25, 10), (40, 25, 10), (25, 10, 5), (32, 16, 8)]
    plans = [Plan(s, CELL, torch.float32) for s in shapes]
    ms = [torch.from_numpy(inputs.random_unit(s, 4200 + g)).to("cuda", torch.float32) for g, s in enumerate(shapes)]
    hs = [torch.empty_like(m) for m in ms]
    batch = Batch(plans, ms, hs, MS)
    batch.launch()
    torch.cuda.synchronize()
    for p, m, h in zip(plans, ms, hs):
        assert torch.equal(p.field(m, MS), h)
    o = oracle.Oracle(shapes[2], CELL)
    mq = inputs.random_unit(shapes[2], 4202).astype(np.float32).astype(np.float64)
    ref = o.field(mq, MS)
    err = float(np.abs(hs[2].double().cpu().numpy() - ref).max() / np.abs(ref).max())
    print(f"generic-length member vs oracle {err:.2e}")
    assert err <= 1e-5
    batch.close()
