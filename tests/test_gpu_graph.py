"""Evaluations captured into a HIP graph by the caller (torch.cuda.graph on
its capture stream): the plan keeps its busy tracking out of the capture, the
evaluation itself records only kernels (no memset), and every replay --
with the program's own eager work and synchronisations between replays --
equals the eager result bit for bit; a changed input is seen by the next
replay.  FP32 and FP64, field with energy and the adjoint."""
import numpy as np
import pytest
import torch

from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu

SHAPE = (64, 32, 8)
CELL = (2e-9, 2e-9, 3e-9)
MS = 8e5


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_field_energy_and_adjoint_in_a_captured_graph(dtype):
    from paper_1204_4302_amd import Plan
    plan = Plan(SHAPE, CELL, dtype)
    m = torch.from_numpy(inputs.random_unit(SHAPE, 7)).to("cuda", dtype)
    g_in = torch.from_numpy(np.random.default_rng(8).standard_normal((3,) + SHAPE[::-1])).to("cuda", dtype)
    H_ref, E_ref = plan.field_energy(m, MS)
    A_ref = plan.adjoint(g_in, MS)
    torch.cuda.synchronize()
    H = torch.empty_like(m)
    A = torch.empty_like(m)
    E = torch.empty((), dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()  # default priority
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # a call on the capture's side stream before capturing
        plan.field_energy(m, MS, out=H, E_out=E)
        plan.adjoint(g_in, MS, out=A)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.field_energy(m, MS, out=H, E_out=E)
        plan.adjoint(g_in, MS, out=A)
    for rep in range(4):
        H.zero_()
        A.zero_()
        E.zero_()
        busy = (m * float(rep + 1)).sum()  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(H, H_ref), f"replay {rep}: field"
        assert torch.equal(A, A_ref), f"replay {rep}: adjoint"
        assert float(E) == float(E_ref), f"replay {rep}: energy"
        del busy
    # the graph reads the input buffer: a negated m gives the negated field
    m.neg_()
    graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(H, -H_ref)
    # and eager calls still work on the plan afterwards
    H2, _ = plan.field_energy(m, MS)
    assert torch.equal(H2, -H_ref)
    del graph
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_energy_alone_in_a_captured_graph(dtype):
    """The energy without a field (X-R2C, Y and the Z pass's spectral sum,
    then the partials' reduction) captured and replayed: every replay equals
    the eager energy bit for bit."""
    from paper_1204_4302_amd import Plan
    plan = Plan(SHAPE, CELL, dtype)
    m = torch.from_numpy(inputs.random_unit(SHAPE, 9)).to("cuda", dtype)
    _, E_ref = plan.field_energy(m, MS, with_field=False)
    torch.cuda.synchronize()
    E = torch.empty((), dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.field_energy(m, MS, with_field=False, E_out=E)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.field_energy(m, MS, with_field=False, E_out=E)
    for rep in range(4):
        E.zero_()
        busy = (m * float(rep + 2)).sum()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert float(E) == float(E_ref), f"replay {rep}"
        del busy
    m.mul_(2.0)  # quadratic: the next replay sees the new input
    graph.replay()
    torch.cuda.synchronize()
    assert abs(float(E) - 4.0 * float(E_ref)) <= 1e-12 * abs(float(E_ref))
    del graph
    plan.close()
