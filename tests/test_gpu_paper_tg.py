"""Sec. 5 experiments with the tensor-grid method on low-rank magnetization,
end to end on the GPU: the paper's states on the 40^3 unit cube, compressed
by ALS from a seeded random guess (or, for the uniform state, written in
exact CP rank 1), then the low-rank field and energy.  Compared, like the
paper's Tables cube_homo / cube_flower / cube_vortex, with DM on the same
grid (our DM FP64 plan, itself pinned to the oracle): the energy and the
field error of eq. (relerr).  The paper leaves the TG difference stencil
open; with the stencil read here (central inside, second-order one-sided on
the faces) the TG energies agree with the paper's printed TG energies to the
printed digits, and are held to them; the field errors, whose printed values
also depend on the paper's unstated DM reference resolution, to within a
factor of two.  Units: Ms = 1, lengths in the cube edge, energies in
mu0 Ms^2 L^3."""
import numpy as np
import pytest
import torch

from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu

N40 = (40, 40, 40)
CELL = (1 / 40,) * 3
MU0 = 4e-7 * np.pi


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float64)


def _dm(m):
    from paper_1204_4302_amd import Plan
    plan = Plan(N40, CELL, torch.float64)
    H, E = plan.field_energy(_gpu(m), 1.0)
    return H.cpu().numpy(), float(E) / MU0


def _relerr_h(H, Hdm):
    """Eq. (relerr): RMS over cells of |H - H_DM| (Ms = 1)."""
    return float(np.sqrt(((H - Hdm) ** 2).sum() / np.prod(N40)))


def _lowrank(fmt, core, factors):
    from paper_1204_4302_amd import Plan
    plan = Plan(N40, CELL, torch.float64)
    plan.tg_lowrank_prepare()
    _, H, E = plan.tg_lowrank_field(fmt, core, factors, 1.0)
    return H.cpu().numpy(), float(E) / MU0


def _compress(fmt, m, r, sweeps, seed):
    from paper_1204_4302_amd import Plan
    plan = Plan(N40, CELL, torch.float64)
    _, init = inputs.lowrank(N40, fmt, r, seed)
    return plan.lowrank_compress(_gpu(m), fmt, r, sweeps, [_gpu(f) for f in init])


def test_cube_homogeneous_cp_rank1():
    """Table cube_homo: TG (CP r = 1), energy error vs the exact 1/6 printed
    as 3.8e-4, field error vs DM 2.3e-3."""
    m = inputs.uniform(N40, (0, 0, 1))
    core = np.zeros((3, 1))
    core[2, 0] = 1.0
    factors = [np.ones((3, 1, 40)) for _ in range(3)]
    H, E = _lowrank(1, _gpu(core), [_gpu(f) for f in factors])
    Hdm, Edm = _dm(m)
    e_err = abs(E * 6 - 1)
    h_err = _relerr_h(H, Hdm)
    print(f"cube_homo TG CP1: relerr e {e_err:.2e} (paper 3.8e-4), relerr h {h_err:.2e} (paper 2.3e-3); "
          f"DM e {abs(Edm * 6 - 1):.1e}")
    assert abs(e_err - 3.8e-4) < 0.05e-4
    assert 2.3e-3 / 2 < h_err < 2.3e-3 * 2


def test_cube_flower_cp_rank6():
    """Table cube_flower: TG (CP r = 6), e printed as 1.529e-1 (DM 1.528e-1),
    field error 1.8e-3."""
    m = inputs.paper_flower(N40, CELL, a=1.0, b=2.0, c=1.0)
    core, factors, relerr = _compress(1, m, 6, 60, seed=61)
    H, E = _lowrank(1, core, factors)
    Hdm, Edm = _dm(m)
    h_err = _relerr_h(H, Hdm)
    print(f"cube_flower TG CP6: compression relerr {relerr:.2e}, e {E:.4e} (paper 1.529e-1, DM {Edm:.4e}), "
          f"relerr h {h_err:.2e} (paper 1.8e-3)")
    assert Edm == pytest.approx(1.528e-1, abs=0.0005e-1)  # the paper's DM energy
    assert E == pytest.approx(1.529e-1, abs=0.0005e-1)
    assert 1.8e-3 / 2 < h_err < 1.8e-3 * 2


def test_cube_vortex_tucker_rank10():
    """Table cube_vortex: TG (Tucker r = 10), e printed as 2.193e-2 (DM
    2.189e-2), field error 4.0e-3."""
    m = inputs.paper_vortex(N40, CELL, rc=0.14)
    core, factors, relerr = _compress(0, m, 10, 12, seed=71)
    H, E = _lowrank(0, core, factors)
    Hdm, Edm = _dm(m)
    h_err = _relerr_h(H, Hdm)
    print(f"cube_vortex TG Tucker10: compression relerr {relerr:.2e}, e {E:.4e} (paper 2.193e-2, DM {Edm:.4e}), "
          f"relerr h {h_err:.2e} (paper 4.0e-3)")
    assert Edm == pytest.approx(2.189e-2, abs=0.0005e-2)
    assert E == pytest.approx(2.193e-2, abs=0.0005e-2)
    assert 4.0e-3 / 2 < h_err < 4.0e-3 * 2


THIN = (80, 80, 8)
THIN_CELL = (1 / 80, 1 / 80, 0.1 / 8)


def _thin(fmt, core, factors, m):
    from paper_1204_4302_amd import Plan
    lr = Plan(THIN, THIN_CELL, torch.float64)
    lr.tg_lowrank_prepare()
    _, H, E = lr.tg_lowrank_field(fmt, core, factors, 1.0)
    dm = Plan(THIN, THIN_CELL, torch.float64)
    Hdm, Edm = dm.field_energy(_gpu(m), 1.0)
    h_err = float(np.sqrt(((H - Hdm) ** 2).sum().item() / np.prod(THIN)))
    return float(E) / MU0, float(Edm) / MU0, h_err  # energies in mu0 Ms^2 L^3, L = 1


def test_thin_film_homogeneous_cp_rank1():
    """Table thin_homo (1 x 1 x 0.1 film, 80 x 80 x 8, out of plane): TG
    (CP r = 1) e printed as 4.025e-2 (DM 4.025e-2), field error 3.7e-3."""
    m = inputs.uniform(THIN, (0, 0, 1))
    core = np.zeros((3, 1))
    core[2, 0] = 1.0
    factors = [np.ones((3, 1, n)) for n in THIN]
    E, Edm, h_err = _thin(1, _gpu(core), [_gpu(f) for f in factors], m)
    print(f"thin_homo TG CP1: e {E:.4e} (paper 4.025e-2, DM {Edm:.4e}), relerr h {h_err:.2e} (paper 3.7e-3)")
    assert Edm == pytest.approx(4.025e-2, abs=0.0005e-2)
    assert E == pytest.approx(4.025e-2, abs=0.0005e-2)
    assert 3.7e-3 / 2 < h_err < 3.7e-3 * 2


def test_thin_film_vortex_tucker():
    """Table thin_vortex: the vortex of eq. (config1) (r_c = 0.14) in the thin
    film; TG e printed as 1.569e-3 (DM 1.569e-3), field error 2.9e-3.  The
    table's "CP r = 1" cannot hold a vortex (not a separable state); a Tucker
    rank 8 compression is used instead."""
    from paper_1204_4302_amd import Plan
    m = inputs.paper_vortex(THIN, THIN_CELL, rc=0.14)
    plan = Plan(THIN, THIN_CELL, torch.float64)
    _, init = inputs.lowrank(THIN, 0, 8, seed=81)
    core, factors, relerr = plan.lowrank_compress(_gpu(m), 0, 8, 12, [_gpu(f) for f in init])
    E, Edm, h_err = _thin(0, core, factors, m)
    print(f"thin_vortex TG Tucker8: compression relerr {relerr:.2e}, e {E:.4e} (paper 1.569e-3, DM {Edm:.4e}), "
          f"relerr h {h_err:.2e} (paper 2.9e-3)")
    assert Edm == pytest.approx(1.569e-3, abs=0.0005e-3)
    assert E == pytest.approx(1.569e-3, abs=0.0005e-3)
    assert 2.9e-3 / 2 < h_err < 2.9e-3 * 2
