"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here re-types the oracle's own formulas: each check compares it with
an independent route (closed forms, identities, quadrature of the defining
integral, the point-dipole expansion, the paper's printed energies).
"""
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_1204_4302_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_dm_energies.txt")
CELLS = [(1.0, 1.0, 1.0), (2e-9, 2e-9, 3e-9), (1.95e-9, 1.95e-9, 0.75e-9), (1.0, 0.3, 2.2)]
XX, YY, ZZ, XY, XZ, YZ = range(6)
COMP_AXES = {XX: (0, 0), YY: (1, 1), ZZ: (2, 2), XY: (0, 1), XZ: (0, 2), YZ: (1, 2)}


from closed_forms import aharoni_dz, body_factors  # noqa: E402


# ---- independent far field: point dipole plus cell-size moments ----------
def dipole_series(R, cell, order):
    """V * sum_beta c_beta d^beta D(R), D_ab = (delta_ab r^2 - 3 r_a r_b)/(4 pi r^5),
    with c_beta the even moments of the triangle (box autocorrelation) weight:
    <s^2> = d^2/6, <s^4> = d^4/15.  Derivatives by mpmath numerical
    differentiation at 50 digits.  order = 0 (dipole), 2 or 4."""
    with mp.workdps(50):
        R = [mp.mpf(v) for v in R]
        d = [mp.mpf(v) for v in cell]
        V = d[0] * d[1] * d[2]
        mom = {0: mp.mpf(1), 2: None, 4: None}
        betas = [((0, 0, 0), mp.mpf(1))]
        if order >= 2:
            for k in range(3):
                b = [0, 0, 0]; b[k] = 2
                betas.append((tuple(b), d[k] ** 2 / 6 / 2))
        if order >= 4:
            for k in range(3):
                b = [0, 0, 0]; b[k] = 4
                betas.append((tuple(b), d[k] ** 4 / 15 / 24))
            for k in range(3):
                for l in range(k + 1, 3):
                    b = [0, 0, 0]; b[k] = 2; b[l] = 2
                    betas.append((tuple(b), (d[k] ** 2 / 6) * (d[l] ** 2 / 6) / 4))
        out = np.zeros(6)
        for comp, (ia, ib) in COMP_AXES.items():
            def Dab(x, y, z, ia=ia, ib=ib):
                r = [x, y, z]
                r2 = x * x + y * y + z * z
                return ((r2 if ia == ib else 0) - 3 * r[ia] * r[ib]) / (4 * mp.pi * r2 ** mp.mpf(2.5))
            s = mp.mpf(0)
            for beta, coef in betas:
                s += coef * (Dab(*R) if beta == (0, 0, 0) else mp.diff(Dab, tuple(R), beta))
            out[comp] = float(V * s)
        return out


# ---- independent mid range: Gauss-Legendre of the defining integral ------
def cell_average_quadrature(offset, cell, q=20):
    """N(R) = V * int D(R+u) prod_k W_k(u_k) du over u in [-d,d]^3, with
    W_k(s) = (d_k - |s|)/d_k^2 (autocorrelation of two cells, normalised).
    Product Gauss-Legendre, q nodes on each half [-d_k,0], [0,d_k].  Valid
    only when the cells do not touch (integrand smooth on the domain)."""
    xg, wg = np.polynomial.legendre.leggauss(q)
    axes = []
    for k in range(3):
        d = cell[k]
        s = np.concatenate([(xg - 1) * d / 2, (xg + 1) * d / 2])
        w = np.concatenate([wg, wg]) * d / 2 * (d - np.abs(s)) / d ** 2
        axes.append((s, w))
    R = [offset[k] * cell[k] for k in range(3)]
    X = R[0] + axes[0][0][:, None, None]
    Y = R[1] + axes[1][0][None, :, None]
    Z = R[2] + axes[2][0][None, None, :]
    W = axes[0][1][:, None, None] * axes[1][1][None, :, None] * axes[2][1][None, None, :]
    r2 = X * X + Y * Y + Z * Z
    r5 = r2 ** 2.5
    pos = (X, Y, Z)
    V = cell[0] * cell[1] * cell[2]
    out = np.zeros(6)
    for comp, (ia, ib) in COMP_AXES.items():
        D = ((r2 if ia == ib else 0.0) - 3 * pos[ia] * pos[ib]) / (4 * np.pi * r5)
        out[comp] = V * np.sum(W * D)
    return out


def octant(shape, cell):
    return oracle.Oracle(shape, cell)


# ======================================================================
@pytest.mark.parametrize("cell", CELLS)
def test_self_term_trace_is_one(cell):
    o = octant((1, 1, 1), cell)
    N0 = o.Noct[:, 0, 0, 0]
    assert abs(N0[XX] + N0[YY] + N0[ZZ] - 1.0) < 1e-15
    assert np.all(np.abs(N0[3:]) < 1e-15)


def test_cubic_cell_is_one_third():
    o = octant((2, 2, 2), (2e-9, 2e-9, 2e-9))
    assert np.allclose(o.Noct[:3, 0, 0, 0], 1.0 / 3.0, rtol=0, atol=1e-16)


@pytest.mark.parametrize("cell", CELLS)
def test_self_term_equals_aharoni(cell):
    """The self term of one cell is the demag factor of that cuboid."""
    o = octant((1, 1, 1), cell)
    D = body_factors(*cell)
    assert np.allclose(o.Noct[:3, 0, 0, 0], D, rtol=2e-15, atol=0)
    assert abs(sum(D) - 1.0) < 1e-14


def test_aharoni_cube_closed_form():
    assert abs(aharoni_dz(0.5, 0.5, 0.5) - 1.0 / 3.0) < 1e-15


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("off", [(1, 0, 0), (0, 1, 1), (2, -1, 0), (-3, 2, 1), (5, 4, -3), (12, 0, 7)])
def test_trace_vanishes_off_origin(cell, off):
    """tr N(o) = 0 for o != 0 (tr of -grad grad 1/(4 pi r) is a delta at 0)."""
    diag = [oracle.tensor_at(c, off, cell) for c in (XX, YY, ZZ)]
    scale = max(abs(v) for v in diag)
    assert abs(sum(diag)) <= 1e-13 * scale + 1e-18


@pytest.mark.parametrize("cell", CELLS[:3])
def test_parity_and_octant_consistency(cell):
    """N at negative offsets equals the octant value times the parity sign:
    diagonal even in every axis; xy odd in x,y; xz odd in x,z; yz odd in y,z."""
    o = octant((4, 3, 3), cell)
    parity = {XX: (0, 0, 0), YY: (0, 0, 0), ZZ: (0, 0, 0), XY: (1, 1, 0), XZ: (1, 0, 1), YZ: (0, 1, 1)}
    for ox, oy, oz in [(1, 2, 1), (3, 1, 2), (2, 2, 0), (1, 0, 2)]:
        for sx in (1, -1):
            for sy in (1, -1):
                for sz in (1, -1):
                    for comp in range(6):
                        px, py, pz = parity[comp]
                        sign = (sx if px else 1) * (sy if py else 1) * (sz if pz else 1)
                        direct = oracle.tensor_at(comp, (sx * ox, sy * oy, sz * oz), cell)
                        ref = sign * o.Noct[comp, oz, oy, ox]
                        assert abs(direct - ref) <= 1e-15 * max(1e-3, abs(ref))


def test_octant_matches_single_offset_evaluation():
    cell = CELLS[2]
    o = octant((5, 4, 3), cell)
    for (ox, oy, oz) in [(0, 0, 0), (4, 3, 2), (2, 0, 1)]:
        for comp in range(6):
            assert oracle.tensor_at(comp, (ox, oy, oz), cell) == o.Noct[comp, oz, oy, ox]


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("off", [(2, 0, 0), (2, 1, 1), (0, 3, 2), (3, -2, 2), (4, 4, 4)])
def test_mid_range_equals_cell_average_quadrature(cell, off):
    """f/g against Gauss-Legendre of the defining double-cell average."""
    ref = cell_average_quadrature(off, cell, q=24)
    got = np.array([oracle.tensor_at(c, off, cell) for c in range(6)])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("off", [(40, 0, 0), (30, 20, 10), (-25, 31, 17), (7, 0, 60)])
def test_far_field_point_dipole_with_moments(cell, off):
    """At large offsets the cell-averaged tensor tends to the point dipole;
    with the 2nd and 4th moment corrections the residual is O((d/R)^6)."""
    got = np.array([oracle.tensor_at(c, off, cell) for c in range(6)])
    R = [off[k] * cell[k] for k in range(3)]
    scale = np.max(np.abs(got))
    d0 = dipole_series(R, cell, 0)
    d4 = dipole_series(R, cell, 4)
    rho = np.linalg.norm(R) / max(cell)
    assert np.max(np.abs(got - d0)) <= 1.0 / rho ** 2 * scale
    assert np.max(np.abs(got - d4)) <= (3.0 / rho ** 6 + 1e-12) * scale


def test_symmetric_operator_matrix_and_sums():
    """A = A^T on the explicit matrix; field() and field_T() are A m, A^T g."""
    shape, cell, Ms = (4, 3, 2), (1.95e-9, 1.95e-9, 0.75e-9), 8e5
    o = octant(shape, cell)
    A = o.matrix(Ms)
    assert np.max(np.abs(A - A.T)) <= 1e-15 * np.max(np.abs(A))
    m = inputs.random_unit(shape, 11)
    g = np.random.default_rng(12).standard_normal(m.shape)
    H = o.field(m, Ms)
    assert np.allclose(H.ravel(), A @ m.ravel(), rtol=0, atol=1e-12 * np.abs(H).max())
    gT = o.field_T(g, Ms)
    assert np.allclose(gT.ravel(), A.T @ g.ravel(), rtol=0, atol=1e-12 * np.abs(gT).max())
    # positive semi-definite energy form: -m.A m >= 0 for every m
    w = np.linalg.eigvalsh(-(A + A.T) / 2)
    assert w.min() >= -1e-12 * w.max()


def test_field_targets_agree_with_full_field():
    shape, cell = (6, 5, 4), (2e-9, 2e-9, 3e-9)
    o = octant(shape, cell)
    m = inputs.random_unit(shape, 3)
    H = o.field(m, 1.4e6)
    t = inputs.sample_targets(shape, 20, 5)
    Ht = o.field_targets(m, 1.4e6, t)
    assert np.array_equal(Ht, H.reshape(3, -1)[:, t])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_energy_positive(seed):
    shape, cell, Ms = (7, 5, 3), (2e-9, 2e-9, 3e-9), 1.4e6
    o = octant(shape, cell)
    m = inputs.random_unit(shape, seed)
    assert o.energy(m, o.field(m, Ms), Ms) > 0


@pytest.mark.parametrize("shape,cell", [((5, 3, 2), (2e-9, 2e-9, 3e-9)),
                                        ((8, 8, 8), (2e-9, 2e-9, 2e-9)),
                                        ((9, 4, 3), (1.95e-9, 1.95e-9, 0.75e-9))])
def test_uniform_body_average_equals_cuboid_factors(shape, cell):
    """For uniform m the cell-averaged field averaged over the whole body is
    -Ms N_body m, N_body = diag of the body's cuboid demag factors."""
    Ms = 8e5
    o = octant(shape, cell)
    direction = np.array([1.0, 1.0, 1.0]) / np.sqrt(3)
    m = inputs.uniform(shape, direction)
    H = o.field(m, Ms)
    mean = H.reshape(3, -1).mean(axis=1)
    D = np.array(body_factors(*(shape[k] * cell[k] for k in range(3))))
    assert np.allclose(mean, -Ms * D * direction, rtol=1e-13, atol=0)


def test_cube_uniform_is_one_sixth_any_grid():
    """Sec. 5.1: homogeneous unit cube, e = 1/6 mu0 Ms^2 exactly; DM reaches it
    up to rounding for every grid (tensor built for homogeneous cells)."""
    for n in (3, 6, 10):
        o = octant((n, n, n), (1.0 / n,) * 3)
        for direction in [(0, 0, 1), (1, 2, 3)]:
            m = inputs.uniform((n, n, n), direction)
            e = o.energy(m, o.field(m, 1.0), 1.0) / oracle.MU0
            assert abs(e * 6 - 1) < 1e-13


def _golden():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                p = line.split()
                rows.append((p[0], tuple(int(v) for v in p[1:4]), tuple(float(v) for v in p[4:7]),
                             p[7], float(p[8]), p[9]))
    return rows


@pytest.mark.slow
@pytest.mark.parametrize("row", _golden(), ids=lambda r: r[0])
def test_paper_dm_energies(row):
    """The five DM energies printed in the paper's tables, to the printed digits."""
    name, shape, body, state, value, digits = row
    cell = tuple(body[k] / shape[k] for k in range(3))
    o = octant(shape, cell)
    if state == "uniform_z":
        m = inputs.uniform(shape, (0, 0, 1))
    elif state == "flower":
        m = inputs.paper_flower(shape, cell, a=1.0, b=2.0, c=1.0)
    else:
        m = inputs.paper_vortex(shape, cell, rc=0.14)
    e = o.energy(m, o.field(m, 1.0), 1.0) / oracle.MU0
    if digits == "exact":
        assert abs(e / value - 1) < 1e-12
    else:
        assert float(f"{e:.{int(digits) - 1}e}") == value
    if name == "thin_homo":
        # closed form: E = 1/2 D_z(1,1,0.1) * volume (uniform out of plane)
        assert abs(e - 0.5 * body_factors(1, 1, 0.1)[2] * 0.1) < 1e-13
