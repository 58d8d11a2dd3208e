"""Pins of the low-rank format reference (Appendix, eqs. (CP), (tucker),
(relr)) against what the definitions fix independently of its code:
brute-force index sums on tiny tensors, the composition rule of n-mode
products (which fails for a transposed operand), CP as Tucker with a
superdiagonal core, norm preservation under orthonormal factors, the cell
layout of the expanded magnetization, and eq. (relr) on known cases."""
import itertools

import numpy as np
import pytest

from oracle import lowrank as lr
from paper_1204_4302_amd import inputs


def brute_tucker(C, U1, U2, U3):
    n1, n2, n3 = U1.shape[0], U2.shape[0], U3.shape[0]
    r1, r2, r3 = C.shape
    A = np.zeros((n1, n2, n3))
    for i, j, k in itertools.product(range(n1), range(n2), range(n3)):
        s = 0.0
        for a, b, c in itertools.product(range(r1), range(r2), range(r3)):
            s += C[a, b, c] * U1[i, a] * U2[j, b] * U3[k, c]
        A[i, j, k] = s
    return A


def test_tucker_brute_force():
    rng = np.random.default_rng(1)
    C = rng.standard_normal((2, 3, 2))
    U1, U2, U3 = rng.standard_normal((4, 2)), rng.standard_normal((3, 3)), rng.standard_normal((5, 2))
    assert np.allclose(lr.tucker_full(C, U1, U2, U3), brute_tucker(C, U1, U2, U3), rtol=1e-13, atol=1e-13)


def test_cp_brute_force_and_superdiagonal_core():
    rng = np.random.default_rng(2)
    r = 3
    lam = rng.standard_normal(r)
    U1, U2, U3 = rng.standard_normal((4, r)), rng.standard_normal((2, r)), rng.standard_normal((3, r))
    ref = np.zeros((4, 2, 3))
    for i, j, k in itertools.product(range(4), range(2), range(3)):
        ref[i, j, k] = sum(lam[l] * U1[i, l] * U2[j, l] * U3[k, l] for l in range(r))
    assert np.allclose(lr.cp_full(lam, U1, U2, U3), ref, rtol=1e-13, atol=1e-13)
    C = np.zeros((r, r, r))
    for l in range(r):
        C[l, l, l] = lam[l]
    assert np.allclose(lr.tucker_full(C, U1, U2, U3), ref, rtol=1e-13, atol=1e-13)


def test_mode_product_rules():
    """A x_n I = A; (A x_n U) x_n V = A x_n (V U); products in distinct modes commute."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 3, 5))
    for n in range(3):
        assert np.array_equal(lr.mode_product(A, np.eye(A.shape[n]), n), A)
        U = rng.standard_normal((6, A.shape[n]))
        V = rng.standard_normal((2, 6))
        assert np.allclose(lr.mode_product(lr.mode_product(A, U, n), V, n), lr.mode_product(A, V @ U, n), rtol=1e-12)
    U0, U2 = rng.standard_normal((2, 4)), rng.standard_normal((7, 5))
    assert np.allclose(lr.mode_product(lr.mode_product(A, U0, 0), U2, 2),
                       lr.mode_product(lr.mode_product(A, U2, 2), U0, 0), rtol=1e-12)
    # fiber definition: (A x_1 U)[:, j, k] = U @ A[:, j, k]
    U = rng.standard_normal((3, 4))
    B = lr.mode_product(A, U, 0)
    assert np.allclose(B[:, 1, 2], U @ A[:, 1, 2], rtol=1e-13)


def test_orthonormal_factors_keep_the_norm():
    rng = np.random.default_rng(4)
    C = rng.standard_normal((3, 2, 4))
    Us = [np.linalg.qr(rng.standard_normal((n, r)))[0] for n, r in [(7, 3), (5, 2), (6, 4)]]
    A = lr.tucker_full(C, *Us)
    assert np.linalg.norm(A) == pytest.approx(np.linalg.norm(C), rel=1e-13)


def test_magnetization_layout():
    """Rank one with unit-vector factors puts one value at cell (x, y, z) of
    component p in the [3][nz][ny][nx] array."""
    shape = (5, 4, 3)
    for fmt in (0, 1):
        core, factors = inputs.lowrank(shape, fmt, 1, seed=0)
        core = np.zeros_like(core)
        factors = [np.zeros_like(f) for f in factors]
        p, (x, y, z) = 1, (3, 2, 1)
        core[(p, 0, 0, 0) if fmt == 0 else (p, 0)] = 2.5
        factors[0][p, 0, x] = 1.0
        factors[1][p, 0, y] = 1.0
        factors[2][p, 0, z] = 1.0
        m = lr.magnetization(fmt, core, factors)
        assert m.shape == (3, 3, 4, 5)
        assert m[p, z, y, x] == 2.5 and np.count_nonzero(m) == 1


def test_core_index_order():
    """Tucker core [p][s3][s2][s1]: the entry at [p][0][0][1] couples factor
    column 1 of axis x with column 0 of axes y and z."""
    shape = (4, 3, 2)
    core, factors = inputs.lowrank(shape, 0, 2, seed=5)
    core = np.zeros_like(core)
    core[0, 0, 0, 1] = 1.0
    m = lr.magnetization(0, core, factors)
    U1, U2, U3 = (factors[q][0].T for q in range(3))
    ref = np.multiply.outer(np.multiply.outer(U1[:, 1], U2[:, 0]), U3[:, 0]).transpose(2, 1, 0)
    assert np.allclose(m[0], ref, rtol=1e-14) and not m[1].any() and not m[2].any()


def test_relerr():
    rng = np.random.default_rng(6)
    a = rng.standard_normal((3, 4, 5, 6))
    assert lr.relerr(a, a) == 0.0
    assert lr.relerr(a, 0.9 * a) == pytest.approx(0.1, rel=1e-13)
    assert lr.relerr(a, np.zeros_like(a)) == pytest.approx(1.0, rel=1e-15)
    assert lr.relerr(3 * a, 3 * 1.1 * a) == pytest.approx(0.1, rel=1e-12)


def test_smooth_factors_are_cosine_modes():
    core, factors = inputs.lowrank((8, 6, 4), 0, 3, seed=0, smooth=True)
    f = factors[0][2]
    G = f @ f.T
    assert np.allclose(G - np.diag(np.diag(G)), 0, atol=1e-12)  # DCT-II modes are orthogonal
