"""Pins of the ALS compression reference (Sec. 3.2: CP and Tucker
approximations by alternating least squares from random initial guesses)
against what the mathematics fixes: the unfolding / Khatri-Rao identity
behind the CP normal equations, exact recovery of exactly low-rank tensors,
agreement of the Tucker subspaces with the SVD of the unfoldings (HOSVD),
the monotone decrease of the ALS residual, and exactness at full rank."""
import numpy as np
import pytest

from oracle import lowrank as lr


def _rng(seed):
    return np.random.default_rng(seed)


def test_unfolding_khatri_rao_identity():
    """X_(n) (U_c (.) U_b) equals the brute-force MTTKRP sum."""
    rng = _rng(1)
    X = rng.standard_normal((4, 3, 5))
    U = [rng.standard_normal((n, 2)) for n in X.shape]
    for n in range(3):
        o = [m for m in range(3) if m != n]
        got = lr.unfold(X, n) @ lr.khatri_rao(U[o[1]], U[o[0]])
        ref = np.zeros((X.shape[n], 2))
        for idx in np.ndindex(*X.shape):
            for s in range(2):
                ref[idx[n], s] += X[idx] * U[o[0]][idx[o[0]], s] * U[o[1]][idx[o[1]], s]
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)
    # unfolding keeps every fiber: column j of X_(1) is the mode-1 fiber
    assert np.array_equal(lr.unfold(X, 0)[:, 1 + 3 * 2], X[:, 1, 2])


def test_tucker_recovers_exact_low_rank_and_matches_hosvd():
    rng = _rng(2)
    shape, r = (9, 7, 6), 3
    Us = [np.linalg.qr(rng.standard_normal((n, r)))[0] for n in shape]
    X = lr.tucker_full(rng.standard_normal((r, r, r)), *Us)
    U0 = [rng.standard_normal((n, r)) for n in shape]
    C, U = lr.tucker_hooi(X, U0, 3)
    assert lr.relerr(X, lr.tucker_full(C, *U)) < 1e-13
    for n in range(3):
        Uh = np.linalg.svd(lr.unfold(X, n), full_matrices=False)[0][:, :r]  # HOSVD subspace
        assert np.allclose(U[n] @ U[n].T, Uh @ Uh.T, atol=1e-12)
        assert np.allclose(U[n].T @ U[n], np.eye(r), atol=1e-13)


def test_tucker_full_rank_is_exact():
    rng = _rng(3)
    X = rng.standard_normal((4, 3, 3))
    U0 = [rng.standard_normal((n, 3)) for n in (4, 3, 3)]
    C, U = lr.tucker_hooi(X, [U0[0][:, :3], U0[1], U0[2]], 1)
    # rank 3 in every mode covers modes 2 and 3 completely; mode 1 (4 rows) not:
    err = lr.relerr(X, lr.tucker_full(C, *U))
    assert err < 1.0
    C4, U4 = lr.tucker_hooi(np.ascontiguousarray(X[:3]), [rng.standard_normal((3, 3)) for _ in range(3)], 1)
    assert lr.relerr(X[:3], lr.tucker_full(C4, *U4)) < 1e-13


def test_cp_recovers_exact_low_rank():
    rng = _rng(4)
    shape, r = (8, 7, 6), 2
    A = [rng.standard_normal((n, r)) for n in shape]
    lam0 = np.array([3.0, 1.5])
    X = lr.cp_full(lam0, *A)
    lam, U = lr.cp_als(X, [rng.standard_normal((n, r)) for n in shape], 200)
    assert lr.relerr(X, lr.cp_full(lam, *U)) < 1e-8
    for u in U:
        assert np.allclose(np.linalg.norm(u, axis=0), 1.0, atol=1e-13)


def test_cp_rank_one_weight_is_norm_product():
    rng = _rng(5)
    a, b, c = (rng.standard_normal(n) for n in (5, 4, 3))
    X = np.multiply.outer(np.multiply.outer(a, b), c)
    lam, U = lr.cp_als(X, [rng.standard_normal((n, 1)) for n in (5, 4, 3)], 3)
    assert lam[0] == pytest.approx(np.linalg.norm(a) * np.linalg.norm(b) * np.linalg.norm(c), rel=1e-12)
    assert lr.relerr(X, lr.cp_full(lam, *U)) < 1e-13


@pytest.mark.parametrize("fmt", [0, 1])
def test_residual_does_not_increase(fmt):
    """Each ALS mode update is an exact least-squares step (CP) or an
    orthogonal-iteration step on Y_(n) Y_(n)^T (Tucker): the residual never
    grows from sweep to sweep."""
    rng = _rng(6)
    X = rng.standard_normal((8, 7, 6)) + lr.cp_full(np.array([5.0, 4.0, 3.0]),
                                                   *[rng.standard_normal((n, 3)) for n in (8, 7, 6)])
    U0 = [rng.standard_normal((n, 3)) for n in X.shape]
    errs = []
    for k in range(1, 12):
        if fmt == 0:
            C, U = lr.tucker_hooi(X, U0, k)
            errs.append(lr.relerr(X, lr.tucker_full(C, *U)))
        else:
            lam, U = lr.cp_als(X, U0, k)
            errs.append(lr.relerr(X, lr.cp_full(lam, *U)))
    assert all(b <= a + 1e-12 for a, b in zip(errs, errs[1:])), errs


def test_compress_layouts_round_trip():
    """compress() in the device layouts reproduces an exactly low-rank
    magnetization built with the same layouts."""
    from paper_1204_4302_amd import inputs
    shape = (7, 6, 5)
    for fmt, r, sweeps in ((0, 2, 3), (1, 2, 300)):
        core, factors = inputs.lowrank(shape, fmt, r, seed=7)
        m = lr.magnetization(fmt, core, factors)
        _, init = inputs.lowrank(shape, fmt, r, seed=8)
        c2, f2 = lr.compress(fmt, m, init, sweeps)
        assert lr.relerr(m, lr.magnetization(fmt, c2, f2)) < 1e-7


def test_orth_completes_dependent_columns():
    """Dependent columns are replaced by the unit vector with the largest
    remainder; full-rank input gives the QR factor with diag(R) > 0."""
    rng = _rng(9)
    P = rng.standard_normal((7, 3))
    Q = lr.orth(P)
    Qr, R = np.linalg.qr(P)
    assert np.allclose(Q, Qr * np.sign(np.diag(R)), atol=1e-14)
    D = np.stack([P[:, 0], 2 * P[:, 0], P[:, 1]], axis=1)  # column 1 depends on column 0
    Q = lr.orth(D)
    assert np.allclose(Q.T @ Q, np.eye(3), atol=1e-14)
    assert np.allclose(Q[:, 0], P[:, 0] / np.linalg.norm(P[:, 0]), atol=1e-15)
    res = 1 - Q[:, 0] ** 2
    e = np.zeros(7)
    e[np.argmax(res)] = 1.0
    e -= (Q[:, 0] @ e) * Q[:, 0]
    assert np.allclose(Q[:, 1], e / np.linalg.norm(e), atol=1e-14)
    Z = lr.orth(np.zeros((5, 2)))
    assert np.allclose(Z.T @ Z, np.eye(2)) and Z[0, 0] == 1.0


def test_tucker_on_axis_invariant_state():
    """A state constant along z has mode-3 rank 1: rank 2 still compresses it
    exactly, the second mode-3 direction being a weightless completion."""
    rng = _rng(10)
    A = rng.standard_normal((6, 5))
    X = np.repeat(A[:, :, None], 4, axis=2)
    C, U = lr.tucker_hooi(X, [rng.standard_normal((n, 2)) for n in (6, 5, 4)], 200)
    assert np.allclose(U[2].T @ U[2], np.eye(2), atol=1e-14)
    assert np.abs(C[:, :, 1]).max() < 1e-12 * np.abs(C).max()
    rec = lr.tucker_full(C, *U)
    sv = np.linalg.svd(A, compute_uv=False)
    best = np.sqrt((sv[2:] ** 2).sum() / (sv ** 2).sum())  # rank-2 truncation of A is optimal here
    assert lr.relerr(X, rec) <= best + 1e-9
