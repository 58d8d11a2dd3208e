"""Plain reference of the low-rank magnetization formats -- TEST
INFRASTRUCTURE ONLY (nothing in the product imports it).

Appendix, eqs. (CP) and (tucker): a tensor in CP format is a weighted sum of
r outer products of vectors; in Tucker format it is a core tensor multiplied
along every mode by a factor matrix, the n-mode product multiplying each
mode-n fiber by the matrix.  The low-rank tensor-grid method (Sec. 3.2,
"Low-Rank Magnetization") computes the same potential, field and energy as
the dense method applied to the expanded magnetization, so the reference for
it is: expand the compressed components to the dense grid with the plain
definitions below, then take the SP oracle (direct sum of the cell potential
and the difference stencils), which is the exact quantity the Sinc
quadrature approximates.  relerr is eq. (relr).  numpy, FP64.

Layouts (those of the device calls): core [3][r][r][r] indexed [p][s3][s2][s1]
(Tucker) or lambda [3][r] (CP); factors a list of three arrays (3, r, n_q),
factor s of component p along axis q at [p][s]; tensor index (i1, i2, i3) =
cell (x, y, z); a dense field is [3][nz][ny][nx].
"""
from __future__ import annotations

import numpy as np


def mode_product(A: np.ndarray, U: np.ndarray, n: int) -> np.ndarray:
    """A x_n U: every mode-n fiber of A multiplied by U (M x N_n)."""
    An = np.moveaxis(A, n, 0)
    out = (U @ An.reshape(An.shape[0], -1)).reshape((U.shape[0],) + An.shape[1:])
    return np.moveaxis(out, 0, n)


def tucker_full(C: np.ndarray, U1: np.ndarray, U2: np.ndarray, U3: np.ndarray) -> np.ndarray:
    """C x_1 U1 x_2 U2 x_3 U3 (eq. (tucker)); C r1 x r2 x r3, U_j N_j x r_j."""
    return mode_product(mode_product(mode_product(C, U1, 0), U2, 1), U3, 2)


def cp_full(lam: np.ndarray, U1: np.ndarray, U2: np.ndarray, U3: np.ndarray) -> np.ndarray:
    """sum_l lam_l u1_l o u2_l o u3_l (eq. (CP)); U_j N_j x r."""
    A = np.zeros((U1.shape[0], U2.shape[0], U3.shape[0]))
    for l in range(lam.shape[0]):
        A += lam[l] * np.multiply.outer(np.multiply.outer(U1[:, l], U2[:, l]), U3[:, l])
    return A


def component(fmt: int, core: np.ndarray, factors, p: int) -> np.ndarray:
    """Component p as a dense N1 x N2 x N3 tensor (index (x, y, z))."""
    U = [np.asarray(f[p], dtype=np.float64).T for f in factors]  # N_q x r
    if fmt == 0:
        C = np.asarray(core[p], dtype=np.float64).transpose(2, 1, 0)  # [s1][s2][s3]
        return tucker_full(C, *U)
    return cp_full(np.asarray(core[p], dtype=np.float64), *U)


def magnetization(fmt: int, core: np.ndarray, factors) -> np.ndarray:
    """The expanded magnetization [3][nz][ny][nx] (not renormalised)."""
    return np.stack([component(fmt, core, factors, p).transpose(2, 1, 0) for p in range(3)])


def relerr(dense: np.ndarray, lowrank: np.ndarray) -> float:
    """Eq. (relr): Frobenius error over the three components, relative."""
    return float(np.sqrt(((dense - lowrank) ** 2).sum()) / np.sqrt((dense ** 2).sum()))


# ---- ALS compression (Sec. 3.2: CP and Tucker approximations by alternating
# least squares from random initial guesses) ---------------------------------
def unfold(A: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding: rows the mode-n index, columns the other indices with
    the lower remaining mode varying fastest."""
    return np.reshape(np.moveaxis(A, n, 0), (A.shape[n], -1), order="F")


def khatri_rao(B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Column-wise Kronecker product: (B (.) C)[j + J k, s] = C[j, s] B[k, s]
    for C with J rows (the first factor's index varies slowest)."""
    r = B.shape[1]
    return np.stack([np.kron(B[:, s], C[:, s]) for s in range(r)], axis=1)


ORTH_TOL = 1e-13  # dependence threshold relative to the largest column norm of P


def orth(P: np.ndarray, tol: float = ORTH_TOL) -> np.ndarray:
    """Orthonormal basis of range(P) by Gram-Schmidt, each column
    orthogonalised twice against the accepted ones (for full-rank P this is
    the Q of QR with diag(R) > 0).  A column whose remainder is not above
    tol * max column norm is dependent and replaced by the unit vector e_i
    with the largest remainder 1 - sum_k Q[i, k]^2 (first i on ties),
    orthogonalised the same way."""
    n, r = P.shape
    pmax = max(float(np.linalg.norm(P[:, j])) for j in range(r)) if r else 0.0
    Q = np.zeros((n, r))
    for j in range(r):
        v = np.array(P[:, j], dtype=np.float64)
        scale = pmax
        for _attempt in range(2):
            for _pass in range(2):
                for k in range(j):
                    v = v - (Q[:, k] @ v) * Q[:, k]
            nv = float(np.linalg.norm(v))
            if nv > tol * scale and nv > 0:
                Q[:, j] = v / nv
                break
            res = 1.0 - (Q[:, :j] ** 2).sum(axis=1)
            v = np.zeros(n)
            v[int(np.argmax(res))] = 1.0
            scale = 1.0
    return Q


def cp_als(X: np.ndarray, U_init, sweeps: int):
    """CP-ALS: per mode, U_n = X_(n) (Khatri-Rao of the other factors, higher
    mode first) V^-1 with V the Hadamard product of their Gram matrices, then
    unit 2-norm columns; returns (lambda, [U1, U2, U3])."""
    U = [np.array(u, dtype=np.float64) for u in U_init]
    lam = np.ones(U[0].shape[1])
    if not (X ** 2).sum() > 0:  # a zero component: weights 0, factors as given
        return np.zeros(U[0].shape[1]), U
    for _ in range(sweeps):
        for n in range(3):
            others = [m for m in range(3) if m != n]
            V = np.ones((U[0].shape[1],) * 2)
            for m in others:
                V = V * (U[m].T @ U[m])
            KR = khatri_rao(U[others[1]], U[others[0]])
            M = unfold(X, n) @ KR
            Un = np.linalg.solve(V, M.T).T  # M V^-1 (V symmetric)
            lam = np.linalg.norm(Un, axis=0)
            U[n] = Un / np.where(lam > 0, lam, 1.0)
    return lam, U


def tucker_hooi(X: np.ndarray, U_init, sweeps: int):
    """Higher-order orthogonal iteration with the leading subspace of each
    Y_(n) = (X x_{m != n} U_m^T)_(n) taken by one step of orthogonal iteration
    from the current factor, U_n <- orth(Y_(n) Y_(n)^T U_n); the initial
    factors are orthonormalised first.  Returns (core, [U1, U2, U3])."""
    U = [orth(np.array(u, dtype=np.float64)) for u in U_init]
    for _ in range(sweeps):
        for n in range(3):
            Y = X
            for m in range(3):
                if m != n:
                    Y = mode_product(Y, U[m].T, m)
            Yn = unfold(Y, n)
            U[n] = orth(Yn @ (Yn.T @ U[n]))
    C = tucker_full(X, U[0].T, U[1].T, U[2].T)
    return C, U


def compress(fmt: int, m: np.ndarray, factors_init, sweeps: int):
    """Both formats for the three components of m ([3][nz][ny][nx]) in the
    device layouts: returns (core, factors) like the device call."""
    r = factors_init[0].shape[1]
    cores, facs = [], [np.zeros_like(np.asarray(f, dtype=np.float64)) for f in factors_init]
    for p in range(3):
        X = np.asarray(m[p], dtype=np.float64).transpose(2, 1, 0)  # (x, y, z)
        U0 = [np.asarray(factors_init[q][p], dtype=np.float64).T for q in range(3)]
        if fmt == 0:
            C, U = tucker_hooi(X, U0, sweeps)
            cores.append(C.transpose(2, 1, 0))  # [s3][s2][s1]
        else:
            lam, U = cp_als(X, U0, sweeps)
            cores.append(lam)
        for q in range(3):
            facs[q][p] = U[q].T
    del r
    return np.stack(cores), facs
