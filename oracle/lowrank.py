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
