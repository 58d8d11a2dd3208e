"""Plain CPU oracle for the DM stray-field method -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does.

The arithmetic lives in ``demag_oracle.c`` (FP64 direct O(N^2) sums over all
cell pairs; Newell f/g lattice in binary128).  This module only loads the
shared object with ctypes and marshals numpy arrays.

Functions and the passages they follow (Abert et al., arXiv:1204.4302):

* ``tensor``      -- cell-averaged demagnetization tensor N for homogeneously
                     magnetized cells (Sec. 5.1, "Homogeneously Magnetized
                     Cube"; closed forms of Newell et al. 1993, which the paper
                     cites only by property).
* ``field``       -- H = -Ms N * m as a plain sum, Sec. 3.1 eq. (demag).
* ``field_targets`` -- the same sum evaluated at selected cells only.
* ``field_T``     -- the transposed operator as its own loop (also at
                     selected cells: ``field_T_targets``).
* ``energy``      -- E = -(mu0/2) Ms V sum m.H, Sec. 2 (stray-field energy).
* ``matrix``      -- the explicit 3N x 3N operator for tiny grids.

The scalar-potential method (SP, Sec. 3.1 eqs. (scpot), (convolution),
(field)) is in ``sp_oracle.c``, class ``SPOracle``: the kernel S of
homogeneously magnetized cells (two charged faces per cell), the potential as
a plain sum, and the field as its finite-difference gradient.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "demag_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "sp_oracle.c")]
_LIB = os.path.join(_HERE, "_demag_oracle.so")
_lib = None

MU0 = 4.0e-7 * np.pi


def build(force: bool = False, extra_flags: list[str] | None = None,
          out: str | None = None) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, libquadmath)."""
    out = out or _LIB
    if not force and os.path.exists(out) and all(os.path.getmtime(out) >= os.path.getmtime(f) for f in _SRCS):
        return out
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=gnu11",
           *_SRCS, "-o", out + ".tmp", "-lquadmath", "-lm"]
    if extra_flags:
        cmd[1:1] = list(extra_flags)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def load(path: str | None = None):
    """Load (building first if needed) and declare the C signatures."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    lib = ctypes.CDLL(path or build())
    d, i, l, p = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
    lib.oracle_tensor.argtypes = [i, i, i, d, d, d, p]
    lib.oracle_tensor.restype = i
    lib.oracle_tensor_at.argtypes = [i, l, l, l, d, d, d]
    lib.oracle_tensor_at.restype = d
    lib.oracle_f.argtypes = [d, d, d]
    lib.oracle_f.restype = d
    lib.oracle_g.argtypes = [d, d, d]
    lib.oracle_g.restype = d
    lib.oracle_field.argtypes = [i, i, i, p, p, d, p]
    lib.oracle_field.restype = i
    lib.oracle_field_targets.argtypes = [i, i, i, p, p, d, p, l, p]
    lib.oracle_field_targets.restype = i
    lib.oracle_field_T.argtypes = [i, i, i, p, p, d, p]
    lib.oracle_field_T.restype = i
    lib.oracle_field_T_targets.argtypes = [i, i, i, p, p, d, p, l, p]
    lib.oracle_field_T_targets.restype = i
    lib.oracle_energy.argtypes = [i, i, i, d, d, d, p, p, d]
    lib.oracle_energy.restype = d
    lib.oracle_matrix.argtypes = [i, i, i, p, d, p]
    lib.oracle_matrix.restype = i
    lib.oracle_mu0.argtypes = []
    lib.oracle_mu0.restype = d
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = i
    lib.sp_face_potential.argtypes = [d, d, d, d, d]
    lib.sp_face_potential.restype = d
    lib.oracle_sp_kernel_at.argtypes = [i, l, l, l, d, d, d]
    lib.oracle_sp_kernel_at.restype = d
    lib.oracle_sp_kernel.argtypes = [i, i, i, d, d, d, p]
    lib.oracle_sp_kernel.restype = i
    lib.oracle_sp_potential.argtypes = [i, i, i, p, p, d, p]
    lib.oracle_sp_potential.restype = i
    lib.oracle_sp_gradient.argtypes = [i, i, i, d, d, d, p, p]
    lib.oracle_sp_gradient.restype = i
    lib.oracle_sp_field.argtypes = [i, i, i, d, d, d, p, p, d, p]
    lib.oracle_sp_field.restype = i
    lib.oracle_sp_field_targets.argtypes = [i, i, i, d, d, d, p, p, d, p, l, p]
    lib.oracle_sp_field_targets.restype = i
    if path is None:
        _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _vec(m: np.ndarray, shape) -> np.ndarray:
    nx, ny, nz = shape
    m = np.ascontiguousarray(m, dtype=np.float64)
    if m.shape != (3, nz, ny, nx):
        raise ValueError(f"expected a [3][nz][ny][nx] field, got {m.shape}")
    return m


class Oracle:
    """One grid (shape (nx, ny, nz), cell (dx, dy, dz)) with its FP64 tensor."""

    def __init__(self, shape, cell, lib=None, cache_dir: str | None = None):
        """cache_dir: optional folder where the tensor this oracle computed is
        kept (.npy, keyed by shape and cell) and reused by later instances."""
        self.lib = lib or load()
        self.shape = tuple(int(v) for v in shape)
        self.cell = tuple(float(v) for v in cell)
        nx, ny, nz = self.shape
        path = None
        if cache_dir:
            key = "noct_%dx%dx%d_%s_%s_%s.npy" % (nx, ny, nz, *(v.hex() for v in self.cell))
            path = os.path.join(cache_dir, key)
            if os.path.exists(path):
                self.Noct = np.load(path)
                self.tensor_seconds = 0.0
                return
        import time
        t0 = time.perf_counter()
        self.Noct = np.empty((6, nz, ny, nx), dtype=np.float64)
        rc = self.lib.oracle_tensor(nx, ny, nz, *self.cell, _ptr(self.Noct))
        if rc != 0:
            raise ValueError(f"oracle_tensor failed ({rc})")
        self.tensor_seconds = time.perf_counter() - t0
        if path:
            os.makedirs(cache_dir, exist_ok=True)
            np.save(path + ".tmp.npy", self.Noct)
            os.replace(path + ".tmp.npy", path)

    @property
    def volume(self) -> float:
        dx, dy, dz = self.cell
        return dx * dy * dz

    def field(self, m, Ms):
        m = _vec(m, self.shape)
        H = np.empty_like(m)
        self.lib.oracle_field(*self.shape, _ptr(self.Noct), _ptr(m), float(Ms), _ptr(H))
        return H

    def field_targets(self, m, Ms, targets):
        m = _vec(m, self.shape)
        t = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.empty((3, t.size), dtype=np.float64)
        rc = self.lib.oracle_field_targets(*self.shape, _ptr(self.Noct), _ptr(m),
                                           float(Ms), _ptr(t), t.size, _ptr(out))
        if rc != 0:
            raise ValueError("target index out of range")
        return out

    def field_T(self, g, Ms):
        g = _vec(g, self.shape)
        out = np.empty_like(g)
        self.lib.oracle_field_T(*self.shape, _ptr(self.Noct), _ptr(g), float(Ms), _ptr(out))
        return out

    def field_T_targets(self, g, Ms, targets):
        g = _vec(g, self.shape)
        t = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.empty((3, t.size), dtype=np.float64)
        rc = self.lib.oracle_field_T_targets(*self.shape, _ptr(self.Noct), _ptr(g),
                                             float(Ms), _ptr(t), t.size, _ptr(out))
        if rc != 0:
            raise ValueError("target index out of range")
        return out

    def energy(self, m, H, Ms) -> float:
        m = _vec(m, self.shape)
        H = _vec(H, self.shape)
        return self.lib.oracle_energy(*self.shape, *self.cell, _ptr(m), _ptr(H), float(Ms))

    def matrix(self, Ms):
        n = 3 * int(np.prod(self.shape))
        A = np.empty((n, n), dtype=np.float64)
        if self.lib.oracle_matrix(*self.shape, _ptr(self.Noct), float(Ms), _ptr(A)) != 0:
            raise ValueError("grid too large for an explicit matrix")
        return A


class SPOracle:
    """The SP method on one grid: kernel octant S (FP64, from binary128 face
    potentials), potential phi = Ms S * m as a plain sum, H = -grad phi by
    finite differences (central inside, second-order one-sided on the faces)."""

    def __init__(self, shape, cell, lib=None, cache_dir: str | None = None):
        """cache_dir: optional folder keeping the kernel octant (.npy, keyed by
        shape and cell) for later instances."""
        self.lib = lib or load()
        self.shape = tuple(int(v) for v in shape)
        self.cell = tuple(float(v) for v in cell)
        nx, ny, nz = self.shape
        path = None
        if cache_dir:
            key = "soct_%dx%dx%d_%s_%s_%s.npy" % (nx, ny, nz, *(v.hex() for v in self.cell))
            path = os.path.join(cache_dir, key)
            if os.path.exists(path):
                self.Soct = np.load(path)
                self.kernel_seconds = 0.0
                return
        import time
        t0 = time.perf_counter()
        self.Soct = np.empty((3, nz, ny, nx), dtype=np.float64)
        if self.lib.oracle_sp_kernel(nx, ny, nz, *self.cell, _ptr(self.Soct)) != 0:
            raise ValueError("oracle_sp_kernel failed")
        self.kernel_seconds = time.perf_counter() - t0
        if path:
            os.makedirs(cache_dir, exist_ok=True)
            np.save(path + ".tmp.npy", self.Soct)
            os.replace(path + ".tmp.npy", path)

    @property
    def volume(self) -> float:
        dx, dy, dz = self.cell
        return dx * dy * dz

    def potential(self, m, Ms):
        m = _vec(m, self.shape)
        nx, ny, nz = self.shape
        phi = np.empty((nz, ny, nx), dtype=np.float64)
        self.lib.oracle_sp_potential(*self.shape, _ptr(self.Soct), _ptr(m), float(Ms), _ptr(phi))
        return phi

    def gradient(self, phi):
        nx, ny, nz = self.shape
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(nz, ny, nx)
        H = np.empty((3, nz, ny, nx), dtype=np.float64)
        self.lib.oracle_sp_gradient(*self.shape, *self.cell, _ptr(phi), _ptr(H))
        return H

    def field(self, m, Ms):
        m = _vec(m, self.shape)
        H = np.empty_like(m)
        if self.lib.oracle_sp_field(*self.shape, *self.cell, _ptr(self.Soct), _ptr(m), float(Ms), _ptr(H)) != 0:
            raise MemoryError("oracle_sp_field")
        return H

    def field_targets(self, m, Ms, targets):
        m = _vec(m, self.shape)
        t = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.empty((3, t.size), dtype=np.float64)
        rc = self.lib.oracle_sp_field_targets(*self.shape, *self.cell, _ptr(self.Soct), _ptr(m), float(Ms),
                                              _ptr(t), t.size, _ptr(out))
        if rc != 0:
            raise ValueError("target index out of range")
        return out

    def energy(self, m, H, Ms) -> float:
        m = _vec(m, self.shape)
        H = _vec(H, self.shape)
        return load().oracle_energy(*self.shape, *self.cell, _ptr(m), _ptr(H), float(Ms))


def sp_kernel_at(a: int, offset, cell) -> float:
    """S_a at one signed integer offset, straight from the two faces (binary128)."""
    ox, oy, oz = (int(v) for v in offset)
    return load().oracle_sp_kernel_at(int(a), ox, oy, oz, *(float(c) for c in cell))


def face_potential(X, Y, W, A, B) -> float:
    """Newton potential at (X, Y, W) of the unit-density rectangle A x B
    centred at the origin in the plane W = 0."""
    return load().sp_face_potential(float(X), float(Y), float(W), float(A), float(B))


def threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(load().oracle_threads())


def tensor_at(comp: int, offset, cell) -> float:
    """N_comp at one signed integer offset, straight from f/g (binary128)."""
    ox, oy, oz = (int(v) for v in offset)
    return load().oracle_tensor_at(int(comp), ox, oy, oz, *(float(c) for c in cell))
