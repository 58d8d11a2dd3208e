"""Python face of the DM stray-field library: Plan, Batch, autograd Functions.

Torch supplies device memory and streams only; each method hands raw device
pointers and the current HIP stream to the C ABI (include/demag.h).

Conventions (Abert et al., Sec. 2 and Sec. 3.1): a magnetization direction
field m has shape (3, nz, ny, nx) on the GPU; H = -Ms N * m in A/m;
E = -(mu0/2) Ms V sum m.H in J.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

MU0 = 4.0e-7 * np.pi
_DT = {torch.float32: _lib.DEMAG_F32, torch.float64: _lib.DEMAG_F64}


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """One grid (shape (nx, ny, nz), cell (dx, dy, dz) in metres) and precision.

    Creating a plan computes the tensor spectrum on the current CUDA device
    (FP64 setup, stored in `dtype`)."""

    def __init__(self, shape, cell, dtype=torch.float32, far_cut=None, fg_cut=None):
        if dtype not in _DT:
            raise TypeError("dtype must be torch.float32 or torch.float64")
        self.shape = tuple(int(v) for v in shape)
        self.cell = tuple(float(v) for v in cell)
        self.dtype = dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        nx, ny, nz = self.shape
        _lib.call("demag_plan_create", ctypes.byref(h), nx, ny, nz, *self.cell, _DT[dtype], _stream_ptr())
        self._h = h
        if far_cut is not None:
            self.set_option("far_cut", far_cut)
        if fg_cut is not None:
            self.set_option("fg_cut", fg_cut)

    # -- lifetime -------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.call("demag_plan_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- facts ------------------------------------------------------------
    @property
    def volume(self) -> float:
        dx, dy, dz = self.cell
        return dx * dy * dz

    @property
    def vec_shape(self):
        nx, ny, nz = self.shape
        return (3, nz, ny, nx)

    def info(self) -> dict:
        v = (ctypes.c_int64 * 16)()
        _lib.call("demag_plan_info", self._h, v)
        keys = ["nx", "ny", "nz", "Px", "Py", "Pz", "Kx", "dtype", "scratch_bytes", "tensor_bytes", "setup_us"]
        return {k: int(v[i]) for i, k in enumerate(keys)}

    def set_option(self, key: str, value: float):
        _lib.call("demag_plan_set_option", self._h, key.encode(), float(value))

    PASSES = ("x_r2c", "y_fwd", "z_conv", "y_inv", "x_c2r", "energy")

    def pass_times(self) -> tuple[dict, int]:
        """Average ms per pass over the evaluations recorded by "pass_timing"."""
        ms = (ctypes.c_double * 6)()
        n = ctypes.c_int64()
        _lib.call("demag_plan_pass_times", self._h, ms, ctypes.byref(n))
        return {k: ms[i] for i, k in enumerate(self.PASSES)}, int(n.value)

    def describe(self) -> str:
        """Launch shape of every pass."""
        buf = ctypes.create_string_buffer(1024)
        _lib.call("demag_plan_describe", self._h, buf, 1024)
        return buf.value.decode()

    def autotune(self):
        _lib.call("demag_autotune", self._h, _stream_ptr())

    def spectrum(self) -> np.ndarray:
        """Stored tensor spectrum, [Py/2+1][6][Kx][Pz/2+1], -1/(PxPyPz) folded in."""
        i = self.info()
        a = np.empty((i["Py"] // 2 + 1, 6, i["Kx"], i["Pz"] // 2 + 1),
                     dtype=np.float32 if self.dtype == torch.float32 else np.float64)
        _lib.call("demag_plan_spectrum", self._h, a.ctypes.data_as(ctypes.c_void_p))
        return a

    def tensor(self) -> np.ndarray:
        """FP64 real-space tensor octant N(o), [6][nz][ny][nx]."""
        nx, ny, nz = self.shape
        a = np.empty((6, nz, ny, nx), dtype=np.float64)
        _lib.call("demag_plan_tensor", self._h, a.ctypes.data_as(ctypes.c_void_p))
        return a

    # -- evaluation -------------------------------------------------------
    def _check(self, t: torch.Tensor, name: str):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.dtype != self.dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, plan has {self.dtype}")
        if tuple(t.shape) != self.vec_shape:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {self.vec_shape}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def _ptr(self, t):
        return ctypes.c_void_p(t.data_ptr())

    def field(self, m: torch.Tensor, Ms: float, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check(m, "m")
        H = torch.empty_like(m) if out is None else out
        self._check(H, "out")
        _lib.call("demag_field", self._h, self._ptr(m), float(Ms), self._ptr(H), _stream_ptr())
        return H

    def adjoint(self, gH: torch.Tensor, Ms: float, out: torch.Tensor | None = None,
                accumulate: bool = False) -> torch.Tensor:
        self._check(gH, "gH")
        gm = torch.empty_like(gH) if out is None else out
        self._check(gm, "out")
        _lib.call("demag_field_adjoint", self._h, self._ptr(gH), float(Ms), self._ptr(gm),
                  1 if accumulate else 0, _stream_ptr())
        return gm

    def field_energy(self, m: torch.Tensor, Ms: float, with_field: bool = True,
                     out: torch.Tensor | None = None, E_out: torch.Tensor | None = None):
        """(H or None, E) with E a 0-dim float64 CUDA tensor."""
        self._check(m, "m")
        H = (torch.empty_like(m) if out is None else out) if with_field else None
        if H is not None:
            self._check(H, "out")
        E = torch.empty((), dtype=torch.float64, device=m.device) if E_out is None else E_out
        if E.dtype != torch.float64 or E.device.type != "cuda" or E.numel() != 1:
            raise TypeError("E_out must be a one-element float64 CUDA tensor")
        _lib.call("demag_field_energy", self._h, self._ptr(m), float(Ms),
                  self._ptr(H) if H is not None else None, ctypes.c_void_p(E.data_ptr()), _stream_ptr())
        return H, E

    def energy_gradient(self, H: torch.Tensor, Ms: float, gE: torch.Tensor | None = None,
                        out: torch.Tensor | None = None, accumulate: bool = False) -> torch.Tensor:
        """gE * dE/dm = gE * (-mu0 Ms V H) from the field H of m (gE: a
        one-element float64 CUDA tensor, None = 1)."""
        self._check(H, "H")
        gm = torch.empty_like(H) if out is None else out
        self._check(gm, "out")
        if gE is not None and (gE.dtype != torch.float64 or gE.device.type != "cuda" or gE.numel() != 1):
            raise TypeError("gE must be a one-element float64 CUDA tensor")
        _lib.call("demag_energy_gradient", self._h, self._ptr(H), float(Ms),
                  ctypes.c_void_p(gE.data_ptr()) if gE is not None else None, self._ptr(gm),
                  1 if accumulate else 0, _stream_ptr())
        return gm

    # -- scalar-potential method (SP) ---------------------------------------
    def sp_prepare(self):
        """Build the SP kernel spectrum (synchronous, once)."""
        _lib.call("demag_sp_prepare", self._h, _stream_ptr())

    def sp_field(self, m: torch.Tensor, Ms: float, out: torch.Tensor | None = None) -> torch.Tensor:
        """H = -grad (Ms S * m) by finite differences (SP method)."""
        self._check(m, "m")
        H = torch.empty_like(m) if out is None else out
        self._check(H, "out")
        _lib.call("demag_sp_field", self._h, self._ptr(m), float(Ms), self._ptr(H), _stream_ptr())
        return H

    def sp_field_energy(self, m: torch.Tensor, Ms: float, with_field: bool = True,
                        out: torch.Tensor | None = None, E_out: torch.Tensor | None = None):
        """(H or None, E) of the SP method, E a 0-dim float64 CUDA tensor."""
        self._check(m, "m")
        H = (torch.empty_like(m) if out is None else out) if with_field else None
        if H is not None:
            self._check(H, "out")
        E = torch.empty((), dtype=torch.float64, device=m.device) if E_out is None else E_out
        if E.dtype != torch.float64 or E.device.type != "cuda" or E.numel() != 1:
            raise TypeError("E_out must be a one-element float64 CUDA tensor")
        _lib.call("demag_sp_field_energy", self._h, self._ptr(m), float(Ms),
                  self._ptr(H) if H is not None else None, ctypes.c_void_p(E.data_ptr()), _stream_ptr())
        return H, E

    def sp_kernel(self) -> np.ndarray:
        """FP64 SP kernel octant S_a(o) in metres, [3][nz][ny][nx]."""
        nx, ny, nz = self.shape
        a = np.empty((3, nz, ny, nx), dtype=np.float64)
        _lib.call("demag_sp_kernel", self._h, a.ctypes.data_as(ctypes.c_void_p))
        return a

    # -- LLG driver (Sec. 2) ------------------------------------------------
    GAMMA = 2.2128e5  # m/(A s): free-electron gyromagnetic ratio times mu0

    def llg_heun(self, m: torch.Tensor, Ms: float, alpha: float, dt: float, steps: int,
                 H_ext=(0.0, 0.0, 0.0), gamma: float = GAMMA, work: torch.Tensor | None = None) -> torch.Tensor:
        """Advance the unit magnetization m in place by `steps` Heun steps of
        the LLG equation with H = H_demag(m) + H_ext; returns m."""
        self._check(m, "m")
        if work is None:
            work = torch.empty((9,) + tuple(m.shape[1:]), dtype=m.dtype, device=m.device)
        if work.dtype != m.dtype or work.numel() < 3 * m.numel() or not work.is_contiguous():
            raise ValueError("work must be a contiguous tensor of 3 m.numel() values of m's dtype")
        hx, hy, hz = (float(v) for v in H_ext)
        _lib.call("demag_llg_heun", self._h, self._ptr(m), float(Ms), float(alpha), float(gamma), hx, hy, hz,
                  float(dt), int(steps), ctypes.c_void_p(work.data_ptr()), _stream_ptr())
        return m

    # -- tensor-grid method (TG, dense) --------------------------------------
    def tg_prepare(self):
        """Sinc nodes, Gaussian matrices and mode-product scratch (synchronous, once)."""
        _lib.call("demag_tg_prepare", self._h, _stream_ptr())

    def tg_info(self) -> dict:
        out = (ctypes.c_int64 * 3)()
        _lib.call("demag_tg_info", self._h, out)
        return {"nodes": out[0], "scratch_bytes": out[1], "flops_per_eval": out[2]}

    def tg_path(self) -> dict:
        """Which mode-product path runs (fused FP32 kernel or library GEMMs) and its flops."""
        out = (ctypes.c_int64 * 2)()
        _lib.call("demag_tg_path", self._h, out)
        return {"fused": bool(out[0]), "flops_issued": out[1]}

    def tg_field(self, m: torch.Tensor, Ms: float, out: torch.Tensor | None = None) -> torch.Tensor:
        """H = -grad phi, phi by the block-CP sum of Gaussian mode products."""
        self._check(m, "m")
        H = torch.empty_like(m) if out is None else out
        self._check(H, "out")
        _lib.call("demag_tg_field", self._h, self._ptr(m), float(Ms), self._ptr(H), _stream_ptr())
        return H

    def tg_field_energy(self, m: torch.Tensor, Ms: float, with_field: bool = True,
                        out: torch.Tensor | None = None, E_out: torch.Tensor | None = None):
        """(H or None, E) of the TG method, E a 0-dim float64 CUDA tensor."""
        self._check(m, "m")
        H = (torch.empty_like(m) if out is None else out) if with_field else None
        if H is not None:
            self._check(H, "out")
        E = torch.empty((), dtype=torch.float64, device=m.device) if E_out is None else E_out
        if E.dtype != torch.float64 or E.device.type != "cuda" or E.numel() != 1:
            raise TypeError("E_out must be a one-element float64 CUDA tensor")
        _lib.call("demag_tg_field_energy", self._h, self._ptr(m), float(Ms),
                  self._ptr(H) if H is not None else None, ctypes.c_void_p(E.data_ptr()), _stream_ptr())
        return H, E

    # -- tensor grid on low-rank magnetization --------------------------------
    def tg_lowrank_prepare(self):
        """Sinc nodes and the stacked Gaussian matrices of the three axes
        (synchronous, once)."""
        _lib.call("demag_tg_lowrank_prepare", self._h, _stream_ptr())

    def tg_lowrank_info(self) -> dict:
        out = (ctypes.c_int64 * 3)()
        _lib.call("demag_tg_lowrank_info", self._h, out)
        h_max = np.frombuffer(bytes(ctypes.c_int64(out[2])), dtype=np.float64)[0]
        return {"nodes": out[0], "bytes": out[1], "h_max": float(h_max)}

    def tg_lowrank_field(self, fmt: int, core: torch.Tensor, factors, Ms: float, dense: bool = True,
                         energy: bool = True, FG: torch.Tensor | None = None):
        """Field of a low-rank magnetization (fmt TUCKER: core [3][r][r][r]
        indexed [p][s3][s2][s1]; CP: lambda [3][r]; factors: three tensors
        (3, r, n_q), factor s of component p along axis q at [p][s]).
        Returns (FG, H or None, E or None): FG the compressed potential and
        field, one (3, R, r, 2 n_q) view per axis (rows [:n_q] potential
        factors F, [n_q:] field factors G), H the dense field, E a 0-dim float64
        CUDA tensor."""
        r = int(core.shape[1])
        want = (3, r, r, r) if fmt == TUCKER else (3, r)
        if fmt not in (TUCKER, CP):
            raise ValueError("fmt must be TUCKER or CP")
        if tuple(core.shape) != want:
            raise ValueError(f"core has shape {tuple(core.shape)}, expected {want}")
        if len(factors) != 3:
            raise ValueError("three factor tensors (one per axis) expected")
        for q, f in enumerate(factors):
            if tuple(f.shape) != (3, r, self.shape[q]):
                raise ValueError(f"factor {q} has shape {tuple(f.shape)}, expected {(3, r, self.shape[q])}")
        for t, name in [(core, "core")] + [(f, f"factor {q}") for q, f in enumerate(factors)]:
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != self.dtype:
                raise TypeError(f"{name} must be a CUDA tensor of {self.dtype}")
        core = core.contiguous()
        U = torch.cat([f.contiguous().reshape(-1) for f in factors])
        R = self.tg_lowrank_info()["nodes"]
        nfg = 6 * R * r * sum(self.shape)
        if FG is None:
            FG = torch.empty(nfg, dtype=self.dtype, device=core.device)
        elif FG.dtype != self.dtype or FG.device.type != "cuda" or FG.numel() != nfg or not FG.is_contiguous():
            raise ValueError(f"FG must be a contiguous CUDA tensor of {nfg} {self.dtype} values")
        H = torch.empty(self.vec_shape, dtype=self.dtype, device=core.device) if dense else None
        E = torch.empty((), dtype=torch.float64, device=core.device) if energy else None
        _lib.call("demag_tg_lowrank_field", self._h, int(fmt), r, self._ptr(core), self._ptr(U), float(Ms),
                  self._ptr(FG), self._ptr(H) if H is not None else None,
                  ctypes.c_void_p(E.data_ptr()) if E is not None else None, _stream_ptr())
        return FG, H, E

    def lowrank_compress(self, m: torch.Tensor, fmt: int, rank: int, sweeps: int, factors):
        """ALS compression of the dense m ([3][nz][ny][nx]) into `fmt` with
        `rank`, from the initial factors (three tensors (3, r, n_q), not
        modified).  Returns (core, factors, relerr) in the layouts of
        tg_lowrank_field; relerr is eq. (relr) of the result."""
        self._check(m, "m")
        r = int(rank)
        if fmt not in (TUCKER, CP):
            raise ValueError("fmt must be TUCKER or CP")
        if len(factors) != 3:
            raise ValueError("three factor tensors (one per axis) expected")
        for q, f in enumerate(factors):
            if tuple(f.shape) != (3, r, self.shape[q]):
                raise ValueError(f"factor {q} has shape {tuple(f.shape)}, expected {(3, r, self.shape[q])}")
            if not isinstance(f, torch.Tensor) or f.device.type != "cuda" or f.dtype != self.dtype:
                raise TypeError(f"factor {q} must be a CUDA tensor of {self.dtype}")
        U = torch.cat([f.contiguous().reshape(-1) for f in factors])
        core = torch.empty((3, r, r, r) if fmt == TUCKER else (3, r), dtype=self.dtype, device=m.device)
        err = ctypes.c_double()
        _lib.call("demag_lowrank_compress", self._h, int(fmt), r, int(sweeps), self._ptr(m), self._ptr(core),
                  self._ptr(U), ctypes.byref(err), _stream_ptr())
        out, off = [], 0
        for n in self.shape:
            out.append(U[off:off + 3 * r * n].view(3, r, n))
            off += 3 * r * n
        return core, out, err.value

    def lowrank_fg_views(self, FG: torch.Tensor, rank: int):
        """The per-axis (3, R, r, 2 n_q) views of a compressed field buffer."""
        R = self.tg_lowrank_info()["nodes"]
        out, off = [], 0
        for n in self.shape:
            size = 6 * R * rank * n
            out.append(FG[off:off + size].view(3, R, rank, 2 * n))
            off += size
        return out

    def energy(self, m: torch.Tensor, Ms: float) -> float:
        self._check(m, "m")
        e = ctypes.c_double()
        _lib.call("demag_energy", self._h, self._ptr(m), float(Ms), ctypes.byref(e), _stream_ptr())
        return e.value


TUCKER, CP = 0, 1  # low-rank formats of the magnetization


def tg_sinc_nodes(rmin: float, rmax: float, step: float):
    """Host-side Sinc nodes and weights of the TG kernel quadrature:
    1/r^3 ~ 4 pi sum_l w_l exp(-tau_l^2 r^2) for r in [rmin, rmax]."""
    lib = _lib.load()
    R = lib.demag_tg_sinc_nodes(float(rmin), float(rmax), float(step), None, None, 0)
    if R < 0:
        _lib.check("demag_tg_sinc_nodes", R)
    tau = np.empty(R)
    w = np.empty(R)
    rc = lib.demag_tg_sinc_nodes(float(rmin), float(rmax), float(step), tau.ctypes.data_as(ctypes.c_void_p),
                                 w.ctypes.data_as(ctypes.c_void_p), R)
    if rc != R:
        _lib.check("demag_tg_sinc_nodes", rc)
    return tau, w


class Batch:
    """Field evaluations of several plans recorded into one HIP graph."""

    def __init__(self, plans, ms, hs, Ms: float):
        n = len(plans)
        self._keep = (list(plans), list(ms), list(hs))
        for p, m, h in zip(plans, ms, hs):
            p._check(m, "m")
            p._check(h, "H")
        arr_p = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
        arr_m = (ctypes.c_void_p * n)(*[m.data_ptr() for m in ms])
        arr_h = (ctypes.c_void_p * n)(*[h.data_ptr() for h in hs])
        b = ctypes.c_void_p()
        _lib.call("demag_batch_create", ctypes.byref(b), arr_p, n, arr_m, arr_h, float(Ms), _stream_ptr())
        self._h = b

    def autotune(self):
        """Tune each geometry group's launch shapes on the group launch itself
        (synchronous; the next launch() recomputes every H)."""
        _lib.call("demag_batch_autotune", self._h, _stream_ptr())

    def launch(self):
        _lib.call("demag_batch_launch", self._h, _stream_ptr())

    def info(self) -> dict:
        """Members, geometry groups and the streams the recorded graph uses."""
        out = (ctypes.c_int64 * 3)()
        _lib.call("demag_batch_info", self._h, out)
        return {"members": out[0], "groups": out[1], "streams": out[2]}

    def close(self):
        if getattr(self, "_h", None):
            _lib.call("demag_batch_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DemagField(torch.autograd.Function):
    """H = -Ms N * m with the hand-written adjoint as its backward:
    dL/dm = A^T dL/dH, A = -Ms N * (A = A^T; same passes on the cotangent)."""

    @staticmethod
    def forward(ctx, m, plan: Plan, Ms: float):
        ctx.plan, ctx.Ms = plan, float(Ms)
        return plan.field(m.contiguous(), Ms)

    @staticmethod
    def backward(ctx, gH):
        gm = ctx.plan.adjoint(gH.contiguous(), ctx.Ms)
        return gm, None, None


class DemagEnergy(torch.autograd.Function):
    """E = -(mu0/2) Ms V sum m.H; the backward hands the saved field and the
    cotangent to demag_energy_gradient (dE/dm = -mu0 Ms V H: the operator is
    symmetric, so no further convolution)."""

    @staticmethod
    def forward(ctx, m, plan: Plan, Ms: float):
        H, E = plan.field_energy(m.contiguous(), Ms)
        ctx.save_for_backward(H)
        ctx.plan, ctx.Ms = plan, float(Ms)
        return E

    @staticmethod
    def backward(ctx, gE):
        (H,) = ctx.saved_tensors
        g = gE.detach().to(device=H.device, dtype=torch.float64).contiguous()
        return ctx.plan.energy_gradient(H, ctx.Ms, gE=g), None, None


def demag_field(m, plan: Plan, Ms: float):
    return DemagField.apply(m, plan, Ms)


def demag_energy(m, plan: Plan, Ms: float):
    return DemagEnergy.apply(m, plan, Ms)
