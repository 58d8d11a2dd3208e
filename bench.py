#!/usr/bin/env python3
"""Throughput of the DM stray-field path on one MI355X.

Workload: 256 x 256 x 64 cells of 2 x 2 x 3 nm, Ms = 1.4e6 A/m, seeded i.i.d.
random unit magnetization, FP32 bulk path (tensor set up in FP64).  One step
is one forward field evaluation with the fused energy (H = -Ms N * m and
E = -(mu0/2) Ms V sum m.H) plus one adjoint evaluation (gm = A^T gH) of a
fixed cotangent: two field evaluations.  `value` counts field evaluations per
second (forward and adjoint each count one); inputs are resident in HBM.

Also reported: the same step in FP64 on the GPU, the FP32 error against the
FP64 oracle at sampled cells, the roofline of the dominant pass (live HIP
events over the timed region) and the CPU oracle timed on a bounded sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W]
  python bench.py --summarize-profile DIR --out FILE   (rocprofv3 output -> text)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SHAPE = (256, 256, 64)
CELL = (2e-9, 2e-9, 3e-9)
MS = 1.4e6
SEED_M, SEED_G, SEED_T = 3, 33, 7
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "traffic_z_conv_256x256x64_f32.txt")
KERNEL_SOURCES = ["paper_1204_4302_amd/csrc/passes_p2.hip", "paper_1204_4302_amd/csrc/fft_reg.hpp",
                  "paper_1204_4302_amd/csrc/fft_lds.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pass_bytes(shape, Px, Py, Pz, Kx, real_bytes):
    """Algorithmic HBM bytes per launch of each pass (read + write, each byte
    of every array a pass must touch once)."""
    nx, ny, nz = shape
    N = nx * ny * nz
    c = 2 * real_bytes
    vec = 3 * N * real_bytes
    B1 = 3 * nz * Kx * ny * c
    B2 = 3 * Py * Kx * nz * c
    nhat = (Py // 2 + 1) * 6 * Kx * (Pz // 2 + 1) * real_bytes
    return {
        "x_r2c": vec + B1,
        "y_fwd": B1 + B2,
        "z_conv": 2 * B2 + nhat,
        "y_inv": B2 + B1,
        "x_c2r": B1 + vec,          # + another vec when the energy reads m
    }


def sp_pass_bytes(shape, Px, Py, Pz, Kx, real_bytes):
    """Algorithmic bytes per launch of each kernel of one scalar-potential
    evaluation with energy (X and Y forward as for DM; the SP Z pass reads
    three components and the kernel spectrum, writes one; one-component
    inverse passes; the gradient reads phi and m, writes H)."""
    nx, ny, nz = shape
    N = nx * ny * nz
    c = 2 * real_bytes
    vec = 3 * N * real_bytes
    B1c = nz * Kx * ny * c
    B2c = Py * Kx * nz * c
    shat = (Py // 2 + 1) * 3 * Kx * (Pz // 2 + 1) * real_bytes
    return {
        "x_r2c": vec + 3 * B1c,
        "y_fwd": 3 * B1c + 3 * B2c,
        "z_sp": 3 * B2c + shat + B2c,
        "y_inv_1": B2c + B1c,
        "x_c2r_1": B1c + N * real_bytes,
        "gradient": N * real_bytes + 2 * vec,
    }


def bench_sp(args, torch, np, m_np, dm_value):
    """Scalar-potential method on the same workload, FP32: field + energy.
    Its energy is compared with DM's on a smooth state (the Gaussian vortex):
    on i.i.d. random directions the finite-difference gradient cannot resolve
    the cell-scale structure, and the two methods differ at O(1) there."""
    from paper_1204_4302_amd import Plan, inputs
    plan = Plan(SHAPE, CELL, torch.float32)
    if not args.no_autotune:
        plan.autotune()
    plan.sp_prepare()
    m = torch.from_numpy(m_np).to("cuda", torch.float32)
    H = torch.empty_like(m)
    E = torch.empty((), dtype=torch.float64, device="cuda")

    def step():
        plan.sp_field_energy(m, MS, out=H, E_out=E)

    for _ in range(args.warmup):
        step()
    k = args.sp_steps
    secs = run_steps(step, k, torch, "sp")
    i = plan.info()
    pb = sp_pass_bytes(SHAPE, i["Px"], i["Py"], i["Pz"], i["Kx"], 4)
    nbytes = sum(pb.values())
    mv = torch.from_numpy(inputs.gaussian_vortex(SHAPE, CELL, 10e-9)).to("cuda", torch.float32)
    _, e_sp = plan.sp_field_energy(mv, MS, with_field=False)
    e_dm = plan.energy(mv, MS)
    e_sp = float(e_sp.cpu())
    out = {"value": round(k / secs, 2), "unit": "evals/s", "ms_per_eval": round(1e3 * secs / k, 4),
           "modelled_bytes_per_eval": nbytes, "achieved_GBs": round(nbytes * k / secs / 1e9, 1),
           "roofline": hbm_roofline(nbytes * k, secs, "whole SP evaluation (all six kernels)"),
           "bytes_per_kernel": pb, "speedup_over_dm": round(k / secs / dm_value, 3),
           "vortex_energy_rel_diff_vs_dm": abs(e_sp - e_dm) / abs(e_dm),
           "step": "one SP field evaluation with energy (potential by FFT convolution, finite-difference gradient)"}
    plan.close()
    return out


def bench_energy_only(args, torch, np, m_np, dm_value):
    """The energy alone on the same workload, FP32: X-R2C, Y and the fused Z
    pass's forward half with the spectral sum of Re(M^H Nhat M) (no inverse
    passes, no field), against the energy of a field evaluation."""
    from paper_1204_4302_amd import Plan
    plan = Plan(SHAPE, CELL, torch.float32)
    if not args.no_autotune:
        plan.autotune()
    m = torch.from_numpy(m_np).to("cuda", torch.float32)
    E = torch.empty((), dtype=torch.float64, device="cuda")

    def step():
        plan.field_energy(m, MS, with_field=False, E_out=E)

    for _ in range(args.warmup):
        step()
    k = args.energy_steps
    secs = run_steps(step, k, torch, "energy_only")
    e_alone = float(E.cpu())
    _, e_field = plan.field_energy(m, MS)
    e_field = float(e_field.cpu())
    i = plan.info()
    pb = pass_bytes(SHAPE, i["Px"], i["Py"], i["Pz"], i["Kx"], 4)
    nx, ny, nz = SHAPE
    B2 = 3 * i["Py"] * i["Kx"] * nz * 8
    # X-R2C and Y as in a field evaluation; the Z pass reads B2 and the tensor
    # octant and writes nothing but the partials
    z_bytes = pb["z_conv"] - B2
    nbytes = pb["x_r2c"] + pb["y_fwd"] + z_bytes
    out = {"value": round(k / secs, 2), "unit": "energy evals/s", "ms_per_eval": round(1e3 * secs / k, 4),
           "modelled_bytes_per_eval": nbytes, "achieved_GBs": round(nbytes * k / secs / 1e9, 1),
           "roofline": hbm_roofline(nbytes * k, secs, "whole energy evaluation (three passes and the sum)"),
           "speedup_over_field_evals": round(k / secs / dm_value, 3),
           "rel_diff_vs_field_energy": abs(e_alone - e_field) / abs(e_field),
           "step": "energy alone (three passes: X-R2C, Y, Z forward with the spectral quadratic form)"}
    plan.close()
    return out


def bench_llg(args, torch, np, dm_value):
    """LLG driver on the same grid, FP32: explicit Heun steps with the DM field
    (two field evaluations and two elementwise kernels per step)."""
    from paper_1204_4302_amd import Plan, inputs
    plan = Plan(SHAPE, CELL, torch.float32)
    if not args.no_autotune:
        plan.autotune()
    m = torch.from_numpy(inputs.gaussian_vortex(SHAPE, CELL, 10e-9)).to("cuda", torch.float32)
    work = torch.empty((9,) + tuple(m.shape[1:]), dtype=torch.float32, device="cuda")
    dt = 1e-13

    def step():
        plan.llg_heun(m, MS, 0.5, dt, 1, H_ext=(0.0, 0.0, 5e4), work=work)

    for _ in range(3):
        step()
    k = args.llg_steps
    secs = run_steps(step, k, torch, "llg")
    i = plan.info()
    field = sum(pass_bytes(SHAPE, i["Px"], i["Py"], i["Pz"], i["Kx"], 4).values())
    vec = 3 * SHAPE[0] * SHAPE[1] * SHAPE[2] * 4
    nbytes = 2 * field + 4 * vec + 5 * vec  # two fields, predictor (m, H -> k1, m*), corrector (m, H, k1, m* -> m)
    out = {"value": round(k / secs, 2), "unit": "Heun steps/s", "ms_per_step": round(1e3 * secs / k, 4),
           "modelled_bytes_per_step": nbytes, "achieved_GBs": round(nbytes * k / secs / 1e9, 1),
           "roofline": hbm_roofline(nbytes * k, secs, "whole Heun step (two field evaluations, two update kernels)"),
           "field_evals_per_s": round(2 * k / secs, 1),
           "step": "one explicit Heun step of the LLG equation (alpha 0.5, dt 1e-13 s, H_ext 5e4 A/m along z, "
                   "Gaussian vortex start), demag field by DM"}
    plan.close()
    return out


MFMA_FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix peak


def bench_tg(args, torch, np, m_np, dm_value):
    """Tensor-grid method (dense block-CP sum of Gaussian mode products) on the
    same workload, FP32: the default path (the fused mode-1/2 kernel on the
    matrix cores, the third mode product a library GEMM) and, as a second
    record, the library chain of three GEMMs (option "tg_mode12" 0); the
    field by differences."""
    from paper_1204_4302_amd import Plan
    m = torch.from_numpy(m_np).to("cuda", torch.float32)
    H = torch.empty_like(m)
    E = torch.empty((), dtype=torch.float64, device="cuda")
    k = args.tg_steps
    res, fields = {}, {}
    for mode, name in ((1, "tg"), (0, "tg_library")):
        plan = Plan(SHAPE, CELL, torch.float32)
        plan.set_option("tg_mode12", mode)
        t0 = time.perf_counter()
        plan.tg_prepare()  # matrices, scratch, and the timed choice of the GEMMs' rocBLAS solutions
        prepare_s = time.perf_counter() - t0
        info, path = plan.tg_info(), plan.tg_path()

        def step():
            plan.tg_field_energy(m, MS, out=H, E_out=E)

        for _ in range(2):
            step()
        secs = run_steps(step, k, torch, name)
        fields[mode] = H.clone()
        res[mode] = {"secs": secs, "info": info, "path": path, "prepare_s": prepare_s}
        plan.close()
    f, lib = res[1], res[0]
    info = f["info"]
    issued = f["path"]["flops_issued"]
    tflops = issued * k / f["secs"] / 1e12
    lib_tflops = lib["info"]["flops_per_eval"] * k / lib["secs"] / 1e12
    Hf, Hl = fields[1].double(), fields[0].double()
    out = {"value": round(k / f["secs"], 2), "unit": "evals/s", "ms_per_eval": round(1e3 * f["secs"] / k, 3),
           "sinc_nodes": info["nodes"], "flops_per_eval": info["flops_per_eval"], "flops_issued": issued,
           "mode12": "fused kernel" if f["path"]["fused"] else "library GEMMs",
           "scratch_bytes": info["scratch_bytes"], "prepare_s": round(f["prepare_s"], 2),
           "roofline": {"bound": "mfma", "achieved": round(tflops, 1), "peak": MFMA_FP32_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(tflops / MFMA_FP32_PEAK_TFLOPS, 4),
                        "note": "mode-product flops issued (zero blocks of the banded Gaussian matrices "
                                "skipped) over the whole evaluation (gradient included in the time)"},
           "dense_equivalent_tflops": round(info["flops_per_eval"] * k / f["secs"] / 1e12, 1),
           "library": {"value": round(k / lib["secs"], 2), "ms_per_eval": round(1e3 * lib["secs"] / k, 3),
                       "scratch_bytes": lib["info"]["scratch_bytes"], "prepare_s": round(lib["prepare_s"], 2),
                       "roofline": {"bound": "mfma", "achieved": round(lib_tflops, 1),
                                    "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                    "frac": round(lib_tflops / MFMA_FP32_PEAK_TFLOPS, 4)},
                       "step": "the same evaluation with all three mode products as rocBLAS GEMMs "
                               "(option tg_mode12 = 0)"},
           "speedup_over_library": round(lib["secs"] / f["secs"], 3),
           "rel_diff_vs_library": float((Hf - Hl).abs().max() / Hl.abs().max()),
           "speedup_over_dm": round(k / f["secs"] / dm_value, 4),
           "step": "one TG field evaluation with energy (Sinc quadrature, first two Gaussian mode products in the "
                   "fused kernel and the third as a GEMM, on the matrix cores; finite-difference gradient)"}
    return out


def bench_lowrank(args, torch, np, dm_value):
    """Tensor grid on low-rank magnetization, FP32, same grid: compressed
    potential + field + energy from Tucker (rank 8) and CP (rank 16) factors
    of a smooth state (cosine modes); the dense expansion timed on its own."""
    import ctypes
    from paper_1204_4302_amd import CP, Plan, TUCKER, inputs, _lib
    plan = Plan(SHAPE, CELL, torch.float32)
    plan.tg_lowrank_prepare()
    info = plan.tg_lowrank_info()
    R = info["nodes"]
    out = {"sinc_nodes": R, "gaussian_matrix_bytes": info["bytes"]}
    E = torch.empty((), dtype=torch.float64, device="cuda")
    H = torch.empty((3, SHAPE[2], SHAPE[1], SHAPE[0]), dtype=torch.float32, device="cuda")
    n1, n2, n3 = SHAPE
    for name, fmt, rank in (("tucker_r8", TUCKER, 8), ("cp_r16", CP, 16)):
        core_np, fac_np = inputs.lowrank(SHAPE, fmt, rank, seed=8, smooth=True)
        core = torch.from_numpy(core_np).to("cuda", torch.float32).contiguous()
        U = torch.cat([torch.from_numpy(f).to("cuda", torch.float32).reshape(-1) for f in fac_np])
        FG = torch.empty(6 * R * rank * sum(SHAPE), dtype=torch.float32, device="cuda")
        fn = _lib.load().demag_tg_lowrank_field
        args_c = [plan._h, fmt, rank, ctypes.c_void_p(core.data_ptr()), ctypes.c_void_p(U.data_ptr()), MS,
                  ctypes.c_void_p(FG.data_ptr())]
        e_ptr, h_ptr = ctypes.c_void_p(E.data_ptr()), ctypes.c_void_p(H.data_ptr())

        def compressed():
            _lib.check("demag_tg_lowrank_field", fn(*args_c, None, e_ptr, None))

        def dense():
            _lib.check("demag_tg_lowrank_field", fn(*args_c, h_ptr, e_ptr, None))

        for _ in range(3):
            compressed()
            dense()
        k = args.lowrank_steps
        sc = run_steps(compressed, k, torch, f"lowrank_{name}")
        kd = max(1, k // 10)
        sd = run_steps(dense, kd, torch, f"lowrank_dense_{name}")
        # algorithmic bytes of the compressed evaluation: per axis q and node
        # the even and the odd Gaussian matrix (n_q x n_q each, read once for
        # all three components), the magnetization factors and core in, and
        # the factor buffer twice (potential factors written, then read by the
        # difference kernel that writes the field factors; all read by the
        # Gram matrices)
        gbytes = sum(2 * R * n * n * 4 for n in SHAPE)
        fbytes = 4 * (U.numel() + core.numel() + 2 * FG.numel())
        nbytes = gbytes + fbytes
        stored = (core.numel() + U.numel())
        out[name] = {
            "value": round(k / sc, 1), "unit": "evals/s", "ms_per_eval": round(1e3 * sc / k, 4),
            "speedup_over_dm": round(k / sc / dm_value, 2),
            "modelled_bytes_per_eval": nbytes, "achieved_GBs": round(nbytes * k / sc / 1e9, 1),
            "roofline": hbm_roofline(nbytes * k, sc, "whole compressed evaluation (factors, differences, "
                                                     "Gram matrices, contraction, sum)"),
            "magnetization_values": stored, "dense_values": 3 * n1 * n2 * n3,
            "with_dense_field": {"value": round(kd / sd, 2), "unit": "evals/s", "ms_per_eval": round(1e3 * sd / kd, 3),
                                 "expansion_gemm_flops": 2 * 3 * n1 * n2 * n3 * 3 * R * rank},
            "step": f"compressed potential, field and energy from a rank-{rank} "
                    f"{'Tucker' if fmt == TUCKER else 'CP'} magnetization (no dense tensor formed)"}
    # ALS compression of a dense state on the same grid (set-up work): the
    # Gaussian vortex to Tucker rank 8 from a seeded random guess
    m = torch.from_numpy(inputs.gaussian_vortex(SHAPE, CELL, 10e-9)).to("cuda", torch.float32)
    _, init_np = inputs.lowrank(SHAPE, TUCKER, 8, seed=9)
    init = [torch.from_numpy(f).to("cuda", torch.float32) for f in init_np]
    plan.lowrank_compress(m, TUCKER, 8, 1, init)  # warm-up (rocBLAS handle, kernels)
    sweeps = 4
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, relerr = plan.lowrank_compress(m, TUCKER, 8, sweeps, init)
    secs = time.perf_counter() - t0
    out["als_compress"] = {"state": "Gaussian vortex (r0 = 10 nm) on 256x256x64", "format": "Tucker", "rank": 8,
                           "sweeps": sweeps, "seconds": round(secs, 4), "relerr": relerr}
    plan.close()
    return out


def hbm_roofline(nbytes, seconds, what):
    """HBM roofline of a leg measured as a whole (modelled bytes over the
    measured time of the leg's step, every kernel of the step included)."""
    achieved = nbytes / seconds / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "over": what}


def read_traffic():
    """HBM bytes per z_conv launch from the committed --pmc summary, or None if
    the kernels changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def device_copy_rates(torch):
    """Context for the HBM fractions: a plain device-to-device copy (torch
    copy_) of 512 MiB and 2 GiB on the same GPU in the same run, bytes read
    plus bytes written per second (median of 10 after 3 warm-ups)."""
    out = {}
    for label, nbytes in (("512MiB", 512 << 20), ("2GiB", 2 << 30)):
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        ts = []
        for r in range(13):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            if r >= 3:
                ts.append(e0.elapsed_time(e1) * 1e-3)
        ts.sort()
        out[label] = round(2 * nbytes / ts[len(ts) // 2] / 1e9, 1)
        del a, b
    torch.cuda.empty_cache()
    return out


def settle(step, torch, seconds):
    """Run `step` back to back for about `seconds` before the warm-up steps.
    Measured on MI355X: after an idle spell the step time falls from about
    0.76 to 0.61 ms over its first ~30 repetitions (the GPU's clocks ramp up
    under sustained load), so a few warm-up steps alone leave a short timed
    region inside the ramp."""
    if seconds <= 0:
        return
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            step()
        torch.cuda.synchronize()


_ROCTX = []


def _roctx():
    """The ROCTx library (host-side profiler ranges), or None if absent."""
    if not _ROCTX:
        import ctypes
        lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib",
                                                                    "librocprofiler-sdk-roctx.so.1")):
            try:
                lib = ctypes.CDLL(name)
                lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                break
            except OSError:
                lib = None
        _ROCTX.append(lib)
    return _ROCTX[0]


def run_steps(step, k, torch, name=None):
    """Time k calls of `step` between two device synchronisations.  With
    `name`, the region (synchronisations included) is the profiler range
    "bench:<name>" (rocprofv3 --marker-trace), which --summarize-profile
    --range selects."""
    rx = _roctx() if name else None
    torch.cuda.synchronize()
    if rx:
        rx.roctxRangePushA(f"bench:{name}".encode())
    t0 = time.perf_counter()
    for _ in range(k):
        step()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    if rx:
        rx.roctxRangePop()
    return secs


def cpu_baseline(m, target_seconds, Href32, Href64):
    import numpy as np
    import oracle
    from paper_1204_4302_amd import inputs

    o = oracle.Oracle(SHAPE, CELL, cache_dir=os.environ.get("DEMAG_ORACLE_CACHE"))
    N = SHAPE[0] * SHAPE[1] * SHAPE[2]
    # calibrate the per-target cost, then size the sample to ~target_seconds
    probe = inputs.sample_targets(SHAPE, 32, SEED_T)
    t0 = time.perf_counter()
    o.field_targets(m, MS, probe)
    per = (time.perf_counter() - t0) / probe.size
    count = int(max(64, min(20000, target_seconds / max(per, 1e-9))))
    targets = inputs.sample_targets(SHAPE, count, SEED_T + 1)
    t0 = time.perf_counter()
    Ht = o.field_targets(m, MS, targets)
    dt = time.perf_counter() - t0
    flat32 = Href32.reshape(3, -1)[:, targets]
    flat64 = Href64.reshape(3, -1)[:, targets]
    scale = np.max(np.abs(Ht))
    err = {"f32": float(np.max(np.abs(flat32 - Ht)) / scale),
           "f64": float(np.max(np.abs(flat64 - Ht)) / scale),
           "targets": int(targets.size)}
    base = {
        "value": targets.size / dt / N,
        "unit": "evals/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": (f"FP64 direct O(N^2) field at {targets.size} seeded target cells of the "
                   f"256x256x64 grid ({dt:.1f} s), scaled to whole-grid evaluations; "
                   f"binary128 tensor setup {o.tensor_seconds:.1f} s not counted"),
    }
    return base, err


def bench_rocfft_reference(args, torch, np, m_np):
    """Informational, not a target: the same forward DM field written with
    torch.fft (rocFFT) -- the padded magnetization transformed whole, the
    product with the plan's tensor spectrum (mirrored from its octant with the
    parity signs: xy, yz odd in ky; xz, yz odd in kz) as separate tensor
    operations, the inverse transform and the crop -- against the plan's own
    forward field on the same input.  Checked against the plan's field first."""
    from paper_1204_4302_amd import Plan
    plan = Plan(SHAPE, CELL, torch.float32)
    if not args.no_autotune:
        plan.autotune()
    i = plan.info()
    Px, Py, Pz = i["Px"], i["Py"], i["Pz"]
    nx, ny, nz = SHAPE
    full = torch.from_numpy(mirrored_spectrum(np, plan.spectrum(), Py, Pz)).cuda()  # [6][Pz][Py][Kx]
    nxx, nyy, nzz, nxy, nxz, nyz = full
    m = torch.from_numpy(m_np).to("cuda", torch.float32)
    mp = torch.zeros((3, Pz, Py, Px), device="cuda")
    out = torch.empty_like(m)

    def step():
        mp[:, :nz, :ny, :nx] = m
        M = torch.fft.rfftn(mp, dim=(1, 2, 3))
        Hh = torch.stack((nxx * M[0] + nxy * M[1] + nxz * M[2], nxy * M[0] + nyy * M[1] + nyz * M[2],
                          nxz * M[0] + nyz * M[1] + nzz * M[2]))
        h = torch.fft.irfftn(Hh, s=(Pz, Py, Px), dim=(1, 2, 3), norm="forward")
        torch.mul(h[:, :nz, :ny, :nx], MS, out=out)

    step()
    ref = plan.field(m, MS)
    err = float(((out - ref).abs().max() / ref.abs().max()).item())
    H = torch.empty_like(m)
    k = args.rocfft_steps
    for _ in range(3):
        step()
        plan.field(m, MS, out=H)
    t_ref = run_steps(step, k, torch, "rocfft_reference")
    t_dm = run_steps(lambda: plan.field(m, MS, out=H), k, torch, "rocfft_reference_dm")
    plan.close()
    del full, mp, out, ref
    torch.cuda.empty_cache()
    return {"value": round(k / t_ref, 1), "unit": "evals/s", "ms_per_eval": round(1e3 * t_ref / k, 4),
            "dm_forward_evals_per_s": round(k / t_dm, 1), "speedup_dm_over_rocfft": round(t_ref / t_dm, 2),
            "rel_err_vs_dm": err,
            "note": "informational, not a target: forward field with torch.fft (rocFFT) on the padded grid and "
                    "the plan's tensor spectrum, vs the plan's forward field (no energy, no adjoint)"}


def mirrored_spectrum(np, S, Py, Pz):
    """[6][Pz][Py][Kx] from the stored octant [Py/2+1][6][Kx][Pz/2+1] (numpy):
    xy, yz odd in ky; xz, yz odd in kz."""
    ky, kz = np.arange(Py), np.arange(Pz)
    full = S[np.where(ky <= Py // 2, ky, Py - ky)][..., np.where(kz <= Pz // 2, kz, Pz - kz)]
    full = np.ascontiguousarray(full.transpose(1, 3, 0, 2))
    sy = np.where(ky <= Py // 2, 1.0, -1.0)[None, :, None]
    sz = np.where(kz <= Pz // 2, 1.0, -1.0)[:, None, None]
    for c in (3, 5):
        full[c] *= sy
    for c in (4, 5):
        full[c] *= sz
    return full


def cpu_fft_reference(args, np, m_np, plan64, H64):
    """Informational, not a target: the forward DM field on the host with
    scipy.fft in FP64 on the host's threads (the padded magnetization
    transformed whole, the product with the plan's FP64 tensor spectrum, the
    inverse, the crop); best of a few evaluations; checked against the plan's
    FP64 field.  The like-for-like (O(N log N)) CPU counterpart of the GPU
    path, where the oracle baseline is the O(N^2) definition."""
    import scipy.fft
    i = plan64.info()
    Px, Py, Pz = i["Px"], i["Py"], i["Pz"]
    nx, ny, nz = SHAPE
    full = mirrored_spectrum(np, plan64.spectrum(), Py, Pz)
    nxx, nyy, nzz, nxy, nxz, nyz = full
    workers = min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16") or 16))

    def ev():
        mp = np.zeros((3, Pz, Py, Px))
        mp[:, :nz, :ny, :nx] = m_np
        M = scipy.fft.rfftn(mp, axes=(1, 2, 3), workers=workers)
        Hh = np.stack((nxx * M[0] + nxy * M[1] + nxz * M[2], nxy * M[0] + nyy * M[1] + nyz * M[2],
                       nxz * M[0] + nyz * M[1] + nzz * M[2]))
        h = scipy.fft.irfftn(Hh, s=(Pz, Py, Px), axes=(1, 2, 3), norm="forward", workers=workers)
        return MS * h[:, :nz, :ny, :nx]

    best, h = None, None
    for _ in range(max(1, args.cpu_fft_evals)):
        t0 = time.perf_counter()
        h = ev()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    err = float(np.max(np.abs(h - H64)) / np.max(np.abs(H64)))
    return {"value": round(1.0 / best, 3), "unit": "evals/s", "cores": workers, "kind": "scipy.fft FP64 host",
            "rel_err_vs_gpu_f64": err,
            "note": "informational: forward field only, best of %d evaluations" % max(1, args.cpu_fft_evals)}


BATCH_SIZES = [(32, 32, 32), (64, 64, 16), (96, 48, 8), (128, 128, 4), (48, 48, 48)]


XGMI_LINK_GBS, XGMI_LINKS = 153.0, 7  # MI355X: point-to-point xGMI links per GPU


def bench_shard_share(args, torch, np):
    """One GPU's share of the headline grid sharded over G GPUs (the design:
    z-slabs for the X and Y passes, kx-slabs for the fused Z pass, an
    all-to-all of B2 before and after the Z pass), its kernels timed here at
    their real shapes: the X and Y passes of a 256 x 256 x (64/G) slab, and
    the fused Z pass over ceil(257/G) kx columns x 512 ky x 128 (the Z pass of
    a 32 x 256 x 64 plan has exactly Kx = 33 such columns for G = 8).  The
    all-to-alls are a model (bytes over the seven links), not a measurement;
    no second GPU is used."""
    from paper_1204_4302_amd import Plan, inputs
    G = args.shard_share
    nx, ny, nz = SHAPE
    Kx = nx + 1  # padded x length 2 nx
    if nz % G or (Kx + G - 1) // G != 33:
        return {"note": f"modelled for G = 8 only (got {G})"}
    times = {}
    for name, shape in (("slab", (nx, ny, nz // G)), ("kx_slab", (32, ny, nz))):
        plan = Plan(shape, CELL, torch.float32)
        if not args.no_autotune:
            plan.autotune()
        m = torch.from_numpy(inputs.random_unit(shape, SEED_M)).to("cuda", torch.float32)
        H = torch.empty_like(m)
        for _ in range(args.warmup):
            plan.field(m, MS, out=H)
        plan.set_option("pass_timing", 200)
        for _ in range(200):
            plan.field(m, MS, out=H)
        torch.cuda.synchronize()
        times[name], _ = plan.pass_times()
        plan.close()
    local_ms = sum(times["slab"][k] for k in ("x_r2c", "y_fwd", "y_inv", "x_c2r")) + times["kx_slab"]["z_conv"]
    i_b2 = 3 * Kx * (2 * ny) * nz * 8  # B2 bytes of the whole grid (FP32 complex)
    a2a_bytes = i_b2 / G * (G - 1) / G  # one GPU sends (and receives) this much per exchange
    a2a_ms = 1e3 * a2a_bytes / (XGMI_LINKS * XGMI_LINK_GBS * 1e9)
    per_eval_ms = local_ms + 2 * a2a_ms
    return {"gpus_modelled": G, "slab_passes_ms": {k: round(times["slab"][k], 4) for k in
                                                   ("x_r2c", "y_fwd", "y_inv", "x_c2r")},
            "kx_slab_z_conv_ms": round(times["kx_slab"]["z_conv"], 4),
            "local_ms_per_eval": round(local_ms, 4), "all_to_all_bytes_per_gpu": int(a2a_bytes),
            "all_to_all_ms_modelled": round(a2a_ms, 4),
            "evals_per_s_modelled_no_overlap": round(1e3 / per_eval_ms, 1),
            "note": "kernels measured on this GPU at one GPU's share; the two all-to-alls per evaluation are "
                    "modelled (bytes / (7 links x 153 GB/s)), not overlapped; no multi-GPU run"}


def bench_batch(args, torch, np):
    """96 independent grids of seeded uneven shapes (2 nm cubes, Ms = 8e5, FP32):
    one replay of the recorded batch graph vs 96 single-grid calls."""
    from paper_1204_4302_amd import Batch, Plan, inputs
    rng = np.random.default_rng(4)
    shapes = [BATCH_SIZES[i] for i in rng.integers(0, len(BATCH_SIZES), size=96)]
    cell, Ms = (2e-9, 2e-9, 2e-9), 8e5
    plans = [Plan(s, cell, torch.float32) for s in shapes]
    ms = [torch.from_numpy(inputs.random_unit(s, 4000 + g)).to("cuda", torch.float32) for g, s in enumerate(shapes)]
    hs = [torch.empty_like(m) for m in ms]
    batch = Batch(plans, ms, hs, Ms)
    tune_s = None
    if not args.no_autotune:  # launch shapes tuned on each group's whole launch
        t0 = time.perf_counter()
        batch.autotune()
        tune_s = round(time.perf_counter() - t0, 2)

    def seq():
        for p, m, h in zip(plans, ms, hs):
            p.field(m, Ms, out=h)

    k = args.batch_steps
    for _ in range(3):
        seq()
    t_seq = run_steps(seq, k, torch, "batch_sequential")
    for _ in range(20):  # untimed replays before the timed ones
        batch.launch()
    t_graph = run_steps(batch.launch, k, torch, "batch_graph")
    # every member of the timed replays against its single-grid call (the
    # group-tuned launch shapes may differ from the plans' own: FP32 rounding)
    batch.launch()
    torch.cuda.synchronize()
    member_err = max(float((p.field(m, Ms) - h).abs().max() / h.abs().max()) for p, m, h in zip(plans, ms, hs))
    nbytes = 0
    for p in plans:
        i = p.info()
        nbytes += sum(pass_bytes(p.shape, i["Px"], i["Py"], i["Pz"], i["Kx"], 4).values())
    cells = sum(a * b * c for a, b, c in shapes)
    out = {"grids": len(shapes), "cells": cells, "distinct_shapes": len(set(shapes)),
           "graph_batches_per_s": round(k / t_graph, 2), "graph_grid_evals_per_s": round(96 * k / t_graph, 1),
           "sequential_batches_per_s": round(k / t_seq, 2), "speedup_graph_over_sequential": round(t_seq / t_graph, 3),
           "modelled_bytes_per_batch": nbytes, "graph_achieved_GBs": round(nbytes * k / t_graph / 1e9, 1),
           "roofline": hbm_roofline(nbytes * k, t_graph, "whole batch replay (96 grids, five passes each)"),
           "launch_shapes": "autotuned per group" if tune_s is not None else "default", "autotune_s": tune_s,
           "graph": batch.info(),
           "members_max_rel_diff_vs_single_calls": member_err}
    batch.close()
    for p in plans:
        p.close()
    return out


def bench(args):
    import numpy as np
    import torch

    from paper_1204_4302_amd import Plan, inputs

    torch.cuda.set_device(0)
    nx, ny, nz = SHAPE
    # FP32-representable directions, so the FP32 and FP64 paths and the oracle see one input
    m_np = inputs.random_unit(SHAPE, SEED_M).astype(np.float32).astype(np.float64)
    g_np = np.random.default_rng(SEED_G).standard_normal((3, nz, ny, nx))

    results = {}
    for dtype, steps in [(torch.float32, args.steps), (torch.float64, args.fp64_steps)]:
        if steps <= 0:
            continue
        plan = Plan(SHAPE, CELL, dtype)
        tune_s = None
        if not args.no_autotune:
            t0 = time.perf_counter()
            plan.autotune()
            tune_s = time.perf_counter() - t0
        m = torch.from_numpy(m_np).to("cuda", dtype)
        gH = torch.from_numpy(g_np).to("cuda", dtype)
        H = torch.empty_like(m)
        gm = torch.empty_like(m)
        E = torch.empty((), dtype=torch.float64, device="cuda")

        def step():
            plan.field_energy(m, MS, out=H, E_out=E)
            plan.adjoint(gH, MS, out=gm)

        settle(step, torch, args.settle)
        for _ in range(args.warmup):
            step()
        # the timed region runs without instrumentation; the per-pass times
        # come from a second, separately recorded region of the same length
        secs = run_steps(step, steps, torch, "dm_f32" if dtype == torch.float32 else "dm_f64")
        passes, nrec = {}, 0
        if dtype == torch.float32 and not args.no_pass_timing:
            plan.set_option("pass_timing", 2 * steps)
            run_steps(step, steps, torch, "dm_f32_pass_timing")
            passes, nrec = plan.pass_times()
            plan.set_option("pass_timing", 0)
        print(f"# {dtype} launch: {plan.describe()}", file=sys.stderr, flush=True)
        results[dtype] = {"plan": plan, "secs": secs, "steps": steps, "H": H.double().cpu().numpy(), "tune_s": tune_s,
                          "E": float(E.cpu()), "passes": passes, "nrec": nrec, "info": plan.info()}
        print(f"# {dtype}: {steps} steps in {secs:.3f} s ({1e3 * secs / steps:.3f} ms/step)", file=sys.stderr,
              flush=True)

    r32 = results[torch.float32]
    info = r32["info"]
    ms_step = 1e3 * r32["secs"] / r32["steps"]
    value = 2 * r32["steps"] / r32["secs"]

    # roofline of the dominant pass, from the per-pass events of the second region
    pb = pass_bytes(SHAPE, info["Px"], info["Py"], info["Pz"], info["Kx"], 4)
    passes = r32["passes"]
    roofline = None
    if passes:
        dom = max(pb, key=lambda k: passes.get(k, 0.0))
        achieved = pb[dom] / (passes[dom] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": read_traffic() if dom == "z_conv" else None,
                    "bytes_per_launch": pb[dom], "avg_launch_ms": round(passes[dom], 5),
                    "pass_ms": {k: round(v, 5) for k, v in passes.items()},
                    "pass_ms_region": f"separate region of {r32['steps']} steps with per-pass HIP events "
                                      "(the timed region runs without them)"}
        # the whole step against HBM: modelled bytes of all passes of both evaluations
        step_bytes = 2 * sum(pb.values()) + 3 * nx * ny * nz * 4  # + m read by the energy epilogue
        roofline["step_achieved_GBs"] = round(step_bytes / (ms_step * 1e-3) / 1e9, 1)
        roofline["device_copy_GBs"] = device_copy_rates(torch)

    out = {
        "metric": "demag field evals/s at 256x256x64 FP32 (fwd+adjoint), achieved HBM GB/s, vs FP64",
        "value": round(value, 2),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": r32["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256x256x64 cells, 2x2x3 nm, Ms=1.4e6 A/m, seeded random unit m; "
                               "step = forward field+energy and adjoint (2 field evaluations)",
                   "padded": [info["Px"], info["Py"], info["Pz"]], "parallelism": "none (1 GPU)",
                   "launch": r32["plan"].describe(),
                   "launch_shapes": "autotuned" if r32["tune_s"] is not None else "default",
                   "settle_s": args.settle,
                   "autotune_s": None if r32["tune_s"] is None else round(r32["tune_s"], 2)},
        "roofline": roofline,
        # once per plan, not in the timed region: Newell tensor on the octant
        # (FP64, three distance bands) and its spectrum (FP64 FFTs), stored in
        # the plan precision
        "setup": {"tensor_setup_ms": round(info["setup_us"] / 1e3, 2), "tensor_bytes": info["tensor_bytes"],
                  "scratch_bytes": info["scratch_bytes"]},
    }
    if torch.float64 in results:
        r64 = results[torch.float64]
        v64 = 2 * r64["steps"] / r64["secs"]
        i64 = r64["info"]
        pb64 = pass_bytes(SHAPE, i64["Px"], i64["Py"], i64["Pz"], i64["Kx"], 8)
        step64 = 2 * sum(pb64.values()) + 3 * nx * ny * nz * 8  # as the FP32 step, 8-byte reals
        out["fp64"] = {"value": round(v64, 2), "unit": "evals/s",
                       "ms_per_step": round(1e3 * r64["secs"] / r64["steps"], 4),
                       "speedup_fp32_over_fp64": round(value / v64, 3),
                       "roofline": hbm_roofline(step64 * r64["steps"], r64["secs"],
                                                "whole FP64 step (modelled bytes of both evaluations)")}
        H64 = r64["H"]
        out["accuracy"] = {"f32_vs_f64_gpu_field": float(np.max(np.abs(r32["H"] - H64)) / np.max(np.abs(H64))),
                           "f32_vs_f64_gpu_energy": abs(r32["E"] - r64["E"]) / abs(r64["E"])}
    if args.energy_steps > 0:
        out["energy_only"] = bench_energy_only(args, torch, np, m_np, value)
        print(f"# energy_only: {out['energy_only']}", file=sys.stderr, flush=True)
    if args.sp_steps > 0:
        out["sp"] = bench_sp(args, torch, np, m_np, value)
        print(f"# sp: {out['sp']}", file=sys.stderr, flush=True)
    if args.lowrank_steps > 0:
        out["tg_lowrank"] = bench_lowrank(args, torch, np, value)
        print(f"# tg_lowrank: {out['tg_lowrank']}", file=sys.stderr, flush=True)
    if args.llg_steps > 0:
        out["llg"] = bench_llg(args, torch, np, value)
        print(f"# llg: {out['llg']}", file=sys.stderr, flush=True)
    if args.rocfft_steps > 0:
        out["rocfft_reference"] = bench_rocfft_reference(args, torch, np, m_np)
        print(f"# rocfft_reference: {out['rocfft_reference']}", file=sys.stderr, flush=True)
    if args.tg_steps > 0:
        out["tg"] = bench_tg(args, torch, np, m_np, value)
        print(f"# tg: {out['tg']}", file=sys.stderr, flush=True)
    if args.batch_steps > 0:
        out["batch"] = bench_batch(args, torch, np)
        print(f"# batch: {out['batch']}", file=sys.stderr, flush=True)
    if args.shard_share > 0:
        out["shard_share"] = bench_shard_share(args, torch, np)
        print(f"# shard_share: {out['shard_share']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        H64 = results[torch.float64]["H"] if torch.float64 in results else r32["H"]
        base, err = cpu_baseline(m_np, args.cpu_seconds, r32["H"], H64)
        out["cpu_baseline"] = base
        out.setdefault("accuracy", {})["vs_oracle_sampled"] = err
        if args.cpu_fft_evals > 0 and torch.float64 in results:
            out["cpu_fft_reference"] = cpu_fft_reference(args, np, m_np, results[torch.float64]["plan"], H64)
            print(f"# cpu_fft_reference: {out['cpu_fft_reference']}", file=sys.stderr, flush=True)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# rocprofv3 output (its SQLite results database) -> short text summaries
def _find(d, pattern):
    return sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))


def _short(name):
    name = name.replace("demag::(anonymous namespace)::", "").replace("demag::", "")
    return name.split("(")[0].replace("void ", "")


def _union_ns(intervals):
    """Total length of the union of [start, end) intervals."""
    busy, cur_s, cur_e = 0, None, None
    for a, b in sorted(intervals):
        if cur_e is None or a > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = a, b
        else:
            cur_e = max(cur_e, b)
    return busy + (cur_e - cur_s if cur_e is not None else 0)


def summarize_profile(d, out_path, command, match=None, region=None):
    """Per-kernel calls / average / total from a --kernel-trace --stats run
    (only kernels whose name contains one of the comma-separated `match`
    strings, when given).  With `region`, only the kernels that ran inside
    the bench's profiler range "bench:<region>" (a run with --marker-trace),
    with the range's length and the fraction of it during which a kernel ran."""
    import sqlite3
    lines = [f"# command: {command}", f"# kernel_source_hash = {kernel_source_hash()}",
             "# per kernel and grid size (work-items), from the trace's dispatch records",
             f"{'kernel':44s} {'grid':>9s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for db in _find(d, "*results.db"):
        con = sqlite3.connect(db)
        where = ""
        if region:
            # the range's message is the name (older layouts) or in the JSON extdata
            ranges = []
            for a, b, nm, ext in con.execute("select start, end, name, extdata from regions"):
                try:
                    msg = json.loads(ext or "{}").get("message")
                except ValueError:
                    msg = None
                if f"bench:{region}" in (nm, msg):
                    ranges.append((a, b))
            if not ranges:
                raise SystemExit(f"no profiler range bench:{region} in {db} (run rocprofv3 with --marker-trace)")
            where = " where " + " or ".join(f"(start >= {a} and end <= {b})" for a, b in ranges)
            spans = con.execute(f"select start, end from kernels{where}").fetchall()
            window = sum(b - a for a, b in ranges)
            lines.insert(3, f"# range bench:{region}: {len(ranges)} range(s), {window / 1e6:.3f} ms, "
                            f"{len(spans)} dispatches, a kernel running {100.0 * _union_ns(spans) / window:.1f}% "
                            "of the time")
        rows = con.execute("select name, grid_x * grid_y * grid_z, count(*), sum(end - start), avg(end - start) "
                           f"from kernels{where} group by name, grid_x, grid_y, grid_z").fetchall()
        total_ns = sum(r[3] for r in rows) or 1
        if match:
            keys = [k for k in match.split(",") if k]
            rows = [r for r in rows if any(k in r[0] for k in keys)]
            lines.insert(3, f"# kernels matching: {match}")
        for name, grid, calls, tot, avg in sorted(rows, key=lambda r: -r[3]):
            # dispatch timestamps are in nanoseconds
            lines.append(f"{_short(name)[:44]:44s} {grid:9d} {calls:6d} {avg / 1e3:10.2f} {tot / 1e6:10.3f} "
                         f"{100.0 * tot / total_ns:6.2f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_means(d, counter):
    """{kernel: (mean value per dispatch, dispatches)} of one --pmc counter."""
    import sqlite3
    agg = {}
    for db in _find(d, "*results.db"):
        con = sqlite3.connect(db)
        for name, val, grid in con.execute(
                "select kernel_name, value, grid_size from counters_collection where counter_name = ?", (counter,)):
            agg.setdefault((_short(name), grid), []).append(val)
    return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}


# --copy-calibration: a 256 MiB device copy (the runtime's copy kernel) and,
# as a check, a 1 GiB elementwise copy (torch's kernel, y = 1 * x)
CALIBRATION = ((256, "copyBuffer"), (1024, "elementwise"))


def traffic_summary(fetch_dir, write_dir, out_path, command):
    """HBM bytes per launch of every pass kernel from FETCH_SIZE / WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for the
    plain 256 MiB device copy of --copy-calibration (runtime copy kernel); the
    1 GiB elementwise copy of the same run is reported beside it as a check
    that the factor depends neither on the size nor on the copying kernel."""
    fetch, write = _counter_means(fetch_dir, "FETCH_SIZE"), _counter_means(write_dir, "WRITE_SIZE")

    def calib(mib, kind):
        # the copy of `mib` MiB: among the dispatches (name, grid) of that kind
        # of kernel that write about the copied size, the one that reads most
        # (the fill that initialised the source writes as much but reads nothing)
        kib = mib * 1024.0
        keys = [key for key, (v, n) in write.items() if kind in key[0] and 0.5 * kib < v < 2.0 * kib]
        if not keys:
            return None, None
        key = max(keys, key=lambda kk: fetch.get(kk, (0.0, 0))[0])
        return fetch.get(key, (None, 0))[0], write[key][0]

    cal = {mib: calib(mib, kind) for mib, kind in CALIBRATION}
    fc, wc = cal[256]
    f_fetch = 256 * 1024.0 / fc if fc else None
    f_write = 256 * 1024.0 / wc if wc else None
    lines = [f"# command: {command}", f"kernel_source_hash = {kernel_source_hash()}"]
    for mib, (cf, cw) in cal.items():
        ff = f"{mib * 1024.0 / cf:.4f}" if cf else "n/a"
        fw = f"{mib * 1024.0 / cw:.4f}" if cw else "n/a"
        what = "device copy (runtime copy kernel)" if mib == 256 else "elementwise copy (check)"
        lines.append(f"# calibration: a {mib} MiB {what} reads {cf} KiB (FETCH_SIZE) and writes {cw} KiB "
                     f"(WRITE_SIZE): factors {ff} / {fw}")
    lines += [f"copy_calibration_fetch_factor = {f_fetch}", f"copy_calibration_write_factor = {f_write}",
              f"# {'kernel':40s} {'grid':>9s} {'FETCH_KiB':>11s} {'WRITE_KiB':>11s} {'scaled_MB':>10s}"]
    zconv = None
    for key in sorted(set(fetch) | set(write)):
        fv, wv = fetch.get(key, (0.0, 0))[0], write.get(key, (0.0, 0))[0]
        if fv + wv < 1024:
            continue
        scaled = (fv * f_fetch + wv * f_write) * 1024.0 if (f_fetch and f_write) else None
        lines.append(f"  {key[0][:40]:40s} {key[1]:9d} {fv:11.1f} {wv:11.1f} "
                     f"{(scaled or 0) / 1e6:10.1f}")
        # the headline's fused Z pass: the largest FP32 field launch (template
        # arguments: type, length, schedule, energy alone, streamed tensor)
        args_ = key[0][len("kz_conv<"):-1].split(", ") if key[0].startswith("kz_conv<float") else []
        if len(args_) >= 4 and args_[3] == "false" and scaled is not None:
            zconv = max(zconv or 0.0, scaled)
    if zconv is not None:
        lines.append(f"traffic_bytes_per_launch = {zconv}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--fp64-steps", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle sample budget")
    ap.add_argument("--batch-steps", type=int, default=50, help="replays of the 96-grid batch (0: skip)")
    ap.add_argument("--shard-share", type=int, default=8,
                    help="time one GPU's share of the headline grid sharded over this many GPUs (0: skip)")
    ap.add_argument("--sp-steps", type=int, default=200, help="scalar-potential evaluations (0: skip)")
    ap.add_argument("--energy-steps", type=int, default=200, help="energy-alone evaluations (0: skip)")
    ap.add_argument("--tg-steps", type=int, default=10, help="tensor-grid evaluations (0: skip)")
    ap.add_argument("--llg-steps", type=int, default=100, help="LLG Heun steps (0: skip)")
    ap.add_argument("--lowrank-steps", type=int, default=200, help="low-rank TG evaluations (0: skip)")
    ap.add_argument("--cpu-fft-evals", type=int, default=2,
                    help="informational host scipy.fft FP64 forward fields (0: skip)")
    ap.add_argument("--rocfft-steps", type=int, default=30,
                    help="informational torch.fft (rocFFT) forward fields beside the plan's (0: skip)")
    ap.add_argument("--settle", type=float, default=0.15,
                    help="seconds of back-to-back steps before the warm-up steps (clock ramp; 0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pass-timing", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default launch shapes (default: tune them first; DEMAG_AUTOTUNE_CACHE keeps the result)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 256 MiB (counter calibration)")
    ap.add_argument("--summarize-profile", metavar="DIR")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--out", metavar="FILE")
    ap.add_argument("--command", default="", help="command line recorded in the summary")
    ap.add_argument("--match", default=None, help="--summarize-profile: keep kernels whose name contains one of "
                                                  "these comma-separated strings")
    ap.add_argument("--range", default=None, help="--summarize-profile: only kernels inside the bench's profiler "
                                                  "range bench:RANGE (e.g. batch_graph, dm_f32)")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary, args.out or "/dev/stdout", args.command)
        return 0
    if args.summarize_profile:
        summarize_profile(args.summarize_profile, args.out or "/dev/stdout", args.command, args.match, args.range)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU and measures the one-GPU path only; --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        return 2
    if args.copy_calibration:
        import torch
        for mib, kind in CALIBRATION:
            a = torch.empty(mib * 256 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
            b = torch.empty_like(a)
            for _ in range(3):
                if kind == "copyBuffer":
                    b.copy_(a)
                else:
                    torch.mul(a, 1.0, out=b)
            torch.cuda.synchronize()
            del a, b
        print("# copy calibration: 3 x 256 MiB device copies, 3 x 1 GiB elementwise copies", file=sys.stderr)
    bench(args)
    return 0


if __name__ == "__main__":
    sys.exit(main())
