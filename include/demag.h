/*
 * demag.h -- C ABI of the MI355X (gfx950) demagnetization-tensor (DM) stray
 * field library.
 *
 * The operation (Abert et al., "Numerical Methods for the Stray-Field
 * Calculation: A Comparison of recently developed Algorithms", Sec. 3.1,
 * eq. (demag)): for a cell-wise constant magnetization M = Ms m on a regular
 * nx x ny x nz grid of dx x dy x dz cuboid cells, the cell-averaged stray
 * field is the discrete matrix-vector convolution
 *
 *      H_i = -Ms * sum_j N(r_i - r_j) m_j ,
 *
 * N the demagnetization tensor of homogeneously magnetized cells averaged over
 * the target cell (Sec. 5.1).  The convolution is evaluated with the
 * convolution theorem (eq. (convolution)) on a grid zero-padded to P = 2L
 * points per axis (L >= n), as an element-wise 3x3 matrix-vector product in
 * Fourier space (Sec. 3.1).  The energy is the stray-field energy of Sec. 2,
 *
 *      E = -(mu0/2) * Ms * V * sum_i m_i . H_i ,   V = dx dy dz, mu0 = 4 pi 1e-7.
 *
 * Conventions for every call:
 *  - Vector fields (m, H, gH, gm) are DEVICE pointers owned by the caller,
 *    contiguous structure-of-arrays [3][nz][ny][nx] (x fastest), in the plan's
 *    precision (float for DEMAG_F32, double for DEMAG_F64).  Input and output
 *    buffers must not overlap.
 *  - m is used as given (not renormalised).  NaN/Inf in m propagate.
 *  - Ms in A/m; H in A/m; E in J.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Field calls only enqueue work and return; they do not synchronise.
 *  - Every function returns DEMAG_OK (0) or a negative demag_status; the text
 *    of the last error of the calling thread is demag_last_error().
 *  - A plan owns its scratch (two spectrum buffers) and must not be used on
 *    two streams at the same time; a call on another stream while work of the
 *    plan is still pending returns DEMAG_ESTATE.
 */
#ifndef DEMAG_H
#define DEMAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct demag_plan_s* demag_plan_t;
typedef struct demag_batch_s* demag_batch_t;

typedef enum { DEMAG_F32 = 0, DEMAG_F64 = 1 } demag_dtype;

typedef enum {
    DEMAG_OK = 0,
    DEMAG_EINVAL = -1,      /* bad argument (shape, cell size, pointer, option) */
    DEMAG_ENOMEM = -2,      /* device allocation failed */
    DEMAG_EHIP = -3,        /* a HIP runtime call failed */
    DEMAG_EUNSUPPORTED = -4,/* shape beyond what the kernels handle */
    DEMAG_ESTATE = -5       /* plan busy on another stream, or wrong object state */
} demag_status;

/* Create a plan for an nx x ny x nz grid of dx x dy x dz cells (metres, > 0,
 * finite).  Computes the tensor N in FP64 on the current device and stores
 * the real, symmetric spectrum of N on its non-redundant octant in `dtype`
 * (Sec. 4: the constants depend on the geometry only and are computed once).
 * Runs on `setup_stream` and synchronises it.  Padded length per axis:
 * 2L, L the smallest 2^a 3^b 5^c >= n; 2L <= 4096 per axis, else
 * DEMAG_EUNSUPPORTED.  Along z the fused Z pass runs on the register kernels
 * for powers of two up to 4096 (a pencil and its mirror per workgroup up to
 * 2048, one pencil per workgroup at 4096) and, in FP32, 3 * 2^a up to 3072;
 * other lengths up to 1365 (six pencils in one workgroup); longer z lengths
 * are DEMAG_EUNSUPPORTED (put the longest axis along x or y).  The register
 * Z kernels address a spectrum component (ny' Kx nz complex values, ny' the
 * padded y length, Kx = nx' / 2 + 1, nx' the padded x length) with 32-bit
 * offsets: above 4 GB per component the generic kernel is used, so z lengths
 * above 1365 need smaller x-y extents.  Device memory
 * bounds the grid: about 96 bytes per cell for an FP32 plan (192 in FP64)
 * plus about 240 bytes per cell of FP64 set-up scratch while this call runs
 * (DEMAG_ENOMEM when it cannot be allocated).  *out receives the plan (caller destroys it
 * once). */
int demag_plan_create(demag_plan_t* out, int nx, int ny, int nz, double dx, double dy, double dz,
                      demag_dtype dtype, void* setup_stream);

/* Tensor-setup options; the spectrum is recomputed at once (synchronous).
 *  "far_cut" (also "far_cutoff"): offsets with |o (.) d| / max(d) >= far_cut
 *             (cell-size units) use the moment series of the dipole kernel
 *             (default 40; 0 < v).
 *  "fg_cut" (also "fg_cutoff"):  offsets with Chebyshev distance <= fg_cut use the Newell f/g
 *             closed form (default 1; integer >= 0); the rest of the near field
 *             uses Gauss-Legendre quadrature of the cell-average integral.
 *  "generic_kernels": 1 runs every pass on the generic (any-length)
 *             kernels, 0 (default) uses the compile-time power-of-two kernels
 *             on the axes whose padded length allows them; resets the launch
 *             shapes to their defaults.  DEMAG_EUNSUPPORTED (plan unchanged)
 *             when the generic Z pass cannot hold the padded z length.
 *  "pass_timing": K > 0 records HIP events around every pass of the next
 *             field evaluations on their own stream (a ring of K evaluations;
 *             0 turns it off; evaluations of the energy alone are not
 *             recorded); read the averages with demag_plan_pass_times.
 *  "radix_schedule": S = 0, 1 or 2 sets the radix schedule of every pass on
 *             the register kernels whose length has schedule S (the others
 *             take 0); launch shapes are kept.  The schedules of a length
 *             2^a = 8^k r (same number of stages each): 0 = 8, ..., 8, r;
 *             1 = 8, r, 8, ..., 8 (k >= 2, r = 2 or 4); 2 = 8, ..., 8, 4, 4
 *             (k >= 2, r = 2).  demag_autotune searches them per pass.
 *  "lowrank_scratch": byte cap of the low-rank dense-expansion scratch
 *             (default 256 MB; at least one z slice is always held).
 *  "tg_mode12": 1 (default) runs the first two mode products of the dense
 *             tensor grid as one fused FP32 kernel on the matrix cores where
 *             it applies (FP32 plans with ny <= 512; otherwise, and in FP64,
 *             library GEMMs): half the scratch (R N values instead of 2 R N)
 *             and about 0.96x the evaluation time of the GEMMs at
 *             256 x 256 x 64; 0 as two library GEMMs (rocBLAS).  A prepared
 *             tensor grid is rebuilt (synchronously) for the chosen path. */
int demag_plan_set_option(demag_plan_t plan, const char* key, double value);
int demag_plan_destroy(demag_plan_t plan);

/* Plan facts, written to info[0..15] (host):
 * nx ny nz Px Py Pz Kx dtype scratch_bytes tensor_bytes setup_us 0... */
int demag_plan_info(demag_plan_t plan, int64_t* info);

/* H = -Ms N * m  (Sec. 3.1 eq. (demag)); asynchronous on `stream`.
 * demag_field, demag_field_adjoint, demag_field_energy and
 * demag_energy_async record only kernels (no memset, no synchronisation) and
 * may be captured into a HIP graph by stream capture: while `stream` is
 * capturing, the plan's busy tracking and pass timing are skipped; a replay
 * reads the buffers given at capture.  Replays of such a graph are outside the
 * plan's busy tracking (DEMAG_ESTATE cannot see them): they use the plan's
 * scratch like any call, so the caller must order them against every other
 * call on the plan and must not run two at once. */
int demag_field(demag_plan_t plan, const void* m, double Ms, void* H, void* stream);

/* Adjoint (transpose) of m -> H applied to a cotangent gH:
 * gm (+)= A^T gH with A = -Ms N * (restricted to the grid).  N(o) is symmetric
 * and even under o -> -o, so A^T = A and the same passes run on gH.
 * accumulate = 0 overwrites gm, 1 adds to it.  Asynchronous. */
int demag_field_adjoint(demag_plan_t plan, const void* gH, double Ms, void* gm, int accumulate, void* stream);

/* Field and energy in one evaluation: H (may be NULL: energy only) and
 * E_dev, a DEVICE double receiving E = -(mu0/2) Ms V sum m.H (Sec. 2).
 * FP32 plans form m.H in FP32 and accumulate in FP64.  With H == NULL and the
 * register kernel on the Z pass (power-of-two padded z up to 4096; 3 * 2^a in
 * FP32), the field is not formed: after the forward X and Y passes the Z pass
 * transforms m and sums Re(M^H Nhat M) over the spectrum (Parseval's identity
 * on the padded grid, where m is zero off the grid equals sum m.H), three
 * passes instead of five; the result agrees with the field's m.H sum to
 * rounding (FP32 products, FP64 sums).  Asynchronous. */
int demag_field_energy(demag_plan_t plan, const void* m, double Ms, void* H, double* E_dev, void* stream);

/* Gradient of the energy of Sec. 2 with respect to m, from the field H that
 * demag_field / demag_field_energy returned for that m: E is quadratic in m
 * and the grid operator is symmetric, so dE/dm = -mu0 Ms V H (no further
 * convolution).  gm (+)= gE * dE/dm, gE = *gE_dev (a DEVICE double, the
 * cotangent of E; NULL means 1); accumulate = 0 overwrites gm, 1 adds to it.
 * H and gm: device [3][nz][ny][nx] in the plan precision, distinct buffers.
 * Asynchronous. */
int demag_energy_gradient(demag_plan_t plan, const void* H, double Ms, const double* gE_dev, void* gm, int accumulate,
                          void* stream);

/* Energy only (demag_field_energy with H == NULL), result to a HOST double;
 * synchronises `stream`. */
int demag_energy(demag_plan_t plan, const void* m, double Ms, double* E_host, void* stream);
/* Energy only (demag_field_energy with H == NULL), result to a DEVICE double;
 * asynchronous. */
int demag_energy_async(demag_plan_t plan, const void* m, double Ms, double* E_dev, void* stream);

/* Copy the stored tensor spectrum (plan precision) to HOST memory `out`,
 * layout [Py/2+1][6][Kx][Pz/2+1], components xx yy zz xy xz yz, with the
 * factor -1/(Px Py Pz) folded in (device storage keeps the six components of
 * a frequency side by side; the copy reorders).  Synchronous. */
int demag_plan_spectrum(demag_plan_t plan, void* out);

/* Recompute the FP64 real-space tensor octant N(o), o in [0,n), to HOST
 * memory `out` [6][nz][ny][nx] (components xx yy zz xy xz yz).  Synchronous. */
int demag_plan_tensor(demag_plan_t plan, double* out);

/* ---- Scalar-potential method (SP), Sec. 3.1 eqs. (scpot), (convolution),
 * (field) -------------------------------------------------------------------
 * phi = Ms S * m on the cell centres, S_a(R) the potential at R of a cell
 * magnetized along axis a with unit magnetization (two charged faces), then
 * H = -grad phi by finite differences: central inside, second-order one-sided
 * on the grid's faces (first order with two cells along an axis, zero with
 * one).  Same plan, buffers, layouts and units as the DM calls.
 *
 * demag_sp_prepare builds the kernel spectrum (FP64 setup; distance bands as
 * for the tensor; Im of the transform of the odd kernel on the octant with
 * h/(Px Py Pz) folded in) once; synchronous.  DEMAG_EUNSUPPORTED unless the
 * padded z length is 2^a or 3 * 2^a (FP64: 2^a); idempotent. */
int demag_sp_prepare(demag_plan_t plan, void* stream);
/* H (device, [3][nz][ny][nx]) for m; asynchronous on `stream`.  DEMAG_ESTATE
 * before demag_sp_prepare.  m and H must not alias. */
int demag_sp_field(demag_plan_t plan, const void* m, double Ms, void* H, void* stream);
/* The same and the energy -(mu0/2) Ms V sum m.H into the device double
 * *E_dev; H may be NULL (energy only). */
int demag_sp_field_energy(demag_plan_t plan, const void* m, double Ms, void* H, double* E_dev, void* stream);
/* Recompute the FP64 kernel octant S_a(o), o in [0,n), in metres (potential
 * per unit magnetization), to HOST memory `out` [3][nz][ny][nx].  Synchronous. */
int demag_sp_kernel(demag_plan_t plan, double* out);

/* ---- LLG driver, Sec. 2 (the LLG equation) ------------------------------------
 * nsteps explicit Heun steps of
 *     m_t = -g (m x H) - alpha g (m x (m x H)),  g = gamma / (1 + alpha^2),
 * H = H_demag(m) (this plan, Ms) + (hx, hy, hz) (uniform, A/m), gamma > 0 in
 * m/(A s) (2.2128e5 for the free electron), dt in s; each step renormalises
 * the predictor and the result to unit length.  m (device, [3][nz][ny][nx],
 * plan dtype) is updated in place; `work` is caller-owned device scratch of
 * 9 nx ny nz values of the plan dtype (H, k1, predictor); nothing is
 * allocated.  Asynchronous on `stream`. */
int demag_llg_heun(demag_plan_t plan, void* m, double Ms, double alpha, double gamma, double hx, double hy, double hz,
                   double dt, int nsteps, void* work, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * steps as demag_llg_heun with the 9 nx ny nz-value workspace taken from a
 * static device array of the library instead of a `work` argument.  The array
 * holds DEMAG_LLG_STATIC_SCRATCH_BYTES (64 MiB) on every GPU the library runs
 * on, from the library's load until the process ends; a plan whose workspace
 * would exceed it (9 N sizeof(real) bytes: N up to 1,864,135 cells in FP32,
 * 932,067 in FP64) gets DEMAG_EINVAL.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).  All calls on one GPU
 * share the array and it keeps the last call's contents (none need to start at
 * zero); calls that overlap on one GPU -- on different streams, or replays of
 * graphs that captured it -- race and must be ordered by the caller.
 * Asynchronous on `stream`. */
#define DEMAG_LLG_STATIC_SCRATCH_BYTES (64ull << 20)
int demag_llg_heun_static(demag_plan_t plan, void* m, double Ms, double alpha, double gamma, double hx, double hy,
                          double hz, double dt, int nsteps, void* stream);

/* ---- Tensor-grid method (TG, dense), Sec. 3.2 eqs. (transform), (gausspot),
 * (sumpot), (Dmat), (gs) -----------------------------------------------------
 * The same potential phi as the SP calls (exact for cell-wise constant m up
 * to the quadrature), computed as the block-CP sum of eq. (sumpot): Sinc
 * quadrature of the Gaussian representation of 1/r^3 in t = log(tau) (step
 * 0.25 in FP32, 0.15 in FP64; relative kernel error about 2e-7 and 6e-13 on
 * distances from the smallest cell edge to the body diagonal), closed-form
 * Gaussian matrices per axis and node; H = -grad phi with the SP difference
 * stencils.  In FP32 (ny <= 512, option "tg_mode12" 1, the default) the
 * first two mode products of every node and z-plane, D_1 M(:,:,k) D_2^T, run
 * as one fused kernel on the matrix cores that keeps the intermediate on chip
 * and skips the 16-column groups of the banded Gaussian matrices that are
 * exactly zero (finite m: the same sums); the third mode product and the node
 * sum are one GEMM (rocBLAS).  Otherwise all three mode products are GEMMs
 * (rocBLAS).
 *
 * demag_tg_prepare builds nodes and matrices and allocates the scratch (R N
 * values on the fused path, 2 R N on the library path; R nodes, about 75 in
 * FP32 and 125 in FP64 at 256 x 256 x 64); in FP32 it also times the rocBLAS
 * solutions of the library GEMM shapes on these buffers and keeps, per
 * shape, the fastest whose result agrees with rocBLAS's default to 1e-5
 * (preparation takes about 2 s at 256 x 256 x 64; the plan's spectrum scratch
 * is overwritten); synchronous; idempotent; DEMAG_ENOMEM if the scratch does
 * not fit. */
int demag_tg_prepare(demag_plan_t plan, void* stream);
/* H (device, [3][nz][ny][nx]) for m; asynchronous.  DEMAG_ESTATE before
 * demag_tg_prepare. */
int demag_tg_field(demag_plan_t plan, const void* m, double Ms, void* H, void* stream);
/* The same and the energy into the device double *E_dev; H may be NULL. */
int demag_tg_field_energy(demag_plan_t plan, const void* m, double Ms, void* H, double* E_dev, void* stream);
/* out[0] = R (nodes), out[1] = scratch bytes, out[2] = flops per evaluation. */
int demag_tg_info(demag_plan_t plan, int64_t* out);
/* out[0] = 1 when the first two mode products run fused (see above), 0 for
 * the library GEMMs; out[1] = the mode-product flops one evaluation issues
 * (out[2] of demag_tg_info less the skipped zero blocks).  DEMAG_ESTATE before
 * demag_tg_prepare. */
int demag_tg_path(demag_plan_t plan, int64_t* out);
/* Host only: the Sinc nodes tau_l and weights w_l (w_l = step tau_l^3 /
 * pi^(3/2), so that 1/r^3 ~ 4 pi sum_l w_l exp(-tau_l^2 r^2)) for
 * distances in [rmin, rmax]; returns R (the count) and fills tau, w when both
 * are non-NULL and cap >= R; negative status on bad arguments. */
int demag_tg_sinc_nodes(double rmin, double rmax, double step, double* tau, double* w, int cap);

/* ---- Tensor-grid method on low-rank magnetization, Sec. 3.2 (Low-Rank
 * Magnetization), Tables 1 and 2 (TG Tucker / TG CP rows), Appendix eqs. (CP)
 * and (tucker) ------------------------------------------------------------------
 * Each component M_p (p = x, y, z) is given compressed, with one rank r for
 * every mode:
 *   DEMAG_TUCKER: M_p = C_p x_1 U_1^p x_2 U_2^p x_3 U_3^p, core C_p r x r x r;
 *   DEMAG_CP:     M_p(i1,i2,i3) = sum_s lambda_p(s) U_1^p(i1,s) U_2^p(i2,s) U_3^p(i3,s).
 * Tensor index (i1, i2, i3) = cell (x, y, z).  The potential and the field
 * are block-CP tensors on the same grid as the dense TG calls (same Sinc
 * nodes, same difference stencils), computed on the factors only:
 *   Phi   = sum_{p,l} alpha c_l  C_p x_1 F_1^{pl} x_2 F_2^{pl} x_3 F_3^{pl},
 *   H_a   = the same with F_a replaced by G_a^{pl} (a = x, y, z),
 *   F_q^{pl} = D_q^{l,p} U_q^p  (the Gaussian matrix of node l, odd kind when
 *   q = p), G_q^{pl} = -delta_q F_q^{pl} (difference along axis q, 1/m),
 *   alpha = Ms h_max (h_max the largest cell edge, m), c_l = w_l of
 *   demag_tg_sinc_nodes for this plan's nodes;
 * the energy -(mu0/2) Ms V sum_a <M_a, H_a> from inner products of the
 * compressed tensors (no dense tensor is formed); the dense field on the grid
 * only when H is given.
 *
 * demag_tg_lowrank_prepare builds the nodes and the stacked Gaussian matrices
 * of the three axes (4 R (n1^2 + n2^2 + n3^2) values); synchronous;
 * idempotent. */
#define DEMAG_TUCKER 0
#define DEMAG_CP 1
#define DEMAG_TUCKER_MAX_RANK 16
#define DEMAG_CP_MAX_RANK 64
int demag_tg_lowrank_prepare(demag_plan_t plan, void* stream);
/* One evaluation; asynchronous on `stream`.  All pointers are device memory
 * of the plan dtype (E_dev: double), caller-owned:
 *   core  Tucker: [3][r][r][r] (s1 fastest), C_p(s1,s2,s3) at
 *         p r^3 + s1 + r s2 + r^2 s3;  CP: lambda [3][r];
 *   U     the three axis blocks one after another; block q (n_q x 3r,
 *         column-major) holds U_q^x, U_q^y, U_q^z side by side: U_q^p(i, s) at
 *         offset(q) + i + n_q (p r + s), offset(q) = 3 r (n_1 + .. + n_{q-1});
 *   FG    output, the compressed potential and field: block q
 *         (2 n_q x 3 R r, column-major) at 6 R r (n_1 + .. + n_{q-1}); column
 *         (p R + l) r + s holds F_q^{pl}(:, s) in rows [0, n_q) and
 *         G_q^{pl}(:, s) in rows [n_q, 2 n_q);
 *   H     optional dense field [3][nz][ny][nx] (NULL: not formed);
 *   E_dev optional energy (one double, J).
 * rank in [1, DEMAG_TUCKER_MAX_RANK] (Tucker) or [1, DEMAG_CP_MAX_RANK] (CP),
 * else DEMAG_EINVAL; DEMAG_ESTATE before demag_tg_lowrank_prepare.  The dense
 * expansion uses plan-owned scratch (within the "lowrank_scratch" cap, at
 * least one z slice; allocated on first use and grown when a later call needs
 * more), taking as many z slices per GEMM as fit. */
int demag_tg_lowrank_field(demag_plan_t plan, int format, int rank, const void* core, const void* U, double Ms,
                           void* FG, void* H, double* E_dev, void* stream);
/* out[0] = R (nodes), out[1] = bytes of the stacked Gaussian matrices and
 * scratch held, out[2] = alpha / Ms = h_max in metres. */
int demag_tg_lowrank_info(demag_plan_t plan, int64_t* out);
/* Alternating least squares compression of a dense magnetization m (device,
 * [3][nz][ny][nx], plan dtype) into the format above, each component on its
 * own, from the caller's initial factors (Sec. 3.2: ALS from random initial
 * guesses), `sweeps` >= 1 sweeps over the three modes:
 *   DEMAG_TUCKER: higher-order orthogonal iteration; per mode the leading
 *     rank-r left singular subspace of Y_(n) = (X x_{m != n} U_m^T)_(n) by one
 *     step of orthogonal iteration from the current factor (Cholesky QR,
 *     twice); the factors are orthonormalised first; afterwards
 *     core = X x_1 U1^T x_2 U2^T x_3 U3^T.  rank <= min(nx, ny, nz).
 *   DEMAG_CP: CP-ALS; per mode U_n = X_(n) (U_c (.) U_b) V^-1 with
 *     V = (U_b^T U_b) * (U_c^T U_c), then columns normalised to unit 2-norm,
 *     core = the weights lambda.  The initial factor of axis x is not read.
 * U (in: initial factors, out: result) and core use the layouts of
 * demag_tg_lowrank_field.  *relerr (host, may be NULL) receives eq. (relr)
 * of the result, from the factor identities in FP64 (Tucker:
 * ||X||^2 - ||C||^2; CP: ||X||^2 - 2 <X, X^> + ||X^||^2), so values below
 * about 1e-7 (FP64) or 1e-3 (FP32) are rounding-limited.  Allocates its
 * scratch for the call and synchronises `stream`.  DEMAG_EINVAL for a rank
 * outside the format's range, sweeps < 1, or a Gram matrix that is not
 * positive definite (a rank above the numerical rank of the data or of the
 * initial guess). */
int demag_lowrank_compress(demag_plan_t plan, int format, int rank, int sweeps, const void* m, void* core, void* U,
                           double* relerr, void* stream);

/* Text description of the launch shape of every pass (kernel family, threads,
 * tiles) into `buf` (len bytes, NUL-terminated); DEMAG_EINVAL if too small. */
int demag_plan_describe(demag_plan_t plan, char* buf, int len);

/* Average duration in ms of each pass over the evaluations recorded since the
 * last call (at most the ring size), from the events of "pass_timing":
 * ms[0..5] = X-R2C, Y, fused Z, Y-inverse, X-C2R, energy reduction (0 when the
 * evaluations had no energy).  *count = evaluations averaged.  Synchronises
 * the device and empties the ring. */
int demag_plan_pass_times(demag_plan_t plan, double* ms, int64_t* count);

/* Time the candidate launch shapes and radix schedules of every pass on this
 * plan's buffers, keep the fastest, and update the cache file named by
 * $DEMAG_AUTOTUNE_CACHE (if set).  Synchronous; clobbers the plan's scratch.
 * On failure the plan keeps the launch shapes it had. */
int demag_autotune(demag_plan_t plan, void* stream);

/* Batch: `count` independent field evaluations H_i = -Ms N_i * m_i (one per
 * plan; plans may have different grids and cells but one precision) with their
 * m / H device buffers.  Plans of equal geometry form a group that runs each
 * pass as one launch over all its members (and uses the first member's
 * tensor spectrum and launch shapes); all groups' launches are recorded once
 * into a HIP graph, replayed by demag_batch_launch (asynchronous), with the
 * groups spread over one forked stream per hardware queue ($GPU_MAX_HW_QUEUES,
 * default 4), largest first onto the least loaded stream.  The batch
 * references (does not own) plans and buffers; all must stay alive and
 * unchanged until demag_batch_destroy.  Plans must be distinct (each owns the
 * scratch its evaluation uses).  demag_batch_create synchronises `stream`. */
int demag_batch_create(demag_batch_t* out, const demag_plan_t* plans, int count, const void* const* m,
                       void* const* H, double Ms, void* stream);
/* Time the candidate launch shapes of every pass of every group on the
 * group's own buffers (each candidate launch covering all members), keep the
 * fastest per group, then spread the groups (by their measured times) over
 * 1 .. (hardware queues) forked streams, time whole replays of each and keep
 * the fastest graph.  Synchronous; overwrites the
 * members' H and scratch (the next demag_batch_launch recomputes them); plans'
 * own launch shapes are unchanged.  Groups then may run other kernels than
 * single-plan calls, so members agree with demag_field to rounding only. */
int demag_batch_autotune(demag_batch_t batch, void* stream);
int demag_batch_launch(demag_batch_t batch, void* stream);
/* out[0] = members, out[1] = geometry groups (one launch per pass each),
 * out[2] = streams the recorded graph spreads the groups over (host). */
int demag_batch_info(demag_batch_t batch, int64_t* out);
int demag_batch_destroy(demag_batch_t batch);

/* Test hook (environment): while DEMAG_FAIL_ALLOC_AT=k is set, the k-th
 * device allocation of the library counted since the value last changed
 * fails as out of memory (DEMAG_ENOMEM), so that callers can exercise every
 * failure path of plan creation and set-up; unset, allocations are plain. */

/* Last error message of the calling thread ("" if none). */
const char* demag_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DEMAG_H */
