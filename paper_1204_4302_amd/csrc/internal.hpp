// Internal declarations shared by the pass kernels, the tensor setup and the
// plan runtime (not part of the public C ABI).
#pragma once
#include <vector>
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"

namespace demag {

constexpr int kMaxThreads = 256;  // workgroup size bound of every pass kernel

// Launch shape of one pass: threads per workgroup, elements per thread per
// FFT stage (compile-time instance), and two tile extents whose meaning
// depends on the pass:
//   X fwd / X inv : t0 = rows per workgroup (Ty)
//   Y fwd / Y inv : t0 = kx per workgroup (Tx), t1 = z per workgroup (Tz)
//   Z conv / fwd  : t0 = kx per workgroup (Tx)
//
// p2 = 1 selects the compile-time register kernels (passes_p2.hip; lengths
// 2^a and 3 * 2^a); then
// t0, t1 are log2 of the tile extents (X: Ty; Y: Tx, Tz) and the workgroup
// size follows from them (pencils x threads per pencil); for the Z pass t0 is
// log2 of the consecutive ky' rows of one kx per tile and t1 the rows per
// group (2: a row with its mirror, 1: single rows).
struct LaunchCfg {
    int threads = 256;
    int E = 16;
    int t0 = 1;
    int t1 = 1;
    int p2 = 0;
    int sched = 0;  // p2: radix schedule of the pass's length (p2::num_schedules); one per axis
};

// Several grids of one shape in one launch: per-grid device pointers of the
// pass's input and output (arrays of `count` pointers in device memory).
// in == nullptr: a single grid, whose pointers are the launcher's arguments.
struct BatchIO {
    const void* const* in = nullptr;
    void* const* out = nullptr;
    int count = 1;
};

template <typename T>
hipError_t launch_x_fwd(const LaunchCfg&, hipStream_t, const T* in, cx<T>* out, int Xin, int Yr, int Zr, int Kx,
                        int C, const FftPlanDev&, const cx<T>* tw, const BatchIO& bio = BatchIO());
template <typename T>
hipError_t launch_y_fwd(const LaunchCfg&, hipStream_t, const cx<T>* in, cx<T>* out, int Yin, int Zr, int Kx, int Zs,
                        int C, const FftPlanDev&, const cx<T>* tw, const BatchIO& bio = BatchIO());
template <typename T>
hipError_t launch_z_conv(const LaunchCfg&, hipStream_t, cx<T>* B2, const T* nhat, T Ms, int nz, int Py, int Kx,
                         const FftPlanDev&, const cx<T>* tw, const BatchIO& bio = BatchIO());
template <typename T>
hipError_t launch_z_fwd(const LaunchCfg&, hipStream_t, cx<T>* B2, int Py, int Kx, const FftPlanDev&,
                        const cx<T>* tw);
template <typename T>
hipError_t launch_y_inv(const LaunchCfg&, hipStream_t, const cx<T>* in, cx<T>* out, int ny, int nz, int Kx, int C,
                        const FftPlanDev&, const cx<T>* tw, const BatchIO& bio = BatchIO());
template <typename T>
hipError_t launch_x_inv(const LaunchCfg&, hipStream_t, const cx<T>* in, T* out, const T* m, double* partials, int nx,
                        int ny, int nz, int Kx, int C, int accumulate, const FftPlanDev&, const cx<T>* tw,
                        const BatchIO& bio = BatchIO());
hipError_t launch_energy_reduce(hipStream_t, const double* partials, int n, double scale, double* out);
// gm (+)= gE c H over n values (gE: device scalar, NULL = 1): the energy gradient.
template <typename T>
hipError_t launch_energy_grad(hipStream_t, size_t n, const T* H, const double* gE, double c, T* gm, int accumulate);

// lengths 2^a and 3 * 2^a (2 <= P <= 4096): compile-time instances
// compile-time register kernels ("p2" family): lengths 2^a and 3 * 2^a up to
// 4096; the fused Z pass in FP64 only for 2^a
bool p2_supported(int P);
bool p2_z_supported(int P, size_t cbytes);
int p2_threads_per_pencil(int P);
int p2_slab_elems(int P);
// The X and Y passes stage twiddle tables of at most this many bytes in LDS
// per workgroup (larger ones would cost workgroups per CU); the dynamic LDS of
// such a launch is its slabs plus p2_twiddle_lds_bytes.  The fused Z pass loads
// its twiddles once per thread for six transforms and reads them from memory.
constexpr size_t kP2TwLdsMax = 8192;
size_t p2_twiddle_lds_bytes(int P, size_t cbytes);
size_t p2_z_twiddle_lds_bytes(int P, size_t cbytes);  // extra LDS of a fused Z launch
// dynamic LDS of a fused Z launch: slabs, twiddle table, tensor staging
size_t p2_z_lds_bytes(int P, int rows, int lgTx, size_t cbytes);
extern int kXcds;                       // XCDs of the device: 8 on MI355X; 1 turns the swizzle off
int p2_max_threads(int P);              // X and Y passes: 1024 (2^a) or 512 (3 * 2^a)
int p2_num_schedules(int P);            // radix schedules of a register-kernel length (0: not one)
constexpr int kP2MaxThreadsZ = 512;     // fused Z pass (three pencils per thread)
// The register-kernel Z pass reaches B2 and the tensor octant through 32-bit
// buffer offsets: one B2 component and the whole octant must each span fewer
// bytes than this (larger shapes run the generic Z pass).
constexpr size_t kP2BufLimit = 0xFFFFF000u;

// One-thread-per-element launches over `total` elements in pieces of at most
// kLaunchPiece work-items (a 1-D grid holds fewer than 2^32 work-items, and
// set-up arrays of a large padded grid hold more elements): launch(base,
// blocks) enqueues the piece starting at element `base`.
constexpr size_t kLaunchPiece = size_t(1) << 30;
template <typename F>
hipError_t launch_pieces(size_t total, unsigned threads, F&& launch) {
    for (size_t base = 0; base < total; base += kLaunchPiece) {
        const size_t n = total - base < kLaunchPiece ? total - base : kLaunchPiece;
        launch(base, (unsigned)((n + threads - 1) / threads));
        if (hipError_t e = hipGetLastError()) return e;
    }
    return hipSuccess;
}
// The p2 kernels read their twiddles from a thread-major table: the values of
// tw (exp(-2 pi i t / P), t < P) rearranged so that the threads of one pencil
// load consecutive entries.  Empty if P is not a supported power of two.
// (the table of radix schedule `sched`; every launcher below takes the
// schedule of its length and the table built for it)
template <typename T>
std::vector<cx<T>> p2_thread_twiddles(int P, int sched, const std::vector<cx<T>>& tw);
template <typename T>
hipError_t launch_x_fwd_p2(int lgTy, int sched, hipStream_t, const T* in, cx<T>* out, int nx, int ny, int nz, int C,
                           int P, const cx<T>* twt, const BatchIO& bio = BatchIO());
template <typename T>
hipError_t launch_x_inv_p2(int lgTy, int sched, hipStream_t, const cx<T>* in, T* out, const T* m, double* partials,
                           int nx, int ny, int nz, int C, int accumulate, int P, const cx<T>* twt,
                           const BatchIO& bio = BatchIO());
template <typename T>
hipError_t launch_y_fwd_p2(int lgTz, int lgTx, int sched, hipStream_t, const cx<T>* in, cx<T>* out, int ny, int nz,
                           int Kx, int C, int P, const cx<T>* twt, const BatchIO& bio = BatchIO());
template <typename T>
hipError_t launch_y_inv_p2(int lgTz, int lgTx, int sched, hipStream_t, const cx<T>* in, cx<T>* out, int ny, int nz,
                           int Kx, int C, int P, const cx<T>* twt, const BatchIO& bio = BatchIO());
template <typename T>
// rows: 2 = a row ky' and its mirror Py - ky' per workgroup (lengths whose
// pair fits kP2MaxThreadsZ), 1 = one row per workgroup (the others)
hipError_t launch_z_conv_p2(int lgTx, int rows, int sched, hipStream_t, cx<T>* B2, const T* nhat, T Ms, int nz,
                            int Py, int Kx, int P, const cx<T>* twt, const BatchIO& bio = BatchIO());

// scalar-potential method: fused Z pass (3 components in, Ms phi out in
// component 0 of B2), register-kernel lengths only
template <typename T>
hipError_t launch_z_energy_p2(int lgTx, int rows, int sched, hipStream_t, cx<T>* B2, const T* nhat, int nz, int Py,
                              int Kx, int P, const cx<T>* twt, double* epart, int* nparts);
template <typename T>
hipError_t launch_z_sp_p2(int lgTx, int rows, int sched, hipStream_t, cx<T>* B2, const T* shat, T Ms, int nz, int Py,
                          int Kx, int P, const cx<T>* twt);

// ---- tensor setup (FP64) ----------------------------------------------------
struct TensorBands {
    double far_cut = 40.0;  // rho = |o (.) d| / max d >= far_cut -> moment series
    int fg_cut = 1;         // Chebyshev distance <= fg_cut -> Newell f/g
    int gl_q = 12;          // Gauss-Legendre nodes per panel (mid band)
    int max_panels = 16;    // panels per half-axis cap (mid band)
};

// Octant N(o), o in [0,n) per axis, written [6][nz][ny][nx] (FP64, device).
hipError_t launch_tensor_octant(hipStream_t, int nx, int ny, int nz, const double dt[3], const TensorBands&,
                                const double* gl_x_dev, const double* gl_w_dev, double* Noct);
// Mirror component `comp` of the octant into the P-periodic real array
// A [Pz][Py][Px] (zero in the padding gap), with the parity signs.
hipError_t launch_tensor_embed(hipStream_t, int comp, int nx, int ny, int nz, int Px, int Py, int Pz,
                               const double* Noct, double* A);
// Take the real part of the FFT'd component (B2 [Kx][Py][Pz], complex FP64)
// on the octant ky <= Ly, kz <= Lz, scale, cast to T into
// nhat [Kx][Ly+1][Lz+1][6] (the six components of a frequency side by side).
template <typename T>
hipError_t launch_tensor_extract(hipStream_t, int comp, int Px, int Py, int Pz, int Kx, double scale,
                                 const cx<double>* B2, T* nhat);

// ---- scalar-potential method (sp.hip) ----------------------------------------
// Kernel octant S_a(o), o in [0,n) per axis, [3][nz][ny][nx] (FP64, device),
// with the same distance bands as the tensor.
hipError_t launch_sp_kernel_octant(hipStream_t, int nx, int ny, int nz, const double dt[3], const TensorBands&,
                                   const double* gl_x_dev, const double* gl_w_dev, double* Soct);
// Component a mirrored into A [Pz][Py][Px] (odd in axis a, zero in the gap).
hipError_t launch_sp_embed(hipStream_t, int a, int nx, int ny, int nz, int Px, int Py, int Pz, const double* Soct,
                           double* A);
// Im of the FFT'd component on the octant, scaled, into shat [Kx][Ly+1][3][Lz+1].
template <typename T>
hipError_t launch_sp_extract(hipStream_t, int a, int Py, int Pz, int Kx, double scale, const cx<double>* B2,
                             T* shat);
// ---- tensor-grid method (tg.hip) ----------------------------------------------
// Sinc nodes tau_l and weights h tau_l^3 / pi^(3/2) for 1/r^3 on [rmin, rmax]
// (reduced units), step h; returns R (or -1 for bad arguments).
int tg_sinc_nodes(double rmin, double rmax, double h, std::vector<double>& tau, std::vector<double>& w);
template <typename T>
hipError_t launch_tg_axis(hipStream_t, int n, double d, int R, const double* tau, T* E, T* O);
template <typename T>
hipError_t launch_tg_stack3(hipStream_t, int n3, int R, const double* c, const T* D3, T* B3);
template <typename T>
int tg_potential(void* handle, hipStream_t st, int n1, int n2, int n3, int R, const T* m, const T* D1E,
                 const T* D1O, const T* const* D2p[3], const T* const* Y1k, T* const* Y2k, const T* const B3[3], T* Y1,
                 T* Y2, T* phi, double alpha, int sol1 = 0, int sol2 = 0, int sol3 = 0);
// rocBLAS solutions for the three GEMMs of tg_potential, chosen by timing on
// the given buffers (Mp: a mode-1 input; Y1, Y2 (behind Y2k) and phi are
// overwritten); 0 (the default) for FP64 or when no faster solution agrees
// with the default's result.  With Y1 NULL only the mode-3 GEMM is tuned.
template <typename T>
int tg_tune(void* handle, hipStream_t st, int n1, int n2, int n3, int R, const T* D1, const T* Mp, T* Y1,
            const T* const* Y1k, const T* const* D2k, T* const* Y2k, T* Y2, const T* B3, T* phi, int* sol1, int* sol2,
            int* sol3);

// ---- fused first and second TG mode products, FP32 (tg_fused.hip) -------------
// Y2[l](:,:,k) = D1[l] M(:,:,k) D2[l]^T for every node and plane in one launch
// (the intermediate stays in LDS); D1, D2 [R][tg_tiled_floats(n)] in the tiled
// operand order of launch_tg_axis_tiled, M [n3][n2][n1], Y2 [R][n3][n2][n1];
// lo/hi per matrix [R][tg_band_blocks(n)] from launch_tg_band.
constexpr int kTgMode12MaxN2 = 512;  // LDS holds 64 rows of the intermediate
bool tg_mode12_fits(int n2);
int tg_band_blocks(int n);
size_t tg_tiled_floats(int n);  // per node: ceil(n/16)^2 tiles of 256 values
// the Gaussian matrices of one axis for every node in the tiled operand order
hipError_t launch_tg_axis_tiled(hipStream_t st, int n, double d, int R, const double* tau, float* E, float* O);
// allows the launch's dynamic LDS for n2 (once, before the first launch)
hipError_t tg_mode12_init(int n2);
// columns [lo, hi] holding the nonzero entries of each block of 64 rows (hi -1: none)
hipError_t launch_tg_band(hipStream_t st, int n, int R, const float* D, int* lo, int* hi);
hipError_t launch_tg_mode12(hipStream_t st, int n1, int n2, int n3, int R, const float* D1, const int* lo1,
                            const int* hi1, const float* M, const float* D2, const int* lo2, const int* hi2, float* Y2);
// Operands of the fused chain per component p (the odd matrix on axis p).
struct TGFused {
    const float* D1[3];
    const float* D2[3];
    const int *lo1[3], *hi1[3], *lo2[3], *hi2[3];
};
// phi by the fused mode-1/2 kernel and the mode-3 GEMM (rocBLAS solution sol3)
int tg_potential_fused(void* handle, hipStream_t st, int n1, int n2, int n3, int R, const float* m, const TGFused& f,
                       const float* const B3[3], float* Y2, float* phi, double alpha, int sol3);

// ---- low-rank tensor grid (lowrank.hip) ---------------------------------------
// Stacked Gaussian matrices of one axis for every node: [R][2n x n] column-major,
// rows [0, n) D, rows [n, 2n) -delta D (spacing h).
template <typename T>
hipError_t launch_lr_axis(hipStream_t, int n, double d, double h, int R, const double* tau, T* E, T* O);
// Factors FG, then (partials != null) 9 R energy partials via 27 R r^2 Gram
// values in gram, then (H != null) the dense field using W (w_elems values of
// scratch).  Returns 0 or a negative code.
// FP32 plans keep the Gaussian matrices swizzled for the MFMA factor product
// (R lr_swizzled_elems(n) values per kind and axis, no difference rows); FP64
// plans keep the stacked [D; -delta D] matrices.
hipError_t launch_lr_axis_sw(hipStream_t, int n, double d, int R, const double* tau, float* E, float* O);
size_t lr_swizzled_elems(int n);
template <typename T>
int lr_evaluate(void* handle, hipStream_t st, const int n[3], const double h[3], int R, int r, bool tucker,
                const T* core, const T* U, const T* const DE[3], const T* const DO[3], const double* c, double alpha,
                T* FG, double* partials, double* gram, T* H, T* W, size_t w_elems);

// ---- ALS compression (als.hip) ------------------------------------------------
// Device scratch of one compression (sizes for rank r, n_max = max n_q):
// Tm max(n1 n2, n2 n3) r; Y n_max r^2; W r^3; P n_max r; Q max(n_max r, r^3);
// Rinv r^2; G[4] r^2 doubles; partials 1024 doubles; scal 1 double; flag 1 int
// (set when a Gram matrix is not positive definite).
template <typename T>
struct AlsScratch {
    T *Tm, *Y, *W, *P, *Q, *Rinv;
    double* G[4];
    double* partials;
    double* scal;
    int* flag;
};
// Compress the three components of m in place of the initial factors U
// (layout of the low-rank calls), writing core (Tucker core / CP weights) and
// err2[3][2] = (residual^2, ||X||^2) per component.  Returns 0 or a negative code.
template <typename T>
int als_compress(void* handle, hipStream_t st, const int n[3], int r, bool tucker, int sweeps, const T* m, T* core,
                 T* U, double* err2, const AlsScratch<T>& w);

// ---- LLG driver (llg.hip) ------------------------------------------------------
// Heun predictor: k1 = f(m, H + hext), ms = unit(m + dt k1); corrector:
// m = unit(m + dt/2 (k1 + f(ms, H2 + hext))); f = -g m x h - alpha g m x (m x h).
template <typename T>
hipError_t launch_llg_predict(hipStream_t, size_t N, const T* m, const T* H, const double hext[3], double g,
                              double alpha, double dt, T* k1, T* ms);
template <typename T>
hipError_t launch_llg_correct(hipStream_t, size_t N, T* m, const T* H2, const T* k1, const T* ms,
                              const double hext[3], double g, double alpha, double dt);

// H = -grad phi (d = cell edges), optional energy partials m.H, one per
// workgroup; *nparts (if given) receives their count, at most
// sp_gradient_tiles(nx, ny, nz, 1).
template <typename T>
hipError_t launch_sp_gradient(hipStream_t, int nx, int ny, int nz, const double d[3], const T* phi, T* H,
                              const T* m, double* partials, int* nparts);
long sp_gradient_tiles(int nx, int ny, int nz, int zc);

}  // namespace demag
