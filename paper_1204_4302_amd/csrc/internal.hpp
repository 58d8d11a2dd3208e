// Internal declarations shared by the pass kernels, the tensor setup and the
// plan runtime (not part of the public C ABI).
#pragma once
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
struct LaunchCfg {
    int threads = 256;
    int E = 16;
    int t0 = 1;
    int t1 = 1;
};

template <typename T>
hipError_t launch_x_fwd(const LaunchCfg&, hipStream_t, const T* in, cx<T>* out, int Xin, int Yr, int Zr, int Kx,
                        int C, const FftPlanDev&, const cx<T>* tw);
template <typename T>
hipError_t launch_y_fwd(const LaunchCfg&, hipStream_t, const cx<T>* in, cx<T>* out, int Yin, int Zr, int Kx, int Zs,
                        int C, const FftPlanDev&, const cx<T>* tw);
template <typename T>
hipError_t launch_z_conv(const LaunchCfg&, hipStream_t, cx<T>* B2, const T* nhat, T Ms, int nz, int Py, int Kx,
                         const FftPlanDev&, const cx<T>* tw);
template <typename T>
hipError_t launch_z_fwd(const LaunchCfg&, hipStream_t, cx<T>* B2, int Py, int Kx, const FftPlanDev&,
                        const cx<T>* tw);
template <typename T>
hipError_t launch_y_inv(const LaunchCfg&, hipStream_t, const cx<T>* in, cx<T>* out, int ny, int nz, int Kx, int C,
                        const FftPlanDev&, const cx<T>* tw);
template <typename T>
hipError_t launch_x_inv(const LaunchCfg&, hipStream_t, const cx<T>* in, T* out, const T* m, double* partials, int nx,
                        int ny, int nz, int Kx, int C, int accumulate, const FftPlanDev&, const cx<T>* tw);
hipError_t launch_energy_reduce(hipStream_t, const double* partials, int n, double scale, double* out);

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
// Take the real part of the FFT'd component (B2 [Py][Kx][Pz], complex FP64)
// on the octant ky <= Ly, kz <= Lz, scale, cast to T into
// nhat [Ly+1][6][Kx][Lz+1].
template <typename T>
hipError_t launch_tensor_extract(hipStream_t, int comp, int Px, int Py, int Pz, int Kx, double scale,
                                 const cx<double>* B2, T* nhat);

}  // namespace demag
