// The five streaming passes of one DM field evaluation (gfx950).
//
// H = -Ms N * m (Sec. 3.1, eq. (demag)) is evaluated as a zero-padded circular
// convolution on P = 2L points per axis (L >= n), where the convolution
// theorem (eq. (convolution)) turns it into a pointwise 3x3 real-symmetric
// matrix-vector product in Fourier space.  Each pass keeps whole pencils in
// LDS; between passes the data makes one round trip through HBM in layouts
// chosen so that one side of every pass is a long contiguous run and the other
// side is a tile of T adjacent pencils:
//
//   m   [C][nz][ny][nx]  real
//   B1  [C][nz][Kx][ny]  complex   Kx = Px/2 + 1     (after X-R2C / Y-inverse)
//   B2  [C][Kx][Py][Zs]  complex   Zs = nz (field)   (after Y / fused Z)
//   H   [C][nz][ny][nx]  real
//
// X-R2C transforms two real rows at once as one complex pencil (even row in
// the real part, odd row in the imaginary part) and splits the spectra; the
// padded half of every forward pencil is never read (zero-filled in LDS) and
// the discarded half of every inverse pencil is never written.  The tensor
// product is fused into the Z pass between its forward and inverse FFTs.
#include <algorithm>

#include "fft_lds.hpp"
#include "internal.hpp"

namespace demag {

template <typename T>
__device__ __forceinline__ cx<T>* lds_buf() {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    return reinterpret_cast<cx<T>*>(smem_raw);
}

// ---------------------------------------------------------------------------
// X forward: real rows -> half spectra, output transposed to y-fastest.
// grid (ceil(Yr/Ty), Zr, C); in [C][Zr][Yr][Xin]; out [C][Zr][Kx][Yr].
template <typename T, int E>
__global__ void __launch_bounds__(kMaxThreads) k_x_fwd(const T* __restrict__ in, cx<T>* __restrict__ out,
                                                     int Xin, int Yr, int Zr, int Kx, int Ty, int C, FftPlanDev pl,
                                                     const cx<T>* __restrict__ tw, BatchIO bio) {
    cx<T>* buf = lds_buf<T>();
    const int P = pl.P, tid = threadIdx.x, nthr = blockDim.x;
    const int y0 = blockIdx.x * Ty, z = blockIdx.y, c = blockIdx.z % C, g = blockIdx.z / C;
    if (bio.in) {
        in = (const T*)bio.in[g];
        out = (cx<T>*)bio.out[g];
    }
    const int ty = min(Ty, Yr - y0);
    const int B = (ty + 1) >> 1;
    const T* src = in + (((size_t)c * Zr + z) * Yr + y0) * (size_t)Xin;
    for (int e = tid; e < B * Xin; e += nthr) {
        int p = e / Xin, x = e - p * Xin;
        T re = src[(size_t)(2 * p) * Xin + x];
        T im = (2 * p + 1 < ty) ? src[(size_t)(2 * p + 1) * Xin + x] : T(0);
        buf[p * P + x] = mk(re, im);
    }
    const int pad = P - Xin;
    for (int e = tid; e < B * pad; e += nthr) {
        int p = e / pad, x = Xin + (e - p * pad);
        buf[p * P + x] = mk(T(0), T(0));
    }
    __syncthreads();
    fft_lds<-1, E>(buf, B, P, pl, tw);
    cx<T>* dst = out + ((size_t)c * Zr + z) * (size_t)Kx * Yr + y0;
    for (int e = tid; e < Kx * ty; e += nthr) {
        int k = e / ty, y = e - k * ty;
        const cx<T>* pen = buf + (y >> 1) * P;
        cx<T> a = pen[k], b = pen[k == 0 ? 0 : P - k];
        cx<T> r = (y & 1) ? mk(T(0.5) * (a.im + b.im), T(0.5) * (b.re - a.re))
                          : mk(T(0.5) * (a.re + b.re), T(0.5) * (a.im - b.im));
        dst[(size_t)k * Yr + y] = r;
    }
}

// ---------------------------------------------------------------------------
// Y forward: y-pencils (contiguous) -> ky, written with z fastest.
// grid (ceil(Zr/Tz), ceil(Kx/Tx), C); in [C][Zr][Kx][Yin]; out [C][Kx][Py][Zs].
template <typename T, int E>
__global__ void __launch_bounds__(kMaxThreads) k_y_fwd(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                     int Yin, int Zr, int Kx, int Zs, int Tx, int Tz, int C,
                                                     FftPlanDev pl, const cx<T>* __restrict__ tw, BatchIO bio) {
    cx<T>* buf = lds_buf<T>();
    const int P = pl.P, tid = threadIdx.x, nthr = blockDim.x;
    const int kx0 = blockIdx.y * Tx, z0 = blockIdx.x * Tz, c = blockIdx.z % C, g = blockIdx.z / C;
    if (bio.in) {
        in = (const cx<T>*)bio.in[g];
        out = (cx<T>*)bio.out[g];
    }
    const int tx = min(Tx, Kx - kx0), tz = min(Tz, Zr - z0);
    const int B = tx * tz;
    for (int e = tid; e < B * Yin; e += nthr) {
        int p = e / Yin, y = e - p * Yin;
        int zi = p / tx, xi = p - zi * tx;
        buf[p * P + y] = in[(((size_t)c * Zr + z0 + zi) * Kx + kx0 + xi) * (size_t)Yin + y];
    }
    const int pad = P - Yin;
    for (int e = tid; e < B * pad; e += nthr) {
        int p = e / pad, y = Yin + (e - p * pad);
        buf[p * P + y] = mk(T(0), T(0));
    }
    __syncthreads();
    fft_lds<-1, E>(buf, B, P, pl, tw);
    for (int e = tid; e < P * B; e += nthr) {
        int zi = e % tz, r = e / tz;
        int xi = r % tx, ky = r / tx;
        out[(((size_t)c * Kx + kx0 + xi) * P + ky) * (size_t)Zs + z0 + zi] = buf[(zi * tx + xi) * P + ky];
    }
}

// ---------------------------------------------------------------------------
// Fused Z pass: forward z-FFT of the three components, multiply by Ms * Nhat
// (real symmetric 3x3, stored for the octant kx <= Lx, ky <= Ly, kz <= Lz with
// -1/(Px Py Pz) folded in), inverse z-FFT, keep the first nz outputs, in place.
// A workgroup takes ky' and its mirror Py - ky' together, so each tensor value
// is read once.  Mirroring ky (kz) flips the sign of the components odd in y
// (z): xy, yz (xz, yz).
// grid (Ly + 1, ceil(Kx/Tx)); B2 [3][Kx][Py][nz]; nhat [Kx][Ly+1][Lz+1][6].
template <typename T, int E>
__global__ void __launch_bounds__(kMaxThreads) k_z_conv(cx<T>* __restrict__ B2, const T* __restrict__ nhat, T Ms,
                                                      int nz, int Py, int Kx, int Tx, FftPlanDev pl,
                                                      const cx<T>* __restrict__ tw, BatchIO bio) {
    cx<T>* buf = lds_buf<T>();
    const int P = pl.P, Lz = P >> 1, Ly = Py >> 1, tid = threadIdx.x, nthr = blockDim.x;
    const int kx0 = blockIdx.y * Tx, kyp = blockIdx.x;
    if (bio.in) B2 = (cx<T>*)bio.out[blockIdx.z];
    const int tx = min(Tx, Kx - kx0);
    const int ns = (kyp == 0 || kyp == Ly) ? 1 : 2;
    const int B = ns * 3 * tx;
    // pencil p = (s * 3 + comp) * tx + xi
    for (int e = tid; e < B * nz; e += nthr) {
        int p = e / nz, zz = e - p * nz;
        int sc = p / tx, xi = p - sc * tx;
        int s = sc / 3, comp = sc - s * 3;
        int ky = s ? Py - kyp : kyp;
        buf[p * P + zz] = B2[(((size_t)comp * Kx + kx0 + xi) * Py + ky) * (size_t)nz + zz];
    }
    const int pad = P - nz;
    for (int e = tid; e < B * pad; e += nthr) {
        int p = e / pad, zz = nz + (e - p * pad);
        buf[p * P + zz] = mk(T(0), T(0));
    }
    __syncthreads();
    fft_lds<-1, E>(buf, B, P, pl, tw);
    for (int e = tid; e < ns * tx * P; e += nthr) {
        int kz = e % P, r = e / P;
        int xi = r % tx, s = r / tx;
        int kzp = kz <= Lz ? kz : P - kz;
        T sz = kz > Lz ? T(-1) : T(1);
        T sy = s ? T(-1) : T(1);
        const T* nh = nhat + (((size_t)(kx0 + xi) * (Ly + 1) + kyp) * (Lz + 1) + kzp) * 6;
        T nxx = nh[0], nyy = nh[1], nzz = nh[2];
        T nxy = sy * nh[3], nxz = sz * nh[4], nyz = sy * sz * nh[5];
        cx<T>* px = buf + ((s * 3 + 0) * tx + xi) * P + kz;
        cx<T>* py = buf + ((s * 3 + 1) * tx + xi) * P + kz;
        cx<T>* pz = buf + ((s * 3 + 2) * tx + xi) * P + kz;
        cx<T> mx = *px, my = *py, mz = *pz;
        *px = mk(Ms * (nxx * mx.re + nxy * my.re + nxz * mz.re), Ms * (nxx * mx.im + nxy * my.im + nxz * mz.im));
        *py = mk(Ms * (nxy * mx.re + nyy * my.re + nyz * mz.re), Ms * (nxy * mx.im + nyy * my.im + nyz * mz.im));
        *pz = mk(Ms * (nxz * mx.re + nyz * my.re + nzz * mz.re), Ms * (nxz * mx.im + nyz * my.im + nzz * mz.im));
    }
    __syncthreads();
    fft_lds<+1, E>(buf, B, P, pl, tw);
    for (int e = tid; e < B * nz; e += nthr) {
        int p = e / nz, zz = e - p * nz;
        int sc = p / tx, xi = p - sc * tx;
        int s = sc / 3, comp = sc - s * 3;
        int ky = s ? Py - kyp : kyp;
        B2[(((size_t)comp * Kx + kx0 + xi) * Py + ky) * (size_t)nz + zz] = buf[p * P + zz];
    }
}

// Plain forward z-FFT of full-length pencils, in place (tensor setup).
// grid (ceil(Py/Ty), Kx); B2 [Kx][Py][P]: Ty consecutive pencils (kx, ky0 ..).
template <typename T, int E>
__global__ void __launch_bounds__(kMaxThreads) k_z_fwd(cx<T>* __restrict__ B2, int Py, int Ty, FftPlanDev pl,
                                                     const cx<T>* __restrict__ tw) {
    cx<T>* buf = lds_buf<T>();
    const int P = pl.P, tid = threadIdx.x, nthr = blockDim.x;
    const int ky0 = blockIdx.x * Ty, kx = blockIdx.y;
    const int ty = min(Ty, Py - ky0);
    cx<T>* base = B2 + ((size_t)kx * Py + ky0) * (size_t)P;
    for (int e = tid; e < ty * P; e += nthr) buf[e] = base[e];
    __syncthreads();
    fft_lds<-1, E>(buf, ty, P, pl, tw);
    for (int e = tid; e < ty * P; e += nthr) base[e] = buf[e];
}

// ---------------------------------------------------------------------------
// Y inverse: ky -> first ny outputs, written y-fastest.
// grid (ceil(nz/Tz), ceil(Kx/Tx), C); in [C][Kx][Py][nz]; out [C][nz][Kx][ny].
template <typename T, int E>
__global__ void __launch_bounds__(kMaxThreads) k_y_inv(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                     int ny, int nz, int Kx, int Tx, int Tz, int C, FftPlanDev pl,
                                                     const cx<T>* __restrict__ tw, BatchIO bio) {
    cx<T>* buf = lds_buf<T>();
    const int P = pl.P, tid = threadIdx.x, nthr = blockDim.x;
    const int kx0 = blockIdx.y * Tx, z0 = blockIdx.x * Tz, c = blockIdx.z % C, g = blockIdx.z / C;
    if (bio.in) {
        in = (const cx<T>*)bio.in[g];
        out = (cx<T>*)bio.out[g];
    }
    const int tx = min(Tx, Kx - kx0), tz = min(Tz, nz - z0);
    const int B = tx * tz;
    for (int e = tid; e < P * B; e += nthr) {
        int zi = e % tz, r = e / tz;
        int xi = r % tx, ky = r / tx;
        buf[(zi * tx + xi) * P + ky] = in[(((size_t)c * Kx + kx0 + xi) * P + ky) * (size_t)nz + z0 + zi];
    }
    __syncthreads();
    fft_lds<+1, E>(buf, B, P, pl, tw);
    for (int e = tid; e < B * ny; e += nthr) {
        int p = e / ny, y = e - p * ny;
        int zi = p / tx, xi = p - zi * tx;
        out[(((size_t)c * nz + z0 + zi) * Kx + kx0 + xi) * (size_t)ny + y] = buf[p * P + y];
    }
}

// ---------------------------------------------------------------------------
// X inverse (C2R of two rows per complex pencil), keep the first nx outputs.
// Epilogue: optional store (overwrite or accumulate) and optional energy
// partial sum_i m_i . h_i (FP32 products in FP32 paths, FP64 accumulation),
// one FP64 partial per workgroup.
// grid (ceil(ny/Ty), nz, C); in [C][nz][Kx][ny]; out, m [C][nz][ny][nx].
template <typename T, int E>
__global__ void __launch_bounds__(kMaxThreads) k_x_inv(const cx<T>* __restrict__ in, T* __restrict__ out,
                                                     const T* __restrict__ m, double* __restrict__ partials,
                                                     int nx, int ny, int nz, int Kx, int Ty, int accumulate, int C,
                                                     FftPlanDev pl, const cx<T>* __restrict__ tw, BatchIO bio) {
    cx<T>* buf = lds_buf<T>();
    const int P = pl.P, Lx = P >> 1, tid = threadIdx.x, nthr = blockDim.x;
    const int y0 = blockIdx.x * Ty, z = blockIdx.y, c = blockIdx.z % C, g = blockIdx.z / C;
    if (bio.in) {  // batches carry no energy
        in = (const cx<T>*)bio.in[g];
        out = (T*)bio.out[g];
        m = nullptr;
        partials = nullptr;
    }
    const int ty = min(Ty, ny - y0);
    const int B = (ty + 1) >> 1;
    const cx<T>* src = in + ((size_t)c * nz + z) * (size_t)Kx * ny + y0;
    for (int e = tid; e < Kx * B; e += nthr) {
        int k = e / B, p = e - k * B;
        cx<T> xe = src[(size_t)k * ny + 2 * p];
        cx<T> xo = (2 * p + 1 < ty) ? src[(size_t)k * ny + 2 * p + 1] : mk(T(0), T(0));
        if (k == 0 || k == Lx) {  // C2R ignores the imaginary parts of DC and Nyquist
            xe.im = T(0);
            xo.im = T(0);
        }
        cx<T>* pen = buf + p * P;
        pen[k] = mk(xe.re - xo.im, xe.im + xo.re);  // xe + i xo
        if (k > 0 && k < Lx) pen[P - k] = mk(xe.re + xo.im, xo.re - xe.im);  // conj(xe) + i conj(xo)
    }
    __syncthreads();
    fft_lds<+1, E>(buf, B, P, pl, tw);
    const size_t rowbase = (((size_t)c * nz + z) * ny + y0) * (size_t)nx;
    T* dst = out ? out + rowbase : nullptr;
    const T* msrc = m ? m + rowbase : nullptr;
    double acc = 0.0;
    for (int e = tid; e < ty * nx; e += nthr) {
        int row = e / nx, x = e - row * nx;
        cx<T> v = buf[(row >> 1) * P + x];
        T h = (row & 1) ? v.im : v.re;
        size_t idx = (size_t)row * nx + x;
        if (msrc) acc += (double)(msrc[idx] * h);
        if (dst) dst[idx] = accumulate ? dst[idx] + h : h;
    }
    if (partials) {
        __syncthreads();  // the pencils are consumed; reuse their LDS for the reduction
        double* red = reinterpret_cast<double*>(buf);
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if ((tid & 63) == 0) red[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < (nthr + 63) / 64; ++w) s += red[w];
            partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
        }
    }
}

// Deterministic FP64 sum of the partials (fixed order), scaled.  Thread i
// sums partials i, i + 1024, ... in that order; each iteration issues its
// four loads before the first add, so the latency of a few thousand partials
// is paid about once rather than once per element.
constexpr int kReduceThreads = 1024;
__global__ void __launch_bounds__(kReduceThreads) k_energy_reduce(const double* __restrict__ partials, int n,
                                                                  double scale, double* __restrict__ out) {
    __shared__ double red[kReduceThreads];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int base = 0; base < n; base += 4 * kReduceThreads) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * kReduceThreads + tid;
            a[u] = i < n ? partials[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s += a[u];
    }
    red[tid] = s;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) out[0] = scale * red[0];
}

// Energy gradient (Sec. 2): E = -(mu0/2) Ms V sum m.H(m) is quadratic in m
// and the grid operator is symmetric, so dE/dm = -mu0 Ms V H(m); with the
// cotangent gE (device scalar, NULL = 1), gm (+)= gE c H, c = -mu0 Ms V.
template <typename T>
__global__ void __launch_bounds__(256) k_energy_grad(size_t n, const T* __restrict__ H,
                                                     const double* __restrict__ gE, double c, T* __restrict__ gm,
                                                     int accumulate) {
    const T s = (T)(gE ? gE[0] * c : c);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        gm[i] = accumulate ? gm[i] + s * H[i] : s * H[i];
}

// ---------------------------------------------------------------------------
// Host launchers (E dispatch).
#define DEMAG_E_SWITCH(E, CALL)                              \
    switch (E) {                                             \
    case 4: CALL(4); break;                                  \
    case 8: CALL(8); break;                                  \
    case 16: CALL(16); break;                                \
    default: CALL(32); break;                                \
    }

template <typename T>
hipError_t launch_x_fwd(const LaunchCfg& lc, hipStream_t st, const T* in, cx<T>* out, int Xin, int Yr, int Zr,
                        int Kx, int C, const FftPlanDev& pl, const cx<T>* tw, const BatchIO& bio) {
    dim3 grid((Yr + lc.t0 - 1) / lc.t0, Zr, C * bio.count);
    size_t lds = (size_t)((lc.t0 + 1) / 2) * pl.P * sizeof(cx<T>);
#define CALL(EE) hipLaunchKernelGGL((k_x_fwd<T, EE>), grid, dim3(lc.threads), lds, st, in, out, Xin, Yr, Zr, Kx, lc.t0, C, pl, tw, bio)
    DEMAG_E_SWITCH(lc.E, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_y_fwd(const LaunchCfg& lc, hipStream_t st, const cx<T>* in, cx<T>* out, int Yin, int Zr, int Kx,
                        int Zs, int C, const FftPlanDev& pl, const cx<T>* tw, const BatchIO& bio) {
    dim3 grid((Zr + lc.t1 - 1) / lc.t1, (Kx + lc.t0 - 1) / lc.t0, C * bio.count);
    size_t lds = (size_t)lc.t0 * lc.t1 * pl.P * sizeof(cx<T>);
#define CALL(EE) hipLaunchKernelGGL((k_y_fwd<T, EE>), grid, dim3(lc.threads), lds, st, in, out, Yin, Zr, Kx, Zs, lc.t0, lc.t1, C, pl, tw, bio)
    DEMAG_E_SWITCH(lc.E, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_z_conv(const LaunchCfg& lc, hipStream_t st, cx<T>* B2, const T* nhat, T Ms, int nz, int Py, int Kx,
                         const FftPlanDev& pl, const cx<T>* tw, const BatchIO& bio) {
    dim3 grid(Py / 2 + 1, (Kx + lc.t0 - 1) / lc.t0, bio.count);
    size_t lds = (size_t)6 * lc.t0 * pl.P * sizeof(cx<T>);
    // dynamic LDS above 64 KB must be allowed per kernel before its launch
#define CALL(EE)                                                                                                   \
    if (lds > 65536) {                                                                                             \
        hipError_t e_ = hipFuncSetAttribute((const void*)&k_z_conv<T, EE>,                                         \
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                 \
        if (e_ != hipSuccess) return e_;                                                                           \
    }                                                                                                              \
    hipLaunchKernelGGL((k_z_conv<T, EE>), grid, dim3(lc.threads), lds, st, B2, nhat, Ms, nz, Py, Kx, lc.t0, pl, tw, bio)
    DEMAG_E_SWITCH(lc.E, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_z_fwd(const LaunchCfg& lc, hipStream_t st, cx<T>* B2, int Py, int Kx, const FftPlanDev& pl,
                        const cx<T>* tw) {
    dim3 grid((Py + lc.t0 - 1) / lc.t0, Kx, 1);
    size_t lds = (size_t)lc.t0 * pl.P * sizeof(cx<T>);
#define CALL(EE) hipLaunchKernelGGL((k_z_fwd<T, EE>), grid, dim3(lc.threads), lds, st, B2, Py, lc.t0, pl, tw)
    DEMAG_E_SWITCH(lc.E, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_y_inv(const LaunchCfg& lc, hipStream_t st, const cx<T>* in, cx<T>* out, int ny, int nz, int Kx,
                        int C, const FftPlanDev& pl, const cx<T>* tw, const BatchIO& bio) {
    dim3 grid((nz + lc.t1 - 1) / lc.t1, (Kx + lc.t0 - 1) / lc.t0, C * bio.count);
    size_t lds = (size_t)lc.t0 * lc.t1 * pl.P * sizeof(cx<T>);
#define CALL(EE) hipLaunchKernelGGL((k_y_inv<T, EE>), grid, dim3(lc.threads), lds, st, in, out, ny, nz, Kx, lc.t0, lc.t1, C, pl, tw, bio)
    DEMAG_E_SWITCH(lc.E, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_x_inv(const LaunchCfg& lc, hipStream_t st, const cx<T>* in, T* out, const T* m, double* partials,
                        int nx, int ny, int nz, int Kx, int C, int accumulate, const FftPlanDev& pl,
                        const cx<T>* tw, const BatchIO& bio) {
    dim3 grid((ny + lc.t0 - 1) / lc.t0, nz, C * bio.count);
    size_t lds = (size_t)((lc.t0 + 1) / 2) * pl.P * sizeof(cx<T>);
    lds = std::max(lds, (size_t)(kMaxThreads / 64) * sizeof(double));  // the epilogue reduction reuses it
#define CALL(EE) hipLaunchKernelGGL((k_x_inv<T, EE>), grid, dim3(lc.threads), lds, st, in, out, m, partials, nx, ny, nz, Kx, lc.t0, accumulate, C, pl, tw, bio)
    DEMAG_E_SWITCH(lc.E, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_energy_reduce(hipStream_t st, const double* partials, int n, double scale, double* out) {
    hipLaunchKernelGGL(k_energy_reduce, dim3(1), dim3(kReduceThreads), 0, st, partials, n, scale, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_energy_grad(hipStream_t st, size_t n, const T* H, const double* gE, double c, T* gm, int accumulate) {
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((k_energy_grad<T>), dim3((unsigned)blocks), dim3(256), 0, st, n, H, gE, c, gm, accumulate);
    return hipGetLastError();
}

#define DEMAG_INSTANTIATE(T)                                                                                      \
    template hipError_t launch_x_fwd<T>(const LaunchCfg&, hipStream_t, const T*, cx<T>*, int, int, int, int, int, \
                                        const FftPlanDev&, const cx<T>*, const BatchIO&);                         \
    template hipError_t launch_y_fwd<T>(const LaunchCfg&, hipStream_t, const cx<T>*, cx<T>*, int, int, int, int,  \
                                        int, const FftPlanDev&, const cx<T>*, const BatchIO&);                    \
    template hipError_t launch_z_conv<T>(const LaunchCfg&, hipStream_t, cx<T>*, const T*, T, int, int, int,       \
                                         const FftPlanDev&, const cx<T>*, const BatchIO&);                        \
    template hipError_t launch_z_fwd<T>(const LaunchCfg&, hipStream_t, cx<T>*, int, int, const FftPlanDev&,       \
                                        const cx<T>*);                                                            \
    template hipError_t launch_y_inv<T>(const LaunchCfg&, hipStream_t, const cx<T>*, cx<T>*, int, int, int, int,  \
                                        const FftPlanDev&, const cx<T>*, const BatchIO&);                         \
    template hipError_t launch_x_inv<T>(const LaunchCfg&, hipStream_t, const cx<T>*, T*, const T*, double*, int,  \
                                        int, int, int, int, int, const FftPlanDev&, const cx<T>*, const BatchIO&); \
    template hipError_t launch_energy_grad<T>(hipStream_t, size_t, const T*, const double*, double, T*, int);

DEMAG_INSTANTIATE(float)
DEMAG_INSTANTIATE(double)

}  // namespace demag
