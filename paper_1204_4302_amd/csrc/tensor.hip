// FP64 setup of the demagnetization-tensor spectrum (once per plan).
//
// The auxiliary constants of DM depend on the geometry only and are computed
// once (Sec. 4, storage and complexity); this file builds them on the GPU:
//   1. N(o) on the octant o in [0,n) in FP64, per offset by distance band
//      (Newell f/g near, Gauss-Legendre of the cell-average integral in the
//      middle, moment series of the dipole kernel far) -- see newell.hpp;
//   2. the parity mirror into P-periodic real arrays (exact by construction:
//      diagonal components even in every axis, xy odd in x and y, xz odd in x
//      and z, yz odd in y and z, zero in the padding gap);
//   3. (plan runtime) the same X/Y/Z FFT passes in FP64;
//   4. the real part on the spectral octant, with -1/(Px Py Pz) folded in,
//      cast to the plan's precision.
#include <algorithm>

#include "internal.hpp"
#include "newell.hpp"

namespace demag {

namespace {

__device__ __forceinline__ bool in_far(int ox, int oy, int oz, const double* dt, double far_cut) {
    double X = ox * dt[0], Y = oy * dt[1], Z = oz * dt[2];
    return X * X + Y * Y + Z * Z >= far_cut * far_cut;
}

// Near and far bands: one thread per octant offset.
__global__ void __launch_bounds__(256) k_tensor_pointwise(size_t base, int nx, int ny, int nz, double dt0, double dt1,
                                                          double dt2, double far_cut, int fg_cut,
                                                          double* __restrict__ Noct) {
    const size_t ncell = (size_t)nx * ny * nz;
    size_t t = base + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncell) return;
    int ox = (int)(t % nx), oy = (int)((t / nx) % ny), oz = (int)(t / ((size_t)nx * ny));
    const double dt[3] = {dt0, dt1, dt2};
    int cheb = max(ox, max(oy, oz));
    double v[6];
    if (cheb <= fg_cut) {
        newell::near_fg(ox, oy, oz, dt, v);
    } else if (in_far(ox, oy, oz, dt, far_cut)) {
        newell::far_series(ox, oy, oz, dt, v);
    } else {
        return;  // mid band: k_tensor_mid
    }
    for (int c = 0; c < 6; ++c) Noct[c * ncell + t] = v[c];
}

// Mid band: one 64-lane workgroup per offset of the bounding box
// [0,bx) x [0,by) x [0,bz); offsets outside the band return at once.
__global__ void __launch_bounds__(64) k_tensor_mid(long base, int nx, int ny, int nz, int bx, int by, double dt0, double dt1,
                                                   double dt2, double far_cut, int fg_cut, int q, int max_panels,
                                                   const double* __restrict__ gl_x, const double* __restrict__ gl_w,
                                                   double* __restrict__ Noct) {
    const long b = base + blockIdx.x;
    const int ox = (int)(b % bx), oy = (int)((b / bx) % by), oz = (int)(b / ((long)bx * by));
    if (ox >= nx || oy >= ny || oz >= nz) return;
    const double dt[3] = {dt0, dt1, dt2};
    if (max(ox, max(oy, oz)) <= fg_cut || in_far(ox, oy, oz, dt, far_cut)) return;
    const double gap = newell::cell_gap(ox, oy, oz, dt);
    int m[3], Q[3];
    for (int k = 0; k < 3; ++k) {
        m[k] = newell::mid_panels(dt[k], gap, max_panels);
        Q[k] = 2 * m[k] * q;
    }
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const double R[3] = {ox * dt[0], oy * dt[1], oz * dt[2]};
    const int total = Q[0] * Q[1] * Q[2];
    for (int n = threadIdx.x; n < total; n += 64) {
        int i = n % Q[0], j = (n / Q[0]) % Q[1], k = n / (Q[0] * Q[1]);
        double sx, wx, sy, wy, sz, wz;
        newell::mid_node(i, dt[0], m[0], q, gl_x, gl_w, &sx, &wx);
        newell::mid_node(j, dt[1], m[1], q, gl_x, gl_w, &sy, &wy);
        newell::mid_node(k, dt[2], m[2], q, gl_x, gl_w, &sz, &wz);
        newell::dipole_add(R[0] + sx, R[1] + sy, R[2] + sz, wx * wy * wz, acc);
    }
    const double V = dt[0] * dt[1] * dt[2];
    const size_t ncell = (size_t)nx * ny * nz;
    const size_t t = ((size_t)oz * ny + oy) * nx + ox;
    for (int c = 0; c < 6; ++c) {
        double s = acc[c];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (threadIdx.x == 0) Noct[c * ncell + t] = V * s;
    }
}

// Signed offset of padded index i (period P, n valid offsets each side), or
// a flag for the zero gap.
__device__ __forceinline__ bool unpad(int i, int n, int P, int* o) {
    if (i < n) { *o = i; return true; }
    if (i > P - n) { *o = i - P; return true; }
    return false;
}

__global__ void __launch_bounds__(256) k_tensor_embed(size_t base, int comp, int nx, int ny, int nz, int Px, int Py,
                                                      int Pz, const double* __restrict__ Noct,
                                                      double* __restrict__ A) {
    const size_t total = (size_t)Px * Py * Pz;
    size_t t = base + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    int x = (int)(t % Px), y = (int)((t / Px) % Py), z = (int)(t / ((size_t)Px * Py));
    int ox, oy, oz;
    double v = 0.0;
    if (unpad(x, nx, Px, &ox) && unpad(y, ny, Py, &oy) && unpad(z, nz, Pz, &oz)) {
        const size_t ncell = (size_t)nx * ny * nz;
        v = Noct[comp * ncell + ((size_t)abs(oz) * ny + abs(oy)) * nx + abs(ox)];
        const bool odd_x = (comp == 3 || comp == 4), odd_y = (comp == 3 || comp == 5), odd_z = (comp == 4 || comp == 5);
        if (odd_x && ox < 0) v = -v;
        if (odd_y && oy < 0) v = -v;
        if (odd_z && oz < 0) v = -v;
    }
    A[t] = v;
}

template <typename T>
__global__ void __launch_bounds__(256) k_tensor_extract(size_t base, int comp, int Py, int Pz, int Kx, double scale,
                                                        const cx<double>* __restrict__ B2, T* __restrict__ nhat) {
    const int Ly = Py / 2, Lz = Pz / 2;
    const size_t total = (size_t)(Ly + 1) * Kx * (Lz + 1);
    size_t t = base + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    int kz = (int)(t % (Lz + 1)), ky = (int)((t / (Lz + 1)) % (Ly + 1)), kx = (int)(t / ((size_t)(Lz + 1) * (Ly + 1)));
    double v = B2[((size_t)kx * Py + ky) * Pz + kz].re * scale;  // B2 [Kx][Py][Pz]
    // A component odd in an axis has an exactly zero transform on that axis's
    // Nyquist plane (its samples at o and P - o cancel, and the sample at P/2
    // is zero); store the exact zero rather than the transform's rounding.
    // xy (3) is odd in x and y, xz (4) in x and z, yz (5) in y and z.
    const int Lx = Kx - 1;
    const bool oddx = comp == 3 || comp == 4, oddy = comp == 3 || comp == 5, oddz = comp == 4 || comp == 5;
    if ((oddx && kx == Lx) || (oddy && ky == Ly) || (oddz && kz == Lz)) v = 0.0;
    nhat[t * 6 + comp] = (T)v;  // [Kx][Ly+1][Lz+1][6]
}

}  // namespace

hipError_t launch_tensor_octant(hipStream_t st, int nx, int ny, int nz, const double dt[3], const TensorBands& tb,
                                const double* gl_x_dev, const double* gl_w_dev, double* Noct) {
    const size_t ncell = (size_t)nx * ny * nz;
    hipError_t e = launch_pieces(ncell, 256, [&](size_t base, unsigned blocks) {
        hipLaunchKernelGGL(k_tensor_pointwise, dim3(blocks), dim3(256), 0, st, base, nx, ny, nz, dt[0], dt[1], dt[2],
                           tb.far_cut, tb.fg_cut, Noct);
    });
    if (e != hipSuccess) return e;
    // bounding box of the mid band: |o_k| dt_k < far_cut
    // (in floating point: far_cut / dt may exceed the int range)
    auto box = [&](int n, double d) { return (int)std::min<double>(n, ceil(tb.far_cut / d) + 1.0); };
    const int bx = box(nx, dt[0]), by = box(ny, dt[1]), bz = box(nz, dt[2]);
    const long nb = (long)bx * by * bz;
    if (nb > 0 && tb.far_cut > 0) {  // one 64-lane workgroup per offset of the box
        e = launch_pieces((size_t)nb * 64, 64, [&](size_t base, unsigned blocks) {
            hipLaunchKernelGGL(k_tensor_mid, dim3(blocks), dim3(64), 0, st, (long)(base / 64), nx, ny, nz, bx, by,
                               dt[0], dt[1], dt[2], tb.far_cut, tb.fg_cut, tb.gl_q, tb.max_panels, gl_x_dev, gl_w_dev,
                               Noct);
        });
    }
    return e;
}

hipError_t launch_tensor_embed(hipStream_t st, int comp, int nx, int ny, int nz, int Px, int Py, int Pz,
                               const double* Noct, double* A) {
    const size_t total = (size_t)Px * Py * Pz;
    return launch_pieces(total, 256, [&](size_t base, unsigned blocks) {
        hipLaunchKernelGGL(k_tensor_embed, dim3(blocks), dim3(256), 0, st, base, comp, nx, ny, nz, Px, Py, Pz, Noct, A);
    });
}

template <typename T>
hipError_t launch_tensor_extract(hipStream_t st, int comp, int Px, int Py, int Pz, int Kx, double scale,
                                 const cx<double>* B2, T* nhat) {
    (void)Px;
    const size_t total = (size_t)(Py / 2 + 1) * Kx * (Pz / 2 + 1);
    return launch_pieces(total, 256, [&](size_t base, unsigned blocks) {
        hipLaunchKernelGGL((k_tensor_extract<T>), dim3(blocks), dim3(256), 0, st, base, comp, Py, Pz, Kx, scale, B2,
                           nhat);
    });
}

template hipError_t launch_tensor_extract<float>(hipStream_t, int, int, int, int, int, double, const cx<double>*,
                                                 float*);
template hipError_t launch_tensor_extract<double>(hipStream_t, int, int, int, int, int, double, const cx<double>*,
                                                  double*);

}  // namespace demag
