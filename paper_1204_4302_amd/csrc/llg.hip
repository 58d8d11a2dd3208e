// Landau-Lifshitz-Gilbert driver (Sec. 2, the LLG equation): the consumer of
// the stray field the paper names.  For the unit magnetization m = M/Ms,
//     m_t = -g (m x H) - alpha g (m x (m x H)),   g = gamma / (1 + alpha^2),
// H = H_demag(m) + H_ext (uniform), gamma > 0 (the damping term is taken
// dissipative: with a positive gamma the printed sign of the second term
// would feed energy in).  Explicit Heun steps with renormalisation:
//     k1 = f(m),  m* = (m + dt k1)/|.|,  k2 = f(m*),  m <- (m + dt (k1 + k2)/2)/|.|
// Two field evaluations and two fused elementwise kernels per step.
#include "internal.hpp"

namespace demag {

namespace {

template <typename T>
struct V3 {
    T x, y, z;
};
template <typename T>
__device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ V3<T> rhs(V3<T> m, V3<T> h, T g, T ag) {
    const V3<T> mh = cross(m, h), mmh = cross(m, mh);
    return {-g * mh.x - ag * mmh.x, -g * mh.y - ag * mmh.y, -g * mh.z - ag * mmh.z};
}
template <typename T>
__device__ __forceinline__ V3<T> unit(V3<T> v) {
    const T r = T(1) / sqrt(v.x * v.x + v.y * v.y + v.z * v.z);
    return {v.x * r, v.y * r, v.z * r};
}
// Loads and stores are non-temporal: every array an update touches is read
// once more at most, after a field evaluation that streams far more than the
// 256 MB memory-side cache holds (or, for m*, by the field's first pass,
// whose loads are non-temporal themselves), so caching them only displaces
// the field passes' data.
template <typename T>
__device__ __forceinline__ V3<T> ld(const T* __restrict__ a, size_t N, size_t i) {
    return {__builtin_nontemporal_load(a + i), __builtin_nontemporal_load(a + N + i),
            __builtin_nontemporal_load(a + 2 * N + i)};
}
template <typename T>
__device__ __forceinline__ void st(T* __restrict__ a, size_t N, size_t i, V3<T> v) {
    __builtin_nontemporal_store(v.x, a + i);
    __builtin_nontemporal_store(v.y, a + N + i);
    __builtin_nontemporal_store(v.z, a + 2 * N + i);
}

template <typename T>
__global__ void __launch_bounds__(256) k_llg_predict(size_t N, const T* __restrict__ m, const T* __restrict__ H,
                                                     T hx, T hy, T hz, T g, T ag, T dt, T* __restrict__ k1,
                                                     T* __restrict__ ms) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const V3<T> mi = ld(m, N, i), hi = ld(H, N, i);
        const V3<T> k = rhs(mi, V3<T>{hi.x + hx, hi.y + hy, hi.z + hz}, g, ag);
        st(k1, N, i, k);
        st(ms, N, i, unit(V3<T>{mi.x + dt * k.x, mi.y + dt * k.y, mi.z + dt * k.z}));
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_llg_correct(size_t N, T* __restrict__ m, const T* __restrict__ H2,
                                                     const T* __restrict__ k1, const T* __restrict__ ms, T hx, T hy,
                                                     T hz, T g, T ag, T dt) {
    const T half = dt * T(0.5);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const V3<T> hi = ld(H2, N, i), a = ld(k1, N, i), mi = ld(m, N, i);
        const V3<T> b = rhs(ld(ms, N, i), V3<T>{hi.x + hx, hi.y + hy, hi.z + hz}, g, ag);
        st(m, N, i, unit(V3<T>{mi.x + half * (a.x + b.x), mi.y + half * (a.y + b.y), mi.z + half * (a.z + b.z)}));
    }
}

unsigned blocks_for(size_t N) {
    const size_t b = (N + 255) / 256;
    return (unsigned)(b < 65536 ? b : 65536);
}

}  // namespace

template <typename T>
hipError_t launch_llg_predict(hipStream_t st, size_t N, const T* m, const T* H, const double hext[3], double g,
                              double alpha, double dt, T* k1, T* ms) {
    hipLaunchKernelGGL((k_llg_predict<T>), dim3(blocks_for(N)), dim3(256), 0, st, N, m, H, (T)hext[0], (T)hext[1],
                       (T)hext[2], (T)g, (T)(alpha * g), (T)dt, k1, ms);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_llg_correct(hipStream_t st, size_t N, T* m, const T* H2, const T* k1, const T* ms,
                              const double hext[3], double g, double alpha, double dt) {
    hipLaunchKernelGGL((k_llg_correct<T>), dim3(blocks_for(N)), dim3(256), 0, st, N, m, H2, k1, ms, (T)hext[0],
                       (T)hext[1], (T)hext[2], (T)g, (T)(alpha * g), (T)dt);
    return hipGetLastError();
}

template hipError_t launch_llg_predict<float>(hipStream_t, size_t, const float*, const float*, const double[3],
                                              double, double, double, float*, float*);
template hipError_t launch_llg_predict<double>(hipStream_t, size_t, const double*, const double*, const double[3],
                                               double, double, double, double*, double*);
template hipError_t launch_llg_correct<float>(hipStream_t, size_t, float*, const float*, const float*, const float*,
                                              const double[3], double, double, double);
template hipError_t launch_llg_correct<double>(hipStream_t, size_t, double*, const double*, const double*,
                                               const double*, const double[3], double, double, double);

}  // namespace demag
