// One-dimensional Gaussian cell integrals of the tensor-grid method (Sec. 3.2,
// eqs. (Dmat), (gs)) in closed form, lengths in one unit:
//     even:  int_{cell} exp(-s^2 (a - x)^2) dx
//     odd:   int_{cell} (a - x) exp(-s^2 (a - x)^2) dx
// for the cell [c - d/2, c + d/2], target coordinate a and s = tau.
#pragma once
#include <hip/hip_runtime.h>

namespace demag {

// int_{c - d/2}^{c + d/2} exp(-s^2 (a - x)^2) dx, with the erf difference taken
// through erfc where both arguments have one sign (no cancellation)
__device__ inline double gauss_even(double a, double c, double d, double s) {
    const double A = s * (a - c + 0.5 * d), B = s * (a - c - 0.5 * d);  // A > B
    double diff;
    if (B >= 0) diff = erfc(B) - erfc(A);
    else if (A <= 0) diff = erfc(-A) - erfc(-B);
    else diff = erf(A) - erf(B);
    return 0.5 * 1.7724538509055160273 / s * diff;
}

// int_{c - d/2}^{c + d/2} (a - x) exp(-s^2 (a - x)^2) dx
__device__ inline double gauss_odd(double a, double c, double d, double s) {
    const double ua = a - c + 0.5 * d, ub = a - c - 0.5 * d;  // a - x at x = c - d/2 and c + d/2
    return (exp(-s * s * ub * ub) - exp(-s * s * ua * ua)) / (2.0 * s * s);
}

}  // namespace demag
