// Device building blocks shared by the libuqc kernels: Boys function, wavefront reductions, Cartesian component
// scale factors.
#pragma once
#include "uqc_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>

namespace uqc {

// Cartesian component scale relative to the axis component: 1/sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!).  Only d shells
// have two values: xx, yy, zz (components 0, 3, 5) carry 1/sqrt(3).
__host__ __device__ constexpr double comp_factor(int l, int c) {
    return (l == 2 && (c == 0 || c == 3 || c == 5)) ? 0.57735026918962576451 : 1.0;
}

constexpr double kPi = 3.14159265358979323846;

// Read-only data that is the same for the whole wavefront (bra-pair records and headers, work lists, the density
// block of the bra pair) is read through the constant address space, so uniform addresses become scalar loads.
// None of it is written while a kernel runs.
typedef const __attribute__((address_space(4))) double* cdptr;
typedef const __attribute__((address_space(4))) int* ciptr;
__device__ __forceinline__ cdptr as_const(const double* p) { return (cdptr)p; }
__device__ __forceinline__ ciptr as_const(const int* p) { return (ciptr)p; }

// 1/x for positive normal x: the hardware approximation refined by two Newton steps to full double precision.
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// 1/sqrt(x) for positive normal x: the hardware approximation y0 (relative error about 2^-23) refined by one
// third-order step of the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - x y0^2: y1 = y0 + y0 e (1/2 + 3e/8).
// The dropped terms are below 5/16 |e|^3 < 2^-68, so the result has the accuracy of two Newton steps (a few
// rounding errors) in two fewer instructions.
__device__ __forceinline__ double rsqrt64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// A double constant materialised in scalar registers at its use (two scalar moves), so that an FMA takes it as its
// scalar operand.  Left to itself the compiler keeps the exp(d) coefficients below in vector registers across the
// primitive loop, and then copies each one before the accumulating FMA that consumes it (six vector moves per
// evaluation).
__device__ __forceinline__ double sgpr_const(double c) {
    asm volatile("" : "+s"(c));
    return c;
}

// ------------------------------------------------------------------------------------------------ Boys function
// F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt, returned multiplied by `pref` (`tab`: the per-order FP64 slices).
// For T < T_L (L the highest order needed): Taylor series of order 8 around the nearest grid point T_g = g/8
// (|d| = |T_g - T| <= 1/16, truncation error < 1e-16 relative), using dF_m/dT = -F_{m+1}, for order L (the table
// holds the coefficients F_{L+k}(T_g)/k!); exp(-T) = exp(-T_g) exp(d) with exp(-T_g) tabulated and exp(d) from its
// Taylor series to order 9 (truncation < 3e-19); then the downward recursion F_m = (2T F_{m+1} + exp(-T)) / (2m+1).
// For T >= T_L: F_0 = sqrt(pi/T)/2 and the upward recursion F_{m+1} = (2m+1) F_m / (2T), i.e.
// F_m = Gamma(m+1/2) / (2 T^{m+1/2}); the exact value is this times the regularised lower incomplete gamma
// P(m+1/2, T), so the relative error is Q(m+1/2, T) <= Q(L+1/2, T), which the cut-offs
// T_L = 37, 41, 44, 47, 50, 53, 55, 58, 60 (L = 0..8) keep below 2e-17 (the grid covers [0, 60) for every L).
// The two halves of boys64: the table row for T (grid index clamped, so the row can be fetched ahead of the test
// on T), then the evaluation from that row.
template <int L>
__device__ __forceinline__ int boys64_row(double T, const double* __restrict__ tab, double2* r) {
    const int g = (int)fmin(T * (double)kBoysGridPerUnit + 0.5, (double)(kBoysNg - 1));
    // uniform slice base + 32-bit byte offset of the row
    const char* slice = reinterpret_cast<const char*>(tab + (size_t)L * kBoysNg * kBoysRow);
    const double2* row =
        reinterpret_cast<const double2*>(slice + __umul24((unsigned)g, (unsigned)(kBoysRow * sizeof(double))));
#pragma unroll
    for (int x = 0; x < kBoysRow / 2; ++x) r[x] = row[x];
    return g;
}

// T_L of the comment above: the smallest integer T with Q(L+1/2, T) <= 2e-17
constexpr int kBoysAsymTi[9] = {37, 41, 44, 47, 50, 53, 55, 58, 60};
__device__ constexpr double kBoysAsymT[9] = {37, 41, 44, 47, 50, 53, 55, 58, 60};

// Rows of the order-L slice an evaluation can use: below T_L the nearest grid point is at most T_L * 8.
template <int L>
__host__ __device__ constexpr int boys_rows() {
    return kBoysAsymTi[L] * kBoysGridPerUnit + 1;
}

// boys64_row from a copy of the slice's first boys_rows<L>() rows in LDS (5 double2 per row).
template <int L>
__device__ __forceinline__ int boys64_row_lds(double T, const double2* lds, double2* r) {
    const int g = (int)fmin(T * (double)kBoysGridPerUnit + 0.5, (double)(boys_rows<L>() - 1));
    // 24-bit multiply (full rate; g < 2^24): the row's double2 offset
    const double2* row = lds + __umul24((unsigned)g, (unsigned)(kBoysRow / 2));
#pragma unroll
    for (int x = 0; x < kBoysRow / 2; ++x) r[x] = row[x];
    return g;
}

template <int L>
__device__ __forceinline__ void boys64_eval(double T, int g, double pref, const double2* r, double* F) {
    static_assert(L >= 0 && L <= 8 && kBoysTmax >= 60, "Boys orders 0..8 with the grid covering [0, 60)");
    if (T < kBoysAsymT[L]) {
        const double d = (double)g * (1.0 / kBoysGridPerUnit) - T;  // exact grid point
        double p = r[4].x;
        p = fma(p, d, r[3].y);
        p = fma(p, d, r[3].x);
        p = fma(p, d, r[2].y);
        p = fma(p, d, r[2].x);
        p = fma(p, d, r[1].y);
        p = fma(p, d, r[1].x);
        p = fma(p, d, r[0].y);
        p = fma(p, d, r[0].x);
        F[L] = p * pref;
        if constexpr (L > 0) {
            double x = sgpr_const(1.0 / 362880.0);
            x = fma(x, d, sgpr_const(1.0 / 40320.0));
            x = fma(x, d, sgpr_const(1.0 / 5040.0));
            x = fma(x, d, sgpr_const(1.0 / 720.0));
            x = fma(x, d, sgpr_const(1.0 / 120.0));
            x = fma(x, d, sgpr_const(1.0 / 24.0));
            x = fma(x, d, sgpr_const(1.0 / 6.0));
            x = fma(x, d, 0.5);
            x = fma(x, d, 1.0);
            x = fma(x, d, 1.0);
            const double e = r[4].y * x * pref;
            const double t2 = T + T;
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = fma(t2, F[m + 1], e) * (1.0 / (2 * m + 1));
        }
    } else {
        const double rs = rsqrt64(T);
        F[0] = (0.88622692545275801365 * pref) * rs;  // sqrt(pi)/2
        if constexpr (L > 0) {
            const double h = 0.5 * rs * rs;
#pragma unroll
            for (int m = 0; m < L; ++m) F[m + 1] = ((double)(2 * m + 1) * h) * F[m];
        }
    }
}

template <int L>
__device__ __forceinline__ void boys64(double T, double pref, const double* __restrict__ tab, double* F) {
    double2 r[kBoysRow / 2];
    const int g = boys64_row<L>(T, tab, r);
    boys64_eval<L>(T, g, pref, r, F);
}

// FP32 variant (mixed mode, T <= 30 only): Taylor order 5 around the same grid points (truncation < 1e-10
// relative).  The argument arrives in FP64: the grid point and the offset d = T_g - T are taken from it before
// rounding (rounding T itself to FP32 first would move F_m by up to (m + 1/2) units of FP32 rounding through
// dF_m/dT = -F_{m+1}), so only the series and the downward recursion run in FP32.  No step rounds the same way for
// every argument (no library exp, no rounded reciprocal constant), so the FP32 errors of many small integrals do
// not add up to a bias.
template <int L>
__device__ __forceinline__ void boys32(double Td, const float* __restrict__ tab, float* F) {
    const int g = (int)(Td * (double)kBoysGridPerUnit + 0.5);
    const float d = (float)((double)g * (1.0 / kBoysGridPerUnit) - Td);
    const float T = (float)Td;
    const float* r = tab + g * kBoysNm + L;
    float p = r[5];
    p = fmaf(p, d * 0.2f, r[4]);
    p = fmaf(p, d * 0.25f, r[3]);
    p = fmaf(p, d * (1.0f / 3.0f), r[2]);
    p = fmaf(p, d * 0.5f, r[1]);
    p = fmaf(p, d, r[0]);
    F[L] = p;
    if constexpr (L > 0) {
        // exp(-T) = exp(-T_g) exp(d), exp(d) to order 5 (truncation < 1e-10); the division by 2m+1 uses the
        // reciprocal split into two floats, so that its rounding does not bias every result the same way
        float x = fmaf(d, 1.0f / 120.0f, 1.0f / 24.0f);
        x = fmaf(x, d, 1.0f / 6.0f);
        x = fmaf(x, d, 0.5f);
        x = fmaf(x, d, 1.0f);
        x = fmaf(x, d, 1.0f);
        const float e = tab[g * kBoysNm + kBoysExpCol] * x;
        const float t2 = T + T;
#pragma unroll
        for (int m = L - 1; m >= 0; --m) {
            const float rh = (float)(1.0 / (2 * m + 1));
            const float rl = (float)(1.0 / (2 * m + 1) - (double)rh);
            const float y = fmaf(t2, F[m + 1], e);
            F[m] = fmaf(y, rh, y * rl);
        }
    }
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// Largest x over the wavefront (every lane active), as a wavefront-uniform value.
__device__ __forceinline__ int wave_max_int(int x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, kWave));
    return __builtin_amdgcn_readfirstlane(x);
}

__device__ __forceinline__ void atomic_add(double* p, double v) { (void)unsafeAtomicAdd(p, v); }

__device__ __forceinline__ void atomic_add_lds(double* p, double v) {
    (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

}  // namespace uqc
