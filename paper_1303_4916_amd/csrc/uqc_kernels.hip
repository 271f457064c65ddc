// Dispatch of the per-class quartet kernels and the small helper kernels of libuqc (density preparation, Fock
// finalisation, Boys verification, serving-side density perturbation).
#include "uqc_device_common.h"
#include "generated/eri_flops.h"

namespace uqc {

#define UQC_DECL(n) ClassLaunchers class_launchers_##n();
UQC_DECL(0) UQC_DECL(1) UQC_DECL(2) UQC_DECL(3) UQC_DECL(4) UQC_DECL(5) UQC_DECL(6) UQC_DECL(7) UQC_DECL(8)
UQC_DECL(9) UQC_DECL(10) UQC_DECL(11) UQC_DECL(12) UQC_DECL(13) UQC_DECL(14) UQC_DECL(15) UQC_DECL(16)
UQC_DECL(17) UQC_DECL(18) UQC_DECL(19) UQC_DECL(20)

static const ClassLaunchers& launchers(int cls) {
    static const ClassLaunchers tab[kNumClasses] = {
        class_launchers_0(),  class_launchers_1(),  class_launchers_2(),  class_launchers_3(),  class_launchers_4(),
        class_launchers_5(),  class_launchers_6(),  class_launchers_7(),  class_launchers_8(),  class_launchers_9(),
        class_launchers_10(), class_launchers_11(), class_launchers_12(), class_launchers_13(), class_launchers_14(),
        class_launchers_15(), class_launchers_16(), class_launchers_17(), class_launchers_18(), class_launchers_19(),
        class_launchers_20()};
    return tab[cls];
}

static int pair_class(int la, int lb) {
    static const int tab[3][3] = {{0, -1, -1}, {1, 2, -1}, {3, 4, 5}};
    if (la < 0 || la > 2 || lb < 0 || lb > la) return -1;
    return tab[la][lb];
}

int class_index(int la, int lb, int lc, int ld) {
    const int bi = pair_class(la, lb), ki = pair_class(lc, ld);
    if (bi < 0 || ki < 0 || ki > bi) return -1;
    return bi * (bi + 1) / 2 + ki;
}

void class_ls(int idx, int* la, int* lb, int* lc, int* ld) {
    static const int pc[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
    int bi = 0;
    while ((bi + 1) * (bi + 2) / 2 <= idx) ++bi;
    const int ki = idx - bi * (bi + 1) / 2;
    *la = pc[bi][0]; *lb = pc[bi][1]; *lc = pc[ki][0]; *ld = pc[ki][1];
}

double class_flops_prim(int cls) { return kClassFlopsPrim[cls]; }
int class_team(int cls) { return kClassTeam[cls]; }
double class_flops_contr(int cls) { return kClassFlopsContr[cls]; }

hipError_t launch_digest(int cls, bool mixed, int nspin, const TaskDev* d_tasks, const long long* d_task_begin,
                         int ntask, long long item0, long long nitems, const double* boys64tab,
                         const float* boys32tab, const WorkRedirect& wr, unsigned* queue, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (cls < 0 || cls >= kNumClasses || item0 < 0 || (nspin != 1 && nspin != 2) || !queue)
        return hipErrorInvalidValue;
    if (wr.J && (nspin != 1 || !wr.D || !wr.K || !wr.count)) return hipErrorInvalidValue;
    static_assert(kQueueWords % 2 == 0 && kQueueWords >= 2 * kXcds, "queue: whole doubles, one counter per die");
    const hipError_t e = launch_zero(reinterpret_cast<double*>(queue), kQueueWords / 2, s);
    if (e != hipSuccess) return e;
    return launchers(cls).digest(mixed, nspin, d_tasks, d_task_begin, ntask, item0, nitems, boys64tab, boys32tab,
                                 wr, queue, s);
}

hipError_t launch_list_rys(int cls, const ListDev& list, const double* rystab, hipStream_t s) {
    if (list.n <= 0) return hipSuccess;
    if (cls < 0 || cls >= kNumClasses) return hipErrorInvalidValue;
    return launchers(cls).list_rys(list, rystab, s);
}

hipError_t launch_list(int cls, bool mixed, int mode, const ListDev& list, const double* boys64tab,
                       const float* boys32tab, hipStream_t s) {
    if (list.n <= 0) return hipSuccess;
    if (cls < 0 || cls >= kNumClasses) return hipErrorInvalidValue;
    return launchers(cls).list(mixed, mode, list, boys64tab, boys32tab, s);
}

// ------------------------------------------------------------------------------------ density / Fock helpers
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
    return x;
}

// D' = f_i f_j D_ij; maxbits[0] = max |D_ij - D_ji|, maxbits[1] = max |D_ij| (bit patterns of non-negative
// doubles order like the values, so an integer atomic max is a max over doubles).
__global__ __launch_bounds__(kBlock) void k_prepare(const double* __restrict__ D, const double* __restrict__ f,
                                                    double* __restrict__ Dp, int N,
                                                    unsigned long long* __restrict__ maxbits) {
    const long long NN = (long long)N * N;
    double md = 0.0, ma = 0.0;
    for (long long x = (long long)blockIdx.x * kBlock + threadIdx.x; x < NN; x += (long long)gridDim.x * kBlock) {
        const int i = (int)(x / N), j = (int)(x % N);
        const double v = D[x];
        Dp[x] = f[i] * f[j] * v;
        if (!(fabs(v) < INFINITY)) md = INFINITY;  // NaN or infinite entries are rejected like asymmetry
        md = fmax(md, fabs(v - D[(size_t)j * N + i]));
        ma = fmax(ma, fabs(v));
    }
    md = wave_max(md);
    ma = wave_max(ma);
    if ((threadIdx.x % kWave) == 0) {
        atomicMax(maxbits + 0, (unsigned long long)__double_as_longlong(md));
        atomicMax(maxbits + 1, (unsigned long long)__double_as_longlong(ma));
    }
}

__global__ __launch_bounds__(kBlock) void k_zero(double* __restrict__ p, size_t n) {
    for (size_t x = (size_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += (size_t)gridDim.x * kBlock) p[x] = 0.0;
}

// J = f_i f_j (Jacc_ij + Jacc_ji), K likewise, G = J - (xs/2) K, E2 = 1/2 sum D_ij G_ij.
__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ D, const double* __restrict__ Jacc,
                                                     const double* __restrict__ Kacc, const double* __restrict__ f,
                                                     double* __restrict__ J, double* __restrict__ K,
                                                     double* __restrict__ G, double xs, double* __restrict__ E2,
                                                     int N) {
    const long long NN = (long long)N * N;
    const double hx = 0.5 * xs;
    double e = 0.0;
    for (long long x = (long long)blockIdx.x * kBlock + threadIdx.x; x < NN; x += (long long)gridDim.x * kBlock) {
        const int i = (int)(x / N), j = (int)(x % N);
        const size_t t = (size_t)j * N + i;
        const double ff = f[i] * f[j];
        const double jv = ff * (Jacc[x] + Jacc[t]);
        const double kv = ff * (Kacc[x] + Kacc[t]);
        const double gv = jv - hx * kv;
        if (J) J[x] = jv;
        if (K) K[x] = kv;
        if (G) G[x] = gv;
        e = fma(D[x], gv, e);
    }
    e = wave_sum(e);
    if ((threadIdx.x % kWave) == 0) atomic_add(E2, 0.5 * e);
}

// Spin densities: J from the shared accumulator, K^a and K^b from their own, G^s = J - xs K^s,
// E2 = 1/2 sum (Da_ij Ga_ij + Db_ij Gb_ij).
__global__ __launch_bounds__(kBlock) void k_finalize_uhf(const double* __restrict__ Da, const double* __restrict__ Db,
                                                         const double* __restrict__ Jacc,
                                                         const double* __restrict__ Kaacc,
                                                         const double* __restrict__ Kbacc,
                                                         const double* __restrict__ f, double xs,
                                                         double* __restrict__ J, double* __restrict__ Ka,
                                                         double* __restrict__ Kb, double* __restrict__ Ga,
                                                         double* __restrict__ Gb, double* __restrict__ E2, int N) {
    const long long NN = (long long)N * N;
    double e = 0.0;
    for (long long x = (long long)blockIdx.x * kBlock + threadIdx.x; x < NN; x += (long long)gridDim.x * kBlock) {
        const int i = (int)(x / N), j = (int)(x % N);
        const size_t t = (size_t)j * N + i;
        const double ff = f[i] * f[j];
        const double jv = ff * (Jacc[x] + Jacc[t]);
        const double ka = ff * (Kaacc[x] + Kaacc[t]);
        const double kb = ff * (Kbacc[x] + Kbacc[t]);
        const double ga = jv - xs * ka, gb = jv - xs * kb;
        if (J) J[x] = jv;
        if (Ka) Ka[x] = ka;
        if (Kb) Kb[x] = kb;
        if (Ga) Ga[x] = ga;
        if (Gb) Gb[x] = gb;
        e = fma(Da[x], ga, fma(Db[x], gb, e));
    }
    e = wave_sum(e);
    if ((threadIdx.x % kWave) == 0) atomic_add(E2, 0.5 * e);
}

// C = A + B (n elements)
__global__ __launch_bounds__(kBlock) void k_add(const double* __restrict__ A, const double* __restrict__ B,
                                                double* __restrict__ C, size_t n) {
    for (size_t x = (size_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += (size_t)gridDim.x * kBlock)
        C[x] = A[x] + B[x];
}

// W = U diag(w) for a column-major N x N matrix U: column k of U scaled by w_k
__global__ __launch_bounds__(kBlock) void k_scale_cols(const double* __restrict__ U, const double* __restrict__ w,
                                                       double* __restrict__ W, int N) {
    const size_t NN = (size_t)N * N;
    for (size_t x = (size_t)blockIdx.x * kBlock + threadIdx.x; x < NN; x += (size_t)gridDim.x * kBlock)
        W[x] = U[x] * w[x / N];
}

// E = M - M^T (N x N)
__global__ __launch_bounds__(kBlock) void k_antisym(const double* __restrict__ M, double* __restrict__ E, int N) {
    const size_t NN = (size_t)N * N;
    for (size_t x = (size_t)blockIdx.x * kBlock + threadIdx.x; x < NN; x += (size_t)gridDim.x * kBlock) {
        const size_t i = x / N, j = x % N;
        E[x] = M[x] - M[j * N + i];
    }
}

static unsigned grid_for(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_prepare(const double* D, const double* f, double* Dp, int nbf, unsigned long long* maxbits,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_prepare, dim3(grid_for((long long)nbf * nbf)), dim3(kBlock), 0, s, D, f, Dp, nbf, maxbits);
    return hipGetLastError();
}

hipError_t launch_add(const double* A, const double* B, double* C, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_add, dim3(grid_for((long long)n)), dim3(kBlock), 0, s, A, B, C, n);
    return hipGetLastError();
}

hipError_t launch_scale_cols(const double* U, const double* w, double* W, int N, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_cols, dim3(grid_for((long long)N * N)), dim3(kBlock), 0, s, U, w, W, N);
    return hipGetLastError();
}

hipError_t launch_antisym(const double* M, double* E, int N, hipStream_t s) {
    hipLaunchKernelGGL(k_antisym, dim3(grid_for((long long)N * N)), dim3(kBlock), 0, s, M, E, N);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero, dim3(grid_for((long long)n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* D, const double* Jacc, const double* Kacc, const double* f, double* J,
                           double* K, double* G, double xs, double* E2, int nbf, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(grid_for((long long)nbf * nbf)), dim3(kBlock), 0, s, D, Jacc, Kacc, f, J, K,
                       G, xs, E2, nbf);
    return hipGetLastError();
}

hipError_t launch_finalize_uhf(const double* Da, const double* Db, const double* Jacc, const double* Kaacc,
                               const double* Kbacc, const double* f, double xs, double* J, double* Ka, double* Kb,
                               double* Ga, double* Gb, double* E2, int nbf, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_uhf, dim3(grid_for((long long)nbf * nbf)), dim3(kBlock), 0, s, Da, Db, Jacc, Kaacc,
                       Kbacc, f, xs, J, Ka, Kb, Ga, Gb, E2, nbf);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------- Boys verification kernel
template <int L>
__global__ __launch_bounds__(kBlock) void k_boys(int prec, int n, const double* __restrict__ T,
                                                 double* __restrict__ out, const double* __restrict__ b64,
                                                 const float* __restrict__ b32) {
    const int x = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (x >= n) return;
    const double t = T[x];
    if (prec == 0 || t > (double)kBoysTmax32) {
        double F[L + 1];
        boys64<L>(t, 1.0, b64, F);
        for (int m = 0; m <= L; ++m) out[(size_t)x * (L + 1) + m] = F[m];
    } else {
        float F[L + 1];
        boys32<L>(t, b32, F);
        for (int m = 0; m <= L; ++m) out[(size_t)x * (L + 1) + m] = (double)F[m];
    }
}

hipError_t launch_boys(int prec, int mmax, int n, const double* T, double* out, const double* b64, const float* b32,
                       hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 g((unsigned)((n + kBlock - 1) / kBlock)), b(kBlock);
    switch (mmax) {
        case 0: hipLaunchKernelGGL(k_boys<0>, g, b, 0, s, prec, n, T, out, b64, b32); break;
        case 1: hipLaunchKernelGGL(k_boys<1>, g, b, 0, s, prec, n, T, out, b64, b32); break;
        case 2: hipLaunchKernelGGL(k_boys<2>, g, b, 0, s, prec, n, T, out, b64, b32); break;
        case 3: hipLaunchKernelGGL(k_boys<3>, g, b, 0, s, prec, n, T, out, b64, b32); break;
        case 4: hipLaunchKernelGGL(k_boys<4>, g, b, 0, s, prec, n, T, out, b64, b32); break;
        case 5: hipLaunchKernelGGL(k_boys<5>, g, b, 0, s, prec, n, T, out, b64, b32); break;
        case 6: hipLaunchKernelGGL(k_boys<6>, g, b, 0, s, prec, n, T, out, b64, b32); break;
        case 7: hipLaunchKernelGGL(k_boys<7>, g, b, 0, s, prec, n, T, out, b64, b32); break;
        case 8: hipLaunchKernelGGL(k_boys<8>, g, b, 0, s, prec, n, T, out, b64, b32); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------ serving: density perturbation on device
// Counter-based standard normal numbers: for element n of stream (seed, t) the 64-bit counter
// x = seed * 0x9E3779B97F4A7C15 + t * 0xD1B54A32D192ED03 + 2n (mod 2^64) gives two SplitMix64 outputs s(x), s(x+1)
// (s(x) = finaliser of x + 0x9E3779B97F4A7C15); u1 = ((s(x) >> 11) + 1) 2^-53, u2 = (s(x+1) >> 11) 2^-53 and
// z = sqrt(-2 ln u1) cos(2 pi u2) (Box-Muller).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    unsigned long long z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_normal(double* __restrict__ R, long long n, unsigned long long seed,
                                                   unsigned long long t) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const unsigned long long x = seed * 0x9E3779B97F4A7C15ULL + t * 0xD1B54A32D192ED03ULL +
                                     2ULL * (unsigned long long)i;
        const double u1 = (double)((splitmix64(x) >> 11) + 1ULL) * 0x1.0p-53;
        const double u2 = (double)(splitmix64(x + 1ULL) >> 11) * 0x1.0p-53;
        R[i] = sqrt(-2.0 * log(u1)) * cos(2.0 * kPi * u2);
    }
}

hipError_t launch_normal(double* R, long long n, unsigned long long seed, unsigned long long t, hipStream_t s) {
    hipLaunchKernelGGL(k_normal, dim3(grid_for(n)), dim3(kBlock), 0, s, R, n, seed, t);
    return hipGetLastError();
}

// D <- (1 - eps) D + eps R R^T (R is nbf x ncol, row-major); work[0] accumulates the new trace.
__global__ __launch_bounds__(kBlock) void k_perturb(double* __restrict__ D, const double* __restrict__ R, int N,
                                                    int ncol, double eps, double* __restrict__ work) {
    const long long NN = (long long)N * N;
    double tr = 0.0;
    for (long long x = (long long)blockIdx.x * kBlock + threadIdx.x; x < NN; x += (long long)gridDim.x * kBlock) {
        const int i = (int)(x / N), j = (int)(x % N);
        double s = 0.0;
        for (int c = 0; c < ncol; ++c) s = fma(R[(size_t)i * ncol + c], R[(size_t)j * ncol + c], s);
        const double v = (1.0 - eps) * D[x] + eps * s;
        D[x] = v;
        if (i == j) tr += v;
    }
    tr = wave_sum(tr);
    if ((threadIdx.x % kWave) == 0) atomic_add(work, tr);
}

__global__ __launch_bounds__(kBlock) void k_rescale(double* __restrict__ D, long long NN, double trace0,
                                                    const double* __restrict__ work) {
    const double s = trace0 / work[0];
    for (long long x = (long long)blockIdx.x * kBlock + threadIdx.x; x < NN; x += (long long)gridDim.x * kBlock)
        D[x] *= s;
}

hipError_t launch_perturb(double* D, const double* R, int nbf, int ncol, double eps, double trace0, double* work,
                          hipStream_t s) {
    const long long NN = (long long)nbf * nbf;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, s, work, (size_t)1);
    hipLaunchKernelGGL(k_perturb, dim3(grid_for(NN)), dim3(kBlock), 0, s, D, R, nbf, ncol, eps, work);
    hipLaunchKernelGGL(k_rescale, dim3(grid_for(NN)), dim3(kBlock), 0, s, D, NN, trace0, work);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_trace(const double* __restrict__ D, int N, double* __restrict__ out) {
    double tr = 0.0;
    for (int i = (int)(blockIdx.x * kBlock + threadIdx.x); i < N; i += (int)(gridDim.x * kBlock))
        tr += D[(size_t)i * N + i];
    tr = wave_sum(tr);
    if ((threadIdx.x % kWave) == 0) atomic_add(out, tr);
}

hipError_t launch_trace(const double* D, int nbf, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, s, out, (size_t)1);
    hipLaunchKernelGGL(k_trace, dim3(grid_for(nbf)), dim3(kBlock), 0, s, D, nbf, out);
    return hipGetLastError();
}

}  // namespace uqc
