// Closed-shell second-order Moller-Plesset energy over the Fock-build basis (the paper's MP2, spin-adapted form of
// Szabo-Ostlund Sec. 6.5).  The AO integrals (mu nu|lam sig) are computed by the quartet kernels into a dense
// nbf^4 tensor in HBM (canonical shell quartets, each element written to its eight equivalent places), then
// transformed one index at a time by GEMMs on the matrix cores (rocBLAS; row-major tensors are handed over as
// their column-major transposes):
//   Q1  T1[i][nu lam sig] = sum_mu C[mu][i] T0[mu][nu lam sig]          one GEMM, m = nbf^3, n = o, k = nbf
//   Q2  T2[i][a][lam sig] = sum_nu C[nu][a] T1[i][nu][lam sig]          batched over i, m = nbf^2, n = v, k = nbf
//   Q3  Z[i a lam][b]     = sum_sig T2[i a lam][sig] C[sig][b]          one GEMM, m = v, n = o v nbf, k = nbf
//   Q4  V[i][a][j][b]     = sum_lam C[lam][j] Z[i a][lam][b]           batched over (i a), m = v, n = o, k = nbf
// and E2 = sum_{ijab} V_iajb (2 V_iajb - V_ibja) / (e_i + e_j - e_a - e_b), split into its opposite-spin part
// sum V^2/D and same-spin part sum V (V - V_ibja)/D.  i, j run over the active occupied orbitals (frozen core
// excluded), a, b over the virtual ones.
#include "uqc_api_internal.h"
#include "uqc_device_common.h"

#include <rocblas/rocblas.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

using namespace uqc;

namespace {

__global__ __launch_bounds__(kBlock) void k_mp2_energy(const double* __restrict__ V, const double* __restrict__ eo,
                                                       const double* __restrict__ ev, int o, int v,
                                                       double* __restrict__ acc) {
    const long long n = (long long)o * v * o * v;
    double eos = 0.0, ess = 0.0;
    for (long long x = (long long)blockIdx.x * kBlock + threadIdx.x; x < n; x += (long long)gridDim.x * kBlock) {
        const int b = (int)(x % v);
        const long long r = x / v;
        const int j = (int)(r % o);
        const long long r2 = r / o;
        const int a = (int)(r2 % v), i = (int)(r2 / v);
        const double t = V[x];
        const double tx = V[(((long long)i * v + b) * o + j) * v + a];  // (ib|ja)
        const double d = eo[i] + eo[j] - ev[a] - ev[b];
        eos += t * t / d;
        ess += t * (t - tx) / d;
    }
    eos = wave_sum(eos);
    ess = wave_sum(ess);
    if ((threadIdx.x % kWave) == 0) {
        atomic_add(acc, eos);
        atomic_add(acc + 1, ess);
    }
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

#define UQC_BLAS_MP2(expr)                                                                               \
    do {                                                                                                 \
        rocblas_status b_ = (expr);                                                                      \
        if (b_ != rocblas_status_success)                                                                \
            return uqc_fail(UQC_E_DEVICE, std::string(#expr) + " failed: " + rocblas_status_to_string(b_)); \
    } while (0)

uqc_status uqc_mp2(uqc_basis* B, const double* C, const double* eps, int nocc, int nfrozen, double tau,
                   uqc_mp2_result* res) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!B || !C || !eps) return uqc_fail(UQC_E_ARG, "uqc_mp2: NULL argument");
    const int N = B->nbf;
    if (nocc < 1 || nocc > N || nfrozen < 0 || nfrozen >= nocc)
        return uqc_fail(UQC_E_ARG, "uqc_mp2: need 0 <= nfrozen < nocc <= nbf");
    if (!(tau >= 0) || !std::isfinite(tau)) return uqc_fail(UQC_E_ARG, "uqc_mp2: bad tau");
    for (int p = 0; p < N; ++p)
        if (!std::isfinite(eps[p])) return uqc_fail(UQC_E_ARG, "uqc_mp2: non-finite orbital energy");
    const int o = nocc - nfrozen, v = N - nocc;
    if (res) std::memset(res, 0, sizeof(*res));
    if (v == 0) return UQC_OK;  // no virtual orbitals: E2 = 0
    for (int i = nfrozen; i < nocc; ++i)
        for (int a = nocc; a < N; ++a)
            if (!(eps[a] > eps[i])) return uqc_fail(UQC_E_ARG, "uqc_mp2: a virtual orbital lies below an occupied one");
    const double dN = N;
    const double need = 8.0 * (dN * dN * dN * dN + (double)o * dN * dN * dN + (double)o * v * dN * dN +
                               (double)o * v * v * dN + (double)o * o * v * v + dN * dN + dN + 8);
    uqc_ctx* ctx = B->ctx;
    UQC_HIP(hipSetDevice(ctx->device));
    size_t free_b = 0, total_b = 0;
    UQC_HIP(hipMemGetInfo(&free_b, &total_b));
    if (need > 0.95 * (double)free_b) return uqc_fail(UQC_E_NOMEM, "uqc_mp2: the nbf^4 AO tensor and the transformed "
                                                                  "intermediates do not fit in free device memory");
    hipStream_t s = ctx->stream;
    rocblas_handle h = nullptr;
    uqc_status st = uqc::ensure_blas(ctx, &h);
    if (st != UQC_OK) return st;
    const size_t NN = (size_t)N * N, N3 = NN * N, N4 = N3 * N;
    DevBuf t0buf, cbuf, vbuf;
    if (hipMalloc(&t0buf.p, N4 * sizeof(double)) != hipSuccess) return uqc_fail(UQC_E_NOMEM, "uqc_mp2: AO tensor");
    if (hipMalloc(&cbuf.p, (NN + N + 8) * sizeof(double)) != hipSuccess) return uqc_fail(UQC_E_NOMEM, "uqc_mp2: C");
    double* T0 = (double*)t0buf.p;
    double* Cd = (double*)cbuf.p;
    double* ed = Cd + NN;
    double* acc = ed + N;
    UQC_HIP(hipMemcpyAsync(Cd, C, NN * sizeof(double), hipMemcpyHostToDevice, s));
    UQC_HIP(hipMemcpyAsync(ed, eps, N * sizeof(double), hipMemcpyHostToDevice, s));
    UQC_HIP(launch_zero(acc, 8, s));

    // ---- AO tensor: every canonical shell quartet (bra bin >= ket bin; p >= q inside one bin) with Q Q >= tau
    UQC_HIP(launch_zero(T0, N4, s));
    long long quartets = 0;
    {
        // the lists of every bin pair in one host buffer and one upload; the class launches then run side by side on
        // the context's stream and two more (the tensor positions they write are disjoint across canonical quartets)
        struct Seg {
            size_t X, Y, off;
            int n;
        };
        std::vector<Seg> segs;
        std::vector<int> hb, hk;
        for (size_t X = 0; X < B->bins.size(); ++X)
            for (size_t Y = 0; Y <= X; ++Y) {
                const Bin &bx = B->bins[X], &by = B->bins[Y];
                const size_t off = hb.size();
                for (int p = 0; p < bx.np; ++p)
                    for (int q = 0; q < (X == Y ? p + 1 : by.np); ++q)
                        if (bx.Q[p] * by.Q[q] >= tau) {
                            hb.push_back(p);
                            hk.push_back(q);
                        }
                if (hb.size() > off) segs.push_back(Seg{X, Y, off, (int)(hb.size() - off)});
            }
        const size_t total = hb.size();
        DevBuf ib;
        if (hipMalloc(&ib.p, 2 * std::max<size_t>(total, 1) * sizeof(int)) != hipSuccess)
            return uqc_fail(UQC_E_NOMEM, "uqc_mp2: quartet list");
        int* dbra = (int*)ib.p;
        int* dket = dbra + total;
        if (total) {
            UQC_HIP(hipMemcpyAsync(dbra, hb.data(), total * sizeof(int), hipMemcpyHostToDevice, s));
            UQC_HIP(hipMemcpyAsync(dket, hk.data(), total * sizeof(int), hipMemcpyHostToDevice, s));
        }
        constexpr int kStreams = 3;
        hipStream_t S[kStreams] = {s, nullptr, nullptr};
        for (int k = 1; k < kStreams; ++k)
            if (!(S[k] = ctx_stream(ctx, k))) return uqc_fail(UQC_E_DEVICE, "uqc_mp2: stream creation failed");
        UQC_HIP(hipEventRecord(ctx->fork, s));
        for (int k = 1; k < kStreams; ++k) UQC_HIP(hipStreamWaitEvent(S[k], ctx->fork, 0));
        for (size_t i = 0; i < segs.size(); ++i) {
            const Seg& g = segs[i];
            const Bin &bx = B->bins[g.X], &by = B->bins[g.Y];
            ListDev L;
            L.bra = bx.dev;
            L.ket = by.dev;
            L.bra_idx = dbra + g.off;
            L.ket_idx = dket + g.off;
            L.n = g.n;
            L.out = T0;
            L.nbf = N;
            UQC_HIP(launch_list(class_index(bx.la, bx.lb, by.la, by.lb), false, MODE_SCATTER, L, ctx->boys64,
                                ctx->boys32, S[i % kStreams]));
            quartets += g.n;
        }
        for (int k = 1; k < kStreams; ++k) {
            UQC_HIP(hipEventRecord(ctx->join[k - 1], S[k]));
            UQC_HIP(hipStreamWaitEvent(s, ctx->join[k - 1], 0));
        }
        UQC_HIP(hipStreamSynchronize(s));  // the index lists are freed at the end of this block
    }
    const auto t1 = std::chrono::steady_clock::now();

    // ---- four quarter transformations
    const double one = 1.0, zero = 0.0;
    const double* Co = Cd + nfrozen;  // column-major (nbf_p x nbf_mu), ld nbf: rows p = nfrozen.. are the active occupied
    const double* Cv = Cd + nocc;     // rows p = nocc.. are the virtuals
    const size_t nT1 = (size_t)o * N3, nT2 = (size_t)o * v * NN, nZ = (size_t)o * v * v * N, nV = (size_t)o * v * o * v;
    if (hipMalloc(&vbuf.p, (nT1 + nT2) * sizeof(double)) != hipSuccess)
        return uqc_fail(UQC_E_NOMEM, "uqc_mp2: transformation buffers");
    double* T1 = (double*)vbuf.p;
    double* T2 = T1 + nT1;
    // Q1: T1^T (N^3 x o) = T0^T (N^3 x N) * Co^T (N x o)
    UQC_BLAS_MP2(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, (rocblas_int)N3, o, N, &one, T0,
                               (rocblas_int)N3, Co, N, &zero, T1, (rocblas_int)N3));
    // Q2: per i, T2_i^T (N^2 x v) = T1_i^T (N^2 x N) * Cv^T (N x v)
    UQC_BLAS_MP2(rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, (rocblas_int)NN,
                                               v, N, &one, T1, (rocblas_int)NN, (rocblas_stride)N3, Cv, N, 0, &zero,
                                               T2, (rocblas_int)NN, (rocblas_stride)(v * NN), o));
    UQC_HIP(hipStreamSynchronize(s));
    (void)hipFree(t0buf.p);  // the AO tensor is no longer needed
    t0buf.p = nullptr;
    DevBuf zbuf;
    if (hipMalloc(&zbuf.p, (nZ + nV) * sizeof(double)) != hipSuccess)
        return uqc_fail(UQC_E_NOMEM, "uqc_mp2: transformation buffers");
    double* Z = (double*)zbuf.p;
    double* V = Z + nZ;
    // Q3: Z^T (v x o v N) = Cv (v x N, column-major view of C rows nocc..) * T2^T (N x o v N)
    UQC_BLAS_MP2(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, v, (rocblas_int)((size_t)o * v * N), N,
                               &one, Cv, N, T2, N, &zero, Z, v));
    // Q4: per (i a), V_ia^T (v x o) = Z_ia^T (v x N) * Co^T (N x o)
    UQC_BLAS_MP2(rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, v, o, N, &one, Z,
                                               v, (rocblas_stride)((size_t)v * N), Co, N, 0, &zero, V, v,
                                               (rocblas_stride)((size_t)o * v), o * v));
    UQC_HIP(hipStreamSynchronize(s));
    const auto t2 = std::chrono::steady_clock::now();

    // ---- energy
    {
        const long long n = (long long)o * v * o * v;
        const unsigned grid = (unsigned)std::min<long long>((n + kBlock - 1) / kBlock, 4096);
        hipLaunchKernelGGL(k_mp2_energy, dim3(grid), dim3(kBlock), 0, s, V, ed + nfrozen, ed + nocc, o, v, acc);
        UQC_HIP(hipGetLastError());
    }
    double h_acc[2] = {0, 0};
    UQC_HIP(hipMemcpyAsync(h_acc, acc, sizeof(h_acc), hipMemcpyDeviceToHost, s));
    UQC_HIP(hipStreamSynchronize(s));
    const auto t3 = std::chrono::steady_clock::now();
    if (res) {
        auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
            return std::chrono::duration<double, std::milli>(b - a).count();
        };
        res->e_os = h_acc[0];
        res->e_ss = h_acc[1];
        res->e2 = h_acc[0] + h_acc[1];
        res->quartets = quartets;
        res->ao_ms = ms(t0, t1);
        res->transform_ms = ms(t1, t2);
        res->energy_ms = ms(t2, t3);
        res->ms = ms(t0, t3);
        res->transform_flops = 2.0 * ((double)o * N4 + (double)o * v * N3 + (double)o * v * v * NN +
                                      (double)o * o * v * v * N);
    }
    return UQC_OK;
}
