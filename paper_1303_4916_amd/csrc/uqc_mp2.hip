// Closed-shell second-order Moller-Plesset energy over the Fock-build basis (the paper's MP2, spin-adapted form of
// Szabo-Ostlund Sec. 6.5).  The AO integrals are never held as one nbf^4 tensor: the ordered ket index pairs
// (lam sig) are cut into batches along the canonical shell pairs, and for each batch the quartet kernels write
// (mu nu|lam sig) for every (mu nu) and every (lam sig) of the batch into a dense buffer T0b[mu][nu][col] (each
// canonical bra shell pair times each ket shell pair of the batch, both index orders of each pair, so a shell
// quartet is evaluated once for each of its two pairs' batches); the first quarter transformation is applied to
// the batch at once by a bandwidth-bound kernel that writes its columns straight to their places in T1 (a GEMM
// with n = o this thin would pad its tiles):
//   Q1  T1[i][nu lam sig] = sum_mu C[mu][i] T0[mu][nu lam sig]          per batch, k_mp2_q1
// Then the remaining transformations run as GEMMs on the matrix cores (rocBLAS; row-major tensors are handed over
// as their column-major transposes):
//   Q2  T2[i][a][lam sig] = sum_nu C[nu][a] T1[i][nu][lam sig]          batched over i, m = nbf^2, n = v, k = nbf
//   Q3  Z[i a lam][b]     = sum_sig T2[i a lam][sig] C[sig][b]          one GEMM, m = v, n = o v nbf, k = nbf
//   Q4  V[i][a][j][b]     = sum_lam C[lam][j] Z[i a][lam][b]           batched over (i a), m = v, n = o, k = nbf
// and E2 = sum_{ijab} V_iajb (2 V_iajb - V_ibja) / (e_i + e_j - e_a - e_b), split into its opposite-spin part
// sum V^2/D and same-spin part sum V (V - V_ibja)/D.  i, j run over the active occupied orbitals (frozen core
// excluded), a, b over the virtual ones.  Peak memory: the o nbf^3 of T1 plus one batch (nbf^2 + o nbf doubles per
// column), instead of nbf^4.
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

// First quarter transformation of one batch, written straight to the batch columns' places in T1:
//   T1[i nbf^3 + nu nbf^2 + map[col]] = sum_mu C[mu][nfrozen + i] T0b[mu][nu ncols + col],  i0 <= i < i0 + ib,
// ib <= kQ1Orb.  Each thread takes kQ1Cols batch columns j = nu ncols + col, 64 apart, so that a wavefront reads
// kQ1Cols x 512 contiguous bytes of every row mu; the columns' values are read once per block of orbitals (HBM-bound:
// 2 ib FLOPs per 8 bytes), the coefficients Co[mu nbf + i] (the active occupied orbitals of mu, contiguous) as
// wavefront-uniform scalar loads shared by the thread's columns.
constexpr int kQ1Orb = 16, kQ1Cols = 4;
__global__ __launch_bounds__(kBlock) void k_mp2_q1(const double* __restrict__ T0b, const double* __restrict__ Co,
                                                   const int* __restrict__ map, int ncols, int nbf, int i0, int ib,
                                                   double* __restrict__ T1) {
    const long long R = (long long)nbf * ncols;
    const long long j0 = ((long long)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) * (kWave * kQ1Cols) +
                         threadIdx.x % kWave;
    if (j0 >= R) return;
    double a[kQ1Cols][kQ1Orb];
#pragma unroll
    for (int r = 0; r < kQ1Cols; ++r)
#pragma unroll
        for (int k = 0; k < kQ1Orb; ++k) a[r][k] = 0.0;
    const cdptr c = as_const(Co) + i0;
    for (int mu = 0; mu < nbf; ++mu) {
        const double* row = T0b + (long long)mu * R;
        double t[kQ1Cols];
#pragma unroll
        for (int r = 0; r < kQ1Cols; ++r) {
            const long long j = j0 + (long long)r * kWave;
            t[r] = j < R ? row[j] : 0.0;
        }
        const cdptr cm = c + (size_t)mu * nbf;
#pragma unroll
        for (int k = 0; k < kQ1Orb; ++k)
            if (k < ib) {
                const double ck = cm[k];
#pragma unroll
                for (int r = 0; r < kQ1Cols; ++r) a[r][k] = fma(ck, t[r], a[r][k]);
            }
    }
    const long long N2 = (long long)nbf * nbf, N3 = N2 * nbf;
#pragma unroll
    for (int r = 0; r < kQ1Cols; ++r) {
        const long long j = j0 + (long long)r * kWave;
        if (j >= R) break;
        const long long to = (j / ncols) * N2 + map[j % ncols];
#pragma unroll
        for (int k = 0; k < kQ1Orb; ++k)
            if (k < ib) T1[(long long)(i0 + k) * N3 + to] = a[r][k];
    }
}

}  // namespace

#define UQC_BLAS_MP2(expr)                                                                               \
    do {                                                                                                 \
        rocblas_status b_ = (expr);                                                                      \
        if (b_ != rocblas_status_success)                                                                \
            return uqc_fail(UQC_E_DEVICE, std::string(#expr) + " failed: " + rocblas_status_to_string(b_)); \
    } while (0)

uqc_status uqc_mp2(uqc_basis* B, const double* C, const double* eps, int nocc, int nfrozen, double tau,
                   size_t batch_bytes, uqc_mp2_result* res) {
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
    const size_t NN = (size_t)N * N, N3 = NN * N;
    const size_t nT1 = (size_t)o * N3, nT2 = (size_t)o * v * NN, nZ = (size_t)o * v * v * N, nV = (size_t)o * v * o * v;
    uqc_ctx* ctx = B->ctx;
    UQC_HIP(hipSetDevice(ctx->device));
    size_t free_b = 0, total_b = 0;
    UQC_HIP(hipMemGetInfo(&free_b, &total_b));
    // memory: T1 through the first two stages, then T2 + Z + V; a batch takes nbf^2 doubles per column plus its
    // lists; the widest shell pair has 2 x 6 x 6 columns
    const double avail = 0.9 * (double)free_b - 8.0 * ((double)NN + N + 64);
    const double later = 8.0 * std::max((double)nT1 + (double)nT2, (double)nT2 + (double)nZ + (double)nV);
    const double per_col = 8.0 * (double)NN + 64.0 * N;
    double for_batch = avail - 8.0 * (double)nT1;
    if (batch_bytes > 0) for_batch = std::min(for_batch, (double)batch_bytes);
    long long wmax = 1;  // columns of the widest ket shell pair (a batch holds at least one)
    for (const Bin& by : B->bins) {
        const long long w = (long long)((by.la + 1) * (by.la + 2) / 2) * ((by.lb + 1) * (by.lb + 2) / 2);
        if (by.np > 0) wmax = std::max(wmax, 2 * w);  // both orders of a pair of two shells
    }
    // every GEMM operand stays below 2^31 doubles (a batch buffer, T2, Z): beyond that the transformations are not
    // supported
    if ((double)nT2 >= 2147483647.0 || (double)nZ >= 2147483647.0 || (double)N3 >= 2147483647.0)
        return uqc_fail(UQC_E_UNSUPPORTED, "uqc_mp2: an intermediate of the transformation exceeds 2^31 doubles");
    // a batch buffer stays below 2^31 doubles
    const long long max_cols =
        (long long)std::min({for_batch / per_col, (double)NN, (double)(((1LL << 31) - 1) / (long long)NN)});
    if (later > avail || max_cols < std::min<long long>(wmax, (long long)NN))
        return uqc_fail(UQC_E_NOMEM, "uqc_mp2: the transformed intermediates (o nbf^3 doubles and more) do not fit "
                                     "in free device memory");
    hipStream_t s = ctx->stream;
    rocblas_handle h = nullptr;
    uqc_status st = uqc::ensure_blas(ctx, &h);
    if (st != UQC_OK) return st;
    DevBuf cbuf, vbuf;
    // C, the orbital energies, the energy sums, and kQ1Orb doubles of slack after them (k_mp2_q1 reads the
    // coefficients in blocks of kQ1Orb)
    if (hipMalloc(&cbuf.p, (NN + N + 8 + kQ1Orb) * sizeof(double)) != hipSuccess)
        return uqc_fail(UQC_E_NOMEM, "uqc_mp2: C");
    double* Cd = (double*)cbuf.p;
    double* ed = Cd + NN;
    double* acc = ed + N;
    UQC_HIP(hipMemcpyAsync(Cd, C, NN * sizeof(double), hipMemcpyHostToDevice, s));
    UQC_HIP(hipMemcpyAsync(ed, eps, N * sizeof(double), hipMemcpyHostToDevice, s));
    UQC_HIP(launch_zero(acc, 8, s));
    if (hipMalloc(&vbuf.p, (nT1 + nT2) * sizeof(double)) != hipSuccess)
        return uqc_fail(UQC_E_NOMEM, "uqc_mp2: transformation buffers");
    double* T1 = (double*)vbuf.p;
    double* T2 = T1 + nT1;
    const double one = 1.0, zero = 0.0;
    const double* Co = Cd + nfrozen;  // column-major (nbf_p x nbf_mu), ld nbf: rows p = nfrozen.. are the active occupied
    const double* Cv = Cd + nocc;     // rows p = nocc.. are the virtuals

    // ---- AO integrals in ket-pair batches, each transformed over its first index at once
    long long quartets = 0;
    int nbatch = 0;
    double q1_ms = 0;
    {
        struct KetPair {
            int bin, pos, col;  // bin and position of the ket shell pair, first column in its batch
        };
        // batches of consecutive ket shell pairs (bin by bin) of at most max_cols columns
        std::vector<std::vector<KetPair>> batches(1);
        std::vector<long long> bcols(1, 0);
        for (size_t Y = 0; Y < B->bins.size(); ++Y) {
            const Bin& by = B->bins[Y];
            const int nc = (by.la + 1) * (by.la + 2) / 2, nd = (by.lb + 1) * (by.lb + 2) / 2;
            for (int q = 0; q < by.np; ++q) {
                const bool same = by.la == by.lb && by.off_a[q] == by.off_b[q];
                const int w = same ? nc * nd : 2 * nc * nd;
                if (bcols.back() + w > max_cols) {
                    batches.emplace_back();
                    bcols.push_back(0);
                }
                batches.back().push_back(KetPair{(int)Y, q, (int)bcols.back()});
                bcols.back() += w;
            }
        }
        long long widest = 0;
        for (long long c : bcols) widest = std::max(widest, c);
        DevBuf tbuf, mbuf;
        if (hipMalloc(&tbuf.p, std::max<size_t>((size_t)(NN * widest), 1) * sizeof(double)) != hipSuccess ||
            hipMalloc(&mbuf.p, std::max<size_t>((size_t)widest, 1) * sizeof(int)) != hipSuccess)
            return uqc_fail(UQC_E_NOMEM, "uqc_mp2: batch buffers");
        double* T0b = (double*)tbuf.p;
        int* dmap = (int*)mbuf.p;
        // the quartet counter, then each batch's ket positions and columns (2 ints per ket pair of the widest batch)
        size_t maxk = 1;
        for (const auto& b : batches) maxk = std::max(maxk, b.size());
        DevBuf kbuf;
        if (hipMalloc(&kbuf.p, sizeof(unsigned long long) + 2 * maxk * sizeof(int)) != hipSuccess)
            return uqc_fail(UQC_E_NOMEM, "uqc_mp2: batch ket lists");
        unsigned long long* dcount = (unsigned long long*)kbuf.p;
        int* dkp = (int*)(dcount + 1);
        UQC_HIP(launch_zero((double*)dcount, 1, s));
        UQC_HIP(launch_zero(T1, nT1, s));
        std::vector<double> qmax_bin(B->bins.size(), 0.0);  // largest pair bound of each bin
        for (size_t X = 0; X < B->bins.size(); ++X)
            for (int i = 0; i < B->bins[X].np; ++i) qmax_bin[X] = std::max(qmax_bin[X], B->bins[X].Q[i]);
        constexpr int kStreams = 3;
        hipStream_t S[kStreams] = {s, nullptr, nullptr};
        for (int k = 1; k < kStreams; ++k)
            if (!(S[k] = ctx_stream(ctx, k))) return uqc_fail(UQC_E_DEVICE, "uqc_mp2: stream creation failed");
        for (size_t bi = 0; bi < batches.size(); ++bi) {
            const auto& kp = batches[bi];
            const int ncols = (int)bcols[bi];
            if (ncols == 0) continue;
            ++nbatch;
            // columns -> (lam, sig) flat index
            std::vector<int> map(ncols);
            for (const KetPair& k : kp) {
                const Bin& by = B->bins[k.bin];
                const int nc = (by.la + 1) * (by.la + 2) / 2, nd = (by.lb + 1) * (by.lb + 2) / 2;
                const int oc = by.off_a[k.pos], od = by.off_b[k.pos];
                const bool same = by.la == by.lb && oc == od;
                for (int x = 0; x < nc; ++x)
                    for (int y = 0; y < nd; ++y) {
                        map[k.col + x * nd + y] = (oc + x) * N + (od + y);
                        if (!same) map[k.col + nc * nd + y * nc + x] = (od + y) * N + (oc + x);
                    }
            }
            // quartets: every bra shell pair (all bins) x every ket shell pair of the batch, one launch per (bra bin,
            // ket bin) in the kernel's class order (swap: the kernel's bra is the ket pair), lanes running along the
            // batch's ket pairs of the bin for one bra pair so that their columns are adjacent; the kernels screen
            // and count the quartets themselves from the batch's ket positions and columns per bin
            std::vector<std::vector<const KetPair*>> by_bin(B->bins.size());
            for (const KetPair& k : kp) by_bin[k.bin].push_back(&k);
            std::vector<int> hk(2 * kp.size());  // per ket bin in turn: positions, then (after all) columns
            std::vector<size_t> koff(B->bins.size(), 0);
            size_t nk = 0;
            for (size_t Y = 0; Y < B->bins.size(); ++Y) {
                koff[Y] = nk;
                for (const KetPair* k : by_bin[Y]) {
                    hk[nk] = k->pos;
                    hk[kp.size() + nk] = k->col;
                    ++nk;
                }
            }
            UQC_HIP(hipMemcpyAsync(dkp, hk.data(), hk.size() * sizeof(int), hipMemcpyHostToDevice, s));
            UQC_HIP(hipMemcpyAsync(dmap, map.data(), ncols * sizeof(int), hipMemcpyHostToDevice, s));
            UQC_HIP(launch_zero(T0b, NN * (size_t)ncols, s));
            // the class launches side by side (the batch positions they write are disjoint)
            UQC_HIP(hipEventRecord(ctx->fork, s));
            for (int k = 1; k < kStreams; ++k) UQC_HIP(hipStreamWaitEvent(S[k], ctx->fork, 0));
            std::vector<double> kqmax(B->bins.size(), 0.0);  // largest bound among the batch's kets of each bin
            for (const KetPair& k : kp) kqmax[k.bin] = std::max(kqmax[k.bin], B->bins[k.bin].Q[k.pos]);
            size_t seg = 0;
            for (size_t X = 0; X < B->bins.size(); ++X) {
                const Bin& bx = B->bins[X];
                for (size_t Y = 0; Y < B->bins.size(); ++Y) {
                    if (by_bin[Y].empty() || bx.np == 0 || qmax_bin[X] * kqmax[Y] < tau) continue;
                    const Bin& by = B->bins[Y];
                    const int swap = class_index(bx.la, bx.lb, by.la, by.lb) < 0 ? 1 : 0;  // not in class order
                    const Bin &bb = swap ? by : bx, &bk = swap ? bx : by;
                    const long long n = (long long)bx.np * (long long)by_bin[Y].size();
                    if (n > 0x7fffffffLL) return uqc_fail(UQC_E_UNSUPPORTED, "uqc_mp2: too many quartets per launch");
                    ListDev L{};
                    L.bra = bb.dev;
                    L.ket = bk.dev;
                    L.n = (int)n;
                    L.out = T0b;
                    L.nbf = N;
                    L.ncols = ncols;
                    L.swap = swap;
                    L.kpos = dkp + koff[Y];
                    L.col = dkp + kp.size() + koff[Y];
                    L.nket = (int)by_bin[Y].size();
                    L.tau = tau;
                    L.count = dcount;
                    UQC_HIP(launch_list(class_index(bb.la, bb.lb, bk.la, bk.lb), false, MODE_BATCH, L, ctx->boys64,
                                        ctx->boys32, S[seg++ % kStreams]));
                }
            }
            for (int k = 1; k < kStreams; ++k) {
                UQC_HIP(hipEventRecord(ctx->join[k - 1], S[k]));
                UQC_HIP(hipStreamWaitEvent(s, ctx->join[k - 1], 0));
            }
            // Q1 of the batch, straight into T1 (timed as part of the transformations once the batch's integrals
            // are done)
            const long long R = (long long)N * ncols;
            UQC_HIP(hipStreamSynchronize(s));
            const auto tq = std::chrono::steady_clock::now();
            for (int i0 = 0; i0 < o; i0 += kQ1Orb) {
                const unsigned grid = (unsigned)((R + kBlock * kQ1Cols - 1) / (kBlock * kQ1Cols));
                hipLaunchKernelGGL(k_mp2_q1, dim3(grid), dim3(kBlock), 0, s, T0b, Co, dmap, ncols, N, i0,
                                   std::min(kQ1Orb, o - i0), T1);
                UQC_HIP(hipGetLastError());
            }
            UQC_HIP(hipStreamSynchronize(s));  // the batch's ket lists are rewritten by the next batch
            q1_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tq).count();
        }
        unsigned long long nq = 0;
        UQC_HIP(hipMemcpy(&nq, dcount, sizeof(nq), hipMemcpyDeviceToHost));
        quartets = (long long)nq;
    }
    const auto t1 = std::chrono::steady_clock::now();

    // ---- the other three quarter transformations
    // Q2: per i, T2_i^T (N^2 x v) = T1_i^T (N^2 x N) * Cv^T (N x v)
    UQC_BLAS_MP2(rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, (rocblas_int)NN,
                                               v, N, &one, T1, (rocblas_int)NN, (rocblas_stride)N3, Cv, N, 0, &zero,
                                               T2, (rocblas_int)NN, (rocblas_stride)(v * NN), o));
    UQC_HIP(hipStreamSynchronize(s));
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
        res->ao_ms = ms(t0, t1) - q1_ms;
        res->transform_ms = ms(t1, t2) + q1_ms;
        res->batches = nbatch;
        res->energy_ms = ms(t2, t3);
        res->ms = ms(t0, t3);
        res->transform_flops = 2.0 * ((double)o * N3 * N + (double)o * v * N3 + (double)o * v * v * NN +
                                      (double)o * o * v * v * N);
    }
    return UQC_OK;
}
