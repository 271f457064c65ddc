// Shell-quartet electron-repulsion-integral kernels (templates), instantiated once per angular-momentum class in
// uqc_eri_class.hip.
//
// Quartet kernels.  One work item = one bra shell pair x up to 64 ket shell pairs of one (bra bin, ket bin) block.
// A wavefront takes one item: every lane evaluates one contracted shell quartet (ab|cd) of the integrals of
// Eq. (5); the bra pair is the same for the whole wavefront, so its primitive-pair data are wave-uniform (scalar
// registers) while each lane streams its own ket pair's data (coalesced, pairs stored field-major).  Per primitive
// quartet: Boys function (tabulated Taylor grid + downward recursion), Obara-Saika vertical recursion,
// accumulation into FP64 contracted integrals; per contracted quartet: horizontal recursion, then the J/K digest
// of Eq. (12) using the 8-fold permutational symmetry.  J_ab (same for the whole wavefront) is reduced across the
// wavefront before one atomic add; the five per-lane blocks J_cd, K_ac, K_ad, K_bc, K_bd use FP64 atomics in L2.
#pragma once
#include "uqc_device_common.h"

namespace uqc {

template <typename T>
struct PrimGeom {
    T PA[3], WP[3], QC[3], WQ[3];
    T o2z, roz, o2e, roe, o2ze;
};

template <int LA, int LB, int LC, int LD>
struct EriClass;

#include "generated/eri_classes.h"

// ------------------------------------------------------------------------------------- contracted quartet core
// Sums the primitive quartets of (bra pair `bra` of bin B | ket pair `ket` of bin Kt) into the contracted
// [e0|f0] accumulators of class C.
template <class C, bool MIXED>
__device__ __forceinline__ void accumulate(const BinDev& B, int bra, const BinDev& Kt, int ket,
                                           const double* __restrict__ boys64tab, const float* __restrict__ boys32tab,
                                           double* __restrict__ acc) {
    const size_t npb = (size_t)B.np, npk = (size_t)Kt.np;
    const size_t fsb = (size_t)B.K * npb, fsk = (size_t)Kt.K * npk;
    for (int kk = 0; kk < Kt.K; ++kk) {
        const double* kp = Kt.prim + (size_t)kk * npk + ket;
        const double eta = kp[F_Z * fsk];
        const double Qx = kp[F_PX * fsk], Qy = kp[F_PY * fsk], Qz = kp[F_PZ * fsk];
        const double QCx = kp[F_PAX * fsk], QCy = kp[F_PAY * fsk], QCz = kp[F_PAZ * fsk];
        const double prefk = kp[F_PREF * fsk];
        const double o2e = kp[F_O2Z * fsk];
        for (int kb = 0; kb < B.K; ++kb) {
            const double* bp = B.prim + (size_t)kb * npb + bra;
            const double zeta = bp[F_Z * fsb];
            const double Px = bp[F_PX * fsb], Py = bp[F_PY * fsb], Pz = bp[F_PZ * fsb];
            const double PAx = bp[F_PAX * fsb], PAy = bp[F_PAY * fsb], PAz = bp[F_PAZ * fsb];
            const double prefb = bp[F_PREF * fsb];
            const double o2z = bp[F_O2Z * fsb];

            const double ze = zeta + eta;
            const double inv = rcp64(ze);
            const double PQx = Px - Qx, PQy = Py - Qy, PQz = Pz - Qz;
            const double rho = zeta * eta * inv;
            const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
            const double roz = eta * inv, roe = zeta * inv;
            const double pref = prefb * prefk * rsqrt64(ze);
            if constexpr (!MIXED) {
                PrimGeom<double> g;
                g.PA[0] = PAx; g.PA[1] = PAy; g.PA[2] = PAz;
                g.WP[0] = -roz * PQx; g.WP[1] = -roz * PQy; g.WP[2] = -roz * PQz;
                g.QC[0] = QCx; g.QC[1] = QCy; g.QC[2] = QCz;
                g.WQ[0] = roe * PQx; g.WQ[1] = roe * PQy; g.WQ[2] = roe * PQz;
                g.o2z = o2z; g.roz = roz; g.o2e = o2e; g.roe = roe; g.o2ze = 0.5 * inv;
                double F[C::L + 1];
                boys64<C::L>(T, pref, boys64tab, F);
                C::template vrr<double>(F, g, acc);
            } else {
                PrimGeom<float> g;
                g.PA[0] = (float)PAx; g.PA[1] = (float)PAy; g.PA[2] = (float)PAz;
                g.WP[0] = (float)(-roz * PQx); g.WP[1] = (float)(-roz * PQy); g.WP[2] = (float)(-roz * PQz);
                g.QC[0] = (float)QCx; g.QC[1] = (float)QCy; g.QC[2] = (float)QCz;
                g.WQ[0] = (float)(roe * PQx); g.WQ[1] = (float)(roe * PQy); g.WQ[2] = (float)(roe * PQz);
                g.o2z = (float)o2z; g.roz = (float)roz; g.o2e = (float)o2e; g.roe = (float)roe;
                g.o2ze = (float)(0.5 * inv);
                float F[C::L + 1];
                if (T <= (double)kBoysTmax32) {
                    boys32<C::L>((float)T, boys32tab, F);
                    const float pf = (float)pref;
#pragma unroll
                    for (int m = 0; m <= C::L; ++m) F[m] *= pf;
                } else {
                    double Fd[C::L + 1];
                    boys64<C::L>(T, pref, boys64tab, Fd);
#pragma unroll
                    for (int m = 0; m <= C::L; ++m) F[m] = (float)Fd[m];
                }
                C::template vrr<float>(F, g, acc);
            }
        }
    }
}

// Segmented inclusive sum across the wavefront: lanes with equal keys form contiguous runs; inseg[s] tells whether
// lane - 2^s belongs to the same run.  After the scan the last lane of every run holds the run's total.
__device__ __forceinline__ double seg_scan(double x, const bool* inseg) {
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const double y = __shfl_up(x, 1 << st, kWave);
        if (inseg[st]) x += y;
    }
    return x;
}

// J/K digest of one contracted quartet block v = (ab|cd) (raw components), weight w (degeneracy factors; 0 for
// idle lanes):  J_ab += 2w v.D_cd, J_cd += 2w v.D_ab, K_ac += w v.D_bd, K_ad += w v.D_bc, K_bc += w v.D_ad,
// K_bd += w v.D_ac.  The accumulators are symmetrised (J + J^T, K + K^T) in the finalize step.  The bra pair (a, b)
// is the same for every lane of the wavefront, so J_ab is summed over the wavefront before one atomic add; ket
// pairs sharing their first shell c sit in adjacent lanes, so K_ac and K_bc are summed over each such run before
// one atomic add per run; J_cd, K_ad and K_bd are added per lane.
template <int NA, int NB, int NC, int ND>
__device__ __forceinline__ void digest(const double* __restrict__ v, double w, bool act, int lane, int oa, int ob,
                                       int oc, int od, const double* __restrict__ D, double* __restrict__ J,
                                       double* __restrict__ K, int N) {
    constexpr int NAB = NA * NB, NCD = NC * ND;
    double dab[NAB], dcd[NCD], dbd[NB * ND], dbc[NB * NC], dad[NA * ND], dac[NA * NC];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) dab[i * NB + j] = D[(size_t)(oa + i) * N + ob + j];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = 0; l < ND; ++l) dcd[k * ND + l] = D[(size_t)(oc + k) * N + od + l];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
#pragma unroll
        for (int l = 0; l < ND; ++l) dbd[j * ND + l] = D[(size_t)(ob + j) * N + od + l];
#pragma unroll
        for (int k = 0; k < NC; ++k) dbc[j * NC + k] = D[(size_t)(ob + j) * N + oc + k];
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) {
#pragma unroll
        for (int l = 0; l < ND; ++l) dad[i * ND + l] = D[(size_t)(oa + i) * N + od + l];
#pragma unroll
        for (int k = 0; k < NC; ++k) dac[i * NC + k] = D[(size_t)(oa + i) * N + oc + k];
    }
    double jab[NAB], jcd[NCD], kac[NA * NC], kad[NA * ND], kbc[NB * NC], kbd[NB * ND];
#pragma unroll
    for (int x = 0; x < NAB; ++x) jab[x] = 0.0;
#pragma unroll
    for (int x = 0; x < NCD; ++x) jcd[x] = 0.0;
#pragma unroll
    for (int x = 0; x < NA * NC; ++x) kac[x] = 0.0;
#pragma unroll
    for (int x = 0; x < NA * ND; ++x) kad[x] = 0.0;
#pragma unroll
    for (int x = 0; x < NB * NC; ++x) kbc[x] = 0.0;
#pragma unroll
    for (int x = 0; x < NB * ND; ++x) kbd[x] = 0.0;
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int k = 0; k < NC; ++k)
#pragma unroll
                for (int l = 0; l < ND; ++l) {
                    const double x = v[((i * NB + j) * NC + k) * ND + l];
                    jab[i * NB + j] = fma(x, dcd[k * ND + l], jab[i * NB + j]);
                    jcd[k * ND + l] = fma(x, dab[i * NB + j], jcd[k * ND + l]);
                    kac[i * NC + k] = fma(x, dbd[j * ND + l], kac[i * NC + k]);
                    kad[i * ND + l] = fma(x, dbc[j * NC + k], kad[i * ND + l]);
                    kbc[j * NC + k] = fma(x, dad[i * ND + l], kbc[j * NC + k]);
                    kbd[j * ND + l] = fma(x, dac[i * NC + k], kbd[j * ND + l]);
                }
    const double w2 = 2.0 * w;
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const double s = wave_sum(w2 * jab[i * NB + j]);
            if (lane == 0) atomic_add(J + (size_t)(oa + i) * N + ob + j, s);
        }
    // runs of adjacent lanes with equal first ket shell; the same shell may recur in a later, separate run (the
    // wavefront can span two decades of the ket order), so runs are told apart by their index, not by the shell
    const int kprev = __shfl_up(oc, 1, kWave);
    const bool head = lane == 0 || kprev != oc;
    const unsigned long long heads = __ballot(head);
    const unsigned long long upto = lane == kWave - 1 ? ~0ULL : ((1ULL << (lane + 1)) - 1ULL);
    const int run = __popcll(heads & upto);
    bool inseg[6];
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int ro = __shfl_up(run, 1 << st, kWave);
        inseg[st] = lane >= (1 << st) && ro == run;
    }
    const bool run_last = lane == kWave - 1 || ((heads >> (lane + 1)) & 1ULL);
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const double s = seg_scan(w * kac[i * NC + k], inseg);
            if (run_last && s != 0.0) atomic_add(K + (size_t)(oa + i) * N + oc + k, s);
        }
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const double s = seg_scan(w * kbc[j * NC + k], inseg);
            if (run_last && s != 0.0) atomic_add(K + (size_t)(ob + j) * N + oc + k, s);
        }
    if (act) {
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int l = 0; l < ND; ++l) atomic_add(J + (size_t)(oc + k) * N + od + l, w2 * jcd[k * ND + l]);
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int l = 0; l < ND; ++l) atomic_add(K + (size_t)(oa + i) * N + od + l, w * kad[i * ND + l]);
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int l = 0; l < ND; ++l) atomic_add(K + (size_t)(ob + j) * N + od + l, w * kbd[j * ND + l]);
    }
}

template <int LA, int LB, int LC, int LD, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_digest(const TaskDev* __restrict__ tasks,
                                                   const long long* __restrict__ task_begin, int ntask,
                                                   long long nitems, unsigned long long perm,
                                                   const double* __restrict__ boys64tab,
                                                   const float* __restrict__ boys32tab) {
    using C = EriClass<LA, LB, LC, LD>;
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = (int)(threadIdx.x % kWave);
    const long long slot = (long long)blockIdx.x * (kBlock / kWave) + wid;
    if (slot >= nitems) return;
    // Items of one bra pair are consecutive in the work list; a bijective scatter (slot * perm mod nitems, perm
    // coprime to nitems) makes the wavefronts in flight work on different bra pairs, so their atomic updates of
    // J_ab and of the K rows of shells a and b do not pile onto the same addresses.
    const long long item = (long long)(((unsigned long long)slot * perm) % (unsigned long long)nitems);
    int t = 0;
    {
        int lo = 0, hi = ntask - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (task_begin[mid] <= item) lo = mid; else hi = mid - 1;
        }
        t = lo;
    }
    const TaskDev& tk = tasks[t];
    const long long li = item - tk.item_begin;
    int bra = 0;
    {
        int lo = 0, hi = tk.nbra - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tk.item_off[mid] <= li) lo = mid; else hi = mid - 1;
        }
        bra = lo;
    }
    const int kend = tk.hi[bra];
    int ket = tk.lo[bra] + (int)(li - tk.item_off[bra]) * kWave + lane;
    bool act = ket < kend;
    if (!act) ket = kend - 1;  // idle lanes recompute a valid quartet with weight 0 (keeps the wave converged)
    {
        // exact screening and precision routing per lane (the work range is only decade-accurate)
        const double q = tk.bra.Q[bra] * tk.ket.Q[ket];
        act = act && q >= tk.tau && q > tk.lo_excl && q <= tk.hi_incl;
    }
    const unsigned long long live = __ballot(act);
    if (live == 0ULL) return;  // uniform: nothing of this item survives screening
    if (lane == 0) atomicAdd(tk.count, (unsigned long long)__popcll(live));

    double acc[C::NACC];
#pragma unroll
    for (int x = 0; x < C::NACC; ++x) acc[x] = 0.0;
    accumulate<C, MIXED>(tk.bra, bra, tk.ket, ket, boys64tab, boys32tab, acc);

    const BinDev& B = tk.bra;
    const BinDev& Kt = tk.ket;
    double out[C::NA * C::NB * C::NC * C::ND];
    C::hrr(acc, B.AB[bra], B.AB[B.np + bra], B.AB[2 * B.np + bra], Kt.AB[ket], Kt.AB[Kt.np + ket],
           Kt.AB[2 * Kt.np + ket], out);
    double w = act ? B.sdeg[bra] * Kt.sdeg[ket] : 0.0;
    if (tk.same && ket == bra) w *= 0.5;
    digest<C::NA, C::NB, C::NC, C::ND>(out, w, act, lane, B.off_a[bra], B.off_b[bra], Kt.off_a[ket],
                                       Kt.off_b[ket], tk.D, tk.J, tk.K, tk.nbf);
}

template <int LA, int LB, int LC, int LD, bool MIXED, int MODE>
__global__ __launch_bounds__(kBlock) void k_list(ListDev L, const double* __restrict__ boys64tab,
                                                 const float* __restrict__ boys32tab) {
    using C = EriClass<LA, LB, LC, LD>;
    const int q = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (q >= L.n) return;
    const int bra = L.bra_idx[q], ket = L.ket_idx[q];
    double acc[C::NACC];
#pragma unroll
    for (int x = 0; x < C::NACC; ++x) acc[x] = 0.0;
    accumulate<C, MIXED>(L.bra, bra, L.ket, ket, boys64tab, boys32tab, acc);
    constexpr int NOUT = C::NA * C::NB * C::NC * C::ND;
    double out[NOUT];
    C::hrr(acc, L.bra.AB[bra], L.bra.AB[L.bra.np + bra], L.bra.AB[2 * L.bra.np + bra], L.ket.AB[ket],
           L.ket.AB[L.ket.np + ket], L.ket.AB[2 * L.ket.np + ket], out);
    if constexpr (MODE == MODE_STORE) {
        double* o = L.out + (size_t)q * NOUT;
#pragma unroll
        for (int i = 0; i < C::NA; ++i)
#pragma unroll
            for (int j = 0; j < C::NB; ++j)
#pragma unroll
                for (int k = 0; k < C::NC; ++k)
#pragma unroll
                    for (int l = 0; l < C::ND; ++l) {
                        const int x = ((i * C::NB + j) * C::NC + k) * C::ND + l;
                        o[x] = out[x] * (comp_factor(LA, i) * comp_factor(LB, j) * comp_factor(LC, k) *
                                         comp_factor(LD, l));
                    }
    } else {
        // Schwarz bound of a diagonal quartet (ab|ab): sqrt of the largest (ij|ij) over normalised components
        constexpr int NAB = C::NA * C::NB;
        double m = 0.0;
#pragma unroll
        for (int i = 0; i < C::NA; ++i)
#pragma unroll
            for (int j = 0; j < C::NB; ++j) {
                const double f = comp_factor(LA, i) * comp_factor(LB, j);
                m = fmax(m, out[(i * C::NB + j) * NAB + i * C::NB + j] * (f * f));
            }
        L.out[q] = sqrt(m);
    }
}

}  // namespace uqc
