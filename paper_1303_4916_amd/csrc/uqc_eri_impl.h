// Shell-quartet electron-repulsion-integral kernels (templates), instantiated once per angular-momentum class in
// uqc_eri_class.hip.
//
// Quartet kernels.  One work item = one chunk of 64 ket shell pairs x a group of bra shell pairs of one (bra bin,
// ket bin) block.  A wavefront takes one item; every lane evaluates, for each bra pair of the group in turn, one
// contracted shell quartet (ab|cd) of the integrals of Eq. (5).  The bra pair is the same for the whole wavefront
// (wave-uniform, scalar loads) while each lane streams its own ket pair's data (coalesced, pairs stored
// field-major), which stays in cache across the group.  Per primitive quartet: Boys function (tabulated Taylor
// grid + downward recursion), Obara-Saika vertical recursion, accumulation into FP64 contracted integrals; per
// contracted quartet: horizontal recursion, then the J/K digest of Eq. (12) using the 8-fold permutational
// symmetry.
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
// [e0|f0] accumulators of class C: the leading kbn primitive pairs of the bra times the leading kkn of the ket
// (all of them: kbn = B.K, kkn = Kt.K).
// FP64 path: one loop over the primitive quartets (ket primitive outer, bra primitive inner).  The bra records are
// wavefront-uniform scalar loads; the next one is requested before the current quartet is evaluated, which costs
// scalar registers only.  Ket fields are read through 32-bit offsets from the bin's base.
// BLDS: the Boys rows come from the LDS copy `btab` of the order-L slice instead of the global table.
// SCR (Fock builds): cqk is the ket chunk's row of Kt.cq.  At ket primitive position kk, the bra primitive pairs e
// with Q_e * cqk[kk] <= kPrimEps are left out: by the Cauchy-Schwarz inequality each such primitive quartet is at
// most kPrimEps for every ket of the chunk, the same per-quartet bound as the basis-wide cut (Q_e * Q_max).  Both
// sides are ordered by decreasing bound, so the bra count only shrinks as kk grows, and the loop ends when it
// reaches zero.  (cqk is wavefront-uniform: were it not, the whole loop would turn into per-lane control flow.)
// Returns the primitive quartets evaluated per lane (wavefront-uniform).
template <class C, bool BLDS, bool SCR>
__device__ __forceinline__ int accumulate64(const BinDev& B, int bra, int kbn, const BinDev& Kt, int ket, int kkn,
                                             const double* __restrict__ boys64tab, const double2* btab,
                                             double* __restrict__ acc, cdptr cqk) {
    const unsigned npk = (unsigned)Kt.np, fsk = (unsigned)Kt.K * npk;
    const cdptr kbase = as_const(Kt.prim);
    const cdptr brec = as_const(B.rec) + (size_t)bra * B.K * kRec;  // wavefront-uniform: scalar loads
    const int KB = kbn, NPQ = kbn * kkn;
    double eta = 0, Qx = 0, Qy = 0, Qz = 0, QCx = 0, QCy = 0, QCz = 0, prefk = 0, o2e = 0;
    double b[kNumFields];
#pragma unroll
    for (int f = 0; f < kNumFields; ++f) b[f] = brec[f];
    int kb = 0, kk = 0, nb = KB, done = 0;
    for (int p = 0; p < NPQ; ++p) {
        if (kb == 0) {  // wavefront-uniform: next ket primitive
            if constexpr (SCR) {
                const double qf = cqk[kk];
                while (nb > 0 && brec[(nb - 1) * kRec + kRecQ] * qf <= kPrimEps) --nb;
                if (nb == 0) break;
            }
            done += nb;
            const unsigned o = (unsigned)kk * npk + (unsigned)ket;
            eta = kbase[o + F_Z * fsk];
            Qx = kbase[o + F_PX * fsk];
            Qy = kbase[o + F_PY * fsk];
            Qz = kbase[o + F_PZ * fsk];
            QCx = kbase[o + F_PAX * fsk];
            QCy = kbase[o + F_PAY * fsk];
            QCz = kbase[o + F_PAZ * fsk];
            prefk = kbase[o + F_PREF * fsk];
            o2e = kbase[o + F_O2Z * fsk];
        }
        const int kbn = kb + 1 == nb ? 0 : kb + 1;
        double bn[kNumFields];
        const cdptr bp = brec + kbn * kRec;
#pragma unroll
        for (int f = 0; f < kNumFields; ++f) bn[f] = bp[f];
        const double zeta = b[F_Z];
        const double ze = zeta + eta;
        const double rz = rsqrt64(ze);
        const double inv = rz * rz;
        const double PQx = b[F_PX] - Qx, PQy = b[F_PY] - Qy, PQz = b[F_PZ] - Qz;
        const double roz = eta * inv, roe = zeta * inv;
        const double T = zeta * roz * (PQx * PQx + PQy * PQy + PQz * PQz);
        const double pref = b[F_PREF] * prefk * rz;
        PrimGeom<double> g;
        g.PA[0] = b[F_PAX]; g.PA[1] = b[F_PAY]; g.PA[2] = b[F_PAZ];
        g.WP[0] = -roz * PQx; g.WP[1] = -roz * PQy; g.WP[2] = -roz * PQz;
        g.QC[0] = QCx; g.QC[1] = QCy; g.QC[2] = QCz;
        g.WQ[0] = roe * PQx; g.WQ[1] = roe * PQy; g.WQ[2] = roe * PQz;
        g.o2z = b[F_O2Z]; g.roz = roz; g.o2e = o2e; g.roe = roe; g.o2ze = 0.5 * inv;
        double F[C::L + 1];
        if constexpr (BLDS) {
            double2 r[kBoysRow / 2];
            const int gi = boys64_row_lds<C::L>(T, btab, r);
            boys64_eval<C::L>(T, gi, pref, r, F);
        } else {
            boys64<C::L>(T, pref, boys64tab, F);
        }
        C::template vrr<double>(F, g, acc);
#pragma unroll
        for (int f = 0; f < kNumFields; ++f) b[f] = bn[f];
        kb = kbn;
        if (kb == 0 && ++kk == kkn) break;
    }
    return done;
}


// accumulate64, or for MIXED the same loops with FP32 recursions (and the same SCR screen); returns the primitive
// quartets evaluated per lane (wavefront-uniform).
// MIXED: primitive quartets with Boys argument T <= t32 take the FP32 Boys table, the others the FP64 evaluation.
template <class C, bool MIXED, bool BLDS = false, bool SCR = false>
__device__ __forceinline__ int accumulate(const BinDev& B, int bra, int kbn, const BinDev& Kt, int ket, int kkn,
                                          const double* __restrict__ boys64tab, const float* __restrict__ boys32tab,
                                          double* __restrict__ acc, const double2* btab = nullptr,
                                          cdptr cqk = nullptr, double t32 = (double)kBoysTmax32) {
    if constexpr (!MIXED) return accumulate64<C, BLDS, SCR>(B, bra, kbn, Kt, ket, kkn, boys64tab, btab, acc, cqk);
    const size_t npk = (size_t)Kt.np;
    const size_t fsk = (size_t)Kt.K * npk;
    const cdptr brec = as_const(B.rec) + (size_t)bra * B.K * kRec;  // wavefront-uniform: scalar loads
    int nb = kbn, done = 0;
    for (int kk = 0; kk < kkn; ++kk) {
        if constexpr (SCR) {
            const double qf = cqk[kk];
            while (nb > 0 && brec[(nb - 1) * kRec + kRecQ] * qf <= kPrimEps) --nb;
            if (nb == 0) break;
        }
        done += nb;
        const cdptr kp = as_const(Kt.prim) + (size_t)kk * npk + ket;  // per-lane: vector loads
        const double eta = kp[F_Z * fsk];
        const double Qx = kp[F_PX * fsk], Qy = kp[F_PY * fsk], Qz = kp[F_PZ * fsk];
        const double QCx = kp[F_PAX * fsk], QCy = kp[F_PAY * fsk], QCz = kp[F_PAZ * fsk];
        const double prefk = kp[F_PREF * fsk];
        const double o2e = kp[F_O2Z * fsk];
        for (int kb = 0; kb < nb; ++kb) {
            const cdptr bp = brec + kb * kRec;
            const double zeta = bp[F_Z];
            const double Px = bp[F_PX], Py = bp[F_PY], Pz = bp[F_PZ];
            const double PAx = bp[F_PAX], PAy = bp[F_PAY], PAz = bp[F_PAZ];
            const double prefb = bp[F_PREF];
            const double o2z = bp[F_O2Z];

            const double ze = zeta + eta;
            const double rz = rsqrt64(ze);
            const double inv = rz * rz;
            const double PQx = Px - Qx, PQy = Py - Qy, PQz = Pz - Qz;
            const double rho = zeta * eta * inv;
            const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
            const double roz = eta * inv, roe = zeta * inv;
            const double pref = prefb * prefk * rz;
            {
                PrimGeom<float> g;
                g.PA[0] = (float)PAx; g.PA[1] = (float)PAy; g.PA[2] = (float)PAz;
                g.WP[0] = (float)(-roz * PQx); g.WP[1] = (float)(-roz * PQy); g.WP[2] = (float)(-roz * PQz);
                g.QC[0] = (float)QCx; g.QC[1] = (float)QCy; g.QC[2] = (float)QCz;
                g.WQ[0] = (float)(roe * PQx); g.WQ[1] = (float)(roe * PQy); g.WQ[2] = (float)(roe * PQz);
                g.o2z = (float)o2z; g.roz = (float)roz; g.o2e = (float)o2e; g.roe = (float)roe;
                g.o2ze = (float)(0.5 * inv);
                float F[C::L + 1];
                if (T <= t32) {
                    boys32<C::L>(T, boys32tab, F);
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
    return done;
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

// Partial J/K sums of one contracted quartet block v = (ab|cd) (raw components) against the scaled density, two
// at a time (Eq. 12 with the 8-fold permutational symmetry; the accumulators are symmetrised, J + J^T and K + K^T,
// in the finalize step):
//   P = 0:  x = v.D_cd  [NA*NB],  y = v.D_ab  [NC*ND]    (J_ab, J_cd)     -- d1 = D_cd, d2 = D_ab
//   P = 1:  x = v.D_bd  [NA*NC],  y = v.D_ac  [NB*ND]    (K_ac, K_bd)     -- d1 = D_bd, d2 = D_ac
//   P = 2:  x = v.D_bc  [NA*ND],  y = v.D_ad  [NB*NC]    (K_ad, K_bc)     -- d1 = D_bc, d2 = D_ad
template <int NA, int NB, int NC, int ND, int P>
__device__ __forceinline__ void contract_pair(const double* __restrict__ v, const double* d1, const double* d2,
                                              double* x, double* y) {
    constexpr int NX = P == 0 ? NA * NB : (P == 1 ? NA * NC : NA * ND);
    constexpr int NY = P == 0 ? NC * ND : (P == 1 ? NB * ND : NB * NC);
#pragma unroll
    for (int e = 0; e < NX; ++e) x[e] = 0.0;
#pragma unroll
    for (int e = 0; e < NY; ++e) y[e] = 0.0;
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int k = 0; k < NC; ++k)
#pragma unroll
                for (int l = 0; l < ND; ++l) {
                    const double t = v[((i * NB + j) * NC + k) * ND + l];
                    if constexpr (P == 0) {
                        x[i * NB + j] = fma(t, d1[k * ND + l], x[i * NB + j]);
                        y[k * ND + l] = fma(t, d2[i * NB + j], y[k * ND + l]);
                    } else if constexpr (P == 1) {
                        x[i * NC + k] = fma(t, d1[j * ND + l], x[i * NC + k]);
                        y[j * ND + l] = fma(t, d2[i * NC + k], y[j * ND + l]);
                    } else {
                        x[i * ND + l] = fma(t, d1[j * NC + k], x[i * ND + l]);
                        y[j * NC + k] = fma(t, d2[i * ND + l], y[j * NC + k]);
                    }
                }
}

// Work items of a launch of nitems items.  Workgroups are dealt to the kXcds dies round-robin (workgroup b runs on
// die b mod kXcds).  The item list is cut into segments of consecutive items, also dealt to the dies round-robin,
// so items that read the same ket chunk mostly share one die's L2 while every die gets a like mix of cheap and
// costly items (item costs drift along the list: a die owning one contiguous share of it finished long before the
// others).  A segment holds kSegItems items, fewer in launches too short to give every die eight segments (with a
// single 256-item segment for a 300-item launch, one die did nearly all the work).  Inside a die the items are
// handed out one at a time from the die's counter in the launch's queue (cleared before the launch), so a
// wavefront takes its next item when it finishes one: item costs are too uneven for a fixed share per wavefront.
// The host sizes the launch to the workgroups that fit on the chip at once; a workgroup keeps its LDS until its
// last wavefront ends, which with one item per wavefront left most of the LDS held by finished wavefronts.
constexpr long long kSegItems = 256;
struct DieItems {
    long long n;           // items of this die; its local item i is global item ((i / seg) dies + die) seg
    long long die, dies;   //   + i % seg
    long long seg;         // items per segment
    unsigned* counter;     // the die's counter in the launch's queue
};
__device__ __forceinline__ DieItems die_items(long long nitems, unsigned* queue) {
    const long long nb = gridDim.x;
    const long long dies = nb < kXcds ? nb : kXcds;  // dies holding workgroups
    const long long x = blockIdx.x % kXcds;
    long long seg = nitems / (8 * dies);
    seg = seg < 1 ? 1 : (seg > kSegItems ? kSegItems : seg);
    const long long full = nitems / seg, tail = nitems % seg;
    const long long n = (full / dies + (x < full % dies ? 1 : 0)) * seg + (x == full % dies ? tail : 0);
    return {n, x, dies, seg, queue + x};
}
// The wavefront's next local item (every lane gets the same value; n or more once the die's items are gone).
__device__ __forceinline__ long long next_item(const DieItems& di) {
    unsigned t = 0;
    if (threadIdx.x % kWave == 0)
        t = __hip_atomic_fetch_add(di.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (long long)(unsigned)__builtin_amdgcn_readfirstlane((int)t);
}
__device__ __forceinline__ long long global_item(const DieItems& di, long long i) {
    return ((i / di.seg) * di.dies + di.die) * di.seg + i % di.seg;
}

// Task holding launch-wide item `item` (task_begin ascending, task_begin[0] == 0).
__device__ __forceinline__ int find_task(const long long* __restrict__ task_begin, int ntask, long long item) {
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (task_begin[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

#ifndef UQC_WAVES_ATTR
#define UQC_WAVES_ATTR
#endif

// Partial sums a wavefront keeps across its group of bra pairs: J_cd for the whole group, K_ad and K_ac while the
// bra's first shell a stays the same (bra pairs of a chunk are ordered by a), each where registers allow.
#ifndef UQC_KEEP_LIMIT
#define UQC_KEEP_LIMIT 24
#endif
#ifndef UQC_KAC_LDS
#define UQC_KAC_LDS 1
#endif
// 1: the FP64 Fock-build kernel of this class copies the rows of its Boys slice into LDS once per workgroup and
// reads them there (the per-lane row gathers then leave the vector-memory path to the ket data and the density)
#ifndef UQC_BOYS_LDS
#define UQC_BOYS_LDS 0
#endif
constexpr int kKeepLimit = UQC_KEEP_LIMIT;
constexpr bool kKacInLds = UQC_KAC_LDS != 0;

// Quartet kernel of one class.  Work item = one chunk of 64 ket pairs x a group of bra pairs (TaskDev); lane l
// holds ket pair 64 * chunk + l for the whole group and loops over the bra pairs, which are wavefront-uniform.
// Per bra pair: exact per-lane screening and precision routing (the item's ranges are decade-accurate), the
// primitive sums, horizontal recursion, partial J/K sums.  Reductions: J_ab (one bra pair for all lanes) over the
// wavefront, then one atomic add; K_ac and K_bc over each run of adjacent lanes sharing the first ket shell c,
// then one atomic add per run; J_cd, K_ad (and K_bd) per lane.  Idle lanes compute a valid quartet with weight 0.
// NSPIN = 2 (spin densities): J from the total density, the K passes once per spin density into its own
// accumulator, the integrals evaluated once.
template <int LA, int LB, int LC, int LD, bool MIXED, int NSPIN>
__global__ __launch_bounds__(kBlock) UQC_WAVES_ATTR void k_digest(const TaskDev* __restrict__ tasks,
                                                   const long long* __restrict__ task_begin, int ntask,
                                                   long long item0, long long nitems,
                                                   const double* __restrict__ boys64tab,
                                                   const float* __restrict__ boys32tab, const WorkRedirect wr,
                                                   unsigned* __restrict__ queue) {
    using C = EriClass<LA, LB, LC, LD>;
    constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND;
    constexpr int NAB = NA * NB, NCD = NC * ND;
    // where the K_ad and K_ac sums of a same-a run are kept: 1 = registers, 2 = the lane's private LDS slots,
    // 0 = not kept (summed over the lanes of each c-run and added per bra pair)
    constexpr int KAD_MODE = NCD + NSPIN * NA * ND <= kKeepLimit ? 1 : 2;
    constexpr int KAC_MODE =
        (KAD_MODE == 1 && NCD + NSPIN * (NA * ND + NA * NC) <= kKeepLimit) ? 1 : (kKacInLds ? 2 : 0);
    constexpr bool KEEP_KAD = KAD_MODE != 0;
    constexpr bool KEEP_KAC = KAC_MODE != 0;
    constexpr int SLOTS1 = (KAD_MODE == 2 ? NA * ND : 0) + (KAC_MODE == 2 ? NA * NC : 0);  // per spin
    constexpr int SLOTS = NSPIN * SLOTS1;
    __shared__ double slots[kBlock / kWave][SLOTS > 0 ? SLOTS * kWave : 1];
    // (and only where the slots leave room for the rows in the workgroup's 160 KB of LDS)
    constexpr bool BLDS = UQC_BOYS_LDS != 0 && !MIXED &&
                          (kBlock / kWave) * (SLOTS > 0 ? SLOTS * kWave : 1) * 8 +
                                  boys_rows<C::L>() * kBoysRow * 8 <= 160 * 1024 - 1024;
    constexpr int BROWS = BLDS ? boys_rows<C::L>() : 1;
    __shared__ double2 btab[BROWS * (kBoysRow / 2)];
    if constexpr (BLDS) {  // every wavefront of the workgroup takes part before any leaves
        const double2* src = reinterpret_cast<const double2*>(boys64tab + (size_t)C::L * kBoysNg * kBoysRow);
        for (int i = (int)threadIdx.x; i < BROWS * (kBoysRow / 2); i += kBlock) btab[i] = src[i];
        __syncthreads();
    }
    // MIXED, same classes: the FP32 table's rows of the grid points an FP32 evaluation can use (T <= kBoysTmax32,
    // every order of a point in one row) in LDS as well
    constexpr int B32ROWS = kBoysTmax32 * kBoysGridPerUnit + 1;
    constexpr bool B32LDS = UQC_BOYS_LDS != 0 && MIXED &&
                            (kBlock / kWave) * (SLOTS > 0 ? SLOTS * kWave : 1) * 8 + B32ROWS * kBoysNm * 4 <=
                                160 * 1024 - 1024;
    __shared__ float b32tab[B32LDS ? B32ROWS * kBoysNm : 1];
    if constexpr (B32LDS) {
        for (int i = (int)threadIdx.x; i < B32ROWS * kBoysNm; i += kBlock) b32tab[i] = boys32tab[i];
        __syncthreads();
    }
    const float* const b32 = B32LDS ? b32tab : boys32tab;
    const DieItems di = die_items(nitems, queue);
    for (long long i = next_item(di); i < di.n; i = next_item(di)) {
        const long long item = item0 + global_item(di, i);
        const TaskDev& tk = tasks[find_task(task_begin, ntask, item)];
        const long long li = item - tk.item_begin;
        const int2 it = tk.items[li];
        const int gend = tk.items[li + 1].x;
        const BinDev& B = tk.bra;
        const BinDev& Kt = tk.ket;
        const int lane = (int)(threadIdx.x % kWave);
        const int ket = it.y * kWave + lane;
        const bool ket_ok = ket < Kt.np;
        const int kc = ket_ok ? ket : Kt.np - 1;
        const double qk = Kt.Q[kc];
        // ket primitive pairs evaluated: the most any lane's ket needs (the kets stay for the whole item)
        const int kkn = wave_max_int(ket_ok ? Kt.kp[kc] : 1);
        // the chunk's largest primitive bounds (it.y is loaded through a generic pointer: made wavefront-uniform)
        const cdptr cqk = as_const(Kt.cq) + (size_t)__builtin_amdgcn_readfirstlane(it.y) * Kt.K;
        const bool redir = NSPIN == 1 && wr.J != nullptr;  // kernel argument: wavefront-uniform
        const double* __restrict__ D = redir ? wr.D : tk.D;
        // D is read-only while the kernel runs: read through the constant address space with 32-bit offsets (N < 2^16)
        const cdptr Dc = as_const(D);
        const cdptr Dj = NSPIN == 2 ? as_const(tk.DJ) : Dc;  // density of the J pass
        double* __restrict__ J = redir ? wr.J : tk.J;
        double* __restrict__ K0 = redir ? wr.K : tk.K;
        const int N = tk.nbf;
        auto Dk = [&](int sp) { return sp == 0 ? Dc : as_const(tk.D2); };  // density of spin sp's K passes
        auto Kp = [&](int sp) { return sp == 0 ? K0 : tk.K2; };             // its accumulator
        // Only the ket index, its bound and the kept sums live across the loop; everything else about the ket is
        // re-read (from cache) through an index the compiler cannot see through, which keeps register use low.
        auto opaque = [](int x) {
            asm volatile("" : "+v"(x));
            return x;
        };
        // runs of adjacent lanes with equal first ket shell; the same shell may recur in a later, separate run (a
        // chunk can span two decades of the ket order), so runs are told apart by their index, not by the shell
        auto runs = [&](int oc, bool* inseg, bool& run_last) {
            const int kprev = __shfl_up(oc, 1, kWave);
            const bool head = lane == 0 || kprev != oc;
            const unsigned long long heads = __ballot(head);
            const unsigned long long upto = lane == kWave - 1 ? ~0ULL : ((1ULL << (lane + 1)) - 1ULL);
            const int run = __popcll(heads & upto);
#pragma unroll
            for (int st = 0; st < 6; ++st) {
                const int ro = __shfl_up(run, 1 << st, kWave);
                inseg[st] = lane >= (1 << st) && ro == run;
            }
            run_last = lane == kWave - 1 || ((heads >> (lane + 1)) & 1ULL);
        };

        double jcd_s[NCD], kad_s[NSPIN][KAD_MODE == 1 ? NA * ND : 1], kac_s[NSPIN][KAC_MODE == 1 ? NA * NC : 1];
#pragma unroll
        for (int x = 0; x < NCD; ++x) jcd_s[x] = 0.0;
#pragma unroll
        for (int sp = 0; sp < NSPIN; ++sp) {
#pragma unroll
            for (int x = 0; x < (KAD_MODE == 1 ? NA * ND : 1); ++x) kad_s[sp][x] = 0.0;
#pragma unroll
            for (int x = 0; x < (KAC_MODE == 1 ? NA * NC : 1); ++x) kac_s[sp][x] = 0.0;
        }
        // LDS slots of this lane: slot x at kept[x * kWave] (lane-contiguous, no bank conflicts, private to the lane),
        // spin sp's slots after those of the spins before it
        double* kept0 = &slots[threadIdx.x / kWave][lane];
#pragma unroll
        for (int x = 0; x < SLOTS; ++x) kept0[x * kWave] = 0.0;
        auto kad_get = [&](int sp, int x) -> double& {
            if constexpr (KAD_MODE == 2) return kept0[(sp * SLOTS1 + x) * kWave]; else return kad_s[sp][x];
        };
        auto kac_get = [&](int sp, int x) -> double& {
            if constexpr (KAC_MODE == 2) return kept0[(sp * SLOTS1 + (KAD_MODE == 2 ? NA * ND : 0) + x) * kWave];
            else return kac_s[sp][x];
        };
        int cur_a = -1;  // wavefront-uniform: first shell of the bra pairs whose K_ad / K_ac sums are held
        auto flush_a = [&]() {
            const int kl = opaque(kc);
            const int oc = Kt.off_a[kl], od = Kt.off_b[kl];
            bool inseg[6], run_last;
            if constexpr (KEEP_KAC) runs(oc, inseg, run_last);
#pragma unroll
            for (int sp = 0; sp < NSPIN; ++sp) {
                double* __restrict__ K = Kp(sp);
                if constexpr (KEEP_KAD) {
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int l = 0; l < ND; ++l) {
                            double& r = kad_get(sp, i * ND + l);
                            const double s = r;
                            r = 0.0;
                            if (s != 0.0) atomic_add(K + (size_t)(cur_a + i) * N + od + l, s);
                        }
                }
                if constexpr (KEEP_KAC) {
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            double& r = kac_get(sp, i * NC + k);
                            const double s = seg_scan(r, inseg);
                            r = 0.0;
                            if (run_last && s != 0.0) atomic_add(K + (size_t)(cur_a + i) * N + oc + k, s);
                        }
                }
            }
        };
        unsigned long long cnt = 0, pcnt = 0;
        for (int e = it.x; e < gend; ++e) {
            const int bra = __builtin_amdgcn_readfirstlane(as_const(tk.blist)[e]);  // wavefront-uniform
            const cdptr bh = as_const(B.hdr) + (size_t)bra * kHdr;  // AB, sdeg, Q, offsets of the bra pair
            const double q = bh[4] * qk;
            const bool act = ket_ok && ket >= as_const(tk.lo)[bra] && ket < as_const(tk.hi)[bra] && q >= tk.tau &&
                             q > tk.lo_excl && q <= tk.hi_incl;
            const unsigned long long live = __ballot(act);
            if (live == 0ULL) continue;  // uniform: no quartet of this bra pair survives in the chunk
            const int kbn = as_const(B.kp)[bra];
            cnt += (unsigned long long)__popcll(live);
            const int oa = ((ciptr)(bh + 5))[0], ob = ((ciptr)(bh + 5))[1];
            if (oa != cur_a) {
                if (cur_a >= 0) flush_a();
                cur_a = oa;
            }
            const int kl = opaque(kc);
            double out[NAB * NCD];
            {
                double acc[C::NACC];
#pragma unroll
                for (int x = 0; x < C::NACC; ++x) acc[x] = 0.0;
                const int done = accumulate<C, MIXED, BLDS, true>(B, bra, kbn, Kt, kl, kkn, boys64tab, b32, acc, btab,
                                                                  cqk, tk.boys_t);
                pcnt += (unsigned long long)__popcll(live) * (unsigned long long)done;
                C::hrr(acc, bh[0], bh[1], bh[2], Kt.AB[kl], Kt.AB[Kt.np + kl],
                       Kt.AB[2 * Kt.np + kl], out);
            }
            const int oc = Kt.off_a[kl], od = Kt.off_b[kl];
            double w = act ? bh[3] * Kt.sdeg[kl] : 0.0;
            if (tk.same && ket == bra) w *= 0.5;
            // Digest in three passes over the block (J; K_ac with K_bd; K_ad with K_bc), so that only two density
            // slices and two partial blocks are live at a time.
            const double w2 = 2.0 * w;
            {
                double dab[NAB], dcd[NCD], jab[NAB], jcd[NCD];
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) dab[i * NB + j] = Dj[(unsigned)(oa + i) * (unsigned)N + (unsigned)(ob + j)];
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int l = 0; l < ND; ++l) dcd[k * ND + l] = Dj[(unsigned)(oc + k) * (unsigned)N + (unsigned)(od + l)];
                contract_pair<NA, NB, NC, ND, 0>(out, dcd, dab, jab, jcd);
#pragma unroll
                for (int x = 0; x < NAB; ++x) {
                    const double s = wave_sum(w2 * jab[x]);
                    if (lane == 0) atomic_add(J + (size_t)(oa + x / NB) * N + ob + x % NB, s);
                }
#pragma unroll
                for (int x = 0; x < NCD; ++x) jcd_s[x] = fma(w2, jcd[x], jcd_s[x]);
            }
            bool inseg[6], run_last;
            runs(oc, inseg, run_last);
#pragma unroll
            for (int sp = 0; sp < NSPIN; ++sp) {
                const cdptr Ds = Dk(sp);
                double* __restrict__ K = Kp(sp);
                {
                    double dbd[NB * ND], dac[NA * NC], kac[NA * NC], kbd[NB * ND];
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int l = 0; l < ND; ++l) dbd[j * ND + l] = Ds[(unsigned)(ob + j) * (unsigned)N + (unsigned)(od + l)];
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int k = 0; k < NC; ++k) dac[i * NC + k] = Ds[(unsigned)(oa + i) * (unsigned)N + (unsigned)(oc + k)];
                    contract_pair<NA, NB, NC, ND, 1>(out, dbd, dac, kac, kbd);
                    if constexpr (KEEP_KAC) {
#pragma unroll
                        for (int x = 0; x < NA * NC; ++x) kac_get(sp, x) += w * kac[x];
                    } else {
#pragma unroll
                        for (int i = 0; i < NA; ++i)
#pragma unroll
                            for (int k = 0; k < NC; ++k) {
                                const double s = seg_scan(w * kac[i * NC + k], inseg);
                                if (run_last && s != 0.0) atomic_add(K + (size_t)(oa + i) * N + oc + k, s);
                            }
                    }
                    if (act) {
#pragma unroll
                        for (int j = 0; j < NB; ++j)
#pragma unroll
                            for (int l = 0; l < ND; ++l) atomic_add(K + (size_t)(ob + j) * N + od + l, w * kbd[j * ND + l]);
                    }
                }
                {
                    double dbc[NB * NC], dad[NA * ND], kad[NA * ND], kbc[NB * NC];
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int k = 0; k < NC; ++k) dbc[j * NC + k] = Ds[(unsigned)(ob + j) * (unsigned)N + (unsigned)(oc + k)];
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int l = 0; l < ND; ++l) dad[i * ND + l] = Ds[(unsigned)(oa + i) * (unsigned)N + (unsigned)(od + l)];
                    contract_pair<NA, NB, NC, ND, 2>(out, dbc, dad, kad, kbc);
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            const double s = seg_scan(w * kbc[j * NC + k], inseg);
                            if (run_last && s != 0.0) atomic_add(K + (size_t)(ob + j) * N + oc + k, s);
                        }
                    if constexpr (KEEP_KAD) {
#pragma unroll
                        for (int x = 0; x < NA * ND; ++x) kad_get(sp, x) += w * kad[x];
                    } else if (act) {
#pragma unroll
                        for (int i = 0; i < NA; ++i)
#pragma unroll
                            for (int l = 0; l < ND; ++l) atomic_add(K + (size_t)(oa + i) * N + od + l, w * kad[i * ND + l]);
                    }
                }
            }  // spins
        }
        if (cur_a >= 0) flush_a();
        {
            const int kl = opaque(kc);
            const int oc = Kt.off_a[kl], od = Kt.off_b[kl];
#pragma unroll
            for (int k = 0; k < NC; ++k)
#pragma unroll
                for (int l = 0; l < ND; ++l) {
                    const double s = jcd_s[k * ND + l];
                    if (s != 0.0) atomic_add(J + (size_t)(oc + k) * N + od + l, s);
                }
        }
        if (lane == 0 && cnt) {
            atomicAdd(redir ? wr.count + tk.cidx : tk.count, cnt);
            atomicAdd(redir ? wr.count + wr.ncount + tk.cidx : tk.pcount, pcnt);
        }
    }  // items
}

template <int LA, int LB, int LC, int LD, bool MIXED, int MODE>
__global__ __launch_bounds__(kBlock) void k_list(ListDev L, const double* __restrict__ boys64tab,
                                                 const float* __restrict__ boys32tab) {
    using C = EriClass<LA, LB, LC, LD>;
    const int q = (int)(blockIdx.x * kBlock + threadIdx.x);
    int bra, ket, col = 0;
    if constexpr (MODE == MODE_BATCH) {  // implicit quartet list, screened and counted here
        const bool in = q < L.n;
        const int p = in ? q / L.nket : 0, t = in ? q % L.nket : 0;
        const int kp = in ? L.kpos[t] : 0;
        const BinDev& PB = L.swap ? L.ket : L.bra;  // the physical bra and ket bins
        const BinDev& PK = L.swap ? L.bra : L.ket;
        const bool ok = in && PB.Q[p] * PK.Q[kp] >= L.tau;
        const unsigned long long m = __ballot(ok);
        if (threadIdx.x % kWave == 0 && m) atomicAdd(L.count, (unsigned long long)__popcll(m));
        if (!ok) return;
        bra = L.swap ? kp : p;
        ket = L.swap ? p : kp;
        col = L.col[t];
    } else {
        if (q >= L.n) return;
        bra = L.bra_idx[q];
        ket = L.ket_idx[q];
        (void)col;
    }
    double acc[C::NACC];
#pragma unroll
    for (int x = 0; x < C::NACC; ++x) acc[x] = 0.0;
    accumulate<C, MIXED>(L.bra, bra, L.bra.K, L.ket, ket, L.ket.K, boys64tab, boys32tab, acc);
    constexpr int NOUT = C::NA * C::NB * C::NC * C::ND;
    double out[NOUT];
    C::hrr(acc, L.bra.AB[bra], L.bra.AB[L.bra.np + bra], L.bra.AB[2 * L.bra.np + bra], L.ket.AB[ket],
           L.ket.AB[L.ket.np + ket], L.ket.AB[2 * L.ket.np + ket], out);
    if constexpr (MODE == MODE_SCATTER) {
        const size_t N = (size_t)L.nbf;
        const size_t oa = L.bra.off_a[bra], ob = L.bra.off_b[bra], oc = L.ket.off_a[ket], od = L.ket.off_b[ket];
        double* T = L.out;
#pragma unroll
        for (int i = 0; i < C::NA; ++i)
#pragma unroll
            for (int j = 0; j < C::NB; ++j)
#pragma unroll
                for (int k = 0; k < C::NC; ++k)
#pragma unroll
                    for (int l = 0; l < C::ND; ++l) {
                        const int x = ((i * C::NB + j) * C::NC + k) * C::ND + l;
                        const double v = out[x] * (comp_factor(LA, i) * comp_factor(LB, j) * comp_factor(LC, k) *
                                                   comp_factor(LD, l));
                        const size_t a = oa + i, b = ob + j, c = oc + k, d = od + l;
                        T[((a * N + b) * N + c) * N + d] = v;
                        T[((b * N + a) * N + c) * N + d] = v;
                        T[((a * N + b) * N + d) * N + c] = v;
                        T[((b * N + a) * N + d) * N + c] = v;
                        T[((c * N + d) * N + a) * N + b] = v;
                        T[((d * N + c) * N + a) * N + b] = v;
                        T[((c * N + d) * N + b) * N + a] = v;
                        T[((d * N + c) * N + b) * N + a] = v;
                    }
    } else if constexpr (MODE == MODE_BATCH) {
        const int oa = L.bra.off_a[bra], ob = L.bra.off_b[bra], oc = L.ket.off_a[ket], od = L.ket.off_b[ket];
        const bool sab = LA == LB && oa == ob, scd = LC == LD && oc == od;  // a pair of one shell: both orders
        const size_t N = (size_t)L.nbf, W = (size_t)L.ncols;              // already among its components
        const size_t col0 = (size_t)col;
        double* T = L.out;
#pragma unroll
        for (int i = 0; i < C::NA; ++i)
#pragma unroll
            for (int j = 0; j < C::NB; ++j)
#pragma unroll
                for (int k = 0; k < C::NC; ++k)
#pragma unroll
                    for (int l = 0; l < C::ND; ++l) {
                        const int x = ((i * C::NB + j) * C::NC + k) * C::ND + l;
                        const double v = out[x] * (comp_factor(LA, i) * comp_factor(LB, j) * comp_factor(LC, k) *
                                                   comp_factor(LD, l));
                        if (!L.swap) {  // rows from the kernel's bra pair, columns from its ket pair
                            const size_t r1 = (oa + i) * N + (ob + j), r2 = (ob + j) * N + (oa + i);
                            const size_t c1 = col0 + k * C::ND + l, c2 = col0 + C::NC * C::ND + l * C::NC + k;
                            T[r1 * W + c1] = v;
                            if (!scd) T[r1 * W + c2] = v;
                            if (!sab) {
                                T[r2 * W + c1] = v;
                                if (!scd) T[r2 * W + c2] = v;
                            }
                        } else {  // rows from the kernel's ket pair, columns from its bra pair
                            const size_t r1 = (oc + k) * N + (od + l), r2 = (od + l) * N + (oc + k);
                            const size_t c1 = col0 + i * C::NB + j, c2 = col0 + C::NA * C::NB + j * C::NA + i;
                            T[r1 * W + c1] = v;
                            if (!sab) T[r1 * W + c2] = v;
                            if (!scd) {
                                T[r2 * W + c1] = v;
                                if (!sab) T[r2 * W + c2] = v;
                            }
                        }
                    }
    } else if constexpr (MODE == MODE_STORE) {
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
