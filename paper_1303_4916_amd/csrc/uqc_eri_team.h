// Six-lane team kernels for the classes with the largest accumulator sets (see gen_eri.py, "Team evaluation").
// One work item = one chunk of 10 ket pairs x a group of bra pairs, taken in turn; lanes 6t..6t+5 form team t and
// evaluate quartet (bra | ket t), lane 6t+p with the Cartesian axes relabelled by permutation p.  Lanes 60..63
// run with weight 0.  Each lane digests its representative outputs in its own frame; the team's partial J/K blocks
// are summed at their true indices with LDS atomics (wavefront-local, so no block barrier is involved) and flushed
// with one global atomic per element: J_ab, K_bc, K_bd per bra pair, K_ac, K_ad when the bra's first shell
// changes, J_cd once per item.
#pragma once
#include "uqc_eri_impl.h"

namespace uqc {

constexpr int kTeam = 6;
constexpr int kTeamsPerWave = kTeamKets;

// Value of `v` held by lane `src` of the wavefront (team members read each other's accumulators).
__device__ __forceinline__ double fetch(double v, int src) { return __shfl(v, src, kWave); }

template <int LA, int LB, int LC, int LD>
struct TeamClass;

#include "generated/eri_team.h"

__device__ __forceinline__ double sel3(double x, double y, double z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Contracted representative accumulators of one lane: the recursion of class TC with the geometry relabelled by
// the axis permutation (q0, q1, q2).  The primitive screen of accumulate64 (SCR) with the ket bound at position kk
// taken as the larger of the rows cq0, cq1 of Kt.cq (the 64-pair chunks that hold the item's ten kets).  Returns
// the primitive quartets evaluated per lane (wavefront-uniform).  SCR false: every primitive quartet (cq0, cq1
// unused).
template <class TC, bool MIXED, bool SCR = true>
__device__ __forceinline__ int team_accumulate(const BinDev& B, int bra, int kbn, const BinDev& Kt, int ket, int kkn,
                                               int q0, int q1, int q2, const double* __restrict__ boys64tab,
                                               const float* __restrict__ boys32tab, double* __restrict__ acc,
                                               cdptr cq0, cdptr cq1, double t32) {
    const size_t npk = (size_t)Kt.np;
    const size_t fsk = (size_t)Kt.K * npk;
    const cdptr brec = as_const(B.rec) + (size_t)bra * B.K * kRec;  // wavefront-uniform: scalar loads
    int nb = kbn, done = 0;
    for (int kk = 0; kk < kkn; ++kk) {
        if constexpr (SCR) {
            const double qf = fmax(cq0[kk], cq1[kk]);
            while (nb > 0 && brec[(nb - 1) * kRec + kRecQ] * qf <= kPrimEps) --nb;
            if (nb == 0) break;
        }
        done += nb;
        const cdptr kp = as_const(Kt.prim) + (size_t)kk * npk + ket;  // per-lane: vector loads
        const double eta = kp[F_Z * fsk];
        const double Qx = kp[F_PX * fsk], Qy = kp[F_PY * fsk], Qz = kp[F_PZ * fsk];
        const double QC0 = kp[F_PAX * fsk], QC1 = kp[F_PAY * fsk], QC2 = kp[F_PAZ * fsk];
        const double QCx = sel3(QC0, QC1, QC2, q0), QCy = sel3(QC0, QC1, QC2, q1), QCz = sel3(QC0, QC1, QC2, q2);
        const double prefk = kp[F_PREF * fsk];
        const double o2e = kp[F_O2Z * fsk];
        for (int kb = 0; kb < nb; ++kb) {
            const cdptr bp = brec + kb * kRec;
            const double zeta = bp[F_Z];
            const double Px = bp[F_PX], Py = bp[F_PY], Pz = bp[F_PZ];
            const double PA0 = bp[F_PAX], PA1 = bp[F_PAY], PA2 = bp[F_PAZ];
            const double PAx = sel3(PA0, PA1, PA2, q0), PAy = sel3(PA0, PA1, PA2, q1), PAz = sel3(PA0, PA1, PA2, q2);
            const double prefb = bp[F_PREF];
            const double o2z = bp[F_O2Z];

            const double ze = zeta + eta;
            const double rz = rsqrt64(ze);
            const double inv = rz * rz;
            const double PQ0 = Px - Qx, PQ1 = Py - Qy, PQ2 = Pz - Qz;
            const double PQx = sel3(PQ0, PQ1, PQ2, q0), PQy = sel3(PQ0, PQ1, PQ2, q1), PQz = sel3(PQ0, PQ1, PQ2, q2);
            const double rho = zeta * eta * inv;
            const double T = rho * (PQ0 * PQ0 + PQ1 * PQ1 + PQ2 * PQ2);
            const double roz = eta * inv, roe = zeta * inv;
            const double pref = prefb * prefk * rz;
            if constexpr (!MIXED) {
                PrimGeom<double> g;
                g.PA[0] = PAx; g.PA[1] = PAy; g.PA[2] = PAz;
                g.WP[0] = -roz * PQx; g.WP[1] = -roz * PQy; g.WP[2] = -roz * PQz;
                g.QC[0] = QCx; g.QC[1] = QCy; g.QC[2] = QCz;
                g.WQ[0] = roe * PQx; g.WQ[1] = roe * PQy; g.WQ[2] = roe * PQz;
                g.o2z = o2z; g.roz = roz; g.o2e = o2e; g.roe = roe; g.o2ze = 0.5 * inv;
                double F[TC::L + 1];
                boys64<TC::L>(T, pref, boys64tab, F);
                TC::template vrr<double>(F, g, acc);
            } else {
                PrimGeom<float> g;
                g.PA[0] = (float)PAx; g.PA[1] = (float)PAy; g.PA[2] = (float)PAz;
                g.WP[0] = (float)(-roz * PQx); g.WP[1] = (float)(-roz * PQy); g.WP[2] = (float)(-roz * PQz);
                g.QC[0] = (float)QCx; g.QC[1] = (float)QCy; g.QC[2] = (float)QCz;
                g.WQ[0] = (float)(roe * PQx); g.WQ[1] = (float)(roe * PQy); g.WQ[2] = (float)(roe * PQz);
                g.o2z = (float)o2z; g.roz = (float)roz; g.o2e = (float)o2e; g.roe = (float)roe;
                g.o2ze = (float)(0.5 * inv);
                float F[TC::L + 1];
                if (T <= t32) {
                    boys32<TC::L>(T, boys32tab, F);
                    const float pf = (float)pref;
#pragma unroll
                    for (int m = 0; m <= TC::L; ++m) F[m] *= pf;
                } else {
                    double Fd[TC::L + 1];
                    boys64<TC::L>(T, pref, boys64tab, Fd);
#pragma unroll
                    for (int m = 0; m <= TC::L; ++m) F[m] = (float)Fd[m];
                }
                TC::template vrr<float>(F, g, acc);
            }
        }
    }
    return done;
}

// Streaming digest of one lane (classes with too many outputs to hold): all six density slices gathered in the
// lane's frame, every output digested into the six partial blocks as it is formed, then the blocks added into the
// team's LDS block at the true component indices.
// The J slices come from DjC (J added to the team's blocks only if WITH_J), the K slices from DkC.
template <class TC, int LA, int LB, int LC, int LD, bool WITH_J>
__device__ __forceinline__ void team_digest_stream(const double* acc, const int* src, int pidx, double w, cdptr bh,
                                                   const BinDev& Kt, int kl, int q0, int q1, int q2, cdptr DjC,
                                                   cdptr DkC, int N, int oa, int ob, int oc, int od,
                                                   const int* pcA, const int* pcB, const int* pcC, const int* pcD,
                                                   double* t_jab, double* t_jcd, double* t_kac, double* t_kad,
                                                   double* t_kbc, double* t_kbd) {
    constexpr int NA = TC::NA, NB = TC::NB, NC = TC::NC, ND = TC::ND;
    auto Dp = [&](int r, int c) { return DkC[(unsigned)r * (unsigned)N + (unsigned)c]; };
    auto Dq = [&](int r, int c) { return WITH_J ? DjC[(unsigned)r * (unsigned)N + (unsigned)c] : 0.0; };
    double dab[NA * NB], dcd[NC * ND], dbd[NB * ND], dbc[NB * NC], dad[NA * ND], dac[NA * NC];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) dab[i * NB + j] = Dq(oa + pcA[i], ob + pcB[j]);
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = 0; l < ND; ++l) dcd[k * ND + l] = Dq(oc + pcC[k], od + pcD[l]);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
#pragma unroll
        for (int l = 0; l < ND; ++l) dbd[j * ND + l] = Dp(ob + pcB[j], od + pcD[l]);
#pragma unroll
        for (int k = 0; k < NC; ++k) dbc[j * NC + k] = Dp(ob + pcB[j], oc + pcC[k]);
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) {
#pragma unroll
        for (int l = 0; l < ND; ++l) dad[i * ND + l] = Dp(oa + pcA[i], od + pcD[l]);
#pragma unroll
        for (int k = 0; k < NC; ++k) dac[i * NC + k] = Dp(oa + pcA[i], oc + pcC[k]);
    }
    double jab[NA * NB], jcd[NC * ND], kac[NA * NC], kad[NA * ND], kbc[NB * NC], kbd[NB * ND];
#pragma unroll
    for (int x = 0; x < NA * NB; ++x) jab[x] = 0.0;
#pragma unroll
    for (int x = 0; x < NC * ND; ++x) jcd[x] = 0.0;
#pragma unroll
    for (int x = 0; x < NA * NC; ++x) kac[x] = 0.0;
#pragma unroll
    for (int x = 0; x < NA * ND; ++x) kad[x] = 0.0;
#pragma unroll
    for (int x = 0; x < NB * NC; ++x) kbc[x] = 0.0;
#pragma unroll
    for (int x = 0; x < NB * ND; ++x) kbd[x] = 0.0;
    const double ABx = sel3(bh[0], bh[1], bh[2], q0), ABy = sel3(bh[0], bh[1], bh[2], q1);
    const double ABz = sel3(bh[0], bh[1], bh[2], q2);
    const double CDx = sel3(Kt.AB[kl], Kt.AB[Kt.np + kl], Kt.AB[2 * Kt.np + kl], q0);
    const double CDy = sel3(Kt.AB[kl], Kt.AB[Kt.np + kl], Kt.AB[2 * Kt.np + kl], q1);
    const double CDz = sel3(Kt.AB[kl], Kt.AB[Kt.np + kl], Kt.AB[2 * Kt.np + kl], q2);
    TC::hrr_digest(acc, src, pidx, w, ABx, ABy, ABz, CDx, CDy, CDz, dab, dcd, dbd, dbc, dad, dac, jab, jcd, kac, kad,
                   kbc, kbd);
    if constexpr (WITH_J) {
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) atomic_add_lds(t_jab + pcA[i] * NB + pcB[j], jab[i * NB + j]);
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int l = 0; l < ND; ++l) atomic_add_lds(t_jcd + pcC[k] * ND + pcD[l], jcd[k * ND + l]);
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) {
#pragma unroll
        for (int k = 0; k < NC; ++k) atomic_add_lds(t_kac + pcA[i] * NC + pcC[k], kac[i * NC + k]);
#pragma unroll
        for (int l = 0; l < ND; ++l) atomic_add_lds(t_kad + pcA[i] * ND + pcD[l], kad[i * ND + l]);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
#pragma unroll
        for (int k = 0; k < NC; ++k) atomic_add_lds(t_kbc + pcB[j] * NC + pcC[k], kbc[j * NC + k]);
#pragma unroll
        for (int l = 0; l < ND; ++l) atomic_add_lds(t_kbd + pcB[j] * ND + pcD[l], kbd[j * ND + l]);
    }
}

// Entries pidx, pidx + kTeam, ... of the R x Cn density block D[r0 + r][c0 + c] into dst (row-major).
template <int R, int Cn>
__device__ __forceinline__ void gather_slice(double* dst, cdptr Dm, int N, int r0, int c0, int pidx) {
    for (int x = pidx; x < R * Cn; x += kTeam)
        dst[x] = Dm[(unsigned)(r0 + x / Cn) * (unsigned)N + (unsigned)(c0 + x % Cn)];
}

// Doubles of a team's six density slices in LDS (D_ab, D_cd, D_ac, D_ad, D_bc, D_bd, true component order).
template <class TC>
__host__ __device__ constexpr int team_slices() {
    return TC::NA * TC::NB + TC::NC * TC::ND + TC::NA * TC::NC + TC::NA * TC::ND + TC::NB * TC::NC + TC::NB * TC::ND;
}

// team_digest_stream with the density slices and the partial blocks in LDS instead of registers, for classes whose
// accumulators alone take most of a lane's registers ((dd|dd): 185 accumulators, and six 36-element slices plus six
// 36-element partial blocks would need 617 doubles per lane).  The team's six lanes gather the slices into the
// team's slice block `sl` (true component order), then every output adds its six contributions into the team's
// partial blocks with LDS atomics.  The slices are rewritten for every quartet: the calls begin and end with a
// wavefront LDS barrier.
template <class TC, int LA, int LB, int LC, int LD, bool WITH_J>
__device__ __forceinline__ void team_digest_stream_lds(const double* acc, const int* src, int pidx, double w, cdptr bh,
                                                       const BinDev& Kt, int kl, int q0, int q1, int q2, cdptr DjC,
                                                       cdptr DkC, int N, int oa, int ob, int oc, int od,
                                                       const int* pcA, const int* pcB, const int* pcC, const int* pcD,
                                                       double* sl, double* t_jab, double* t_jcd, double* t_kac,
                                                       double* t_kad, double* t_kbc, double* t_kbd) {
    constexpr int NA = TC::NA, NB = TC::NB, NC = TC::NC, ND = TC::ND;
    constexpr int S_AB = 0, S_CD = S_AB + NA * NB, S_AC = S_CD + NC * ND, S_AD = S_AC + NA * NC;
    constexpr int S_BC = S_AD + NA * ND, S_BD = S_BC + NB * NC;
    wave_lds_sync();  // the previous quartet's reads of the slices are done
    if constexpr (WITH_J) {
        gather_slice<NA, NB>(sl + S_AB, DjC, N, oa, ob, pidx);
        gather_slice<NC, ND>(sl + S_CD, DjC, N, oc, od, pidx);
    }
    gather_slice<NA, NC>(sl + S_AC, DkC, N, oa, oc, pidx);
    gather_slice<NA, ND>(sl + S_AD, DkC, N, oa, od, pidx);
    gather_slice<NB, NC>(sl + S_BC, DkC, N, ob, oc, pidx);
    gather_slice<NB, ND>(sl + S_BD, DkC, N, ob, od, pidx);
    wave_lds_sync();
    const double ABx = sel3(bh[0], bh[1], bh[2], q0), ABy = sel3(bh[0], bh[1], bh[2], q1);
    const double ABz = sel3(bh[0], bh[1], bh[2], q2);
    const double CDx = sel3(Kt.AB[kl], Kt.AB[Kt.np + kl], Kt.AB[2 * Kt.np + kl], q0);
    const double CDy = sel3(Kt.AB[kl], Kt.AB[Kt.np + kl], Kt.AB[2 * Kt.np + kl], q1);
    const double CDz = sel3(Kt.AB[kl], Kt.AB[Kt.np + kl], Kt.AB[2 * Kt.np + kl], q2);
    TC::template hrr_digest_lds<WITH_J>(acc, src, pidx, w, ABx, ABy, ABz, CDx, CDy, CDz, sl + S_AB, sl + S_CD,
                                        sl + S_AC, sl + S_AD, sl + S_BC, sl + S_BD, t_jab, t_jcd, t_kac, t_kad, t_kbc,
                                        t_kbd, pcA, pcB, pcC, pcD);
    wave_lds_sync();  // the blocks are complete before anyone flushes them
}

// NSPIN = 2 (spin densities): J from the total density, K_ac, K_ad, K_bc, K_bd once per spin density into its
// own LDS blocks and accumulator.
template <int LA, int LB, int LC, int LD, bool MIXED, int NSPIN>
__global__ __launch_bounds__(kBlock) UQC_WAVES_ATTR void k_digest_team(const TaskDev* __restrict__ tasks,
                                                        const long long* __restrict__ task_begin, int ntask,
                                                        long long item0, long long nitems,
                                                   const double* __restrict__ boys64tab,
                                                        const float* __restrict__ boys32tab, const WorkRedirect wr,
                                                        unsigned* __restrict__ queue) {
    using TC = TeamClass<LA, LB, LC, LD>;
    constexpr int NA = TC::NA, NB = TC::NB, NC = TC::NC, ND = TC::ND;
    constexpr int NAB = NA * NB, NCD = NC * ND;
    // per-team partial blocks: J_cd, then per spin K_ac, K_ad, K_bc, K_bd, then J_ab (J_ab summed over the teams
    // when flushed); the team stride is padded to 1 mod 32 doubles, so the same entry of different teams falls in
    // different LDS banks
    constexpr int KSZ = NA * NC + NA * ND + NB * NC + NB * ND;  // K blocks of one spin
    constexpr int R_JCD = 0, R_KAC = NCD, R_KAD = R_KAC + NA * NC, R_KBC = R_KAD + NA * ND, R_KBD = R_KBC + NB * NC;
    constexpr int R_JAB = NCD + NSPIN * KSZ;
    constexpr int R = R_JAB + NAB;
    constexpr int RS = R + ((33 - R % 32) % 32);
    constexpr int WAVE_LDS = (kTeamsPerWave + 1) * RS;
    __shared__ double lds[kBlock / kWave][WAVE_LDS];
    // streaming classes, where the workgroup's LDS leaves room: every team's six density slices in LDS as well (team
    // stride padded like RS), zeroed once (the idle team's lanes leave some entries unwritten)
    constexpr int SLS = team_slices<TC>() + ((33 - team_slices<TC>() % 32) % 32);
    constexpr bool SLDS =
        TC::STREAM && NSPIN == 1 && (kBlock / kWave) * (WAVE_LDS + (kTeamsPerWave + 1) * SLS) * 8 <= 160 * 1024;
    __shared__ double slices[kBlock / kWave][SLDS ? (kTeamsPerWave + 1) * SLS : 1];
    if constexpr (SLDS) {
        const int w0 = (int)(threadIdx.x / kWave), l0 = (int)(threadIdx.x % kWave);
        for (int x = l0; x < (kTeamsPerWave + 1) * SLS; x += kWave) slices[w0][x] = 0.0;
    }

    const DieItems di = die_items(nitems, queue);
    for (long long i = next_item(di); i < di.n; i = next_item(di)) {
        const long long item = item0 + global_item(di, i);
        const int wid = (int)(threadIdx.x / kWave);
        const int lane = (int)(threadIdx.x % kWave);
        const TaskDev& tk = tasks[find_task(task_begin, ntask, item)];
        const long long li = item - tk.item_begin;
        const int2 it = tk.items[li];
        const int gend = tk.items[li + 1].x;
        const BinDev& B = tk.bra;
        const BinDev& Kt = tk.ket;
        const int team = lane / kTeam;
        const int ket = it.y * kTeamsPerWave + team;
        const bool ket_ok = team < kTeamsPerWave && ket < Kt.np;
        const int kc = ket_ok ? ket : Kt.np - 1;  // idle teams compute a valid quartet with weight 0
        const double qk = Kt.Q[kc];
        // ket primitive pairs evaluated: the most any team's ket needs (the kets stay for the whole item)
        const int kkn = wave_max_int(ket_ok ? Kt.kp[kc] : 1);
        // largest primitive bounds of the 64-pair chunks that hold the item's kets (one or two)
        const int kfirst = __builtin_amdgcn_readfirstlane(it.y) * kTeamsPerWave, klast = min(kfirst + kTeamsPerWave, Kt.np) - 1;
        const cdptr cq0 = as_const(Kt.cq) + (size_t)(kfirst / kWave) * Kt.K;
        const cdptr cq1 = as_const(Kt.cq) + (size_t)(klast / kWave) * Kt.K;
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
        // Only the ket index and its bound live across the loop; the ket's data, the lane's permutation tables and
        // the density blocks are re-read per bra pair through values the compiler cannot see through, which keeps
        // register use (and spills) down.
        auto opaque = [](int x) {
            asm volatile("" : "+v"(x));
            return x;
        };

        double* my = &lds[wid][0];
        for (int x = lane; x < WAVE_LDS; x += kWave) my[x] = 0.0;
        wave_lds_sync();
        double* tm = my + team * RS;
        // flush of the team's partial sums in [e0, e1) of its LDS block (each entry by one lane of the team), then zero;
        // the range lies inside J_cd or inside one spin's K blocks (spin sp: offsets shifted by sp * KSZ)
        auto flush = [&](int e0, int e1, int oa, int ob, int sp) {
            const int kl = opaque(kc);
            const int oc = Kt.off_a[kl], od = Kt.off_b[kl];
            double* __restrict__ K = Kp(sp);
            const int sh = sp * KSZ;
            if (team < kTeamsPerWave) {
                for (int e = e0 + lane - team * kTeam; e < e1; e += kTeam) {
                    const double s = tm[e];
                    tm[e] = 0.0;
                    if (s == 0.0) continue;
                    const int u = e - sh;
                    if (e < R_KAC) atomic_add(J + (size_t)(oc + e / ND) * N + od + e % ND, 2.0 * s);
                    else if (u < R_KAD) atomic_add(K + (size_t)(oa + (u - R_KAC) / NC) * N + oc + (u - R_KAC) % NC, s);
                    else if (u < R_KBC) atomic_add(K + (size_t)(oa + (u - R_KAD) / ND) * N + od + (u - R_KAD) % ND, s);
                    else if (u < R_KBD) atomic_add(K + (size_t)(ob + (u - R_KBC) / NC) * N + oc + (u - R_KBC) % NC, s);
                    else atomic_add(K + (size_t)(ob + (u - R_KBD) / ND) * N + od + (u - R_KBD) % ND, s);
                }
            }
        };
        int cur_a = -1;  // wavefront-uniform: first shell of the bra pairs whose K_ac / K_ad sums are held in LDS
        unsigned long long cnt = 0, pcnt = 0;
        for (int e = it.x; e < gend; ++e) {
            const int bra = __builtin_amdgcn_readfirstlane(as_const(tk.blist)[e]);  // wavefront-uniform
            const cdptr bh = as_const(B.hdr) + (size_t)bra * kHdr;  // AB, sdeg, Q, offsets of the bra pair
            const double q = bh[4] * qk;
            const bool act = ket_ok && ket >= as_const(tk.lo)[bra] && ket < as_const(tk.hi)[bra] && q >= tk.tau &&
                             q > tk.lo_excl && q <= tk.hi_incl;
            const unsigned long long live = __ballot(act);
            if (live == 0ULL) continue;
            const int kbn = as_const(B.kp)[bra];
            cnt += (unsigned long long)(__popcll(live) / kTeam);
            const int oa = ((ciptr)(bh + 5))[0], ob = ((ciptr)(bh + 5))[1];
            if (oa != cur_a) {
                if (cur_a >= 0) {
#pragma unroll
                    for (int sp = 0; sp < NSPIN; ++sp) flush(R_KAC + sp * KSZ, R_KBC + sp * KSZ, cur_a, 0, sp);
                    wave_lds_sync();
                }
                cur_a = oa;
            }
            const int kl = opaque(kc);
            const int pidx = opaque(lane - team * kTeam);
            const int q0 = kPermAxes[pidx][0], q1 = kPermAxes[pidx][1], q2 = kPermAxes[pidx][2];
            double acc[TC::NREP];
#pragma unroll
            for (int x = 0; x < TC::NREP; ++x) acc[x] = 0.0;
            const int done = team_accumulate<TC, MIXED>(B, bra, kbn, Kt, kl, kkn, q0, q1, q2, boys64tab, boys32tab, acc,
                                                        cq0, cq1, tk.boys_t);
            pcnt += (unsigned long long)(__popcll(live) / kTeam) * (unsigned long long)done;

            int src[kTeam];
#pragma unroll
            for (int x = 0; x < kTeam; ++x) src[x] = team * kTeam + kPermCompose[pidx][x];
            int pcA[NA], pcB[NB], pcC[NC], pcD[ND];
#pragma unroll
            for (int k = 0; k < NA; ++k) pcA[k] = kPermComp[LA][pidx][k];
#pragma unroll
            for (int k = 0; k < NB; ++k) pcB[k] = kPermComp[LB][pidx][k];
#pragma unroll
            for (int k = 0; k < NC; ++k) pcC[k] = kPermComp[LC][pidx][k];
#pragma unroll
            for (int k = 0; k < ND; ++k) pcD[k] = kPermComp[LD][pidx][k];
            const int oc = Kt.off_a[kl], od = Kt.off_b[kl];
            double w = act ? bh[3] * Kt.sdeg[kl] : 0.0;
            if (tk.same && ket == bra) w *= 0.5;
            if constexpr (SLDS) {
                team_digest_stream_lds<TC, LA, LB, LC, LD, true>(acc, src, pidx, w, bh, Kt, kl, q0, q1, q2, Dj, Dc, N,
                                                                 oa, ob, oc, od, pcA, pcB, pcC, pcD,
                                                                 &slices[wid][team * SLS], tm + R_JAB, tm + R_JCD,
                                                                 tm + R_KAC, tm + R_KAD, tm + R_KBC, tm + R_KBD);
            } else if constexpr (TC::STREAM) {
                team_digest_stream<TC, LA, LB, LC, LD, true>(acc, src, pidx, w, bh, Kt, kl, q0, q1, q2, Dj, Dc, N, oa, ob,
                                                             oc, od, pcA, pcB, pcC, pcD, tm + R_JAB, tm + R_JCD,
                                                             tm + R_KAC, tm + R_KAD, tm + R_KBC, tm + R_KBD);
                if constexpr (NSPIN == 2)
                    team_digest_stream<TC, LA, LB, LC, LD, false>(acc, src, pidx, w, bh, Kt, kl, q0, q1, q2, Dj,
                                                                  as_const(tk.D2), N, oa, ob, oc, od, pcA, pcB, pcC, pcD,
                                                                  tm + R_JAB, tm + R_JCD, tm + R_KAC + KSZ,
                                                                  tm + R_KAD + KSZ, tm + R_KBC + KSZ, tm + R_KBD + KSZ);
            } else {
            double out[TC::NOUT];
            {
                const double ABx = sel3(bh[0], bh[1], bh[2], q0);
                const double ABy = sel3(bh[0], bh[1], bh[2], q1);
                const double ABz = sel3(bh[0], bh[1], bh[2], q2);
                const double CDx = sel3(Kt.AB[kl], Kt.AB[Kt.np + kl], Kt.AB[2 * Kt.np + kl], q0);
                const double CDy = sel3(Kt.AB[kl], Kt.AB[Kt.np + kl], Kt.AB[2 * Kt.np + kl], q1);
                const double CDz = sel3(Kt.AB[kl], Kt.AB[Kt.np + kl], Kt.AB[2 * Kt.np + kl], q2);
                TC::hrr(acc, src, pidx, w, ABx, ABy, ABz, CDx, CDy, CDz, out);
            }
            // Digest in three passes (J_ab with J_cd; K_ac with K_bd; K_ad with K_bc), each gathering its two density
            // slices in the lane's frame and adding its two partial blocks into LDS at the true component indices.
            auto Dq = [&](int r, int c) { return Dj[(unsigned)r * (unsigned)N + (unsigned)c]; };
            {
                double d1[NCD], d2[NAB], x[NAB], y[NCD];
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int l = 0; l < ND; ++l) d1[k * ND + l] = Dq(oc + pcC[k], od + pcD[l]);
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) d2[i * NB + j] = Dq(oa + pcA[i], ob + pcB[j]);
                TC::digest0(out, d1, d2, x, y);
#pragma unroll
                for (int i = 0; i < NA; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) atomic_add_lds(tm + R_JAB + pcA[i] * NB + pcB[j], x[i * NB + j]);
#pragma unroll
                for (int k = 0; k < NC; ++k)
#pragma unroll
                    for (int l = 0; l < ND; ++l) atomic_add_lds(tm + R_JCD + pcC[k] * ND + pcD[l], y[k * ND + l]);
            }
#pragma unroll
            for (int sp = 0; sp < NSPIN; ++sp) {
                const cdptr Dsp = Dk(sp);
                auto Ds = [&](int r, int c) { return Dsp[(unsigned)r * (unsigned)N + (unsigned)c]; };
                const int sh = sp * KSZ;
                {
                    double d1[NB * ND], d2[NA * NC], x[NA * NC], y[NB * ND];
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int l = 0; l < ND; ++l) d1[j * ND + l] = Ds(ob + pcB[j], od + pcD[l]);
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int k = 0; k < NC; ++k) d2[i * NC + k] = Ds(oa + pcA[i], oc + pcC[k]);
                    TC::digest1(out, d1, d2, x, y);
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int k = 0; k < NC; ++k) atomic_add_lds(tm + R_KAC + sh + pcA[i] * NC + pcC[k], x[i * NC + k]);
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int l = 0; l < ND; ++l) atomic_add_lds(tm + R_KBD + sh + pcB[j] * ND + pcD[l], y[j * ND + l]);
                }
                {
                    double d1[NB * NC], d2[NA * ND], x[NA * ND], y[NB * NC];
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int k = 0; k < NC; ++k) d1[j * NC + k] = Ds(ob + pcB[j], oc + pcC[k]);
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int l = 0; l < ND; ++l) d2[i * ND + l] = Ds(oa + pcA[i], od + pcD[l]);
                    TC::digest2(out, d1, d2, x, y);
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int l = 0; l < ND; ++l) atomic_add_lds(tm + R_KAD + sh + pcA[i] * ND + pcD[l], x[i * ND + l]);
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int k = 0; k < NC; ++k) atomic_add_lds(tm + R_KBC + sh + pcB[j] * NC + pcC[k], y[j * NC + k]);
                }
            }  // spins
            }
            wave_lds_sync();
            // J_ab by the wavefront and the K_bc / K_bd blocks of this bra pair by each team, then cleared
            if (lane < NAB) {
                double s = 0.0;
#pragma unroll
                for (int t = 0; t < kTeamsPerWave; ++t) {
                    s += my[t * RS + R_JAB + lane];
                    my[t * RS + R_JAB + lane] = 0.0;
                }
                if (s != 0.0) atomic_add(J + (size_t)(oa + lane / NB) * N + ob + lane % NB, 2.0 * s);
            }
#pragma unroll
            for (int sp = 0; sp < NSPIN; ++sp)
                flush(R_KBC + sp * KSZ, R_KBC + sp * KSZ + NB * NC + NB * ND, oa, ob, sp);
            wave_lds_sync();
        }
        if (cur_a >= 0) {
            flush(R_JCD, R_KAC, cur_a, 0, 0);
#pragma unroll
            for (int sp = 0; sp < NSPIN; ++sp) flush(R_KAC + sp * KSZ, R_KBC + sp * KSZ, cur_a, 0, sp);
        }
        if (lane == 0 && cnt) {
            atomicAdd(redir ? wr.count + tk.cidx : tk.count, cnt);
            atomicAdd(redir ? wr.count + wr.ncount + tk.cidx : tk.pcount, pcnt);
        }
        wave_lds_sync();  // the next item clears the wavefront's LDS blocks
    }  // items
}

// k_list's BATCH form (implicit quartets of the physical bra bin x the batch's ket pairs of the physical ket bin,
// each (mu nu|lam sig) stored at its row and columns of the batch buffer) for the team classes: ten quartets per
// wavefront, lane 6t+p evaluating quartet t with the axes relabelled by permutation p (every primitive, no
// primitive screen), then storing each output it owns at its true component indices as soon as the horizontal
// recursion forms it.  The other lanes' copies of an output are zero (the owner mask), and so are outputs that
// vanish; the buffer is zero beforehand, so zeros are not stored and every element is written by one lane.
template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(kBlock) void k_list_team_batch(ListDev L, const double* __restrict__ boys64tab) {
    using TC = TeamClass<LA, LB, LC, LD>;
    constexpr int NA = TC::NA, NB = TC::NB, NC = TC::NC, ND = TC::ND;
    const int lane = (int)(threadIdx.x % kWave);
    const int team = lane / kTeam;
    const int pidx = lane - team * kTeam;  // lanes 60..63 (team 10): 0..3, idle
    const long long wave = ((long long)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const long long q = wave * kTeamsPerWave + team;
    const bool in = team < kTeamsPerWave && q < L.n;
    const int qq = in ? (int)q : 0;  // idle lanes evaluate quartet 0 and store nothing
    const int p = qq / L.nket, t = qq % L.nket;
    const int kp = L.kpos[t];
    const BinDev& PB = L.swap ? L.ket : L.bra;  // the physical bra and ket bins
    const BinDev& PK = L.swap ? L.bra : L.ket;
    const bool ok = in && PB.Q[p] * PK.Q[kp] >= L.tau;
    const unsigned long long m = __ballot(ok && pidx == 0);
    if (m == 0ULL) return;  // wavefront-uniform
    if (lane == 0) atomicAdd(L.count, (unsigned long long)__popcll(m));
    const int bra = L.swap ? kp : p, ket = L.swap ? p : kp;
    const int q0 = kPermAxes[pidx][0], q1 = kPermAxes[pidx][1], q2 = kPermAxes[pidx][2];
    double acc[TC::NREP];
#pragma unroll
    for (int x = 0; x < TC::NREP; ++x) acc[x] = 0.0;
    team_accumulate<TC, false, false>(L.bra, bra, L.bra.K, L.ket, ket, L.ket.K, q0, q1, q2, boys64tab, nullptr, acc,
                                      nullptr, nullptr, 0.0);
    int src[kTeam];
#pragma unroll
    for (int x = 0; x < kTeam; ++x) src[x] = team * kTeam + kPermCompose[pidx][x];
    int pcA[NA], pcB[NB], pcC[NC], pcD[ND];  // frame component -> true component
#pragma unroll
    for (int k = 0; k < NA; ++k) pcA[k] = kPermComp[LA][pidx][k];
#pragma unroll
    for (int k = 0; k < NB; ++k) pcB[k] = kPermComp[LB][pidx][k];
#pragma unroll
    for (int k = 0; k < NC; ++k) pcC[k] = kPermComp[LC][pidx][k];
#pragma unroll
    for (int k = 0; k < ND; ++k) pcD[k] = kPermComp[LD][pidx][k];
    const int oa = L.bra.off_a[bra], ob = L.bra.off_b[bra], oc = L.ket.off_a[ket], od = L.ket.off_b[ket];
    const bool sab = LA == LB && oa == ob, scd = LC == LD && oc == od;  // a pair of one shell: both orders
    const size_t N = (size_t)L.nbf, W = (size_t)L.ncols, col0 = ok ? (size_t)L.col[t] : 0;
    double* T = L.out;
    const bool swap = L.swap != 0;
    const auto put = [&](int n, double o) {
        if (!ok || o == 0.0) return;
        const int i = pcA[TC::OUT_IDX[n][0]], j = pcB[TC::OUT_IDX[n][1]];
        const int k = pcC[TC::OUT_IDX[n][2]], l = pcD[TC::OUT_IDX[n][3]];
        const double v = o * (comp_factor(LA, i) * comp_factor(LB, j) * comp_factor(LC, k) * comp_factor(LD, l));
        if (!swap) {  // rows from the kernel's bra pair, columns from its ket pair
            const size_t r1 = (oa + i) * N + (ob + j), r2 = (ob + j) * N + (oa + i);
            const size_t c1 = col0 + k * ND + l, c2 = col0 + NC * ND + l * NC + k;
            T[r1 * W + c1] = v;
            if (!scd) T[r1 * W + c2] = v;
            if (!sab) {
                T[r2 * W + c1] = v;
                if (!scd) T[r2 * W + c2] = v;
            }
        } else {  // rows from the kernel's ket pair, columns from its bra pair
            const size_t r1 = (oc + k) * N + (od + l), r2 = (od + l) * N + (oc + k);
            const size_t c1 = col0 + i * NB + j, c2 = col0 + NA * NB + j * NA + i;
            T[r1 * W + c1] = v;
            if (!sab) T[r1 * W + c2] = v;
            if (!scd) {
                T[r2 * W + c1] = v;
                if (!sab) T[r2 * W + c2] = v;
            }
        }
    };
    const double* ab = L.bra.AB;
    const double* cd = L.ket.AB;
    const size_t nb = (size_t)L.bra.np, nk = (size_t)L.ket.np;
    const double ABx = sel3(ab[bra], ab[nb + bra], ab[2 * nb + bra], q0);
    const double ABy = sel3(ab[bra], ab[nb + bra], ab[2 * nb + bra], q1);
    const double ABz = sel3(ab[bra], ab[nb + bra], ab[2 * nb + bra], q2);
    const double CDx = sel3(cd[ket], cd[nk + ket], cd[2 * nk + ket], q0);
    const double CDy = sel3(cd[ket], cd[nk + ket], cd[2 * nk + ket], q1);
    const double CDz = sel3(cd[ket], cd[nk + ket], cd[2 * nk + ket], q2);
    TC::hrr_emit(acc, src, pidx, 1.0, ABx, ABy, ABz, CDx, CDy, CDz, put);
}

}  // namespace uqc
