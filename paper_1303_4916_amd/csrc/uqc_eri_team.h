// Six-lane team kernels for the classes with the largest accumulator sets (see gen_eri.py, "Team evaluation").
// One wavefront = one bra pair x 10 ket pairs; lanes 6t..6t+5 form team t and evaluate quartet (bra | ket t), lane
// 6t+p with the Cartesian axes relabelled by permutation p.  Lanes 60..63 run with weight 0.  Each lane digests its
// representative outputs in its own frame; the team's partial J/K blocks are summed at their true indices with LDS
// atomics (wavefront-local, so no block barrier is involved), then flushed with one global atomic per element.
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
// the axis permutation (q0, q1, q2).
template <class TC, bool MIXED>
__device__ __forceinline__ void team_accumulate(const BinDev& B, int bra, const BinDev& Kt, int ket, int q0, int q1,
                                                int q2, const double* __restrict__ boys64tab,
                                                const float* __restrict__ boys32tab, double* __restrict__ acc) {
    const size_t npb = (size_t)B.np, npk = (size_t)Kt.np;
    const size_t fsb = (size_t)B.K * npb, fsk = (size_t)Kt.K * npk;
    for (int kk = 0; kk < Kt.K; ++kk) {
        const double* kp = Kt.prim + (size_t)kk * npk + ket;
        const double eta = kp[F_Z * fsk];
        const double Qx = kp[F_PX * fsk], Qy = kp[F_PY * fsk], Qz = kp[F_PZ * fsk];
        const double QC0 = kp[F_PAX * fsk], QC1 = kp[F_PAY * fsk], QC2 = kp[F_PAZ * fsk];
        const double QCx = sel3(QC0, QC1, QC2, q0), QCy = sel3(QC0, QC1, QC2, q1), QCz = sel3(QC0, QC1, QC2, q2);
        const double prefk = kp[F_PREF * fsk];
        const double o2e = kp[F_O2Z * fsk];
        for (int kb = 0; kb < B.K; ++kb) {
            const double* bp = B.prim + (size_t)kb * npb + bra;
            const double zeta = bp[F_Z * fsb];
            const double Px = bp[F_PX * fsb], Py = bp[F_PY * fsb], Pz = bp[F_PZ * fsb];
            const double PA0 = bp[F_PAX * fsb], PA1 = bp[F_PAY * fsb], PA2 = bp[F_PAZ * fsb];
            const double PAx = sel3(PA0, PA1, PA2, q0), PAy = sel3(PA0, PA1, PA2, q1), PAz = sel3(PA0, PA1, PA2, q2);
            const double prefb = bp[F_PREF * fsb];
            const double o2z = bp[F_O2Z * fsb];

            const double ze = zeta + eta;
            const double inv = rcp64(ze);
            const double PQ0 = Px - Qx, PQ1 = Py - Qy, PQ2 = Pz - Qz;
            const double PQx = sel3(PQ0, PQ1, PQ2, q0), PQy = sel3(PQ0, PQ1, PQ2, q1), PQz = sel3(PQ0, PQ1, PQ2, q2);
            const double rho = zeta * eta * inv;
            const double T = rho * (PQ0 * PQ0 + PQ1 * PQ1 + PQ2 * PQ2);
            const double roz = eta * inv, roe = zeta * inv;
            const double pref = prefb * prefk * rsqrt64(ze);
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
                if (T <= (double)kBoysTmax32) {
                    boys32<TC::L>((float)T, boys32tab, F);
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
}

template <int LA, int LB, int LC, int LD, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_digest_team(const TaskDev* __restrict__ tasks,
                                                        const long long* __restrict__ task_begin, int ntask,
                                                        long long nitems, unsigned long long perm,
                                                        const double* __restrict__ boys64tab,
                                                        const float* __restrict__ boys32tab) {
    using TC = TeamClass<LA, LB, LC, LD>;
    constexpr int NA = TC::NA, NB = TC::NB, NC = TC::NC, ND = TC::ND;
    constexpr int NAB = NA * NB, NCD = NC * ND;
    // per-team partial blocks: J_cd, K_ac, K_ad, K_bc, K_bd; per-wavefront partial J_ab
    constexpr int R_JCD = 0, R_KAC = NCD, R_KAD = R_KAC + NA * NC, R_KBC = R_KAD + NA * ND, R_KBD = R_KBC + NB * NC;
    constexpr int R = R_KBD + NB * ND;
    constexpr int WAVE_LDS = (kTeamsPerWave + 1) * R + NAB;
    __shared__ double lds[kBlock / kWave][WAVE_LDS];

    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = (int)(threadIdx.x % kWave);
    const long long slot = (long long)blockIdx.x * (kBlock / kWave) + wid;
    if (slot >= nitems) return;
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
    const int team = lane / kTeam;
    const int pidx = lane - team * kTeam;
    const int kend = tk.hi[bra];
    int ket = tk.lo[bra] + (int)(li - tk.item_off[bra]) * kTeamsPerWave + team;
    bool act = team < kTeamsPerWave && ket < kend;
    if (ket >= kend) ket = kend - 1;  // idle teams recompute a valid quartet with weight 0
    {
        const double q = tk.bra.Q[bra] * tk.ket.Q[ket];
        act = act && q >= tk.tau && q > tk.lo_excl && q <= tk.hi_incl;
    }
    const unsigned long long live = __ballot(act);
    if (live == 0ULL) return;
    if (lane == 0) atomicAdd(tk.count, (unsigned long long)(__popcll(live) / kTeam));

    double* my = &lds[wid][0];
    for (int x = lane; x < WAVE_LDS; x += kWave) my[x] = 0.0;

    const int q0 = kPermAxes[pidx][0], q1 = kPermAxes[pidx][1], q2 = kPermAxes[pidx][2];
    double acc[TC::NREP];
#pragma unroll
    for (int x = 0; x < TC::NREP; ++x) acc[x] = 0.0;
    team_accumulate<TC, MIXED>(tk.bra, bra, tk.ket, ket, q0, q1, q2, boys64tab, boys32tab, acc);

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

    const BinDev& B = tk.bra;
    const BinDev& Kt = tk.ket;
    const int oa = B.off_a[bra], ob = B.off_b[bra], oc = Kt.off_a[ket], od = Kt.off_b[ket];
    const double* __restrict__ D = tk.D;
    const int N = tk.nbf;
    double dab[NAB], dcd[NCD], dbd[NB * ND], dbc[NB * NC], dad[NA * ND], dac[NA * NC];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) dab[i * NB + j] = D[(size_t)(oa + pcA[i]) * N + ob + pcB[j]];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = 0; l < ND; ++l) dcd[k * ND + l] = D[(size_t)(oc + pcC[k]) * N + od + pcD[l]];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
#pragma unroll
        for (int l = 0; l < ND; ++l) dbd[j * ND + l] = D[(size_t)(ob + pcB[j]) * N + od + pcD[l]];
#pragma unroll
        for (int k = 0; k < NC; ++k) dbc[j * NC + k] = D[(size_t)(ob + pcB[j]) * N + oc + pcC[k]];
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) {
#pragma unroll
        for (int l = 0; l < ND; ++l) dad[i * ND + l] = D[(size_t)(oa + pcA[i]) * N + od + pcD[l]];
#pragma unroll
        for (int k = 0; k < NC; ++k) dac[i * NC + k] = D[(size_t)(oa + pcA[i]) * N + oc + pcC[k]];
    }
    double w = act ? B.sdeg[bra] * Kt.sdeg[ket] : 0.0;
    if (tk.same && ket == bra) w *= 0.5;
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
    const double ABx = sel3(B.AB[bra], B.AB[B.np + bra], B.AB[2 * B.np + bra], q0);
    const double ABy = sel3(B.AB[bra], B.AB[B.np + bra], B.AB[2 * B.np + bra], q1);
    const double ABz = sel3(B.AB[bra], B.AB[B.np + bra], B.AB[2 * B.np + bra], q2);
    const double CDx = sel3(Kt.AB[ket], Kt.AB[Kt.np + ket], Kt.AB[2 * Kt.np + ket], q0);
    const double CDy = sel3(Kt.AB[ket], Kt.AB[Kt.np + ket], Kt.AB[2 * Kt.np + ket], q1);
    const double CDz = sel3(Kt.AB[ket], Kt.AB[Kt.np + ket], Kt.AB[2 * Kt.np + ket], q2);
    TC::hrr_digest(acc, src, pidx, w, ABx, ABy, ABz, CDx, CDy, CDz, dab, dcd, dbd, dbc, dad, dac, jab, jcd, kac,
                   kad, kbc, kbd);

    // team and wavefront reductions at the true component indices
    wave_lds_sync();
    double* tm = my + team * R;
    double* wj = my + (kTeamsPerWave + 1) * R;
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) atomic_add_lds(wj + pcA[i] * NB + pcB[j], jab[i * NB + j]);
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = 0; l < ND; ++l) atomic_add_lds(tm + R_JCD + pcC[k] * ND + pcD[l], jcd[k * ND + l]);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
#pragma unroll
        for (int k = 0; k < NC; ++k) atomic_add_lds(tm + R_KAC + pcA[i] * NC + pcC[k], kac[i * NC + k]);
#pragma unroll
        for (int l = 0; l < ND; ++l) atomic_add_lds(tm + R_KAD + pcA[i] * ND + pcD[l], kad[i * ND + l]);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
#pragma unroll
        for (int k = 0; k < NC; ++k) atomic_add_lds(tm + R_KBC + pcB[j] * NC + pcC[k], kbc[j * NC + k]);
#pragma unroll
        for (int l = 0; l < ND; ++l) atomic_add_lds(tm + R_KBD + pcB[j] * ND + pcD[l], kbd[j * ND + l]);
    }
    wave_lds_sync();
    // flush: J_ab by the wavefront, the rest by the lanes of each active team
    double* __restrict__ J = tk.J;
    double* __restrict__ K = tk.K;
    if (lane < NAB) {
        const double s = wj[lane];
        if (s != 0.0) atomic_add(J + (size_t)(oa + lane / NB) * N + ob + lane % NB, 2.0 * s);
    }
    if (act) {
        for (int e = pidx; e < R; e += kTeam) {
            const double s = tm[e];
            if (s == 0.0) continue;
            if (e < R_KAC) atomic_add(J + (size_t)(oc + e / ND) * N + od + e % ND, 2.0 * s);
            else if (e < R_KAD) atomic_add(K + (size_t)(oa + (e - R_KAC) / NC) * N + oc + (e - R_KAC) % NC, s);
            else if (e < R_KBC) atomic_add(K + (size_t)(oa + (e - R_KAD) / ND) * N + od + (e - R_KAD) % ND, s);
            else if (e < R_KBD) atomic_add(K + (size_t)(ob + (e - R_KBC) / NC) * N + oc + (e - R_KBC) % NC, s);
            else atomic_add(K + (size_t)(ob + (e - R_KBD) / ND) * N + od + (e - R_KBD) % ND, s);
        }
    }
}

}  // namespace uqc
