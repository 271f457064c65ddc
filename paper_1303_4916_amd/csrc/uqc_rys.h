// Electron-repulsion integrals by Rys quadrature (the paper's own method for the two-electron integrals, Sec.
// "Implementation details"), one contracted shell quartet per lane, for explicit block output.
//
// Per primitive quartet, with zeta, eta, P, Q, rho = zeta eta / (zeta + eta) and T = rho |PQ|^2, the Boys
// functions of the quartet are moments of the Rys weight: F_m(T) = sum_r W_r t_r^{2m} exactly for m < 2n,
// n = L/2 + 1 roots (L = la + lb + lc + ld).  Replacing F_m by W_r t_r^{2m} in the Obara-Saika recursion makes it
// separate into one-dimensional recursions per root and Cartesian direction d:
//   I(e+1, f) = C00 I(e, f) + e B10 I(e-1, f) + f B00 I(e, f-1),
//   I(e, f+1) = D00 I(e, f) + f B01 I(e, f-1) + e B00 I(e-1, f),
//   C00 = PA_d + WP_d t^2,  D00 = QC_d + WQ_d t^2,  WP = -eta/(zeta+eta) PQ,  WQ = zeta/(zeta+eta) PQ,
//   B10 = (1 - eta/(zeta+eta) t^2)/(2 zeta),  B01 = (1 - zeta/(zeta+eta) t^2)/(2 eta),  B00 = t^2/(2(zeta+eta)),
// with I(0, 0) = 1 in x and y and the root's weight times the quartet prefactor in z.  The transfer to the second
// shell of each pair, (a, b+1) = (a+1, b) + (A - B)_d (a, b) and likewise with C - D, then gives the
// one-dimensional factors of every component, and (ab|cd) = sum over roots of the product of the three.
// Roots and weights: Chebyshev fits on unit intervals of T below kRysTmax (generated/rys_table.h), the scaled
// generalised Gauss-Laguerre rule above.
#pragma once
#include "uqc_device_common.h"

#include <utility>

namespace uqc {

#include "generated/rys_consts.h"

template <int NR>
__device__ __forceinline__ void rys_roots(double T, const double* __restrict__ tab, double* x, double* w) {
    if (T < (double)kRysTmax) {
        const int i = (int)T;
        const double u = 2.0 * (T - (double)i) - 1.0;
        const double* base = tab + kRysOff[NR - 1] + (size_t)i * (2 * NR * (kRysDeg + 1));
#pragma unroll
        for (int f = 0; f < 2 * NR; ++f) {
            const double* c = base + f * (kRysDeg + 1);
            double b1 = 0.0, b2 = 0.0;  // Clenshaw
#pragma unroll
            for (int j = kRysDeg; j >= 1; --j) {
                const double t = fma(2.0 * u, b1, c[j] - b2);
                b2 = b1;
                b1 = t;
            }
            const double v = fma(u, b1, c[0] - b2);
            if (f < NR) x[f] = v; else w[f - NR] = v;
        }
    } else {
        const double it = 1.0 / T;
        const double h = 0.5 * rsqrt64(T);
        const double* lag = tab + kRysOff[kRysNmax] + NR * (NR - 1) / 2;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            x[r] = lag[r] * it;
            w[r] = lag[kRysNlag + r] * h;
        }
    }
}

// One-dimensional factors of one direction: G[a][b][c][d] for a <= LA, b <= LB, c <= LC, d <= LD, from the
// recursion coefficients of one root and the pair separations AB, CD.
template <int LA, int LB, int LC, int LD>
__device__ __forceinline__ void rys_1d(double C00, double D00, double B10, double B01, double B00, double i00,
                                       double AB, double CD, double (&G)[LA + 1][LB + 1][LC + 1][LD + 1]) {
    constexpr int LAB = LA + LB, LCD = LC + LD;
    double I[LAB + 1][LCD + 1];
    I[0][0] = i00;
#pragma unroll
    for (int e = 0; e < LAB; ++e) I[e + 1][0] = C00 * I[e][0] + (e > 0 ? e * B10 * I[e - 1][0] : 0.0);
#pragma unroll
    for (int f = 0; f < LCD; ++f)
#pragma unroll
        for (int e = 0; e <= LAB; ++e)
            I[e][f + 1] = D00 * I[e][f] + (f > 0 ? f * B01 * I[e][f - 1] : 0.0) + (e > 0 ? e * B00 * I[e - 1][f] : 0.0);
    // transfer to the bra's second shell: H[e][b][f], e + b <= LAB
    double H[LAB + 1][LB + 1][LCD + 1];
#pragma unroll
    for (int e = 0; e <= LAB; ++e)
#pragma unroll
        for (int f = 0; f <= LCD; ++f) H[e][0][f] = I[e][f];
#pragma unroll
    for (int b = 0; b < LB; ++b)
#pragma unroll
        for (int e = 0; e + b + 1 <= LAB; ++e)
#pragma unroll
            for (int f = 0; f <= LCD; ++f) H[e][b + 1][f] = H[e + 1][b][f] + AB * H[e][b][f];
    // then to the ket's second shell
#pragma unroll
    for (int a = 0; a <= LA; ++a)
#pragma unroll
        for (int b = 0; b <= LB; ++b) {
            double K2[LCD + 1][LD + 1];
#pragma unroll
            for (int f = 0; f <= LCD; ++f) K2[f][0] = H[a][b][f];
#pragma unroll
            for (int d = 0; d < LD; ++d)
#pragma unroll
                for (int f = 0; f + d + 1 <= LCD; ++f) K2[f][d + 1] = K2[f + 1][d] + CD * K2[f][d];
#pragma unroll
            for (int c = 0; c <= LC; ++c)
#pragma unroll
                for (int d = 0; d <= LD; ++d) G[a][b][c][d] = K2[c][d];
        }
}

template <int L>
struct Comps {
    static constexpr int N = (L + 1) * (L + 2) / 2;
    __device__ static constexpr int x(int i) {
        int n = 0;
        for (int a = L; a >= 0; --a)
            for (int b = L - a; b >= 0; --b) {
                if (n == i) return a;
                ++n;
            }
        return 0;
    }
    __device__ static constexpr int y(int i) {
        int n = 0;
        for (int a = L; a >= 0; --a)
            for (int b = L - a; b >= 0; --b) {
                if (n == i) return b;
                ++n;
            }
        return 0;
    }
    __device__ static constexpr int z(int i) { return L - x(i) - y(i); }
};

// Components [I0, I0 + NI) of shell a of the block (ab|cd) of quartet q: every primitive quartet and root is
// evaluated, and only those outputs are summed and stored (row-major in the whole block, component factors applied).
template <int LA, int LB, int LC, int LD, int I0, int NI>
__device__ __forceinline__ void rys_pass(const ListDev& L, int bra, int ket, const double* __restrict__ rystab,
                                         double* o) {
    constexpr int NR = (LA + LB + LC + LD) / 2 + 1;
    constexpr int NB = Comps<LB>::N, NC = Comps<LC>::N, ND = Comps<LD>::N;
    constexpr int NP = NI * NB * NC * ND;
    const BinDev &Bb = L.bra, &Bk = L.ket;
    const double AB[3] = {Bb.AB[bra], Bb.AB[Bb.np + bra], Bb.AB[2 * Bb.np + bra]};
    const double CD[3] = {Bk.AB[ket], Bk.AB[Bk.np + ket], Bk.AB[2 * Bk.np + ket]};
    double out[NP];
#pragma unroll
    for (int x = 0; x < NP; ++x) out[x] = 0.0;
    const size_t fb = (size_t)Bb.K * Bb.np, fk = (size_t)Bk.K * Bk.np;
    for (int kb = 0; kb < Bb.K; ++kb) {
        const double* bp = Bb.prim + (size_t)kb * Bb.np + bra;
        const double zeta = bp[F_Z * fb], prefb = bp[F_PREF * fb], o2z = bp[F_O2Z * fb];
        const double P[3] = {bp[F_PX * fb], bp[F_PY * fb], bp[F_PZ * fb]};
        const double PA[3] = {bp[F_PAX * fb], bp[F_PAY * fb], bp[F_PAZ * fb]};
        for (int kk = 0; kk < Bk.K; ++kk) {
            const double* kp = Bk.prim + (size_t)kk * Bk.np + ket;
            const double eta = kp[F_Z * fk], prefk = kp[F_PREF * fk], o2e = kp[F_O2Z * fk];
            const double Q[3] = {kp[F_PX * fk], kp[F_PY * fk], kp[F_PZ * fk]};
            const double QC[3] = {kp[F_PAX * fk], kp[F_PAY * fk], kp[F_PAZ * fk]};
            const double ze = zeta + eta, rz = rsqrt64(ze), inv = rz * rz;
            const double roz = eta * inv, roe = zeta * inv;
            const double PQ[3] = {P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
            const double T = zeta * roz * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
            const double pref = prefb * prefk * rz;
            double xr[NR], wr[NR];
            rys_roots<NR>(T, rystab, xr, wr);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const double t2 = xr[r];
                const double B10 = o2z * (1.0 - roz * t2), B01 = o2e * (1.0 - roe * t2), B00 = 0.5 * inv * t2;
                double Gx[LA + 1][LB + 1][LC + 1][LD + 1], Gy[LA + 1][LB + 1][LC + 1][LD + 1],
                    Gz[LA + 1][LB + 1][LC + 1][LD + 1];
                rys_1d<LA, LB, LC, LD>(PA[0] - roz * PQ[0] * t2, QC[0] + roe * PQ[0] * t2, B10, B01, B00, 1.0, AB[0],
                                       CD[0], Gx);
                rys_1d<LA, LB, LC, LD>(PA[1] - roz * PQ[1] * t2, QC[1] + roe * PQ[1] * t2, B10, B01, B00, 1.0, AB[1],
                                       CD[1], Gy);
                rys_1d<LA, LB, LC, LD>(PA[2] - roz * PQ[2] * t2, QC[2] + roe * PQ[2] * t2, B10, B01, B00,
                                       pref * wr[r], AB[2], CD[2], Gz);
#pragma unroll
                for (int ii = 0; ii < NI; ++ii)
#pragma unroll
                    for (int j = 0; j < NB; ++j)
#pragma unroll
                        for (int k = 0; k < NC; ++k)
#pragma unroll
                            for (int l = 0; l < ND; ++l) {
                                const int i = I0 + ii;
                                const int x = ((ii * NB + j) * NC + k) * ND + l;
                                out[x] = fma(Gx[Comps<LA>::x(i)][Comps<LB>::x(j)][Comps<LC>::x(k)][Comps<LD>::x(l)] *
                                                 Gy[Comps<LA>::y(i)][Comps<LB>::y(j)][Comps<LC>::y(k)][Comps<LD>::y(l)],
                                             Gz[Comps<LA>::z(i)][Comps<LB>::z(j)][Comps<LC>::z(k)][Comps<LD>::z(l)],
                                             out[x]);
                            }
            }
        }
    }
#pragma unroll
    for (int ii = 0; ii < NI; ++ii)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int k = 0; k < NC; ++k)
#pragma unroll
                for (int l = 0; l < ND; ++l) {
                    const int i = I0 + ii;
                    o[((i * NB + j) * NC + k) * ND + l] =
                        out[((ii * NB + j) * NC + k) * ND + l] *
                        (comp_factor(LA, i) * comp_factor(LB, j) * comp_factor(LC, k) * comp_factor(LD, l));
                }
}

template <int LA, int LB, int LC, int LD, int NI, int... P>
__device__ __forceinline__ void rys_passes(const ListDev& L, int bra, int ket, const double* __restrict__ rystab,
                                           double* o, std::integer_sequence<int, P...>) {
    (rys_pass<LA, LB, LC, LD, P * NI, NI>(L, bra, ket, rystab, o), ...);
}

// Block (ab|cd) of quartet q of the list (components row-major, component factors applied), as MODE_STORE.  Blocks
// of more than 216 outputs are made in one pass per component of shell a (the primitive quartets and roots evaluated
// again in each): a whole (dd|dd) block held at once took 27 KB of scratch memory per lane.
template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(kBlock) void k_list_rys(ListDev L, const double* __restrict__ rystab) {
    constexpr int NA = Comps<LA>::N, NB = Comps<LB>::N, NC = Comps<LC>::N, ND = Comps<LD>::N;
    constexpr int NOUT = NA * NB * NC * ND;
    constexpr int NI = NOUT > 216 ? 1 : NA;  // components of shell a per pass
    const int q = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (q >= L.n) return;
    const int bra = L.bra_idx[q], ket = L.ket_idx[q];
    rys_passes<LA, LB, LC, LD, NI>(L, bra, ket, rystab, L.out + (size_t)q * NOUT,
                                   std::make_integer_sequence<int, NA / NI>{});
}

}  // namespace uqc
