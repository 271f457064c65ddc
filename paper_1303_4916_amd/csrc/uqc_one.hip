// One-electron integrals of Eq. (2)-(4) over the contracted Cartesian basis: overlap S, kinetic T and the
// attraction V to point nuclei.  One thread per shell pair (a, b) with l_a > l_b, or l_a == l_b and a >= b, of one
// class; it writes the block and its transpose.  Obara-Saika form, per primitive pair (alpha at A, beta at B,
// p = alpha + beta, P = (alpha A + beta B)/p, E_AB = exp(-alpha beta/p |A-B|^2)):
//   one-dimensional overlaps  s_{00} = 1,  s_{i+1,j} = PA s_{ij} + (i s_{i-1,j} + j s_{i,j-1})/(2p),
//                             s_{i,j+1} = PB s_{ij} + (i s_{i-1,j} + j s_{i,j-1})/(2p);
//   S = (pi/p)^{3/2} E_AB s_x s_y s_z;
//   kinetic, symmetric form T = 1/2 <grad a|grad b>, per direction
//     t_{ij} = 1/2 (i j s_{i-1,j-1} - 2 alpha j s_{i+1,j-1} - 2 beta i s_{i-1,j+1} + 4 alpha beta s_{i+1,j+1}),
//   T = (pi/p)^{3/2} E_AB (t_x s_y s_z + s_x t_y s_z + s_x s_y t_z);
//   attraction: V = -sum_C Z_C (2 pi/p) E_AB [a|b]^(0), the auxiliary integrals from the generated recursion
//   (AttractionClass) seeded with F_m(p |P-C|^2).
// Every block is scaled by the component factors f_i f_j at the end (the shell coefficients normalise the axis
// components).
#include "uqc_device_common.h"
#include "uqc_one.h"

namespace uqc {

template <int LA, int LB>
struct AttractionClass;

#include "generated/one_electron.h"

template <int LA, int LB>
__device__ __forceinline__ void overlap_1d(double PA, double PB, double o2p, double (&s)[LA + 2][LB + 2]) {
    s[0][0] = 1.0;
#pragma unroll
    for (int i = 0; i <= LA; ++i) s[i + 1][0] = PA * s[i][0] + (i > 0 ? i * s[i - 1][0] * o2p : 0.0);
#pragma unroll
    for (int j = 0; j <= LB; ++j)
#pragma unroll
        for (int i = 0; i <= LA + 1; ++i)
            s[i][j + 1] = PB * s[i][j] + ((i > 0 ? i * s[i - 1][j] : 0.0) + (j > 0 ? j * s[i][j - 1] : 0.0)) * o2p;
}

template <int LA, int LB>
__global__ __launch_bounds__(kBlock) void k_overlap_kinetic(ShellsDev sh, const int2* __restrict__ pairs,
                                                            int npairs, const double* __restrict__ f,
                                                            double* __restrict__ S, double* __restrict__ T, int N) {
    constexpr int NA = (LA + 1) * (LA + 2) / 2, NB = (LB + 1) * (LB + 2) / 2;
    const int t = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (t >= npairs) return;
    const int a = pairs[t].x, b = pairs[t].y;
    int pa[NA][3], pb[NB][3];
    {
        int n = 0;
#pragma unroll
        for (int x = LA; x >= 0; --x)
#pragma unroll
            for (int y = LA - x; y >= 0; --y) { pa[n][0] = x; pa[n][1] = y; pa[n][2] = LA - x - y; ++n; }
        n = 0;
#pragma unroll
        for (int x = LB; x >= 0; --x)
#pragma unroll
            for (int y = LB - x; y >= 0; --y) { pb[n][0] = x; pb[n][1] = y; pb[n][2] = LB - x - y; ++n; }
    }
    double sacc[NA * NB], tacc[NA * NB];
#pragma unroll
    for (int x = 0; x < NA * NB; ++x) sacc[x] = tacc[x] = 0.0;
    const double Ax = sh.A[3 * a], Ay = sh.A[3 * a + 1], Az = sh.A[3 * a + 2];
    const double Bx = sh.A[3 * b], By = sh.A[3 * b + 1], Bz = sh.A[3 * b + 2];
    const double AB2 = (Ax - Bx) * (Ax - Bx) + (Ay - By) * (Ay - By) + (Az - Bz) * (Az - Bz);
    for (int p1 = 0; p1 < sh.K[a]; ++p1) {
        const double al = sh.alpha[sh.pstart[a] + p1], ca = sh.c[sh.pstart[a] + p1];
        for (int p2 = 0; p2 < sh.K[b]; ++p2) {
            const double be = sh.alpha[sh.pstart[b] + p2], cb = sh.c[sh.pstart[b] + p2];
            const double p = al + be, ip = 1.0 / p, o2p = 0.5 * ip;
            const double Px = (al * Ax + be * Bx) * ip, Py = (al * Ay + be * By) * ip, Pz = (al * Az + be * Bz) * ip;
            const double pref = ca * cb * exp(-al * be * ip * AB2) * (kPi * ip) * sqrt(kPi * ip);
            double sx[LA + 2][LB + 2], sy[LA + 2][LB + 2], sz[LA + 2][LB + 2];
            overlap_1d<LA, LB>(Px - Ax, Px - Bx, o2p, sx);
            overlap_1d<LA, LB>(Py - Ay, Py - By, o2p, sy);
            overlap_1d<LA, LB>(Pz - Az, Pz - Bz, o2p, sz);
            auto kin = [&](const double (&s)[LA + 2][LB + 2], int i, int j) {
                double v = 4.0 * al * be * s[i + 1][j + 1];
                if (j > 0) v -= 2.0 * al * j * s[i + 1][j - 1];
                if (i > 0) v -= 2.0 * be * i * s[i - 1][j + 1];
                if (i > 0 && j > 0) v += (double)(i * j) * s[i - 1][j - 1];
                return 0.5 * v;
            };
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const int ix = pa[i][0], iy = pa[i][1], iz = pa[i][2];
                    const int jx = pb[j][0], jy = pb[j][1], jz = pb[j][2];
                    const double ox = sx[ix][jx], oy = sy[iy][jy], oz = sz[iz][jz];
                    sacc[i * NB + j] = fma(pref, ox * oy * oz, sacc[i * NB + j]);
                    tacc[i * NB + j] = fma(pref, kin(sx, ix, jx) * oy * oz + ox * kin(sy, iy, jy) * oz +
                                                     ox * oy * kin(sz, iz, jz), tacc[i * NB + j]);
                }
        }
    }
    const int oa = sh.off[a], ob = sh.off[b];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const double ff = f[oa + i] * f[ob + j];
            const double sv = ff * sacc[i * NB + j], tv = ff * tacc[i * NB + j];
            if (S) { S[(size_t)(oa + i) * N + ob + j] = sv; S[(size_t)(ob + j) * N + oa + i] = sv; }
            if (T) { T[(size_t)(oa + i) * N + ob + j] = tv; T[(size_t)(ob + j) * N + oa + i] = tv; }
        }
}

template <int LA, int LB>
__global__ __launch_bounds__(kBlock) void k_attraction(ShellsDev sh, const int2* __restrict__ pairs, int npairs,
                                                       int natom, const double* __restrict__ Z,
                                                       const double* __restrict__ R, const double* __restrict__ f,
                                                       double* __restrict__ V, int N,
                                                       const double* __restrict__ boys64tab) {
    using AC = AttractionClass<LA, LB>;
    constexpr int NA = (LA + 1) * (LA + 2) / 2, NB = (LB + 1) * (LB + 2) / 2;
    const int t = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (t >= npairs) return;
    const int a = pairs[t].x, b = pairs[t].y;
    double v[NA * NB];
#pragma unroll
    for (int x = 0; x < NA * NB; ++x) v[x] = 0.0;
    const double Ax = sh.A[3 * a], Ay = sh.A[3 * a + 1], Az = sh.A[3 * a + 2];
    const double Bx = sh.A[3 * b], By = sh.A[3 * b + 1], Bz = sh.A[3 * b + 2];
    const double ABx = Ax - Bx, ABy = Ay - By, ABz = Az - Bz;
    const double AB2 = ABx * ABx + ABy * ABy + ABz * ABz;
    for (int p1 = 0; p1 < sh.K[a]; ++p1) {
        const double al = sh.alpha[sh.pstart[a] + p1], ca = sh.c[sh.pstart[a] + p1];
        for (int p2 = 0; p2 < sh.K[b]; ++p2) {
            const double be = sh.alpha[sh.pstart[b] + p2], cb = sh.c[sh.pstart[b] + p2];
            const double p = al + be, ip = 1.0 / p;
            const double Px = (al * Ax + be * Bx) * ip, Py = (al * Ay + be * By) * ip, Pz = (al * Az + be * Bz) * ip;
            const double pref = -ca * cb * exp(-al * be * ip * AB2) * 2.0 * kPi * ip;
            for (int n = 0; n < natom; ++n) {
                const double PCx = Px - R[3 * n], PCy = Py - R[3 * n + 1], PCz = Pz - R[3 * n + 2];
                double F[AC::L + 1];
                boys64<AC::L>(p * (PCx * PCx + PCy * PCy + PCz * PCz), pref * Z[n], boys64tab, F);
                AC::add(F, Px - Ax, Py - Ay, Pz - Az, PCx, PCy, PCz, ABx, ABy, ABz, 0.5 * ip, v);
            }
        }
    }
    const int oa = sh.off[a], ob = sh.off[b];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const double vv = f[oa + i] * f[ob + j] * v[i * NB + j];
            V[(size_t)(oa + i) * N + ob + j] = vv;
            V[(size_t)(ob + j) * N + oa + i] = vv;
        }
}

template <int LA, int LB>
static hipError_t launch_pair_class(const ShellsDev& sh, const int2* pairs, int npairs, int natom, const double* Z,
                                    const double* R, const double* f, double* S, double* T, double* V, int N,
                                    const double* boys64tab, hipStream_t s) {
    if (npairs <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((npairs + kBlock - 1) / kBlock);
    if (S || T)
        hipLaunchKernelGGL((k_overlap_kinetic<LA, LB>), dim3(nb), dim3(kBlock), 0, s, sh, pairs, npairs, f, S, T, N);
    if (V)
        hipLaunchKernelGGL((k_attraction<LA, LB>), dim3(nb), dim3(kBlock), 0, s, sh, pairs, npairs, natom, Z, R, f, V,
                           N, boys64tab);
    return hipGetLastError();
}

hipError_t launch_one_electron(int pair_class, const ShellsDev& sh, const int2* pairs, int npairs, int natom,
                               const double* Z, const double* R, const double* f, double* S, double* T, double* V,
                               int N, const double* boys64tab, hipStream_t s) {
    switch (pair_class) {
        case 0: return launch_pair_class<0, 0>(sh, pairs, npairs, natom, Z, R, f, S, T, V, N, boys64tab, s);
        case 1: return launch_pair_class<1, 0>(sh, pairs, npairs, natom, Z, R, f, S, T, V, N, boys64tab, s);
        case 2: return launch_pair_class<1, 1>(sh, pairs, npairs, natom, Z, R, f, S, T, V, N, boys64tab, s);
        case 3: return launch_pair_class<2, 0>(sh, pairs, npairs, natom, Z, R, f, S, T, V, N, boys64tab, s);
        case 4: return launch_pair_class<2, 1>(sh, pairs, npairs, natom, Z, R, f, S, T, V, N, boys64tab, s);
        case 5: return launch_pair_class<2, 2>(sh, pairs, npairs, natom, Z, R, f, S, T, V, N, boys64tab, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace uqc
