// CPU oracle for the two-electron integrals and the Coulomb/exchange build.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load
// this library.  It shares no code, header, table or helper with the HIP library; the two meet only through the
// seeded input generator (which draws inputs and does none of this arithmetic).
//
// What it computes (paper, Sec. "Implementation details"):
//   * basis functions: contracted Cartesian Gaussians, Eq. (1);
//   * electron-repulsion integrals (ij|kl), Eq. (5), evaluated exactly (the "analytic" route the paper attributes
//     to Cook, here the McMurchie-Davidson Hermite expansion);
//   * J_ij = sum_kl (ij|kl) D_kl and K_il = sum_jk (ij|kl) D_jk, Eq. (12), for a symmetric density D;
//   * G = J - K/2 and E2 = 1/2 sum_ij D_ij G_ij (closed-shell convention of Szabo-Ostlund, which the paper follows);
//   * overlap, kinetic and nuclear-attraction integrals, Eq. (2)-(4), for the restricted Hartree-Fock reference
//     (the SCF iteration itself is in the Python package, on top of these integrals and J/K).
//
// Readings of points the paper leaves open (each listed in the design notes):
//   * one exponent per primitive, shared by every Cartesian component of a shell;
//   * coefficients refer to normalised primitives; every Cartesian component is normalised on its own (S_ii = 1);
//   * component order inside a shell: descending x power, then descending y power (xx, xy, xz, yy, yz, zz);
//   * units are bohr / hartree;
//   * Schwarz screening keeps a shell quartet iff Q_ab * Q_cd >= tau, Q_ab = sqrt(max_ij (ij|ij)); tau = 0 keeps all.
//
// Precision: double throughout, the Boys function in long double (rounded once to double).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

// ---------------------------------------------------------------------------------------------------------------
// Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt.
//   T < 30 : F_m(T) = exp(-T) * sum_{k>=0} (2T)^k / [(2m+1)(2m+3)...(2m+2k+1)]   (all terms positive)
//   T >= 30: F_0(T) = 1/2 sqrt(pi/T) erf(sqrt(T)), then F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T)   (stable for T >> m)
// ---------------------------------------------------------------------------------------------------------------
long double boys_ld(int m, long double T) {
    if (T == 0.0L) return 1.0L / (2 * m + 1);
    if (T < 30.0L) {
        long double term = 1.0L / (2 * m + 1);
        long double sum = term;
        for (int k = 1; k < 2000; ++k) {
            term *= (2.0L * T) / (2 * m + 2 * k + 1);
            sum += term;
            if (term < 1e-21L * sum) break;
        }
        return std::exp(-T) * sum;
    }
    const long double pi = 3.141592653589793238462643383279502884L;
    long double f = 0.5L * std::sqrt(pi / T) * std::erf(std::sqrt(T));
    const long double e = std::exp(-T);
    for (int k = 0; k < m; ++k) f = ((2 * k + 1) * f - e) / (2.0L * T);
    return f;
}

int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Cartesian exponents of component c of a shell with angular momentum l (descending x, then descending y).
void cart_powers(int l, int c, int& lx, int& ly, int& lz) {
    int idx = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (idx == c) { lx = x; ly = y; lz = l - x - y; return; }
            ++idx;
        }
    lx = ly = lz = -1;
}

double dfact(int n) {  // n!!, with (-1)!! = 1
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

struct Shell {
    int l, K;
    double A[3];
    std::vector<double> alpha;
    // coefficient[comp][prim] = d_prim * N(alpha_prim; comp) / sqrt(S_comp,comp)
    std::vector<std::vector<double>> cc;
    int off;  // first basis-function index
};

struct Basis {
    std::vector<Shell> sh;
    int nbf = 0;
    std::vector<double> Q;  // Schwarz bounds per shell pair, nshell*nshell (symmetric); empty until computed
};

// Primitive normalisation N(alpha; lx,ly,lz) = (2a/pi)^{3/4} (4a)^{l/2} / sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!).
double prim_norm(double a, int lx, int ly, int lz) {
    const double pi = 3.14159265358979323846;
    int l = lx + ly + lz;
    return std::pow(2 * a / pi, 0.75) * std::pow(4 * a, 0.5 * l) /
           std::sqrt(dfact(2 * lx - 1) * dfact(2 * ly - 1) * dfact(2 * lz - 1));
}

// Same-centre overlap of two primitives with equal Cartesian powers:
// prod_x (2l_x-1)!! / (2g)^{l_x} * (pi/g)^{3/2}, g = a + b.
double same_centre_overlap(double a, double b, int lx, int ly, int lz) {
    const double pi = 3.14159265358979323846;
    double g = a + b;
    return dfact(2 * lx - 1) / std::pow(2 * g, lx) * dfact(2 * ly - 1) / std::pow(2 * g, ly) *
           dfact(2 * lz - 1) / std::pow(2 * g, lz) * std::pow(pi / g, 1.5);
}

// ---------------------------------------------------------------------------------------------------------------
// McMurchie-Davidson pieces.
// Hermite expansion coefficients of the 1D overlap distribution of a pair (one Cartesian direction):
//   E_0^{00} = exp(-mu X_AB^2)
//   E_t^{i+1,j} = E_{t-1}^{ij}/(2p) + X_PA E_t^{ij} + (t+1) E_{t+1}^{ij}
//   E_t^{i,j+1} = E_{t-1}^{ij}/(2p) + X_PB E_t^{ij} + (t+1) E_{t+1}^{ij}
// ---------------------------------------------------------------------------------------------------------------
struct Ecoef {
    double e[3][5][8];  // [i][j][t], i <= 2, j <= 4 (the kinetic integral raises the ket power by 2), t <= i + j
};

void hermite_E(int imax, int jmax, double p, double XPA, double XPB, double XAB, double mu, Ecoef& E) {
    std::memset(&E, 0, sizeof(E));
    auto get = [&](int i, int j, int t) -> double {
        if (t < 0 || t > i + j) return 0.0;
        return E.e[i][j][t];
    };
    E.e[0][0][0] = std::exp(-mu * XAB * XAB);
    for (int i = 0; i <= imax; ++i) {
        for (int j = 0; j <= jmax; ++j) {
            if (i == 0 && j == 0) continue;
            for (int t = 0; t <= i + j; ++t) {
                double v;
                if (j == 0)
                    v = get(i - 1, 0, t - 1) / (2 * p) + XPA * get(i - 1, 0, t) + (t + 1) * get(i - 1, 0, t + 1);
                else
                    v = get(i, j - 1, t - 1) / (2 * p) + XPB * get(i, j - 1, t) + (t + 1) * get(i, j - 1, t + 1);
                E.e[i][j][t] = v;
            }
        }
    }
}

// Hermite Coulomb integrals R^0_{tuv} for t+u+v <= L:
//   R^n_{000} = (-2 rho)^n F_n(T)
//   R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X_PQ R^{n+1}_{t,u,v}   (likewise for u with Y_PQ, v with Z_PQ)
struct Rtab {
    // R[t][u][v] at n = 0, t,u,v <= 8
    double r[9][9][9];
};

void hermite_R(int L, double rho, double T, const double PQ[3], Rtab& out) {
    // full table over n as well: Rn[n][t][u][v]
    static thread_local double Rn[9][9][9][9];
    for (int n = 0; n <= L; ++n) {
        long double f = boys_ld(n, T);
        Rn[n][0][0][0] = (double)(std::pow(-2.0L * rho, n) * f);
    }
    for (int n = L - 1; n >= 0; --n) {
        int lmax = L - n;
        for (int tot = 1; tot <= lmax; ++tot)
            for (int t = tot; t >= 0; --t)
                for (int u = tot - t; u >= 0; --u) {
                    int v = tot - t - u;
                    double val;
                    if (t > 0)
                        val = (t > 1 ? (t - 1) * Rn[n + 1][t - 2][u][v] : 0.0) + PQ[0] * Rn[n + 1][t - 1][u][v];
                    else if (u > 0)
                        val = (u > 1 ? (u - 1) * Rn[n + 1][t][u - 2][v] : 0.0) + PQ[1] * Rn[n + 1][t][u - 1][v];
                    else
                        val = (v > 1 ? (v - 1) * Rn[n + 1][t][u][v - 2] : 0.0) + PQ[2] * Rn[n + 1][t][u][v - 1];
                    Rn[n][t][u][v] = val;
                }
    }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u + t <= L; ++u)
            for (int v = 0; v + u + t <= L; ++v) out.r[t][u][v] = Rn[0][t][u][v];
}

// Contracted shell quartet block, out[i][j][k][l] row-major over the Cartesian components of a, b, c, d.
void eri_quartet(const Basis& B, int ia, int ib, int ic, int id, double* out) {
    const Shell &a = B.sh[ia], &b = B.sh[ib], &c = B.sh[ic], &d = B.sh[id];
    const int na = ncart(a.l), nb = ncart(b.l), nc = ncart(c.l), nd = ncart(d.l);
    const int nab = na * nb, ncd = nc * nd;
    const int Lab = a.l + b.l, Lcd = c.l + d.l, L = Lab + Lcd;
    const double pi = 3.14159265358979323846;
    std::fill(out, out + (size_t)nab * ncd, 0.0);

    int pa[6][3], pb[6][3], pc[6][3], pd[6][3];
    for (int i = 0; i < na; ++i) cart_powers(a.l, i, pa[i][0], pa[i][1], pa[i][2]);
    for (int i = 0; i < nb; ++i) cart_powers(b.l, i, pb[i][0], pb[i][1], pb[i][2]);
    for (int i = 0; i < nc; ++i) cart_powers(c.l, i, pc[i][0], pc[i][1], pc[i][2]);
    for (int i = 0; i < nd; ++i) cart_powers(d.l, i, pd[i][0], pd[i][1], pd[i][2]);

    std::vector<double> prim((size_t)nab * ncd);
    std::vector<double> X((size_t)ncd * 9 * 9 * 9);  // ket-contracted Hermite intermediates [cd][t][u][v]
    Ecoef Eab[3], Ecd[3];
    Rtab R;

    for (int p1 = 0; p1 < a.K; ++p1)
        for (int p2 = 0; p2 < b.K; ++p2) {
            const double al = a.alpha[p1], be = b.alpha[p2];
            const double p = al + be, mu_ab = al * be / p;
            double P[3];
            for (int x = 0; x < 3; ++x) {
                P[x] = (al * a.A[x] + be * b.A[x]) / p;
                hermite_E(a.l, b.l, p, P[x] - a.A[x], P[x] - b.A[x], a.A[x] - b.A[x], mu_ab, Eab[x]);
            }
            for (int p3 = 0; p3 < c.K; ++p3)
                for (int p4 = 0; p4 < d.K; ++p4) {
                    const double ga = c.alpha[p3], de = d.alpha[p4];
                    const double q = ga + de, mu_cd = ga * de / q;
                    double Qc[3], PQ[3];
                    for (int x = 0; x < 3; ++x) {
                        Qc[x] = (ga * c.A[x] + de * d.A[x]) / q;
                        hermite_E(c.l, d.l, q, Qc[x] - c.A[x], Qc[x] - d.A[x], c.A[x] - d.A[x], mu_cd, Ecd[x]);
                        PQ[x] = P[x] - Qc[x];
                    }
                    const double rho = p * q / (p + q);
                    const double T = rho * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
                    hermite_R(L, rho, T, PQ, R);
                    const double pref = 2.0 * std::pow(pi, 2.5) / (p * q * std::sqrt(p + q));

                    // ket side: X[kl][t][u][v] = sum_{tau,nu,phi} (-1)^{tau+nu+phi} E^cd_tau E^cd_nu E^cd_phi
                    //                                                           R_{t+tau, u+nu, v+phi}
                    for (int k = 0; k < nc; ++k)
                        for (int l = 0; l < nd; ++l) {
                            const int kl = k * nd + l;
                            const int cx = pc[k][0], cy = pc[k][1], cz = pc[k][2];
                            const int dx = pd[l][0], dy = pd[l][1], dz = pd[l][2];
                            for (int t = 0; t <= Lab; ++t)
                                for (int u = 0; u + t <= Lab; ++u)
                                    for (int v = 0; v + u + t <= Lab; ++v) {
                                        double s = 0.0;
                                        for (int ta = 0; ta <= cx + dx; ++ta)
                                            for (int nu = 0; nu <= cy + dy; ++nu)
                                                for (int ph = 0; ph <= cz + dz; ++ph) {
                                                    double sg = ((ta + nu + ph) & 1) ? -1.0 : 1.0;
                                                    s += sg * Ecd[0].e[cx][dx][ta] * Ecd[1].e[cy][dy][nu] *
                                                         Ecd[2].e[cz][dz][ph] * R.r[t + ta][u + nu][v + ph];
                                                }
                                        X[((size_t)kl * 9 + t) * 81 + u * 9 + v] = s;
                                    }
                        }
                    // bra side
                    for (int i = 0; i < na; ++i)
                        for (int j = 0; j < nb; ++j) {
                            const int ax = pa[i][0], ay = pa[i][1], az = pa[i][2];
                            const int bx = pb[j][0], by = pb[j][1], bz = pb[j][2];
                            const double cab = a.cc[i][p1] * b.cc[j][p2];
                            for (int kl = 0; kl < ncd; ++kl) {
                                const int k = kl / nd, l = kl % nd;
                                const double ccd = c.cc[k][p3] * d.cc[l][p4];
                                double s = 0.0;
                                for (int t = 0; t <= ax + bx; ++t)
                                    for (int u = 0; u <= ay + by; ++u)
                                        for (int v = 0; v <= az + bz; ++v)
                                            s += Eab[0].e[ax][bx][t] * Eab[1].e[ay][by][u] * Eab[2].e[az][bz][v] *
                                                 X[((size_t)kl * 9 + t) * 81 + u * 9 + v];
                                out[(size_t)(i * nb + j) * ncd + kl] += pref * cab * ccd * s;
                            }
                        }
                }
        }
}

void compute_schwarz(Basis& B) {
    const int ns = (int)B.sh.size();
    B.Q.assign((size_t)ns * ns, 0.0);
#pragma omp parallel
    {
        std::vector<double> blk(6 * 6 * 6 * 6);
#pragma omp for schedule(dynamic)
        for (int a = 0; a < ns; ++a)
            for (int b = 0; b <= a; ++b) {
                eri_quartet(B, a, b, a, b, blk.data());
                const int na = ncart(B.sh[a].l), nb = ncart(B.sh[b].l), nab = na * nb;
                double m = 0.0;
                for (int ij = 0; ij < nab; ++ij) m = std::max(m, blk[(size_t)ij * nab + ij]);
                const double q = std::sqrt(std::max(m, 0.0));
                B.Q[(size_t)a * ns + b] = q;
                B.Q[(size_t)b * ns + a] = q;
            }
    }
}

bool keep(const Basis& B, int a, int b, int c, int d, double tau) {
    if (tau <= 0.0) return true;
    const int ns = (int)B.sh.size();
    return B.Q[(size_t)a * ns + b] * B.Q[(size_t)c * ns + d] >= tau;
}

}  // namespace

// ---------------------------------------------------------------------------------------------------------------
// One-electron integrals over the same basis (paper, Eq. (2)-(4)), McMurchie-Davidson form, per primitive pair
// (a: alpha, A, powers i; b: beta, B, powers j), p = alpha + beta, P the product centre:
//   overlap     S = E_0^{ix jx} E_0^{iy jy} E_0^{iz jz} (pi/p)^{3/2}
//   kinetic     T = -1/2 <a|nabla^2|b> = sum over directions of t_x s_y s_z, with the one-dimensional pieces
//                 s_{ij} = E_0^{ij} (pi/p)^{1/2}
//                 t_{ij} = -2 beta^2 s_{i,j+2} + beta (2j+1) s_{ij} - j(j-1)/2 s_{i,j-2}
//               (the second derivative of the ket factor x^j exp(-beta x^2))
//   attraction  V = -sum_C Z_C (2 pi / p) sum_{tuv} E_t^x E_u^y E_v^z R_{tuv}(p, P - C)
//               with R the Hermite Coulomb integrals of a point charge (exponent p, argument p |P - C|^2)
// ---------------------------------------------------------------------------------------------------------------
void one_electron_pair(const Basis& B, int ia, int ib, int natom, const double* Z, const double* Rn, double* S,
                       double* T, double* V) {
    const Shell &a = B.sh[ia], &b = B.sh[ib];
    const int na = ncart(a.l), nb = ncart(b.l);
    const double pi = 3.14159265358979323846;
    int pa[6][3], pb[6][3];
    for (int i = 0; i < na; ++i) cart_powers(a.l, i, pa[i][0], pa[i][1], pa[i][2]);
    for (int j = 0; j < nb; ++j) cart_powers(b.l, j, pb[j][0], pb[j][1], pb[j][2]);
    for (int x = 0; x < na * nb; ++x) S[x] = T[x] = V[x] = 0.0;
    Ecoef E[3];
    Rtab R;
    for (int p1 = 0; p1 < a.K; ++p1)
        for (int p2 = 0; p2 < b.K; ++p2) {
            const double al = a.alpha[p1], be = b.alpha[p2];
            const double p = al + be, mu = al * be / p;
            double P[3];
            for (int x = 0; x < 3; ++x) {
                P[x] = (al * a.A[x] + be * b.A[x]) / p;
                hermite_E(a.l, b.l + 2, p, P[x] - a.A[x], P[x] - b.A[x], a.A[x] - b.A[x], mu, E[x]);
            }
            const double r1 = std::sqrt(pi / p);
            auto s1 = [&](int x, int i, int j) { return j < 0 ? 0.0 : E[x].e[i][j][0] * r1; };
            auto t1 = [&](int x, int i, int j) {
                return -2.0 * be * be * s1(x, i, j + 2) + be * (2 * j + 1) * s1(x, i, j) - 0.5 * j * (j - 1) * s1(x, i, j - 2);
            };
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    const double c = a.cc[i][p1] * b.cc[j][p2];
                    const int *u = pa[i], *w = pb[j];
                    const double sx = s1(0, u[0], w[0]), sy = s1(1, u[1], w[1]), sz = s1(2, u[2], w[2]);
                    S[i * nb + j] += c * sx * sy * sz;
                    T[i * nb + j] += c * (t1(0, u[0], w[0]) * sy * sz + sx * t1(1, u[1], w[1]) * sz +
                                          sx * sy * t1(2, u[2], w[2]));
                }
            for (int n = 0; n < natom; ++n) {
                const double PC[3] = {P[0] - Rn[3 * n], P[1] - Rn[3 * n + 1], P[2] - Rn[3 * n + 2]};
                const double Tb = p * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
                hermite_R(a.l + b.l, p, Tb, PC, R);
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j) {
                        const int *u = pa[i], *w = pb[j];
                        double sum = 0.0;
                        for (int t = 0; t <= u[0] + w[0]; ++t)
                            for (int v = 0; v <= u[1] + w[1]; ++v)
                                for (int q = 0; q <= u[2] + w[2]; ++q)
                                    sum += E[0].e[u[0]][w[0]][t] * E[1].e[u[1]][w[1]][v] * E[2].e[u[2]][w[2]][q] *
                                           R.r[t][v][q];
                        V[i * nb + j] -= a.cc[i][p1] * b.cc[j][p2] * Z[n] * (2.0 * pi / p) * sum;
                    }
            }
        }
}

extern "C" {

// Boys values F_0..F_mmax at T (long double evaluation, rounded to double).
void oracle_boys(int mmax, double T, double* out) {
    for (int m = 0; m <= mmax; ++m) out[m] = (double)boys_ld(m, (long double)T);
}

// Build the normalised basis.  Returns NULL on invalid input (l outside 0..2, K < 1).
void* oracle_basis_create(int nshell, const int* l, const int* nprim, const double* center, const double* alpha,
                          const double* coef) {
    Basis* B = new Basis();
    int off = 0, p = 0;
    for (int s = 0; s < nshell; ++s) {
        if (l[s] < 0 || l[s] > 2 || nprim[s] < 1) { delete B; return nullptr; }
        Shell sh;
        sh.l = l[s];
        sh.K = nprim[s];
        for (int x = 0; x < 3; ++x) sh.A[x] = center[3 * s + x];
        sh.alpha.assign(alpha + p, alpha + p + sh.K);
        std::vector<double> d(coef + p, coef + p + sh.K);
        p += sh.K;
        const int nc = ncart(sh.l);
        sh.cc.assign(nc, std::vector<double>(sh.K));
        for (int c = 0; c < nc; ++c) {
            int lx, ly, lz;
            cart_powers(sh.l, c, lx, ly, lz);
            double S = 0.0;
            for (int i = 0; i < sh.K; ++i)
                for (int j = 0; j < sh.K; ++j)
                    S += d[i] * d[j] * prim_norm(sh.alpha[i], lx, ly, lz) * prim_norm(sh.alpha[j], lx, ly, lz) *
                         same_centre_overlap(sh.alpha[i], sh.alpha[j], lx, ly, lz);
            const double r = 1.0 / std::sqrt(S);
            for (int i = 0; i < sh.K; ++i) sh.cc[c][i] = d[i] * prim_norm(sh.alpha[i], lx, ly, lz) * r;
        }
        sh.off = off;
        off += nc;
        B->sh.push_back(std::move(sh));
    }
    B->nbf = off;
    return B;
}

void oracle_basis_destroy(void* h) { delete static_cast<Basis*>(h); }

int oracle_nbf(void* h) { return static_cast<Basis*>(h)->nbf; }

// One contracted block (ab|cd), n_a*n_b*n_c*n_d doubles, row-major [i][j][k][l].
void oracle_eri_quartet(void* h, int a, int b, int c, int d, double* out) {
    eri_quartet(*static_cast<Basis*>(h), a, b, c, d, out);
}

// Full N^4 tensor (tiny bases only), row-major [i][j][k][l] over basis functions.
void oracle_eri_tensor(void* h, double* out) {
    Basis& B = *static_cast<Basis*>(h);
    const int ns = (int)B.sh.size();
    const size_t N = B.nbf;
#pragma omp parallel
    {
        std::vector<double> blk(6 * 6 * 6 * 6);
#pragma omp for schedule(dynamic) collapse(2)
        for (int a = 0; a < ns; ++a)
            for (int b = 0; b < ns; ++b)
                for (int c = 0; c < ns; ++c)
                    for (int d = 0; d < ns; ++d) {
                        eri_quartet(B, a, b, c, d, blk.data());
                        const Shell &A = B.sh[a], &Bs = B.sh[b], &C = B.sh[c], &Dd = B.sh[d];
                        const int na = ncart(A.l), nb = ncart(Bs.l), nc = ncart(C.l), nd = ncart(Dd.l);
                        for (int i = 0; i < na; ++i)
                            for (int j = 0; j < nb; ++j)
                                for (int k = 0; k < nc; ++k)
                                    for (int l = 0; l < nd; ++l)
                                        out[(((A.off + i) * N + Bs.off + j) * N + C.off + k) * N + Dd.off + l] =
                                            blk[((i * nb + j) * nc + k) * nd + l];
                    }
    }
}

// Schwarz bounds Q_ab (nshell*nshell, symmetric).
void oracle_schwarz(void* h, double* Q) {
    Basis& B = *static_cast<Basis*>(h);
    if (B.Q.empty()) compute_schwarz(B);
    std::copy(B.Q.begin(), B.Q.end(), Q);
}

// J and K by the definition of Eq. (12): every shell quartet (no permutational symmetry), screened with the same
// rule as the fast path.  D, J, K are ndens stacked nbf*nbf row-major matrices.
void oracle_jk_direct(void* h, int ndens, const double* D, double tau, double* J, double* K) {
    Basis& B = *static_cast<Basis*>(h);
    if (tau > 0 && B.Q.empty()) compute_schwarz(B);
    const int ns = (int)B.sh.size();
    const size_t N = B.nbf, NN = N * N;
    std::fill(J, J + ndens * NN, 0.0);
    std::fill(K, K + ndens * NN, 0.0);
    const int nt = omp_get_max_threads();
    std::vector<std::vector<double>> Jt(nt, std::vector<double>(ndens * NN, 0.0)), Kt(nt, std::vector<double>(ndens * NN, 0.0));
#pragma omp parallel
    {
        const int tid = omp_get_thread_num();
        double* Jl = Jt[tid].data();
        double* Kl = Kt[tid].data();
        std::vector<double> blk(6 * 6 * 6 * 6);
#pragma omp for schedule(dynamic) collapse(2)
        for (int a = 0; a < ns; ++a)
            for (int b = 0; b < ns; ++b)
                for (int c = 0; c < ns; ++c)
                    for (int d = 0; d < ns; ++d) {
                        if (!keep(B, a, b, c, d, tau)) continue;
                        eri_quartet(B, a, b, c, d, blk.data());
                        const Shell &A = B.sh[a], &Bs = B.sh[b], &C = B.sh[c], &Dd = B.sh[d];
                        const int na = ncart(A.l), nb = ncart(Bs.l), nc = ncart(C.l), nd = ncart(Dd.l);
                        for (int m = 0; m < ndens; ++m) {
                            const double* Dm = D + m * NN;
                            for (int i = 0; i < na; ++i)
                                for (int j = 0; j < nb; ++j)
                                    for (int k = 0; k < nc; ++k)
                                        for (int l = 0; l < nd; ++l) {
                                            const double v = blk[((i * nb + j) * nc + k) * nd + l];
                                            const size_t I = A.off + i, Jx = Bs.off + j, Kx = C.off + k, Lx = Dd.off + l;
                                            Jl[m * NN + I * N + Jx] += v * Dm[Kx * N + Lx];   // J_ij += (ij|kl) D_kl
                                            Kl[m * NN + I * N + Lx] += v * Dm[Jx * N + Kx];   // K_il += (ij|kl) D_jk
                                        }
                        }
                    }
    }
    for (int t = 0; t < nt; ++t)
        for (size_t x = 0; x < ndens * NN; ++x) { J[x] += Jt[t][x]; K[x] += Kt[t][x]; }
}

// J and K over the unique shell quartets (a>=b, c>=d, ab>=cd) using the 8-fold permutational symmetry of (ij|kl):
//   v = (ab|cd) * 1/2^[a=b] * 1/2^[c=d] * 1/2^[ab=cd]
//   J_ab += 2 v D_cd, J_cd += 2 v D_ab, K_ac += v D_bd, K_ad += v D_bc, K_bc += v D_ad, K_bd += v D_ac
//   then J <- J + J^T, K <- K + K^T.
// Bra pairs can be restricted to a list (sample); npairs_sample <= 0 means all.  counts[0] = kept quartets,
// counts[1] = screened-out quartets.
void oracle_jk_symmetric(void* h, int ndens, const double* D, double tau, double* J, double* K, long long* counts,
                         int npairs_sample, const int* pair_sample) {
    Basis& B = *static_cast<Basis*>(h);
    if (tau > 0 && B.Q.empty()) compute_schwarz(B);
    const int ns = (int)B.sh.size();
    const size_t N = B.nbf, NN = N * N;
    std::vector<int> pa, pb;
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b <= a; ++b) { pa.push_back(a); pb.push_back(b); }
    std::vector<int> bras;
    if (npairs_sample > 0) bras.assign(pair_sample, pair_sample + npairs_sample);
    else for (int i = 0; i < (int)pa.size(); ++i) bras.push_back(i);
    std::fill(J, J + ndens * NN, 0.0);
    std::fill(K, K + ndens * NN, 0.0);
    const int nt = omp_get_max_threads();
    std::vector<std::vector<double>> Jt(nt, std::vector<double>(ndens * NN, 0.0)), Kt(nt, std::vector<double>(ndens * NN, 0.0));
    long long kept = 0, dropped = 0;
#pragma omp parallel reduction(+ : kept, dropped)
    {
        const int tid = omp_get_thread_num();
        double* Jl = Jt[tid].data();
        double* Kl = Kt[tid].data();
        std::vector<double> blk(6 * 6 * 6 * 6);
#pragma omp for schedule(dynamic)
        for (int bi = 0; bi < (int)bras.size(); ++bi) {
            const int ab = bras[bi];
            const int a = pa[ab], b = pb[ab];
            for (int cd = 0; cd <= ab; ++cd) {
                const int c = pa[cd], d = pb[cd];
                if (!keep(B, a, b, c, d, tau)) { ++dropped; continue; }
                ++kept;
                eri_quartet(B, a, b, c, d, blk.data());
                double w = 1.0;
                if (a == b) w *= 0.5;
                if (c == d) w *= 0.5;
                if (ab == cd) w *= 0.5;
                const Shell &A = B.sh[a], &Bs = B.sh[b], &C = B.sh[c], &Dd = B.sh[d];
                const int na = ncart(A.l), nb = ncart(Bs.l), nc = ncart(C.l), nd = ncart(Dd.l);
                for (int m = 0; m < ndens; ++m) {
                    const double* Dm = D + m * NN;
                    double* Jm = Jl + m * NN;
                    double* Km = Kl + m * NN;
                    for (int i = 0; i < na; ++i)
                        for (int j = 0; j < nb; ++j)
                            for (int k = 0; k < nc; ++k)
                                for (int l = 0; l < nd; ++l) {
                                    const double v = w * blk[((i * nb + j) * nc + k) * nd + l];
                                    const size_t I = A.off + i, Jx = Bs.off + j, Kx = C.off + k, Lx = Dd.off + l;
                                    Jm[I * N + Jx] += 2.0 * v * Dm[Kx * N + Lx];
                                    Jm[Kx * N + Lx] += 2.0 * v * Dm[I * N + Jx];
                                    Km[I * N + Kx] += v * Dm[Jx * N + Lx];
                                    Km[I * N + Lx] += v * Dm[Jx * N + Kx];
                                    Km[Jx * N + Kx] += v * Dm[I * N + Lx];
                                    Km[Jx * N + Lx] += v * Dm[I * N + Kx];
                                }
                }
            }
        }
    }
    for (int t = 0; t < nt; ++t)
        for (size_t x = 0; x < ndens * NN; ++x) { J[x] += Jt[t][x]; K[x] += Kt[t][x]; }
    for (int m = 0; m < ndens; ++m) {
        double* Jm = J + m * NN;
        double* Km = K + m * NN;
        for (size_t i = 0; i < N; ++i)
            for (size_t j = 0; j <= i; ++j) {
                const double sj = Jm[i * N + j] + Jm[j * N + i];
                const double sk = Km[i * N + j] + Km[j * N + i];
                Jm[i * N + j] = Jm[j * N + i] = sj;
                Km[i * N + j] = Km[j * N + i] = sk;
            }
    }
    if (counts) { counts[0] = kept; counts[1] = dropped; }
}

// Sampled rows of Eq. (12) by the definition, for bases too large for a full build:
//   Jblk[i][j] = sum over all shells c, d and their components of (ab|cd) D_cd      (i in a, j in b)
//   Kblk[i][l] = sum over all shells b, c and their components of (ab|cd) D_bc      (i in a, l in d = sd)
// Quartets are screened with the same rule.  Jblk is n_a*n_b, Kblk is n_a*n_d (d = shell kd).
void oracle_j_block(void* h, const double* D, double tau, int a, int b, double* Jblk) {
    Basis& B = *static_cast<Basis*>(h);
    if (tau > 0 && B.Q.empty()) compute_schwarz(B);
    const int ns = (int)B.sh.size();
    const size_t N = B.nbf;
    const Shell &A = B.sh[a], &Bs = B.sh[b];
    const int na = ncart(A.l), nb = ncart(Bs.l);
    const int nt = omp_get_max_threads();
    std::vector<std::vector<double>> acc(nt, std::vector<double>(na * nb, 0.0));
#pragma omp parallel
    {
        std::vector<double> blk(6 * 6 * 6 * 6);
        double* ac = acc[omp_get_thread_num()].data();
#pragma omp for schedule(dynamic) collapse(2)
        for (int c = 0; c < ns; ++c)
            for (int d = 0; d < ns; ++d) {
                if (!keep(B, a, b, c, d, tau)) continue;
                eri_quartet(B, a, b, c, d, blk.data());
                const Shell &C = B.sh[c], &Dd = B.sh[d];
                const int nc = ncart(C.l), nd = ncart(Dd.l);
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j)
                        for (int k = 0; k < nc; ++k)
                            for (int l = 0; l < nd; ++l)
                                ac[i * nb + j] += blk[((i * nb + j) * nc + k) * nd + l] * D[(C.off + k) * N + Dd.off + l];
            }
    }
    std::fill(Jblk, Jblk + na * nb, 0.0);
    for (int t = 0; t < nt; ++t)
        for (int x = 0; x < na * nb; ++x) Jblk[x] += acc[t][x];
}

void oracle_k_block(void* h, const double* D, double tau, int a, int d, double* Kblk) {
    Basis& B = *static_cast<Basis*>(h);
    if (tau > 0 && B.Q.empty()) compute_schwarz(B);
    const int ns = (int)B.sh.size();
    const size_t N = B.nbf;
    const Shell &A = B.sh[a], &Dd = B.sh[d];
    const int na = ncart(A.l), nd = ncart(Dd.l);
    const int nt = omp_get_max_threads();
    std::vector<std::vector<double>> acc(nt, std::vector<double>(na * nd, 0.0));
#pragma omp parallel
    {
        std::vector<double> blk(6 * 6 * 6 * 6);
        double* ac = acc[omp_get_thread_num()].data();
#pragma omp for schedule(dynamic) collapse(2)
        for (int b = 0; b < ns; ++b)
            for (int c = 0; c < ns; ++c) {
                if (!keep(B, a, b, c, d, tau)) continue;
                eri_quartet(B, a, b, c, d, blk.data());
                const Shell &Bs = B.sh[b], &C = B.sh[c];
                const int nb = ncart(Bs.l), nc = ncart(C.l);
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j)
                        for (int k = 0; k < nc; ++k)
                            for (int l = 0; l < nd; ++l)
                                ac[i * nd + l] += blk[((i * nb + j) * nc + k) * nd + l] * D[(Bs.off + j) * N + C.off + k];
            }
    }
    std::fill(Kblk, Kblk + na * nd, 0.0);
    for (int t = 0; t < nt; ++t)
        for (int x = 0; x < na * nd; ++x) Kblk[x] += acc[t][x];
}

// Overlap S, kinetic T and nuclear attraction V (point nuclei of charges Z at R, [natom][3] bohr) over the basis,
// nbf x nbf row-major each (Eq. (2)-(4)).
void oracle_one_electron(void* basis, int natom, const double* Z, const double* R, double* S, double* T, double* V) {
    const Basis& B = *(const Basis*)basis;
    const int ns = (int)B.sh.size(), N = B.nbf;
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            double s[36], t[36], v[36];
            one_electron_pair(B, a, b, natom, Z, R, s, t, v);
            const Shell &A = B.sh[a], &Bs = B.sh[b];
            const int na = ncart(A.l), nb = ncart(Bs.l);
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    const size_t x = (size_t)(A.off + i) * N + Bs.off + j;
                    S[x] = s[i * nb + j];
                    T[x] = t[i * nb + j];
                    V[x] = v[i * nb + j];
                }
        }
}

int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) { omp_set_num_threads(n); }

}  // extern "C"
