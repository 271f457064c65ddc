// One-electron integrals (Eq. (2)-(4)) and the Hartree-Fock drivers around the Fock build: restricted closed shell
// and unrestricted (the paper's RHF and URHF).
//
// SCF (Szabo-Ostlund closed-shell and Pople-Nesbet equations, which the paper states it follows; Pulay DIIS as in
// the paper's SCF):
//   X = S^{-1/2} (symmetric orthogonalisation), core-Hamiltonian guess F_0 = H = T + V;
//   per iteration: F' = X F X, F' C' = C' eps, C = X C', closed shell P = 2 C_occ C_occ^T and F = H + G(P) from
//   uqc_fock_build; unrestricted P^s = C^s_occ C^s_occ^T and F^s = H + G^s from uqc_fock_build_uhf;
//   E = sum_s P^s H + E2, error e^s = F^s P^s S - S P^s F^s;
//   DIIS: F^s_extrapolated = sum_i c_i F^s_i with sum_i c_i = 1 minimising sum_s |sum_i c_i e^s_i|^2.
// Matrices live on the device; products and eigendecompositions use rocBLAS / rocSOLVER (column-major; every
// matrix handed to them is symmetric except the eigenvector blocks, which stay internal).
#include "uqc_api_internal.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

using namespace uqc;

void release_blas(uqc_ctx* c) {
    if (c && c->blas) {
        (void)rocblas_destroy_handle((rocblas_handle)c->blas);
        c->blas = nullptr;
    }
}

uqc_status uqc::ensure_blas(uqc_ctx* ctx, rocblas_handle* out) {
    if (!ctx->blas) {
        rocblas_handle h;
        if (rocblas_create_handle(&h) != rocblas_status_success)
            return uqc_fail(UQC_E_DEVICE, "rocblas_create_handle failed");
        ctx->blas = h;
    }
    rocblas_handle h = (rocblas_handle)ctx->blas;
    if (rocblas_set_stream(h, ctx->stream) != rocblas_status_success ||
        rocblas_set_pointer_mode(h, rocblas_pointer_mode_host) != rocblas_status_success)
        return uqc_fail(UQC_E_DEVICE, "rocBLAS stream or pointer mode could not be set");
    *out = h;
    return UQC_OK;
}

#define UQC_BLAS(expr)                                                                                   \
    do {                                                                                                 \
        rocblas_status b_ = (expr);                                                                      \
        if (b_ != rocblas_status_success)                                                                \
            return uqc_fail(UQC_E_DEVICE, std::string(#expr) + " failed: " + rocblas_status_to_string(b_)); \
    } while (0)

// ------------------------------------------------------------------------------------- one-electron integrals
static int pair_class_of(int la, int lb) {
    static const int tab[3][3] = {{0, -1, -1}, {1, 2, -1}, {3, 4, 5}};
    return tab[la][lb];
}

// Shell table and the shell pairs of every pair class on the device (once per basis).
static uqc_status ensure_shells(uqc_basis* B) {
    if (B->d_shells) return UQC_OK;
    const int ns = B->nshell;
    std::vector<int> K(ns), off(ns), pst(ns);
    std::vector<double> A(3 * (size_t)ns), al, cc;
    for (int s = 0; s < ns; ++s) {
        const ShellH& sh = B->shells[s];
        K[s] = sh.K;
        off[s] = sh.off;
        pst[s] = (int)al.size();
        for (int x = 0; x < 3; ++x) A[3 * s + x] = sh.A[x];
        for (int k = 0; k < sh.K; ++k) {
            al.push_back(sh.alpha[k]);
            cc.push_back(sh.c[k]);
        }
    }
    std::vector<int2> pairs[6];
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            const int la = B->shells[a].l, lb = B->shells[b].l;
            if (la < lb || (la == lb && a < b)) continue;
            pairs[pair_class_of(la, lb)].push_back(make_int2(a, b));
        }
    auto al8 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t bytes = 3 * al8(ns * sizeof(int)) + al8(A.size() * 8) + 2 * al8(al.size() * 8);
    for (auto& p : pairs) bytes += al8(p.size() * sizeof(int2));
    std::vector<char> host(bytes, 0);
    void* d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) return uqc_fail(UQC_E_NOMEM, "one-electron: shell table allocation");
    size_t pos = 0;
    auto put = [&](const void* src, size_t n) {
        std::memcpy(host.data() + pos, src, n);
        const size_t at = pos;
        pos += al8(n);
        return (char*)d + at;
    };
    ShellsDev& v = B->shells_dev;
    v.K = (const int*)put(K.data(), ns * sizeof(int));
    v.off = (const int*)put(off.data(), ns * sizeof(int));
    v.pstart = (const int*)put(pst.data(), ns * sizeof(int));
    v.A = (const double*)put(A.data(), A.size() * 8);
    v.alpha = (const double*)put(al.data(), al.size() * 8);
    v.c = (const double*)put(cc.data(), cc.size() * 8);
    v.nshell = ns;
    for (int c = 0; c < 6; ++c) {
        B->npairs[c] = (int)pairs[c].size();
        B->d_pairs[c] = pairs[c].empty() ? nullptr : (const int2*)put(pairs[c].data(), pairs[c].size() * sizeof(int2));
    }
    if (hipMemcpy(d, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return uqc_fail(UQC_E_DEVICE, "one-electron: shell table upload failed");
    }
    B->d_shells = d;
    return UQC_OK;
}

// Device arrays: S, T, V (any null); nuclei uploaded to the basis' small buffer; runs on the context stream.
static uqc_status one_electron_device(uqc_basis* B, int natom, const double* Z, const double* R, double* S, double* T,
                                      double* V) {
    uqc_status st = ensure_shells(B);
    if (st != UQC_OK) return st;
    hipStream_t s = B->ctx->stream;
    const size_t need = std::max<size_t>(4 * (size_t)natom, 4);
    if (B->nuc_cap < need) {
        if (B->d_nuc) (void)hipFree(B->d_nuc);
        B->d_nuc = nullptr;
        B->nuc_cap = 0;
        if (hipMalloc(&B->d_nuc, need * sizeof(double)) != hipSuccess)
            return uqc_fail(UQC_E_NOMEM, "one-electron: nuclei buffer allocation");
        B->nuc_cap = need;
    }
    if (natom > 0) {
        UQC_HIP(hipMemcpyAsync(B->d_nuc, Z, natom * sizeof(double), hipMemcpyHostToDevice, s));
        UQC_HIP(hipMemcpyAsync(B->d_nuc + natom, R, 3 * natom * sizeof(double), hipMemcpyHostToDevice, s));
    }
    for (int c = 0; c < 6; ++c)
        UQC_HIP(launch_one_electron(c, B->shells_dev, B->d_pairs[c], B->npairs[c], natom, B->d_nuc,
                                    B->d_nuc + natom, B->d_f, S, T, natom > 0 ? V : nullptr, B->nbf, B->ctx->boys64,
                                    s));
    if (V && natom == 0) UQC_HIP(launch_zero(V, (size_t)B->nbf * B->nbf, s));
    return UQC_OK;
}

uqc_status uqc_one_electron(uqc_basis* B, int natom, const double* Z, const double* R, double* S, double* T,
                            double* V) {
    if (!B) return uqc_fail(UQC_E_ARG, "uqc_one_electron: NULL basis");
    if (natom < 0 || (natom > 0 && (!Z || !R))) return uqc_fail(UQC_E_ARG, "uqc_one_electron: bad nuclei");
    for (int n = 0; n < natom; ++n)
        if (!std::isfinite(Z[n]) || !std::isfinite(R[3 * n]) || !std::isfinite(R[3 * n + 1]) ||
            !std::isfinite(R[3 * n + 2]))
            return uqc_fail(UQC_E_ARG, "uqc_one_electron: non-finite nuclear charge or position");
    if (!S && !T && !V) return UQC_OK;
    UQC_HIP(hipSetDevice(B->ctx->device));
    const void* first = S ? (const void*)S : (T ? (const void*)T : (const void*)V);
    const bool dev = is_device_ptr(first);
    for (const void* p : {(const void*)S, (const void*)T, (const void*)V})
        if (p && is_device_ptr(p) != dev) return uqc_fail(UQC_E_ARG, "uqc_one_electron: mix of host and device pointers");
    const size_t NN = (size_t)B->nbf * B->nbf;
    hipStream_t s = B->ctx->stream;
    double *dS = S, *dT = T, *dV = V;
    if (!dev) {  // stage in the basis' host-pointer buffers
        dS = S ? B->d_io : nullptr;
        dT = T ? B->d_io + NN : nullptr;
        dV = V ? B->d_io + 2 * NN : nullptr;
    }
    uqc_status st = one_electron_device(B, natom, Z, R, dS, dT, dV);
    if (st != UQC_OK) return st;
    if (!dev) {
        if (S) UQC_HIP(hipMemcpyAsync(S, dS, NN * 8, hipMemcpyDeviceToHost, s));
        if (T) UQC_HIP(hipMemcpyAsync(T, dT, NN * 8, hipMemcpyDeviceToHost, s));
        if (V) UQC_HIP(hipMemcpyAsync(V, dV, NN * 8, hipMemcpyDeviceToHost, s));
    }
    UQC_HIP(hipStreamSynchronize(s));
    return UQC_OK;
}

// ------------------------------------------------------------------------------------------------------ SCF
void uqc_scf_opts_default(uqc_scf_opts* o) {
    if (!o) return;
    o->max_iter = 100;
    o->e_conv = 1e-10;
    o->d_conv = 1e-8;
    o->diis_size = 8;
    uqc_fock_opts_default(&o->fock);
    o->guess_mix = 0.0;
}

// Solves the (m+1) x (m+1) DIIS system [B -1; -1 0] [c; lambda] = [0; -1] by Gaussian elimination with partial
// pivoting; false if singular.
static bool diis_solve(const std::vector<double>& Bm, int m, std::vector<double>& c) {
    const int n = m + 1;
    std::vector<double> A((size_t)n * (n + 1), 0.0);
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < m; ++j) A[i * (n + 1) + j] = Bm[i * m + j];
        A[i * (n + 1) + m] = -1.0;
        A[m * (n + 1) + i] = -1.0;
    }
    A[m * (n + 1) + n] = -1.0;
    // scale the error block so that pivots are comparable
    double mx = 0.0;
    for (int i = 0; i < m; ++i) mx = std::max(mx, std::fabs(Bm[i * m + i]));
    if (!(mx > 0)) return false;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) A[i * (n + 1) + j] /= mx;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r * (n + 1) + col]) > std::fabs(A[piv * (n + 1) + col])) piv = r;
        if (std::fabs(A[piv * (n + 1) + col]) < 1e-300) return false;
        if (piv != col)
            for (int k = 0; k <= n; ++k) std::swap(A[col * (n + 1) + k], A[piv * (n + 1) + k]);
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = A[r * (n + 1) + col] / A[col * (n + 1) + col];
            for (int k = col; k <= n; ++k) A[r * (n + 1) + k] -= f * A[col * (n + 1) + k];
        }
    }
    c.assign(m, 0.0);
    for (int i = 0; i < m; ++i) c[i] = A[i * (n + 1) + n] / A[i * (n + 1) + i];
    return true;
}

// Closed shell (nspin = 1: one density P = 2 C_occ C_occ^T, G from uqc_fock_build) or spin-unrestricted (nspin = 2:
// P^s = C^s_occ C^s_occ^T, G^s from uqc_fock_build_uhf).  nocc[s] occupied orbitals per spin.
static uqc_status scf_run(uqc_basis* B, int natom, const double* Z, const double* R, int nspin, const int* nocc,
                          const uqc_scf_opts* opts, double* const* Pout, double* const* eps_out, uqc_scf_result* res,
                          const char* name) {
    const auto t0 = std::chrono::steady_clock::now();
    const std::string nm(name);
    const int N = B->nbf;
    if (natom < 0 || (natom > 0 && (!Z || !R))) return uqc_fail(UQC_E_ARG, nm + ": bad nuclei");
    uqc_scf_opts o;
    uqc_scf_opts_default(&o);
    if (opts) o = *opts;
    if (o.max_iter < 1 || o.diis_size < 0 || o.diis_size > 16 || !(o.e_conv > 0) || !(o.d_conv > 0) ||
        !std::isfinite(o.guess_mix))
        return uqc_fail(UQC_E_ARG, nm + ": bad options");
    o.fock.progress = nullptr;
    o.fock.timing = 0;
    uqc_ctx* ctx = B->ctx;
    UQC_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    rocblas_handle h = nullptr;
    {
        const uqc_status sb = ensure_blas(ctx, &h);
        if (sb != UQC_OK) return sb;
    }

    const size_t NN = (size_t)N * N;
    const int m_max = o.diis_size;
    // shared: S H X T1 M | per spin: P F G E Fx C | DIIS per slot and spin: F_i, e_i | w, work, info
    const size_t nmat = 5 + 6 * (size_t)nspin + 2 * (size_t)nspin * m_max;
    double* mem = nullptr;
    if (hipMalloc(&mem, (nmat * NN + 3 * (size_t)N + 8) * sizeof(double)) != hipSuccess)
        return uqc_fail(UQC_E_NOMEM, nm + ": workspace allocation failed");
    struct Free {
        double* p;
        ~Free() { if (p) (void)hipFree(p); }
    } guard{mem};
    double *S = mem, *H = S + NN, *X = H + NN, *T1 = X + NN, *M = T1 + NN;
    double *P[2], *F[2], *G[2], *E[2], *Fx[2], *C[2];
    double* q = M + NN;
    for (int sp = 0; sp < nspin; ++sp) {
        P[sp] = q; F[sp] = q + NN; G[sp] = q + 2 * NN; E[sp] = q + 3 * NN; Fx[sp] = q + 4 * NN; C[sp] = q + 5 * NN;
        q += 6 * NN;
    }
    auto Fs = [&](int slot, int sp) { return q + ((size_t)slot * nspin + sp) * NN; };                 // DIIS Fock
    auto Es = [&](int slot, int sp) { return q + ((size_t)(m_max + slot) * nspin + sp) * NN; };      // DIIS error
    double* w = q + 2 * (size_t)m_max * nspin * NN;  // eigenvalues [N]
    double* offd = w + N;                            // work [N]
    rocblas_int* info = (rocblas_int*)(offd + N);

    // one-electron part: S, H = T + V (T in M, V in T1 as scratch)
    uqc_status st = one_electron_device(B, natom, Z, R, S, M, T1);
    if (st != UQC_OK) return st;
    UQC_HIP(launch_add(M, T1, H, NN, s));
    double E_nuc = 0.0;
    for (int a = 0; a < natom; ++a)
        for (int b = 0; b < a; ++b) {
            const double dx = R[3 * a] - R[3 * b], dy = R[3 * a + 1] - R[3 * b + 1], dz = R[3 * a + 2] - R[3 * b + 2];
            E_nuc += Z[a] * Z[b] / std::sqrt(dx * dx + dy * dy + dz * dz);
        }

    auto eig = [&](double* A) -> uqc_status {  // A <- eigenvectors (columns), w <- eigenvalues (ascending)
        UQC_BLAS(rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, N, A, N, w, offd, info));
        rocblas_int hinfo = 0;
        UQC_HIP(hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, s));
        UQC_HIP(hipStreamSynchronize(s));
        if (hinfo != 0) return uqc_fail(UQC_E_DEVICE, nm + ": eigendecomposition did not converge");
        return UQC_OK;
    };
    const double one = 1.0, zero = 0.0;
    const double occ = nspin == 1 ? 2.0 : 1.0;

    // X = U diag(s^-1/2) U^T
    UQC_HIP(hipMemcpyAsync(T1, S, NN * 8, hipMemcpyDeviceToDevice, s));
    if ((st = eig(T1)) != UQC_OK) return st;
    std::vector<double> hw(N);
    UQC_HIP(hipMemcpyAsync(hw.data(), w, N * 8, hipMemcpyDeviceToHost, s));
    UQC_HIP(hipStreamSynchronize(s));
    if (!(hw[0] > 1e-10 * hw[N - 1])) return uqc_fail(UQC_E_DEVICE, nm + ": overlap matrix is numerically singular");
    for (int i = 0; i < N; ++i) hw[i] = 1.0 / std::sqrt(hw[i]);
    UQC_HIP(hipMemcpyAsync(w, hw.data(), N * 8, hipMemcpyHostToDevice, s));
    UQC_HIP(launch_scale_cols(T1, w, M, N, s));
    UQC_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, N, N, N, &one, M, N, T1, N, &zero, X,
                           N));

    // orbitals of Fin in C (X Fin X C' = C' eps, C = X C'; eigenvalues in w)
    auto orbitals = [&](const double* Fin, double* Cout) -> uqc_status {
        UQC_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, N, N, &one, Fin, N, X, N, &zero, T1,
                               N));
        UQC_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, N, N, &one, X, N, T1, N, &zero, M,
                               N));
        uqc_status s2 = eig(M);
        if (s2 != UQC_OK) return s2;
        UQC_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, N, N, &one, X, N, M, N, &zero, Cout,
                               N));
        return UQC_OK;
    };
    // density of spin sp from its orbitals: P = occ C_occ C_occ^T
    auto density = [&](int sp) -> uqc_status {
        if (nocc[sp] == 0) {
            UQC_HIP(launch_zero(P[sp], NN, s));
            return UQC_OK;
        }
        UQC_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, N, N, nocc[sp], &occ, C[sp], N,
                               C[sp], N, &zero, P[sp], N));
        return UQC_OK;
    };

    // core-Hamiltonian guess; for spin densities the alpha highest occupied / lowest virtual pair is rotated
    for (int sp = 0; sp < nspin; ++sp) {
        if ((st = orbitals(H, C[sp])) != UQC_OK) return st;
        if (nspin == 2 && sp == 0 && o.guess_mix != 0.0 && nocc[0] > 0 && nocc[0] < N) {
            const double c = std::cos(o.guess_mix), sn = std::sin(o.guess_mix);
            UQC_BLAS(rocblas_drot(h, N, C[0] + (size_t)(nocc[0] - 1) * N, 1, C[0] + (size_t)nocc[0] * N, 1, &c, &sn));
        }
        if ((st = density(sp)) != UQC_OK) return st;
    }
    double e_prev = 0.0, E_elec = 0.0, err = 0.0, fock_ms = 0.0;
    int it = 0, nstore = 0, head = 0;
    bool converged = false;
    long long quartets = 0;
    std::vector<double> Bm((size_t)m_max * m_max, 0.0), cvec;
    while (it < o.max_iter) {
        ++it;
        uqc_stats fs;
        const auto tf = std::chrono::steady_clock::now();
        if (nspin == 1)
            st = uqc_fock_build(B, P[0], nullptr, nullptr, G[0], &o.fock, &fs);
        else
            st = uqc_fock_build_uhf(B, P[0], P[1], nullptr, nullptr, nullptr, G[0], G[1], &o.fock, &fs);
        if (st != UQC_OK) return st;
        fock_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tf).count();
        quartets = fs.quartets;
        E_elec = fs.E2;
        err = 0.0;
        for (int sp = 0; sp < nspin; ++sp) {
            UQC_HIP(launch_add(H, G[sp], F[sp], NN, s));
            double ph = 0.0;
            UQC_BLAS(rocblas_ddot(h, (rocblas_int)NN, P[sp], 1, H, 1, &ph));
            E_elec += ph;
            // error F P S - S P F
            UQC_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, N, N, &one, F[sp], N, P[sp], N,
                                   &zero, T1, N));
            UQC_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, N, N, &one, T1, N, S, N, &zero,
                                   M, N));
            UQC_HIP(launch_antisym(M, E[sp], N, s));
            rocblas_int imax = 1;
            UQC_BLAS(rocblas_idamax(h, (rocblas_int)NN, E[sp], 1, &imax));
            double e1 = 0.0;
            UQC_HIP(hipMemcpyAsync(&e1, E[sp] + (imax - 1), 8, hipMemcpyDeviceToHost, s));
            UQC_HIP(hipStreamSynchronize(s));
            err = std::max(err, std::fabs(e1));
        }
        if (it > 1 && std::fabs(E_elec - e_prev) < o.e_conv && err < o.d_conv) {
            converged = true;
            break;
        }
        if (it == o.max_iter) break;  // P, F and E stay those of the last build
        e_prev = E_elec;
        const double* Fnext[2] = {F[0], nspin == 2 ? F[1] : nullptr};
        if (m_max > 0) {
            // store (F, e) of every spin in the ring, update the error overlaps, extrapolate with one set of weights
            const int slot = head;
            head = (head + 1) % m_max;
            nstore = std::min(nstore + 1, m_max);
            for (int sp = 0; sp < nspin; ++sp) {
                UQC_HIP(hipMemcpyAsync(Fs(slot, sp), F[sp], NN * 8, hipMemcpyDeviceToDevice, s));
                UQC_HIP(hipMemcpyAsync(Es(slot, sp), E[sp], NN * 8, hipMemcpyDeviceToDevice, s));
            }
            for (int j = 0; j < nstore; ++j) {
                double d = 0.0;
                for (int sp = 0; sp < nspin; ++sp) {
                    double d1 = 0.0;
                    UQC_BLAS(rocblas_ddot(h, (rocblas_int)NN, Es(slot, sp), 1, Es(j, sp), 1, &d1));
                    d += d1;
                }
                Bm[slot * m_max + j] = Bm[j * m_max + slot] = d;
            }
            if (nstore >= 2) {
                std::vector<double> Bs((size_t)nstore * nstore);
                for (int i = 0; i < nstore; ++i)
                    for (int j = 0; j < nstore; ++j) Bs[i * nstore + j] = Bm[i * m_max + j];
                if (diis_solve(Bs, nstore, cvec)) {
                    for (int sp = 0; sp < nspin; ++sp) {
                        UQC_HIP(launch_zero(Fx[sp], NN, s));
                        for (int i = 0; i < nstore; ++i)
                            UQC_BLAS(rocblas_daxpy(h, (rocblas_int)NN, &cvec[i], Fs(i, sp), 1, Fx[sp], 1));
                        Fnext[sp] = Fx[sp];
                    }
                }
            }
        }
        for (int sp = 0; sp < nspin; ++sp) {
            if ((st = orbitals(Fnext[sp], C[sp])) != UQC_OK) return st;
            if ((st = density(sp)) != UQC_OK) return st;
        }
    }
    UQC_HIP(hipStreamSynchronize(s));
    double s2 = 0.0;
    if (nspin == 2) {
        // <S^2> = S_z (S_z + 1) + n_beta - tr(P^a S P^b S); T1 = P^a S and M = S P^b, column-major
        UQC_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, N, N, &one, P[0], N, S, N, &zero,
                               T1, N));
        UQC_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, N, N, &one, S, N, P[1], N, &zero,
                               M, N));
        double tr = 0.0;
        UQC_BLAS(rocblas_ddot(h, (rocblas_int)NN, T1, 1, M, 1, &tr));
        const double sz = 0.5 * (nocc[0] - nocc[1]);
        s2 = sz * (sz + 1.0) + nocc[1] - tr;
    }
    for (int sp = 0; sp < nspin; ++sp) {
        if (Pout[sp]) UQC_HIP(hipMemcpyAsync(Pout[sp], P[sp], NN * 8, hipMemcpyDeviceToHost, s));
        if (eps_out[sp]) {
            // orbital energies of the final Fock matrix
            if ((st = orbitals(F[sp], E[sp])) != UQC_OK) return st;  // E[sp]: scratch for the orbitals
            UQC_HIP(hipMemcpyAsync(eps_out[sp], w, N * 8, hipMemcpyDeviceToHost, s));
        }
    }
    UQC_HIP(hipStreamSynchronize(s));
    if (res) {
        std::memset(res, 0, sizeof(*res));
        res->E_elec = E_elec;
        res->E_nuc = E_nuc;
        res->E_total = E_elec + E_nuc;
        res->iterations = it;
        res->converged = converged ? 1 : 0;
        res->error = err;
        res->fock_ms = fock_ms;
        res->quartets = quartets;
        res->s2 = s2;
        res->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return UQC_OK;
}

uqc_status uqc_scf_rhf(uqc_basis* B, int natom, const double* Z, const double* R, int nocc, const uqc_scf_opts* opts,
                       double* Pout, double* eps_out, uqc_scf_result* res) {
    if (!B) return uqc_fail(UQC_E_ARG, "uqc_scf_rhf: NULL basis");
    if (nocc < 1 || nocc > B->nbf) return uqc_fail(UQC_E_ARG, "uqc_scf_rhf: nocc outside 1..nbf");
    const int n[1] = {nocc};
    double* P[1] = {Pout};
    double* e[1] = {eps_out};
    return scf_run(B, natom, Z, R, 1, n, opts, P, e, res, "uqc_scf_rhf");
}

uqc_status uqc_scf_uhf(uqc_basis* B, int natom, const double* Z, const double* R, int nalpha, int nbeta,
                       const uqc_scf_opts* opts, double* Pa, double* Pb, double* eps_a, double* eps_b,
                       uqc_scf_result* res) {
    if (!B) return uqc_fail(UQC_E_ARG, "uqc_scf_uhf: NULL basis");
    if (nalpha < 0 || nbeta < 0 || nalpha > B->nbf || nbeta > B->nbf || nalpha + nbeta < 1)
        return uqc_fail(UQC_E_ARG, "uqc_scf_uhf: electron counts outside 0..nbf (or none)");
    const int n[2] = {nalpha, nbeta};
    double* P[2] = {Pa, Pb};
    double* e[2] = {eps_a, eps_b};
    return scf_run(B, natom, Z, R, 2, n, opts, P, e, res, "uqc_scf_uhf");
}
