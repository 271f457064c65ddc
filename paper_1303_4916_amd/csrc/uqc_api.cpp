// Host side of libuqc: contexts, basis plans (normalisation, primitive-pair data, Schwarz bounds, pair bins and
// screened work lists), the ERI-block and Fock-build entry points of include/uqc.h.
#include "uqc_api_internal.h"
#include "generated/rys_table.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <tuple>
#include <string>
#include <vector>

using namespace uqc;

namespace {
thread_local std::string g_err;
}

uqc_status uqc_fail(uqc_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

const char* uqc_last_error(void) { return g_err.c_str(); }

void uqc_fock_opts_default(uqc_fock_opts* o) {
    if (!o) return;
    o->schwarz_tau = 1e-12;
    o->precision = UQC_FP64;
    o->fp64_bound = 1e-8;
    o->timing = 0;
    o->progress = nullptr;
    o->progress_user = nullptr;
    o->max_items_per_launch = 0;
    o->exchange_scale = 1.0;
    o->streams = 3;
    o->fp64_boys_T = (double)kBoysTmax32;
}

// ---------------------------------------------------------------------------------------------- Boys table
// F_n(T_g), n = 0..16, and exp(-T_g), T_g = g/8 for g = 0..320; F_n from Gauss-Legendre quadrature (long double,
// 96 nodes) of the
// defining integral F_n(T) = int_0^1 t^{2n} exp(-T t^2) dt; the integrand is entire, so the rule converges to
// the working precision for T <= 40.
static void legendre_nodes(int n, std::vector<long double>& x, std::vector<long double>& w) {
    x.resize(n);
    w.resize(n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        long double z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
        long double dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
            const long double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-21L) break;
        }
        long double p0 = 1, p1 = z;
        for (int k = 2; k <= n; ++k) {
            long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1);
        x[i] = z;
        w[i] = 2 / ((1 - z * z) * dp * dp);
    }
}

static void build_boys_table(std::vector<double>& tab) {
    std::vector<long double> x, w;
    legendre_nodes(96, x, w);
    tab.assign((size_t)kBoysNg * kBoysNm, 0.0);
    for (int g = 0; g < kBoysNg; ++g) {
        const long double T = (long double)g / kBoysGridPerUnit;
        tab[(size_t)g * kBoysNm + kBoysExpCol] = (double)std::exp(-T);
        for (int n = 0; n < kBoysExpCol; ++n) {
            long double s = 0;
            for (size_t i = 0; i < x.size(); ++i) {
                const long double t = 0.5L * (x[i] + 1);  // map [-1, 1] -> [0, 1]
                long double tp = 1;
                for (int k = 0; k < n; ++k) tp *= t * t;
                s += w[i] * tp * std::exp(-T * t * t);
            }
            tab[(size_t)g * kBoysNm + n] = (double)(0.5L * s);
        }
    }
}

// ---------------------------------------------------------------------------------------------- context
uqc_status uqc_init(int device, void* hip_stream, uqc_ctx** out) {
    if (!out) return uqc_fail(UQC_E_ARG, "uqc_init: out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return uqc_fail(UQC_E_DEVICE, "uqc_init: no HIP device");
    if (device < 0 || device >= ndev) return uqc_fail(UQC_E_ARG, "uqc_init: device index out of range");
    UQC_HIP(hipSetDevice(device));
    uqc_ctx* c = new uqc_ctx();
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) {  // blocking: ordered after work on the null stream
            delete c;
            return uqc_fail(UQC_E_DEVICE, "uqc_init: hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    std::vector<double> full;
    build_boys_table(full);
    std::vector<float> tab32(full.size());
    for (size_t i = 0; i < full.size(); ++i) tab32[i] = (float)full[i];
    // per-order slices for the FP64 evaluation
    std::vector<double> tab((size_t)(kBoysLmax + 1) * kBoysNg * kBoysRow);
    for (int L = 0; L <= kBoysLmax; ++L)
        for (int g = 0; g < kBoysNg; ++g) {
            double* row = tab.data() + ((size_t)L * kBoysNg + g) * kBoysRow;
            double inv_fact = 1.0;  // Taylor coefficients F_{L+k}(T_g) / k!
            for (int k = 0; k < 9; ++k) {
                if (k > 0) inv_fact /= k;
                row[k] = full[(size_t)g * kBoysNm + L + k] * inv_fact;
            }
            row[9] = full[(size_t)g * kBoysNm + kBoysExpCol];
        }
    if (hipMalloc(&c->boys64, tab.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->boys32, tab32.size() * sizeof(float)) != hipSuccess) {
        uqc_finalize(c);
        return uqc_fail(UQC_E_NOMEM, "uqc_init: cannot allocate the Boys table");
    }
    if (hipMemcpy(c->boys64, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->boys32, tab32.data(), tab32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        uqc_finalize(c);
        return uqc_fail(UQC_E_DEVICE, "uqc_init: cannot upload the Boys table");
    }
    if (hipMalloc(&c->rys, sizeof(kRysTab)) != hipSuccess ||
        hipMemcpy(c->rys, kRysTab, sizeof(kRysTab), hipMemcpyHostToDevice) != hipSuccess) {
        uqc_finalize(c);
        return uqc_fail(UQC_E_DEVICE, "uqc_init: cannot upload the Rys table");
    }
    // the device address of the fixed workspace of uqc_fock_build_noalloc, taken once per device with it current
    {
        const uqc_status st = uqc::noalloc_setup(device);
        if (st != UQC_OK) {
            uqc_finalize(c);
            return st;
        }
    }
    *out = c;
    return UQC_OK;
}

uqc_status uqc_finalize(uqc_ctx* c) {
    if (!c) return uqc_fail(UQC_E_ARG, "uqc_finalize: NULL context");
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& e : c->events) (void)hipEventDestroy(e);
    for (int i = 0; i < 3; ++i) {
        if (c->side[i]) {
            (void)hipStreamSynchronize(c->side[i]);
            (void)hipStreamDestroy(c->side[i]);
        }
        if (c->join[i]) (void)hipEventDestroy(c->join[i]);
    }
    if (c->fork) (void)hipEventDestroy(c->fork);
    release_blas(c);
    if (c->boys64) (void)hipFree(c->boys64);
    if (c->boys32) (void)hipFree(c->boys32);
    if (c->rys) (void)hipFree(c->rys);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return UQC_OK;
}

hipEvent_t ctx_event(uqc_ctx* c, size_t i) {
    while (c->events.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->events.push_back(e);
    }
    return c->events[i];
}

std::vector<size_t> interleave_ends(const std::vector<size_t>& v) {
    std::vector<size_t> out;
    out.reserve(v.size());
    size_t lo = 0, hi = v.size();
    while (lo < hi) {
        out.push_back(v[lo++]);
        if (lo < hi) out.push_back(v[--hi]);
    }
    return out;
}

hipStream_t ctx_stream(uqc_ctx* c, int i) {
    if (i == 0) return c->stream;
    if (i < 1 || i > 3) return nullptr;
    if (!c->fork && hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess) {
        c->fork = nullptr;
        return nullptr;
    }
    if (!c->join[i - 1] && hipEventCreateWithFlags(&c->join[i - 1], hipEventDisableTiming) != hipSuccess) {
        c->join[i - 1] = nullptr;
        return nullptr;
    }
    if (!c->side[i - 1] && hipStreamCreateWithFlags(&c->side[i - 1], hipStreamNonBlocking) != hipSuccess) {
        c->side[i - 1] = nullptr;
        return nullptr;
    }
    return c->side[i - 1];
}

// ---------------------------------------------------------------------------------------------- basis
static int ncart(int l) { return (l + 1) * (l + 2) / 2; }
static int pclass(int la, int lb) {
    static const int tab[3][3] = {{0, -1, -1}, {1, 2, -1}, {3, 4, 5}};
    return tab[la][lb];
}

uqc_basis::~uqc_basis() {
    (void)hipSetDevice(ctx->device);
    for (auto& b : bins) {
        if (b.d_mem) (void)hipFree(b.d_mem);
    }
    for (auto& kv : plans) free_plan(kv.second);
    if (d_work) (void)hipFree(d_work);
    if (d_uio) (void)hipFree(d_uio);
    if (d_shells) (void)hipFree(d_shells);
    if (d_nuc) (void)hipFree(d_nuc);
}

size_t uqc_basis::device_bytes() const {
    size_t n = work_bytes;
    for (const auto& b : bins) n += b.bytes;
    for (const auto& kv : plans) n += kv.second.bytes;
    return n;
}

uqc_status uqc::check_fock_opts(const uqc_fock_opts& o, const std::string& nm) {
    if (!(o.schwarz_tau >= 0) || !std::isfinite(o.schwarz_tau)) return uqc_fail(UQC_E_ARG, nm + ": bad tau");
    if (o.precision != UQC_FP64 && o.precision != UQC_MIXED) return uqc_fail(UQC_E_ARG, nm + ": bad precision");
    if (o.precision == UQC_MIXED && !(o.fp64_bound >= 0)) return uqc_fail(UQC_E_ARG, nm + ": bad fp64_bound");
    if (o.precision == UQC_MIXED && !(o.fp64_boys_T >= 0 && o.fp64_boys_T <= (double)kBoysTmax32))
        return uqc_fail(UQC_E_ARG, nm + ": fp64_boys_T must be in 0..30 (the FP32 Boys table's range)");
    if (o.max_items_per_launch < 0) return uqc_fail(UQC_E_ARG, nm + ": negative max_items_per_launch");
    if (!std::isfinite(o.exchange_scale)) return uqc_fail(UQC_E_ARG, nm + ": exchange_scale is not finite");
    if (o.streams < 0 || o.streams > 4) return uqc_fail(UQC_E_ARG, nm + ": streams must be in 0..4");
    return UQC_OK;
}

void uqc::free_plan(Plan& p) {
    if (p.d_mem) (void)hipFree(p.d_mem);
    p.d_mem = nullptr;
}

// Device arrays of a bin in one allocation: prim [kNumFields*K*np], AB [3*np], sdeg [np], Q [np], rec
// [np*K*kRec], hdr [np*kHdr], cq [ceil(np/64)*K], off_a [np], off_b [np], kp [np].  Before the primitive bounds are
// known, the record slot of Q_e and cq hold a huge value (nothing is screened by them).
static uqc_status upload_bin(Bin& b) {
    const size_t np = b.np, K = b.K;
    const size_t nchunk = (np + kWave - 1) / kWave;
    const size_t n_prim = kNumFields * K * np, n_rec = np * K * kRec, n_hdr = np * kHdr, n_cq = nchunk * K;
    const size_t nd = n_prim + 3 * np + 2 * np + n_rec + n_hdr + n_cq;
    const bool have_q = b.qprim.size() == K * np;
    constexpr double kUnknown = 1e300;
    const size_t bytes = nd * sizeof(double) + 3 * np * sizeof(int);
    if (!b.d_mem) {
        if (hipMalloc(&b.d_mem, bytes) != hipSuccess) return uqc_fail(UQC_E_NOMEM, "basis: bin allocation failed");
        b.bytes = bytes;
    }
    std::vector<char> host(bytes, 0);
    double* hd = (double*)host.data();
    std::memcpy(hd, b.prim.data(), n_prim * sizeof(double));
    std::memcpy(hd + n_prim, b.AB.data(), 3 * np * sizeof(double));
    std::memcpy(hd + n_prim + 3 * np, b.sdeg.data(), np * sizeof(double));
    std::memcpy(hd + n_prim + 4 * np, b.Q.data(), np * sizeof(double));
    double* rec = hd + n_prim + 5 * np;
    double* hdr = rec + n_rec;
    for (size_t i = 0; i < np; ++i) {
        for (size_t k = 0; k < K; ++k) {
            for (size_t f = 0; f < (size_t)kNumFields; ++f) rec[(i * K + k) * kRec + f] = b.prim[(f * K + k) * np + i];
            rec[(i * K + k) * kRec + kRecQ] = have_q ? b.qprim[k * np + i] : kUnknown;
        }
        double* h = hdr + i * kHdr;
        h[0] = b.AB[i];
        h[1] = b.AB[np + i];
        h[2] = b.AB[2 * np + i];
        h[3] = b.sdeg[i];
        h[4] = b.Q[i];
        int* o = (int*)(h + 5);
        o[0] = b.off_a[i];
        o[1] = b.off_b[i];
    }
    double* cq = hdr + n_hdr;
    for (size_t c = 0; c < nchunk; ++c)
        for (size_t k = 0; k < K; ++k) {
            double m = have_q ? 0.0 : kUnknown;
            if (have_q)
                for (size_t i = c * kWave; i < std::min(np, (c + 1) * kWave); ++i) m = std::max(m, b.qprim[k * np + i]);
            cq[c * K + k] = m;
        }
    int* hi = (int*)(hd + nd);
    std::memcpy(hi, b.off_a.data(), np * sizeof(int));
    std::memcpy(hi + np, b.off_b.data(), np * sizeof(int));
    for (size_t i = 0; i < np; ++i) hi[2 * np + i] = b.kp.empty() ? (int)K : b.kp[i];
    UQC_HIP(hipMemcpy(b.d_mem, host.data(), bytes, hipMemcpyHostToDevice));
    double* dd = (double*)b.d_mem;
    int* di = (int*)(dd + nd);
    b.dev.prim = dd;
    b.dev.AB = dd + n_prim;
    b.dev.sdeg = dd + n_prim + 3 * np;
    b.dev.Q = dd + n_prim + 4 * np;
    b.dev.rec = dd + n_prim + 5 * np;
    b.dev.hdr = b.dev.rec + n_rec;
    b.dev.cq = b.dev.hdr + n_hdr;
    b.dev.off_a = di;
    b.dev.off_b = di + np;
    b.dev.kp = di + 2 * np;
    b.dev.np = (int)np;
    b.dev.K = (int)K;
    return UQC_OK;
}

// Decade of a pair bound, rounded up near powers of ten, and decade of a threshold, rounded down: every pair with
// Q >= t then has decade(Q) >= decade_floor(t), whatever the rounding of log10.
static int decade(double q) { return q > 0 ? (int)std::floor(std::log10(q) + 1e-9) : -400; }
static int decade_floor(double t) { return t > 0 ? (int)std::floor(std::log10(t) - 1e-9) : -400; }

int Bin::first_below(int dec) const {
    for (const auto& x : bstart)
        if (x.first < dec) return x.second;
    return np;
}

int Bin::first_at_or_below(int dec) const {
    for (const auto& x : bstart)
        if (x.first <= dec) return x.second;
    return np;
}

// Reorders the host arrays of a bin by the permutation `perm` (new position i takes old perm[i]).
static void permute_bin(Bin& b, const std::vector<int>& perm) {
    const size_t np = b.np, K = b.K;
    std::vector<double> prim(b.prim.size()), AB(b.AB.size()), sdeg(np), Q(np);
    std::vector<int> oa(np), ob(np), sa(np), sb(np), kp(np);
    std::vector<double> qprim(b.qprim.size());
    for (size_t i = 0; i < np; ++i) {
        const size_t o = perm[i];
        kp[i] = b.kp[o];
        if (!qprim.empty())
            for (size_t k = 0; k < K; ++k) qprim[k * np + i] = b.qprim[k * np + o];
        for (size_t f = 0; f < (size_t)kNumFields; ++f)
            for (size_t k = 0; k < K; ++k) prim[(f * K + k) * np + i] = b.prim[(f * K + k) * np + o];
        for (int x = 0; x < 3; ++x) AB[x * np + i] = b.AB[x * np + o];
        sdeg[i] = b.sdeg[o];
        Q[i] = b.Q[o];
        oa[i] = b.off_a[o];
        ob[i] = b.off_b[o];
        sa[i] = b.sa[o];
        sb[i] = b.sb[o];
    }
    b.prim.swap(prim);
    b.AB.swap(AB);
    b.sdeg.swap(sdeg);
    b.Q.swap(Q);
    b.off_a.swap(oa);
    b.off_b.swap(ob);
    b.sa.swap(sa);
    b.sb.swap(sb);
    b.kp.swap(kp);
    b.qprim.swap(qprim);
}

// Bounds Q_e = sqrt(max_ij (e|e)_ij) of every primitive pair e of a bin (entry e = k * np + i for primitive pair k
// of pair i), from the bin viewed as K = 1: its field-major primitive array [field][k][i] is already laid out as
// [field][e].  didx holds 0..n-1 and dq room for n values, n >= K * np.
static uqc_status prim_schwarz(uqc_ctx* ctx, const Bin& bn, const int* didx, double* dq, std::vector<double>& qp) {
    const size_t np = bn.np, K = bn.K, nv = np * K;
    Bin v;
    v.la = bn.la;
    v.lb = bn.lb;
    v.K = 1;
    v.np = (int)nv;
    v.prim = bn.prim;
    v.AB.resize(3 * nv);
    v.sdeg.assign(nv, 1.0);
    v.Q.assign(nv, 0.0);
    v.off_a.resize(nv);
    v.off_b.resize(nv);
    for (size_t k = 0; k < K; ++k)
        for (size_t i = 0; i < np; ++i) {
            const size_t e = k * np + i;
            for (int x = 0; x < 3; ++x) v.AB[x * nv + e] = bn.AB[x * np + i];
            v.off_a[e] = bn.off_a[i];
            v.off_b[e] = bn.off_b[i];
        }
    uqc_status st = upload_bin(v);
    if (st != UQC_OK) return st;
    ListDev L{};
    L.bra = v.dev;
    L.ket = v.dev;
    L.bra_idx = didx;
    L.ket_idx = didx;
    L.n = (int)nv;
    L.out = dq;
    qp.assign(nv, 0.0);
    const int cls = class_index(bn.la, bn.lb, bn.la, bn.lb);
    if (launch_list(cls, false, MODE_SCHWARZ, L, ctx->boys64, ctx->boys32, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(qp.data(), dq, nv * sizeof(double), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        st = uqc_fail(UQC_E_DEVICE, "basis: primitive Schwarz kernel failed");
    (void)hipFree(v.d_mem);
    return st;
}

// Orders the primitive pairs of every shell pair by decreasing bound and sets kp to the number with
// Q_e * qmax > kPrimEps (at least 1).  qp[b] holds the primitive bounds of bins[b].  Re-uploaded later.
static void order_primitives(std::vector<Bin>& bins, const std::vector<std::vector<double>>& qp, double qmax) {
    for (size_t b = 0; b < bins.size(); ++b) {
        Bin& bn = bins[b];
        const size_t np = bn.np, K = bn.K;
        bn.qprim.assign(K * np, 0.0);
        std::vector<int> ord(K);
        std::vector<double> rec(kNumFields * K);
        for (size_t i = 0; i < np; ++i) {
            std::iota(ord.begin(), ord.end(), 0);
            std::stable_sort(ord.begin(), ord.end(),
                             [&](int x, int y) { return qp[b][(size_t)x * np + i] > qp[b][(size_t)y * np + i]; });
            int keep = 0;
            for (size_t k = 0; k < K; ++k)
                if (qp[b][(size_t)ord[k] * np + i] * qmax > kPrimEps) ++keep;
            bn.kp[i] = std::max(keep, 1);
            for (size_t k = 0; k < K; ++k) bn.qprim[k * np + i] = qp[b][(size_t)ord[k] * np + i];
            for (size_t f = 0; f < (size_t)kNumFields; ++f)
                for (size_t k = 0; k < K; ++k) rec[f * K + k] = bn.prim[(f * K + ord[k]) * np + i];
            for (size_t f = 0; f < (size_t)kNumFields; ++f)
                for (size_t k = 0; k < K; ++k) bn.prim[(f * K + k) * np + i] = rec[f * K + k];
        }
    }
}

uqc_status uqc_basis_create(uqc_ctx* ctx, int nshell, const int* l, const int* nprim, const double* center,
                            const double* alpha, const double* coef, uqc_basis** out) {
    if (!ctx || !out || !l || !nprim || !center || !alpha || !coef)
        return uqc_fail(UQC_E_ARG, "uqc_basis_create: NULL argument");
    *out = nullptr;
    if (nshell <= 0) return uqc_fail(UQC_E_ARG, "uqc_basis_create: nshell must be positive");
    size_t nprim_tot = 0;
    for (int s = 0; s < nshell; ++s) {
        if (l[s] < 0 || nprim[s] < 1) return uqc_fail(UQC_E_ARG, "uqc_basis_create: l < 0 or nprim < 1");
        if (l[s] > 2) return uqc_fail(UQC_E_UNSUPPORTED, "uqc_basis_create: l > 2 is not supported");
        if (nprim[s] > kMaxK) return uqc_fail(UQC_E_UNSUPPORTED, "uqc_basis_create: contraction depth > 16");
        for (int x = 0; x < 3; ++x)
            if (!std::isfinite(center[3 * s + x])) return uqc_fail(UQC_E_ARG, "uqc_basis_create: non-finite centre");
        nprim_tot += nprim[s];
    }
    for (size_t p = 0; p < nprim_tot; ++p)
        if (!(alpha[p] > 0) || !std::isfinite(alpha[p]) || !std::isfinite(coef[p]))
            return uqc_fail(UQC_E_ARG, "uqc_basis_create: exponents must be positive and finite, coefficients finite");
    UQC_HIP(hipSetDevice(ctx->device));

    uqc_basis* B = new uqc_basis();
    B->ctx = ctx;
    B->nshell = nshell;
    B->shells.resize(nshell);
    const double pi = 3.14159265358979323846;
    int off = 0;
    size_t p = 0;
    for (int s = 0; s < nshell; ++s) {
        ShellH& sh = B->shells[s];
        sh.l = l[s];
        sh.K = nprim[s];
        for (int x = 0; x < 3; ++x) sh.A[x] = center[3 * s + x];
        sh.alpha.assign(alpha + p, alpha + p + sh.K);
        // radial normalisation N_r(a) = (2a/pi)^{3/4} (4a)^{l/2}; contracted renormalisation from the self-overlap
        // of the axis component, sum_pq d_p d_q N_r N_r (pi/g)^{3/2} / (2g)^l with g = a_p + a_q
        std::vector<double> nr(sh.K);
        for (int k = 0; k < sh.K; ++k)
            nr[k] = std::pow(2.0 * sh.alpha[k] / pi, 0.75) * std::pow(4.0 * sh.alpha[k], 0.5 * sh.l);
        double S = 0.0;
        for (int i = 0; i < sh.K; ++i)
            for (int j = 0; j < sh.K; ++j) {
                const double g = sh.alpha[i] + sh.alpha[j];
                S += coef[p + i] * coef[p + j] * nr[i] * nr[j] * std::pow(pi / g, 1.5) / std::pow(2.0 * g, sh.l);
            }
        if (!(S > 0) || !std::isfinite(S)) {
            delete B;
            return uqc_fail(UQC_E_ARG, "uqc_basis_create: contracted shell has zero or invalid norm");
        }
        sh.c.resize(sh.K);
        for (int k = 0; k < sh.K; ++k) sh.c[k] = coef[p + k] * nr[k] / std::sqrt(S);
        sh.off = off;
        off += ncart(sh.l);
        p += sh.K;
    }
    B->nbf = off;
    if (off > kMaxNbf) {  // the kernels index N x N matrices with 32-bit offsets
        delete B;
        return uqc_fail(UQC_E_UNSUPPORTED, "uqc_basis_create: more than 65535 basis functions");
    }
    B->fcomp.resize(B->nbf);
    for (int s = 0; s < nshell; ++s)
        for (int c = 0; c < ncart(B->shells[s].l); ++c)
            B->fcomp[B->shells[s].off + c] = (B->shells[s].l == 2 && (c == 0 || c == 3 || c == 5))
                                                 ? 0.57735026918962576451 : 1.0;

    // shell pairs, oriented so that the first shell has the higher l (then the deeper contraction, then the larger
    // index), binned by (l1, l2, K1, K2)
    struct Key { int l1, l2, K1, K2; };
    std::vector<Key> keys;
    B->pair_bin.assign((size_t)nshell * nshell, -1);
    B->pair_pos.assign((size_t)nshell * nshell, -1);
    B->pair_first.assign((size_t)nshell * nshell, -1);
    std::vector<std::vector<std::pair<int, int>>> members;
    for (int a = 0; a < nshell; ++a)
        for (int b = 0; b <= a; ++b) {
            const ShellH &sa = B->shells[a], &sb = B->shells[b];
            int f = a, s = b;
            if (sb.l > sa.l || (sb.l == sa.l && (sb.K > sa.K || (sb.K == sa.K && b > a)))) { f = b; s = a; }
            const ShellH &F = B->shells[f], &Sx = B->shells[s];
            int bi = -1;
            for (size_t k = 0; k < keys.size(); ++k)
                if (keys[k].l1 == F.l && keys[k].l2 == Sx.l && keys[k].K1 == F.K && keys[k].K2 == Sx.K) bi = (int)k;
            if (bi < 0) {
                keys.push_back({F.l, Sx.l, F.K, Sx.K});
                members.emplace_back();
                bi = (int)keys.size() - 1;
            }
            members[bi].push_back({f, s});
        }
    // bin order: pair class, then K1, K2 (a class kernel (X|Y) needs class(X) >= class(Y) for X >= Y)
    std::vector<int> order(keys.size());
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        const int px = pclass(keys[x].l1, keys[x].l2), py = pclass(keys[y].l1, keys[y].l2);
        if (px != py) return px < py;
        if (keys[x].K1 != keys[y].K1) return keys[x].K1 < keys[y].K1;
        return keys[x].K2 < keys[y].K2;
    });
    B->bins.resize(keys.size());
    for (size_t bo = 0; bo < order.size(); ++bo) {
        const Key& k = keys[order[bo]];
        Bin& bn = B->bins[bo];
        bn.la = k.l1;
        bn.lb = k.l2;
        bn.Ka = k.K1;
        bn.Kb = k.K2;
        bn.K = k.K1 * k.K2;
        const auto& mem = members[order[bo]];
        bn.np = (int)mem.size();
        const size_t np = bn.np, K = bn.K;
        bn.prim.assign(kNumFields * K * np, 0.0);
        bn.AB.assign(3 * np, 0.0);
        bn.sdeg.assign(np, 1.0);
        bn.Q.assign(np, 0.0);
        bn.off_a.resize(np);
        bn.off_b.resize(np);
        bn.sa.resize(np);
        bn.sb.resize(np);
        bn.kp.assign(np, (int)K);
        for (size_t i = 0; i < np; ++i) {
            const ShellH& A = B->shells[mem[i].first];
            const ShellH& Bs = B->shells[mem[i].second];
            bn.sa[i] = mem[i].first;
            bn.sb[i] = mem[i].second;
            bn.off_a[i] = A.off;
            bn.off_b[i] = Bs.off;
            bn.sdeg[i] = (mem[i].first == mem[i].second) ? 0.5 : 1.0;
            double AB[3], AB2 = 0.0;
            for (int x = 0; x < 3; ++x) {
                AB[x] = A.A[x] - Bs.A[x];
                AB2 += AB[x] * AB[x];
                bn.AB[x * np + i] = AB[x];
            }
            const double c0 = std::sqrt(2.0) * std::pow(pi, 1.25);
            for (int ia = 0; ia < A.K; ++ia)
                for (int ib = 0; ib < Bs.K; ++ib) {
                    const size_t kk = (size_t)ia * Bs.K + ib;
                    const double al = A.alpha[ia], be = Bs.alpha[ib];
                    const double z = al + be;
                    auto put = [&](int f, double v) { bn.prim[((size_t)f * K + kk) * np + i] = v; };
                    put(F_Z, z);
                    double P[3];
                    for (int x = 0; x < 3; ++x) P[x] = (al * A.A[x] + be * Bs.A[x]) / z;
                    put(F_PX, P[0]);
                    put(F_PY, P[1]);
                    put(F_PZ, P[2]);
                    put(F_PAX, P[0] - A.A[0]);
                    put(F_PAY, P[1] - A.A[1]);
                    put(F_PAZ, P[2] - A.A[2]);
                    put(F_PREF, A.c[ia] * Bs.c[ib] * std::exp(-al * be / z * AB2) * c0 / z);
                    put(F_O2Z, 0.5 / z);
                }
        }
        uqc_status st = upload_bin(bn);
        if (st != UQC_OK) { delete B; return st; }
    }

    // Schwarz bounds on the GPU: diagonal quartets (ab|ab) of every bin
    {
        size_t maxnp = 0;
        for (auto& bn : B->bins) maxnp = std::max(maxnp, (size_t)bn.np);
        void* tmp = nullptr;
        if (hipMalloc(&tmp, maxnp * (2 * sizeof(int) + sizeof(double))) != hipSuccess) {
            delete B;
            return uqc_fail(UQC_E_NOMEM, "basis: Schwarz scratch allocation failed");
        }
        std::vector<int> idx(maxnp);
        std::iota(idx.begin(), idx.end(), 0);
        int* didx = (int*)tmp;
        double* dq = (double*)(didx + 2 * maxnp);
        uqc_status st = UQC_OK;
        if (hipMemcpy(didx, idx.data(), maxnp * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
            st = uqc_fail(UQC_E_DEVICE, "basis: upload failed");
        for (size_t bi = 0; bi < B->bins.size() && st == UQC_OK; ++bi) {
            Bin& bn = B->bins[bi];
            ListDev L{};
            L.bra = bn.dev;
            L.ket = bn.dev;
            L.bra_idx = didx;
            L.ket_idx = didx;
            L.n = bn.np;
            L.out = dq;
            const int cls = class_index(bn.la, bn.lb, bn.la, bn.lb);
            if (launch_list(cls, false, MODE_SCHWARZ, L, ctx->boys64, ctx->boys32, ctx->stream) != hipSuccess ||
                hipMemcpyAsync(bn.Q.data(), dq, bn.np * sizeof(double), hipMemcpyDeviceToHost, ctx->stream) !=
                    hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess)
                st = uqc_fail(UQC_E_DEVICE, "basis: Schwarz kernel failed");
        }
        (void)hipFree(tmp);
        if (st != UQC_OK) { delete B; return st; }
    }
    // primitive-pair screening: bounds of every primitive pair on the GPU, then each pair's primitive pairs ordered
    // by bound with the count above kPrimEps recorded
    {
        double qmax = 0.0;
        size_t maxn = 0;
        for (auto& bn : B->bins) {
            for (int i = 0; i < bn.np; ++i) qmax = std::max(qmax, bn.Q[i]);
            maxn = std::max(maxn, (size_t)bn.np * bn.K);
        }
        void* tmp = nullptr;
        if (hipMalloc(&tmp, (maxn + 1) * (sizeof(int) + sizeof(double))) != hipSuccess) {
            delete B;
            return uqc_fail(UQC_E_NOMEM, "basis: primitive Schwarz scratch allocation failed");
        }
        std::vector<int> idx(maxn);
        std::iota(idx.begin(), idx.end(), 0);
        int* didx = (int*)tmp;
        double* dq = (double*)(didx + maxn + (maxn & 1));
        uqc_status st = UQC_OK;
        if (hipMemcpy(didx, idx.data(), maxn * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
            st = uqc_fail(UQC_E_DEVICE, "basis: upload failed");
        std::vector<std::vector<double>> qp(B->bins.size());
        for (size_t bi = 0; bi < B->bins.size() && st == UQC_OK; ++bi)
            st = prim_schwarz(ctx, B->bins[bi], didx, dq, qp[bi]);
        (void)hipFree(tmp);
        if (st != UQC_OK) { delete B; return st; }
        order_primitives(B->bins, qp, qmax);
    }
    // Morton code of every shell centre (10 bits per axis over the bounding box): pairs that differ only in their
    // second shell are ordered along this curve, so neighbouring lanes hold nearby pairs
    std::vector<uint32_t> morton(nshell);
    {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int s = 0; s < nshell; ++s)
            for (int x = 0; x < 3; ++x) {
                lo[x] = std::min(lo[x], B->shells[s].A[x]);
                hi[x] = std::max(hi[x], B->shells[s].A[x]);
            }
        for (int s = 0; s < nshell; ++s) {
            uint32_t q[3];
            for (int x = 0; x < 3; ++x) {
                const double span = hi[x] > lo[x] ? hi[x] - lo[x] : 1.0;
                q[x] = (uint32_t)std::min(1023.0, std::floor((B->shells[s].A[x] - lo[x]) / span * 1024.0));
            }
            uint32_t m = 0;
            for (int bit = 0; bit < 10; ++bit)
                for (int x = 0; x < 3; ++x) m |= ((q[x] >> bit) & 1u) << (3 * bit + x);
            morton[s] = m;
        }
    }
    // sort each bin and re-upload; record where every shell pair landed
    B->Qfull.assign((size_t)nshell * nshell, 0.0);
    for (size_t bi = 0; bi < B->bins.size(); ++bi) {
        Bin& bn = B->bins[bi];
        std::vector<int> perm(bn.np);
        std::iota(perm.begin(), perm.end(), 0);
        // decade of the bound (descending), then the number of primitive pairs kept (descending: the ket loop of a
        // 64-pair chunk runs to its largest count, and the per-chunk primitive screen ends it sooner when the chunk's
        // pairs keep similar numbers), then first shell, then the second shell along the space-filling curve (then
        // bound, descending)
        std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) {
            const int dx = decade(bn.Q[x]), dy = decade(bn.Q[y]);
            if (dx != dy) return dx > dy;
            if (bn.kp[x] != bn.kp[y]) return bn.kp[x] > bn.kp[y];
            if (bn.off_a[x] != bn.off_a[y]) return bn.off_a[x] < bn.off_a[y];
            const uint32_t mx = morton[bn.sb[x]], my = morton[bn.sb[y]];
            if (mx != my) return mx < my;
            return bn.Q[x] > bn.Q[y];
        });
        permute_bin(bn, perm);
        bn.bucket.resize(bn.np);
        bn.bstart.clear();
        for (int i = 0; i < bn.np; ++i) {
            bn.bucket[i] = decade(bn.Q[i]);
            if (i == 0 || bn.bucket[i] != bn.bucket[i - 1]) bn.bstart.push_back({bn.bucket[i], i});
        }
        uqc_status st = upload_bin(bn);
        if (st != UQC_OK) { delete B; return st; }
        for (int i = 0; i < bn.np; ++i) {
            const int a = bn.sa[i], b = bn.sb[i];
            for (auto key : {(size_t)a * nshell + b, (size_t)b * nshell + a}) {
                B->pair_bin[key] = (int)bi;
                B->pair_pos[key] = i;
                B->pair_first[key] = a;
            }
            B->Qfull[(size_t)a * nshell + b] = B->Qfull[(size_t)b * nshell + a] = bn.Q[i];
        }
        for (int i = 0; i < bn.np; ++i) B->qmax = std::max(B->qmax, bn.Q[i]);
    }
    // workspace: f[nbf], D', J, K accumulators, E2 + symmetry scalars, host-pointer staging for D, J, K, G, and for
    // spin-density builds the second spin's D' and K accumulator and the total D' of the J pass
    {
        const size_t N = B->nbf, NN = N * N;
        const size_t bytes = (N + 3 * NN + 8 + 4 * NN + 3 * NN) * sizeof(double);
        if (hipMalloc(&B->d_work, bytes) != hipSuccess) {
            delete B;
            return uqc_fail(UQC_E_NOMEM, "basis: workspace allocation failed");
        }
        double* w = (double*)B->d_work;
        B->d_f = w;
        B->d_Dp = w + N;
        B->d_J = B->d_Dp + NN;
        B->d_K = B->d_J + NN;
        B->d_scal = B->d_K + NN;
        B->d_io = B->d_scal + 8;
        B->d_Dp2 = B->d_io + 4 * NN;
        B->d_K2 = B->d_Dp2 + NN;
        B->d_Dp3 = B->d_K2 + NN;
        B->work_bytes = bytes;
        if (hipMemcpy(B->d_f, B->fcomp.data(), N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
            delete B;
            return uqc_fail(UQC_E_DEVICE, "basis: upload failed");
        }
    }
    *out = B;
    return UQC_OK;
}

uqc_status uqc_basis_destroy(uqc_basis* b) {
    if (!b) return uqc_fail(UQC_E_ARG, "uqc_basis_destroy: NULL basis");
    (void)hipStreamSynchronize(b->ctx->stream);
    delete b;
    return UQC_OK;
}

uqc_status uqc_basis_info(const uqc_basis* b, int* nbf, int* shell_offset) {
    if (!b) return uqc_fail(UQC_E_ARG, "uqc_basis_info: NULL basis");
    if (nbf) *nbf = b->nbf;
    if (shell_offset)
        for (int s = 0; s < b->nshell; ++s) shell_offset[s] = b->shells[s].off;
    return UQC_OK;
}

uqc_status uqc_schwarz(const uqc_basis* b, double* Q) {
    if (!b || !Q) return uqc_fail(UQC_E_ARG, "uqc_schwarz: NULL argument");
    std::memcpy(Q, b->Qfull.data(), b->Qfull.size() * sizeof(double));
    return UQC_OK;
}

// ---------------------------------------------------------------------------------------------- screened plan
// For every bin pair (X >= Y) the canonical quartets are, per bra pair i of X, the kets j of Y with Q_i Q_j >= tau
// and, if X == Y, j <= i.  Ket bins are ordered by decade of Q (descending), so the kets that can pass form a prefix
// ending one decade below the decade of tau / Q_i; the kernels apply the exact test per lane.  In mixed precision
// the FP64 task takes the kets with Q_i Q_j > bound and the FP32-recursion task those with Q_i Q_j <= bound; the
// decade holding the split is scanned by both tasks with complementary per-lane tests.  The work items of a task
// are (ket chunk, group of bra pairs) pairs, listed chunk by chunk (TaskDev).
void uqc::plan_account(Plan& p) {
    p.quartets = p.prim_quartets = p.fp64_quartets = 0;
    p.flops = 0;
    for (auto& g : p.groups) {
        g.quartets = g.prim_quartets = 0;
        g.flops = 0;
        for (int t = 0; t < g.ntask; ++t) {
            const long long q = (long long)p.h_count[g.task0 + t];
            const long long pq = (long long)p.h_count[p.ntasks + g.task0 + t];
            g.quartets += q;
            g.prim_quartets += pq;
            g.flops += (double)q * class_flops_contr(g.cls) + (double)pq * class_flops_prim(g.cls);
        }
        p.quartets += g.quartets;
        p.prim_quartets += g.prim_quartets;
        if (!g.mixed) p.fp64_quartets += g.quartets;
        p.flops += g.flops;
    }
    p.screened = p.canonical - p.quartets;
}

// Bra pairs per work item: kGroupBras for the 64-ket kernels and kTeamGroupBras for the team kernels, more for the
// classes measured faster with larger groups (the item's ket loads, J_cd flush and task lookup spread over more bra
// pairs, at the price of fewer wavefronts): (ds|ss), (dp|ss), (dd|ss), (ds|ds), (ds|pp), (dp|ds) take 16 (32 is
// slower); the team kernels of (dp|dp) and (dd|dp) take 8, (dd|ds) 12.
// A task (bin pair and precision) with few (bra pair, ket chunk) entries gets smaller groups, down to one bra pair,
// so that it still has about kItemTarget items: a small molecule's class launch would otherwise occupy a fraction
// of the resident wavefronts, each for the whole length of one long item.
constexpr long long kItemTarget = 2048;

static int group_bras(int cls) {
    int la, lb, lc, ld;
    class_ls(cls, &la, &lb, &lc, &ld);
    switch (la * 1000 + lb * 100 + lc * 10 + ld) {
        case 2000: case 2100: case 2200: case 2020: case 2011: case 2120: return 16;
        case 2220: return 12;
        case 2121: case 2221: return 8;
        default: return class_team(cls) ? kTeamGroupBras : kGroupBras;
    }
}

Plan* find_plan(uqc_basis* B, double tau, int prec, double bound, double boys_t) {
    for (auto& kv : B->plans)
        if (kv.first.tau == tau && kv.first.prec == prec &&
            (prec == UQC_FP64 || (kv.first.bound == bound && kv.first.boys_t == boys_t)))
            return &kv.second;
    return nullptr;
}

Plan* get_plan(uqc_basis* B, double tau, int prec, double bound, double boys_t, uqc_status* st) {
    if (Plan* p = find_plan(B, tau, prec, bound, boys_t)) return p;
    PlanKey key{tau, prec, prec == UQC_FP64 ? 0.0 : bound, prec == UQC_FP64 ? 0.0 : boys_t};
    Plan plan;
    struct HostTask {
        int cls, mixed, X, Y, same;
        double lo_excl, hi_incl;
        std::vector<int> lo, hi;
        std::vector<int> blist;   // bra indices, chunk by chunk, ordered by first shell inside a chunk
        std::vector<int> items;   // pairs {first blist entry, chunk}, then the sentinel {blist size, 0}
        long long nitems;
    };
    std::vector<HostTask> tasks;
    const int nb = (int)B->bins.size();
    {
        const long long npair = (long long)B->nshell * (B->nshell + 1) / 2;
        plan.canonical = npair * (npair + 1) / 2;
    }
    const bool mixed = prec == UQC_MIXED;
    for (int X = 0; X < nb; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            const Bin &bx = B->bins[X], &by = B->bins[Y];
            const int cls = class_index(bx.la, bx.lb, by.la, by.lb);
            HostTask t64{cls, 0, X, Y, X == Y, mixed ? bound : -1.0, INFINITY, {}, {}, {}, {}, 0};
            HostTask t32{cls, 1, X, Y, X == Y, -1.0, bound, {}, {}, {}, {}, 0};
            for (int i = 0; i < bx.np; ++i) {
                const double qi = bx.Q[i];
                int h = by.np;
                if (tau > 0) h = qi > 0 ? by.first_below(decade_floor(tau / qi)) : 0;
                if (X == Y) h = std::min(h, i + 1);
                int h64 = h, l32 = h;
                if (mixed) {
                    if (qi > 0) {
                        // FP64 needs Q_j > bound / qi, FP32 needs Q_j <= bound / qi
                        h64 = std::min(h, by.first_below(decade_floor(bound / qi)));
                        l32 = std::min(h, by.first_at_or_below(decade(bound / qi)));
                    } else {
                        h64 = 0;
                        l32 = 0;
                    }
                }
                t64.lo.push_back(0);
                t64.hi.push_back(h64);
                t32.lo.push_back(l32);
                t32.hi.push_back(h);
            }
            // bra pairs by first shell (then bin position): a wavefront keeps its K_ad / K_ac sums across a run
            std::vector<int> by_a(bx.np);
            std::iota(by_a.begin(), by_a.end(), 0);
            std::stable_sort(by_a.begin(), by_a.end(), [&](int x, int y) { return bx.off_a[x] < bx.off_a[y]; });
            const int S = class_team(cls) ? kTeamKets : kWave;
            const int GB0 = group_bras(cls);
            for (HostTask* t : {&t64, &t32}) {
                if (t->mixed && !mixed) continue;
                int nch = 0;
                for (int i = 0; i < bx.np; ++i)
                    if (t->hi[i] > t->lo[i]) nch = std::max(nch, (t->hi[i] + S - 1) / S);
                std::vector<long long> start(nch + 1, 0);
                for (int i = 0; i < bx.np; ++i)
                    if (t->hi[i] > t->lo[i])
                        for (int c = t->lo[i] / S; c <= (t->hi[i] - 1) / S; ++c) ++start[c + 1];
                for (int c = 0; c < nch; ++c) start[c + 1] += start[c];
                if (start[nch] > 0x7fffffffLL) {
                    *st = uqc_fail(UQC_E_NOMEM, "plan: work list exceeds 2^31 entries");
                    return nullptr;
                }
                t->blist.resize(start[nch]);
                const int GB = (int)std::max(1LL, std::min((long long)GB0, start[nch] / kItemTarget));
                std::vector<long long> fill(start.begin(), start.end() - 1);
                for (int i : by_a)
                    if (t->hi[i] > t->lo[i])
                        for (int c = t->lo[i] / S; c <= (t->hi[i] - 1) / S; ++c) t->blist[fill[c]++] = i;
                for (int c = 0; c < nch; ++c)
                    for (long long e = start[c]; e < start[c + 1]; e += GB) {
                        t->items.push_back((int)e);
                        t->items.push_back(c);
                    }
                t->nitems = (long long)t->items.size() / 2;
                t->items.push_back((int)start[nch]);
                t->items.push_back(0);
                if (t->nitems > 0) tasks.push_back(std::move(*t));
            }
        }
    // group tasks into one launch per (class, precision); task order = group order, so the counters of a group
    // are contiguous
    std::vector<std::pair<int, int>> gkeys;
    for (auto& t : tasks) {
        std::pair<int, int> k{t.cls, t.mixed};
        if (std::find(gkeys.begin(), gkeys.end(), k) == gkeys.end()) gkeys.push_back(k);
    }
    std::sort(gkeys.begin(), gkeys.end(), [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
        return a.first != b.first ? a.first > b.first : a.second < b.second;  // heavy classes first
    });
    std::vector<int> order;
    for (auto& gk : gkeys)
        for (size_t ti = 0; ti < tasks.size(); ++ti)
            if (tasks[ti].cls == gk.first && tasks[ti].mixed == gk.second) order.push_back((int)ti);
    plan.ntasks = (int)tasks.size();
    // device memory: counters, per task lo/hi/off, per group TaskDev array + task_begin
    size_t bytes = 0;
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    bytes += align(2 * tasks.size() * sizeof(unsigned long long));
    bytes += align(gkeys.size() * kQueueWords * sizeof(unsigned));
    for (auto& t : tasks) {
        const size_t n = B->bins[t.X].np;
        bytes += align(n * sizeof(int)) * 2 + align(t.blist.size() * sizeof(int)) + align(t.items.size() * sizeof(int));
    }
    for (size_t g = 0; g < gkeys.size(); ++g) bytes += align(tasks.size() * sizeof(TaskDev)) + align(tasks.size() * 8);
    std::vector<char> host(bytes, 0);
    if (hipMalloc(&plan.d_mem, std::max(bytes, (size_t)256)) != hipSuccess) {
        *st = uqc_fail(UQC_E_NOMEM, "plan: allocation failed");
        return nullptr;
    }
    plan.bytes = std::max(bytes, (size_t)256);
    char* dbase = (char*)plan.d_mem;
    size_t pos = 0;
    plan.d_count = (unsigned long long*)dbase;  // [ntasks] quartets, then [ntasks] primitive quartets
    plan.h_count.assign(2 * tasks.size(), 0);
    pos += align(2 * tasks.size() * sizeof(unsigned long long));
    plan.d_queue = (unsigned*)(dbase + pos);  // [groups][kQueueWords] item counters of each group's launches
    pos += align(gkeys.size() * kQueueWords * sizeof(unsigned));
    std::vector<TaskDev> tdev(tasks.size());
    for (size_t oi = 0; oi < order.size(); ++oi) {
        const int ti = order[oi];
        auto& t = tasks[ti];
        const size_t n = B->bins[t.X].np;
        std::memcpy(host.data() + pos, t.lo.data(), n * sizeof(int));
        const int* dlo = (const int*)(dbase + pos);
        pos += align(n * sizeof(int));
        std::memcpy(host.data() + pos, t.hi.data(), n * sizeof(int));
        const int* dhi = (const int*)(dbase + pos);
        pos += align(n * sizeof(int));
        std::memcpy(host.data() + pos, t.blist.data(), t.blist.size() * sizeof(int));
        const int* dblist = (const int*)(dbase + pos);
        pos += align(t.blist.size() * sizeof(int));
        std::memcpy(host.data() + pos, t.items.data(), t.items.size() * sizeof(int));
        const int2* ditems = (const int2*)(dbase + pos);
        pos += align(t.items.size() * sizeof(int));
        TaskDev& d = tdev[oi];
        d.bra = B->bins[t.X].dev;
        d.ket = B->bins[t.Y].dev;
        d.lo = dlo;
        d.hi = dhi;
        d.blist = dblist;
        d.items = ditems;
        d.item_begin = 0;
        d.nitems = t.nitems;
        d.tau = tau;
        d.boys_t = key.boys_t;
        d.lo_excl = t.lo_excl;
        d.hi_incl = t.hi_incl;
        d.count = plan.d_count + oi;
        d.pcount = plan.d_count + tasks.size() + oi;
        d.nbra = (int)n;
        d.same = t.same;
        d.D = B->d_Dp;
        d.J = B->d_J;
        d.K = B->d_K;
        d.DJ = B->d_Dp3;
        d.D2 = B->d_Dp2;
        d.K2 = B->d_K2;
        d.nbf = B->nbf;
        d.cidx = (int)oi;
    }
    size_t oi = 0;
    for (auto& gk : gkeys) {
        LaunchGroup G;
        G.cls = gk.first;
        G.mixed = gk.second;
        G.task0 = (int)oi;
        std::vector<TaskDev> gt;
        std::vector<long long> begin;
        long long items = 0;
        while (oi < order.size() && tasks[order[oi]].cls == gk.first && tasks[order[oi]].mixed == gk.second) {
            TaskDev d = tdev[oi];
            d.item_begin = items;
            begin.push_back(items);
            items += d.nitems;
            gt.push_back(d);
            ++oi;
        }
        G.ntask = (int)gt.size();
        G.nitems = items;
        std::memcpy(host.data() + pos, gt.data(), gt.size() * sizeof(TaskDev));
        G.d_tasks = (const TaskDev*)(dbase + pos);
        pos += align(tasks.size() * sizeof(TaskDev));
        std::memcpy(host.data() + pos, begin.data(), begin.size() * sizeof(long long));
        G.d_begin = (const long long*)(dbase + pos);
        pos += align(tasks.size() * 8);
        G.host_tasks = gt;
        G.host_begin = begin;
        plan.groups.push_back(G);
    }
    if (bytes && hipMemcpy(plan.d_mem, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(plan);
        *st = uqc_fail(UQC_E_DEVICE, "plan: upload failed");
        return nullptr;
    }
    B->plans.push_back({key, plan});
    return &B->plans.back().second;
}

// ---------------------------------------------------------------------------------------------- ERI blocks
bool uqc::is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

uqc_status uqc_eri_blocks(uqc_basis* B, int n, const int* q, int precision, double* out) {
    if (!B || (n > 0 && (!q || !out))) return uqc_fail(UQC_E_ARG, "uqc_eri_blocks: NULL argument");
    if (n < 0) return uqc_fail(UQC_E_ARG, "uqc_eri_blocks: negative count");
    if (precision != UQC_FP64 && precision != UQC_MIXED && precision != UQC_RYS)
        return uqc_fail(UQC_E_ARG, "uqc_eri_blocks: bad precision");
    if (n == 0) return UQC_OK;
    const int ns = B->nshell;
    struct Item {
        int cls, bra_bin, ket_bin, bra, ket;
        int slot[4];   // kernel slot (0..3 = first/second of bra, first/second of ket) of requested shell 0..3
        size_t out_off;
        int dims[4];   // component counts of the kernel slots
    };
    std::vector<Item> items(n);
    size_t total_out = 0;
    for (int x = 0; x < n; ++x) {
        int s[4];
        for (int y = 0; y < 4; ++y) {
            s[y] = q[4 * x + y];
            if (s[y] < 0 || s[y] >= ns) return uqc_fail(UQC_E_ARG, "uqc_eri_blocks: shell index out of range");
        }
        const size_t k1 = (size_t)s[0] * ns + s[1], k2 = (size_t)s[2] * ns + s[3];
        int b1 = B->pair_bin[k1], b2 = B->pair_bin[k2];
        const bool swap_bk = b1 < b2;  // the pair with the higher bin is the bra
        Item& it = items[x];
        const size_t kb = swap_bk ? k2 : k1, kk = swap_bk ? k1 : k2;
        it.bra_bin = B->pair_bin[kb];
        it.ket_bin = B->pair_bin[kk];
        it.bra = B->pair_pos[kb];
        it.ket = B->pair_pos[kk];
        const Bin &bb = B->bins[it.bra_bin], &kb_ = B->bins[it.ket_bin];
        it.cls = class_index(bb.la, bb.lb, kb_.la, kb_.lb);
        // requested slots 0,1 form pair k1; slots 2,3 pair k2
        const int base1 = swap_bk ? 2 : 0, base2 = swap_bk ? 0 : 2;
        const int first1 = B->pair_first[k1], first2 = B->pair_first[k2];
        it.slot[0] = base1 + (s[0] == first1 ? 0 : 1);
        it.slot[1] = base1 + (s[0] == first1 ? 1 : 0);
        if (s[0] == s[1]) { it.slot[0] = base1; it.slot[1] = base1 + 1; }
        it.slot[2] = base2 + (s[2] == first2 ? 0 : 1);
        it.slot[3] = base2 + (s[2] == first2 ? 1 : 0);
        if (s[2] == s[3]) { it.slot[2] = base2; it.slot[3] = base2 + 1; }
        it.dims[0] = ncart(bb.la);
        it.dims[1] = ncart(bb.lb);
        it.dims[2] = ncart(kb_.la);
        it.dims[3] = ncart(kb_.lb);
        it.out_off = total_out;
        total_out += (size_t)it.dims[0] * it.dims[1] * it.dims[2] * it.dims[3];
    }
    uqc_ctx* ctx = B->ctx;
    UQC_HIP(hipSetDevice(ctx->device));
    // one launch per (class, bra bin, ket bin)
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) {
        const Item &x = items[a], &y = items[b];
        if (x.bra_bin != y.bra_bin) return x.bra_bin < y.bra_bin;
        return x.ket_bin < y.ket_bin;
    });
    void* dmem = nullptr;
    const size_t bytes = total_out * sizeof(double) + 2 * (size_t)n * sizeof(int) + 256;
    if (hipMalloc(&dmem, bytes) != hipSuccess) return uqc_fail(UQC_E_NOMEM, "uqc_eri_blocks: allocation failed");
    double* dout = (double*)dmem;
    int* didx = (int*)(dout + total_out);
    // kernel output is grouped by launch; keep the device offset of each item
    std::vector<int> hidx(2 * (size_t)n);
    std::vector<size_t> dev_off(n);
    size_t dpos = 0;
    struct Launch { int cls, bra_bin, ket_bin, first, count; size_t out; };
    std::vector<Launch> launches;
    for (int r = 0; r < n;) {
        const Item& it0 = items[ord[r]];
        int e = r;
        Launch L{it0.cls, it0.bra_bin, it0.ket_bin, r, 0, dpos};
        while (e < n && items[ord[e]].bra_bin == it0.bra_bin && items[ord[e]].ket_bin == it0.ket_bin) {
            const Item& it = items[ord[e]];
            hidx[e] = it.bra;
            hidx[n + e] = it.ket;
            dev_off[ord[e]] = dpos;
            dpos += (size_t)it.dims[0] * it.dims[1] * it.dims[2] * it.dims[3];
            ++e;
        }
        L.count = e - r;
        launches.push_back(L);
        r = e;
    }
    uqc_status st = UQC_OK;
    if (hipMemcpyAsync(didx, hidx.data(), 2 * (size_t)n * sizeof(int), hipMemcpyHostToDevice, ctx->stream) !=
        hipSuccess)
        st = uqc_fail(UQC_E_DEVICE, "uqc_eri_blocks: upload failed");
    for (auto& L : launches) {
        if (st != UQC_OK) break;
        ListDev ld{};
        ld.bra = B->bins[L.bra_bin].dev;
        ld.ket = B->bins[L.ket_bin].dev;
        ld.bra_idx = didx + L.first;
        ld.ket_idx = didx + n + L.first;
        ld.n = L.count;
        ld.out = dout + L.out;
        const hipError_t e = precision == UQC_RYS
                                 ? launch_list_rys(L.cls, ld, ctx->rys, ctx->stream)
                                 : launch_list(L.cls, precision == UQC_MIXED, MODE_STORE, ld, ctx->boys64,
                                               ctx->boys32, ctx->stream);
        if (e != hipSuccess)
            st = uqc_fail(UQC_E_DEVICE, "uqc_eri_blocks: kernel launch failed");
    }
    std::vector<double> hout(total_out);
    if (st == UQC_OK && (hipMemcpyAsync(hout.data(), dout, total_out * sizeof(double), hipMemcpyDeviceToHost,
                                        ctx->stream) != hipSuccess ||
                         hipStreamSynchronize(ctx->stream) != hipSuccess))
        st = uqc_fail(UQC_E_DEVICE, "uqc_eri_blocks: kernel or copy failed");
    (void)hipFree(dmem);
    if (st != UQC_OK) return st;
    // permute every block into the requested (a, b, c, d) order
    for (int x = 0; x < n; ++x) {
        const Item& it = items[x];
        const double* src = hout.data() + dev_off[x];
        double* dst = out + it.out_off;
        int rd[4];
        for (int y = 0; y < 4; ++y) rd[y] = it.dims[it.slot[y]];
        int idx[4];
        for (int i = 0; i < rd[0]; ++i)
            for (int j = 0; j < rd[1]; ++j)
                for (int k = 0; k < rd[2]; ++k)
                    for (int l = 0; l < rd[3]; ++l) {
                        idx[it.slot[0]] = i;
                        idx[it.slot[1]] = j;
                        idx[it.slot[2]] = k;
                        idx[it.slot[3]] = l;
                        const size_t s = ((size_t)(idx[0] * it.dims[1] + idx[1]) * it.dims[2] + idx[2]) * it.dims[3] +
                                         idx[3];
                        *dst++ = src[s];
                    }
    }
    return UQC_OK;
}

uqc_status uqc_eri_block(uqc_basis* B, int a, int b, int c, int d, int precision, double* out) {
    const int q[4] = {a, b, c, d};
    return uqc_eri_blocks(B, 1, q, precision, out);
}

// ---------------------------------------------------------------------------------------------- Fock build
// Fock build for one density (nspin = 1: out = {J, K, G}) or a pair of spin densities (nspin = 2:
// out = {J, Ka, Kb, Ga, Gb}).  With spin densities the class kernels evaluate every integral once and contract it
// with the total density for J and with each spin density for its own K.
uqc_status uqc::fock_run(uqc_basis* B, int nspin, const double* const* Din, double* const* out,
                         const uqc_fock_opts* opts, uqc_stats* stats, const char* name, const FockWorkspace* ws) {
    const auto t0 = std::chrono::steady_clock::now();
    const std::string nm(name);
    uqc_fock_opts o;
    uqc_fock_opts_default(&o);
    if (opts) o = *opts;
    if (const uqc_status e = uqc::check_fock_opts(o, nm)) return e;
    if (ws && (nspin != 1 || o.timing)) return uqc_fail(UQC_E_ARG, nm + ": closed shell only, no timing");
    const long long max_items = o.max_items_per_launch > 0 ? o.max_items_per_launch : kMaxItemsPerLaunch;
    const int nout = nspin == 1 ? 3 : 5;
    uqc_ctx* ctx = B->ctx;
    UQC_HIP(hipSetDevice(ctx->device));
    const bool dev = uqc::is_device_ptr(Din[0]);
    if (ws && !dev) return uqc_fail(UQC_E_ARG, nm + ": D, J, K, G must be device pointers");
    if (nspin == 2 && uqc::is_device_ptr(Din[1]) != dev)
        return uqc_fail(UQC_E_ARG, nm + ": mix of host and device pointers");
    for (int i = 0; i < nout; ++i)
        if (out[i] && uqc::is_device_ptr(out[i]) != dev)
            return uqc_fail(UQC_E_ARG, nm + ": mix of host and device pointers");
    uqc_status st = UQC_OK;
    Plan* plan = ws ? find_plan(B, o.schwarz_tau, o.precision, o.fp64_bound, o.fp64_boys_T)
                    : get_plan(B, o.schwarz_tau, o.precision, o.fp64_bound, o.fp64_boys_T, &st);
    if (!plan && ws)
        return uqc_fail(UQC_E_ARG, nm + ": no screening plan for these options on this basis (an earlier "
                                        "uqc_fock_build with the same tau, precision, fp64_bound and fp64_boys_T "
                                        "makes it)");
    if (!plan) return st;
    if (ws && plan->ntasks > ws->max_tasks)
        return uqc_fail(UQC_E_ARG, nm + ": the plan has more tasks than the fixed workspace holds");
    const size_t N = B->nbf, NN = N * N;
    hipStream_t s = ctx->stream;
    // D' and the accumulators, scalars and counters: the basis's own workspace, or the caller-chosen one
    double* const Dp = ws ? ws->Dp : B->d_Dp;
    double* const Jacc = ws ? ws->J : B->d_J;
    double* const Kacc = ws ? ws->K : B->d_K;
    double* const scal = ws ? ws->scal : B->d_scal;
    unsigned long long* const counts = ws ? ws->count : plan->d_count;
    WorkRedirect wr{};
    if (ws) wr = WorkRedirect{Dp, Jacc, Kacc, counts, plan->ntasks};
    const double* Dd[2] = {Din[0], nspin == 2 ? Din[1] : nullptr};
    double* Od[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    for (int i = 0; i < nout; ++i) Od[i] = out[i];
    if (!dev) {
        // staging: the densities, then one slot per output
        double* io = B->d_io;
        if (nspin == 2) {
            if (!B->d_uio && hipMalloc(&B->d_uio, 7 * NN * sizeof(double)) != hipSuccess) {
                B->d_uio = nullptr;
                return uqc_fail(UQC_E_NOMEM, nm + ": staging allocation failed");
            }
            io = B->d_uio;
        }
        for (int k = 0; k < nspin; ++k) {
            UQC_HIP(hipMemcpyAsync(io + k * NN, Din[k], NN * sizeof(double), hipMemcpyHostToDevice, s));
            Dd[k] = io + k * NN;
        }
        for (int i = 0; i < nout; ++i) Od[i] = out[i] ? io + (nspin + i) * NN : nullptr;
    }
    unsigned long long* maxbits = (unsigned long long*)(scal + 1);
    UQC_HIP(launch_zero(scal, 8, s));
    UQC_HIP(launch_prepare(Dd[0], B->d_f, Dp, (int)N, maxbits, s));
    if (nspin == 2) UQC_HIP(launch_prepare(Dd[1], B->d_f, B->d_Dp2, (int)N, maxbits + 2, s));
    unsigned long long hb[4] = {0, 0, 0, 0};
    UQC_HIP(hipMemcpyAsync(hb, maxbits, sizeof(hb), hipMemcpyDeviceToHost, s));
    UQC_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < nspin; ++k) {
        double md, ma;
        std::memcpy(&md, &hb[2 * k], 8);
        std::memcpy(&ma, &hb[2 * k + 1], 8);
        if (!(md <= 1e-12 * ma))
            return uqc_fail(UQC_E_NOT_SYMMETRIC, nm + ": density is not symmetric (or not finite)");
    }
    if (Kacc == Jacc + NN) {
        UQC_HIP(launch_zero(Jacc, 2 * NN, s));
    } else {
        UQC_HIP(launch_zero(Jacc, NN, s));
        UQC_HIP(launch_zero(Kacc, NN, s));
    }
    if (nspin == 2) {
        UQC_HIP(launch_zero(B->d_K2, NN, s));
        UQC_HIP(launch_add(B->d_Dp, B->d_Dp2, B->d_Dp3, NN, s));
    }
    const bool timing = o.timing != 0;
    std::vector<double> cls_ms(plan->groups.size(), 0.0);
    // Classes spread over several streams: largest first (FLOPs of the previous build, else work items), each to
    // the stream with the least work so far; then queued largest, smallest, second largest, second smallest, ...,
    // so that every stream alternates long and short kernels and their drains overlap.  The extra streams wait for
    // everything queued on the context's stream so far and are joined back into it after their last launch.
    const int nst = ws ? 1 : std::max(1, o.streams);
    const size_t ng = plan->groups.size();
    std::vector<size_t> order(ng);
    std::vector<int> gstream(ng, 0);
    for (size_t gi = 0; gi < ng; ++gi) order[gi] = gi;
    if (nst > 1) {
        auto weight = [&](size_t gi) {
            const LaunchGroup& g = plan->groups[gi];
            return g.flops > 0 ? g.flops : (double)g.nitems;
        };
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return weight(x) > weight(y); });
        std::vector<double> load(nst, 0.0);
        for (size_t gi : order) {
            const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            gstream[gi] = k;
            load[k] += weight(gi);
        }
        order = interleave_ends(order);
    }
    hipStream_t S[4] = {s, nullptr, nullptr, nullptr};
    for (int k = 1; k < nst; ++k)
        if (!(S[k] = ctx_stream(ctx, k))) return uqc_fail(UQC_E_DEVICE, nm + ": stream creation failed");
    // progress on several streams: an event after every sub-launch, waited for in issue order once all are queued
    struct SubLaunch {
        size_t ev;
        int cid;
        long long done, total;
    };
    std::vector<SubLaunch> subs;
    auto pass = [&]() -> uqc_status {
        if (plan->ntasks) UQC_HIP(launch_zero((double*)counts, 2 * (size_t)plan->ntasks, s));
        if (nst > 1) {
            UQC_HIP(hipEventRecord(ctx->fork, s));
            for (int k = 1; k < nst; ++k) UQC_HIP(hipStreamWaitEvent(S[k], ctx->fork, 0));
        }
        for (size_t gi : order) {
            const LaunchGroup& g = plan->groups[gi];
            hipStream_t gs = S[gstream[gi]];
            if (timing) UQC_HIP(hipEventRecord(ctx_event(ctx, 2 * gi), gs));
            int la, lb, lc, ld;
            class_ls(g.cls, &la, &lb, &lc, &ld);
            const int cid = la * 1000 + lb * 100 + lc * 10 + ld + (g.mixed ? 10000 : 0);
            for (long long i0 = 0; i0 < g.nitems; i0 += max_items) {
                const long long n = std::min(max_items, g.nitems - i0);
                // a group's launches share its queue (they run in order on one stream)
                unsigned* q = ws ? ws->queue : plan->d_queue + gi * kQueueWords;
                UQC_HIP(launch_digest(g.cls, g.mixed, nspin, g.d_tasks, g.d_begin, g.ntask, i0, n, ctx->boys64,
                                      ctx->boys32, wr, q, gs));
                if (o.progress && nst == 1) {
                    UQC_HIP(hipStreamSynchronize(gs));
                    o.progress(o.progress_user, cid, i0 + n, g.nitems);
                } else if (o.progress) {
                    const size_t ev = 2 * ng + subs.size();
                    hipEvent_t e = ctx_event(ctx, ev);
                    if (!e) return uqc_fail(UQC_E_DEVICE, nm + ": event creation failed");
                    UQC_HIP(hipEventRecord(e, gs));
                    subs.push_back(SubLaunch{ev, cid, i0 + n, g.nitems});
                }
            }
            if (timing) UQC_HIP(hipEventRecord(ctx_event(ctx, 2 * gi + 1), gs));
        }
        for (int k = 1; k < nst; ++k) {
            UQC_HIP(hipEventRecord(ctx->join[k - 1], S[k]));
            UQC_HIP(hipStreamWaitEvent(s, ctx->join[k - 1], 0));
        }
        for (const SubLaunch& sb : subs) {
            UQC_HIP(hipEventSynchronize(ctx->events[sb.ev]));
            o.progress(o.progress_user, sb.cid, sb.done, sb.total);
        }
        if (timing) {
            UQC_HIP(hipStreamSynchronize(s));
            for (size_t gi = 0; gi < plan->groups.size(); ++gi) {
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, ctx->events[2 * gi], ctx->events[2 * gi + 1]);
                cls_ms[gi] += ms;
            }
        }
        return UQC_OK;
    };
    if ((st = pass()) != UQC_OK) return st;
    if (nspin == 2) {
        UQC_HIP(launch_finalize_uhf(Dd[0], Dd[1], B->d_J, B->d_K, B->d_K2, B->d_f, o.exchange_scale, Od[0], Od[1],
                                    Od[2], Od[3], Od[4], B->d_scal, (int)N, s));
    } else {
        UQC_HIP(launch_finalize(Dd[0], Jacc, Kacc, B->d_f, Od[0], Od[1], Od[2], o.exchange_scale, scal, (int)N, s));
    }
    double E2 = 0.0;
    UQC_HIP(hipMemcpyAsync(&E2, scal, sizeof(double), hipMemcpyDeviceToHost, s));
    if (plan->ntasks)
        UQC_HIP(hipMemcpyAsync(plan->h_count.data(), counts, 2 * plan->ntasks * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s));
    if (!dev)
        for (int i = 0; i < nout; ++i)
            if (out[i]) UQC_HIP(hipMemcpyAsync(out[i], Od[i], NN * sizeof(double), hipMemcpyDeviceToHost, s));
    UQC_HIP(hipStreamSynchronize(s));
    plan_account(*plan);
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->E2 = E2;
        stats->quartets = plan->quartets;
        stats->quartets_screened = plan->screened;
        stats->prim_quartets = plan->prim_quartets;
        stats->fp64_quartets = plan->fp64_quartets;
        stats->flops = plan->flops;
        if (timing) {
            int nc = 0;
            for (size_t gi = 0; gi < plan->groups.size(); ++gi) {
                const auto& g = plan->groups[gi];
                stats->eri_ms += cls_ms[gi];
                if (nc < UQC_MAX_CLASS_STATS) {
                    int la, lb, lc, ld;
                    class_ls(g.cls, &la, &lb, &lc, &ld);
                    stats->class_id[nc] = la * 1000 + lb * 100 + lc * 10 + ld + (g.mixed ? 10000 : 0);
                    stats->class_ms[nc] = cls_ms[gi];
                    stats->class_flops[nc] = g.flops;
                    stats->class_quartets[nc] = g.quartets;
                    ++nc;
                }
            }
            stats->nclass = nc;
        }
        stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return UQC_OK;
}

uqc_status uqc_fock_build(uqc_basis* B, const double* D, double* J, double* K, double* G, const uqc_fock_opts* opts,
                          uqc_stats* stats) {
    if (!B || !D) return uqc_fail(UQC_E_ARG, "uqc_fock_build: NULL basis or density");
    const double* Din[1] = {D};
    double* out[3] = {J, K, G};
    return uqc::fock_run(B, 1, Din, out, opts, stats, "uqc_fock_build", nullptr);
}

uqc_status uqc_fock_build_uhf(uqc_basis* B, const double* Da, const double* Db, double* J, double* Ka, double* Kb,
                              double* Ga, double* Gb, const uqc_fock_opts* opts, uqc_stats* stats) {
    if (!B || !Da || !Db) return uqc_fail(UQC_E_ARG, "uqc_fock_build_uhf: NULL basis or density");
    const double* Din[2] = {Da, Db};
    double* out[5] = {J, Ka, Kb, Ga, Gb};
    return uqc::fock_run(B, 2, Din, out, opts, stats, "uqc_fock_build_uhf", nullptr);
}

// ---------------------------------------------------------------------------------------------- Boys check
uqc_status uqc_boys(uqc_ctx* ctx, int precision, int mmax, int n, const double* T, double* out) {
    if (!ctx || (n > 0 && (!T || !out))) return uqc_fail(UQC_E_ARG, "uqc_boys: NULL argument");
    if (mmax < 0 || mmax > 8 || n < 0) return uqc_fail(UQC_E_ARG, "uqc_boys: mmax must be 0..8, n >= 0");
    if (precision != UQC_FP64 && precision != UQC_MIXED) return uqc_fail(UQC_E_ARG, "uqc_boys: bad precision");
    for (int i = 0; i < n; ++i)
        if (!(T[i] >= 0) || !std::isfinite(T[i])) return uqc_fail(UQC_E_ARG, "uqc_boys: T must be finite and >= 0");
    if (n == 0) return UQC_OK;
    UQC_HIP(hipSetDevice(ctx->device));
    double* d = nullptr;
    const size_t m = (size_t)mmax + 1;
    if (hipMalloc(&d, (size_t)n * (1 + m) * sizeof(double)) != hipSuccess)
        return uqc_fail(UQC_E_NOMEM, "uqc_boys: allocation failed");
    uqc_status st = UQC_OK;
    if (hipMemcpyAsync(d, T, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        launch_boys(precision, mmax, n, d, d + n, ctx->boys64, ctx->boys32, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(out, d + n, (size_t)n * m * sizeof(double), hipMemcpyDeviceToHost, ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        st = uqc_fail(UQC_E_DEVICE, "uqc_boys: kernel or copy failed");
    (void)hipFree(d);
    return st;
}
