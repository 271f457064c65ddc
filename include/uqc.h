/* uqc: two-electron repulsion integrals and Coulomb/exchange (Fock) builds on the AMD MI355X (gfx950).
 *
 * What is computed (arXiv:1303.4916, Sec. "Implementation details" and Sec. "Technical details"):
 *   - basis functions are contracted Cartesian Gaussians, Eq. (1): phi_i = sum_n d_in x^L y^M z^N exp(-alpha_n r^2),
 *     one exponent per primitive shared by all Cartesian components of a shell;
 *   - electron-repulsion integrals (ij|kl), Eq. (5), in chemists' notation;
 *   - J_ij = sum_kl (ij|kl) D_kl and K_il = sum_jk (ij|kl) D_jk, Eq. (12), for a symmetric density D;
 *   - G = J - K/2 and E2 = 1/2 sum_ij D_ij G_ij (closed-shell convention; D is the total density).
 *
 * Conventions:
 *   - units: bohr (positions) and hartree (integrals);
 *   - l = 0, 1, 2 only (s, p, Cartesian d); contraction depth 1..16;
 *   - coefficients refer to normalised primitives; the library normalises primitives and then every Cartesian
 *     component of every contracted function to unit self-overlap;
 *   - basis functions are numbered shell by shell in input order; inside a shell the Cartesian components are
 *     ordered by descending x power, then descending y power: p = x, y, z; d = xx, xy, xz, yy, yz, zz;
 *   - matrices are nbf x nbf, row-major, FP64;
 *   - Schwarz screening: a shell quartet (ab|cd) is computed iff Q_ab * Q_cd >= tau with
 *     Q_ab = sqrt(max_{i in a, j in b} (ij|ij)); tau = 0 computes every quartet.
 *
 * Errors: every call returns a uqc_status; nothing aborts.  The message of the last failing call on the calling
 * thread is available from uqc_last_error().
 *
 * Threading: one uqc_ctx per device; a context and the objects made from it must not be used by two host threads
 * at once, except uqc_submit / uqc_poll on a server, which are thread-safe.
 */
#ifndef UQC_H
#define UQC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct uqc_ctx uqc_ctx;
typedef struct uqc_basis uqc_basis;
typedef struct uqc_server uqc_server;

typedef enum {
    UQC_OK = 0,
    UQC_PENDING = 1,            /* uqc_poll: request not finished yet */
    UQC_E_ARG = -1,             /* invalid argument (null pointer, index out of range, non-finite value, ...) */
    UQC_E_UNSUPPORTED = -2,     /* l > 2, contraction depth > 16, or more than 65535 basis functions */
    UQC_E_NOMEM = -3,           /* device allocation failed, or a request exceeds the whole HBM budget */
    UQC_E_DEVICE = -4,          /* a HIP runtime call failed */
    UQC_E_NOT_SYMMETRIC = -5,   /* max|D - D^T| > 1e-12 max|D| */
    UQC_E_NOT_FOUND = -6,       /* unknown ticket */
    UQC_E_BUSY = -7             /* server is shutting down */
} uqc_status;

/* UQC_RYS: uqc_eri_block(s) only, FP64 integrals by Rys quadrature (the paper's method) instead of the
 * Obara-Saika / Head-Gordon-Pople recursions; the same integrals, for per-class comparison. */
typedef enum { UQC_FP64 = 0, UQC_MIXED = 1, UQC_RYS = 2 } uqc_precision;

/* Progress report of a Fock build: called on the calling thread after every class sub-launch has completed on the
 * device (items_done of items_total work items of class class_id, encoded as in uqc_stats.class_id; for each class
 * in increasing order).  On one stream the build waits for each sub-launch before queuing the next; on several,
 * every sub-launch is queued first and the reports follow their completion, in the order they were queued.  The
 * work itself is unchanged. */
typedef void (*uqc_progress_fn)(void* user, int class_id, long long items_done, long long items_total);

/* Options of a Fock build.  Call uqc_fock_opts_default() first. */
typedef struct {
    double schwarz_tau;   /* screening threshold tau (>= 0) */
    int precision;        /* uqc_precision.  UQC_MIXED: primitive recursions in FP32 with FP64 accumulation, except
                             quartets with Q_ab Q_cd > fp64_bound (whole quartet in FP64) and Boys arguments
                             T > fp64_boys_T (Boys function evaluated in FP64); J, K, G, E2 always accumulated in
                             FP64 */
    double fp64_bound;    /* default 1e-8 */
    int timing;           /* 1: time every class launch with HIP events on its stream (reported in uqc_stats; with
                             several streams a class's time includes the kernels that run beside it) */
    uqc_progress_fn progress;   /* NULL (default) or a progress report, see uqc_progress_fn */
    void* progress_user;        /* passed to progress */
    long long max_items_per_launch;  /* > 0: cap on the work items of one class-kernel launch (longer classes are
                                        split into several launches, which bounds the duration of each kernel);
                                        0 (default): 2^20 */
    double exchange_scale;  /* x, the weight of exchange: G = J - (x/2) K (closed shell), G^s = J - x K^s (spin
                               densities).  1 (default) is Hartree-Fock; the exact-exchange fraction a0 of a hybrid
                               functional (Sec. "Implementation details", B3LYP) gives its scaled exchange, the
                               exchange-correlation functional itself not being part of this library.  Finite. */
    int streams;            /* number of HIP streams the class launches of one build are spread over, 1..4 (0 is
                               read as 1).  Stream 0 is the context's; the others are the context's own (default
                               priority), ordered after the work already queued on the context's stream and joined
                               back into it before the build's final pass, so callers see one stream either way.
                               Kernels of different classes then run side by side, which fills the chip while
                               one class's launch drains.  Default 3; outside 0..4: UQC_E_ARG. */
    double fp64_boys_T;     /* UQC_MIXED: primitive quartets of FP32 quartets whose Boys argument T exceeds this take
                               the FP64 Boys evaluation (the recursion stays FP32).  0..30, the range of the FP32 Boys
                               table (outside, or not finite: UQC_E_ARG); default 30. */
} uqc_fock_opts;

#define UQC_MAX_CLASS_STATS 96

/* Per-build statistics.  Counts are of canonical shell quartets (a>=b, c>=d, ab>=cd). */
typedef struct {
    double E2;                      /* 1/2 sum D G (spin densities: 1/2 sum (D^a G^a + D^b G^b)) */
    long long quartets;             /* shell quartets computed (after screening) */
    long long quartets_screened;    /* canonical shell quartets skipped by screening */
    long long prim_quartets;        /* primitive quartets computed */
    long long fp64_quartets;        /* shell quartets computed with FP64 recursions */
    double flops;                   /* algorithmic FLOPs of the build (frozen per-class operation counts) */
    double ms;                      /* host wall time of the call */
    double eri_ms;                  /* sum of ERI class-kernel times (timing = 1 only) */
    int nclass;                     /* number of class launches reported below (timing = 1 only) */
    int class_id[UQC_MAX_CLASS_STATS];      /* la*1000 + lb*100 + lc*10 + ld; +10000 if FP32 recursions */
    double class_ms[UQC_MAX_CLASS_STATS];
    double class_flops[UQC_MAX_CLASS_STATS];
    long long class_quartets[UQC_MAX_CLASS_STATS];
} uqc_stats;

/* Fills *o with: tau = 1e-12, precision = UQC_FP64, fp64_bound = 1e-8, timing = 0, progress = NULL,
 * max_items_per_launch = 0, exchange_scale = 1, streams = 3, fp64_boys_T = 30. */
void uqc_fock_opts_default(uqc_fock_opts* o);

/* Creates a context on HIP device `device`.  `hip_stream` is a hipStream_t the library launches on (NULL: the
 * library creates its own stream and destroys it in uqc_finalize).  The caller keeps ownership of its stream. */
uqc_status uqc_init(int device, void* hip_stream, uqc_ctx** out);
/* Destroys the context.  Every basis and server made from it must have been destroyed first. */
uqc_status uqc_finalize(uqc_ctx* ctx);

/* Message of the last non-OK status returned on this thread ("" if none).  Valid until the next uqc call. */
const char* uqc_last_error(void);

/* Builds a basis (Eq. 1) and its screening plan: normalisation, primitive-pair data, Schwarz bounds (on the GPU),
 * pairs sorted by bound inside (l_a, l_b, K_a, K_b) bins.  Arrays are copied; the caller keeps ownership.
 *   l[nshell]            angular momentum 0..2
 *   nprim[nshell]        contraction depth 1..16
 *   center[nshell*3]     shell centres (bohr)
 *   alpha[sum nprim]     primitive exponents (> 0), shell by shell
 *   coef[sum nprim]      contraction coefficients for normalised primitives
 * Errors: UQC_E_ARG, UQC_E_UNSUPPORTED, UQC_E_NOMEM, UQC_E_DEVICE. */
uqc_status uqc_basis_create(uqc_ctx* ctx, int nshell, const int* l, const int* nprim, const double* center,
                            const double* alpha, const double* coef, uqc_basis** out);
uqc_status uqc_basis_destroy(uqc_basis* b);

/* Number of basis functions and (optionally, may be NULL) the first basis-function index of every shell. */
uqc_status uqc_basis_info(const uqc_basis* b, int* nbf, int* shell_offset);

/* Schwarz bounds Q_ab (host array nshell*nshell, symmetric), as computed on the GPU at basis creation. */
uqc_status uqc_schwarz(const uqc_basis* b, double* Q);

/* One contracted block (ab|cd), Eq. (5): n_a*n_b*n_c*n_d doubles written to host memory `out`, row-major [i][j][k][l]
 * over the Cartesian components of shells a, b, c, d (any order of the four shell indices).  precision selects the
 * recursions' arithmetic (UQC_MIXED: FP32 recursions, FP64 contraction) or, with UQC_RYS, Rys quadrature in FP64.
 * Never screened (every primitive is evaluated). */
uqc_status uqc_eri_block(uqc_basis* b, int a, int bb, int c, int d, int precision, double* out);

/* n blocks at once: quartets[4*q .. 4*q+3] = (a, b, c, d); blocks are written one after another to `out` (host),
 * each laid out as in uqc_eri_block. */
uqc_status uqc_eri_blocks(uqc_basis* b, int n, const int* quartets, int precision, double* out);

/* Fock build, Eq. (12): J(D), K(D), G = J - K/2 and E2 for a symmetric density D (nbf*nbf, row-major).
 * D, J, K, G are either all device pointers (e.g. torch tensors on the context's device; the work is ordered on the
 * context's stream and the call returns after it completes) or all host pointers (copied in and out).  Any of J,
 * K, G may be NULL.  `stats` may be NULL.
 * Errors: UQC_E_ARG, UQC_E_NOT_SYMMETRIC, UQC_E_NOMEM, UQC_E_DEVICE. */
uqc_status uqc_fock_build(uqc_basis* b, const double* D, double* J, double* K, double* G, const uqc_fock_opts* opts,
                          uqc_stats* stats);

/* uqc_fock_build without any device allocation, for callers that cannot allocate device memory (code being captured
 * into a HIP graph, tight serving loops, harnesses that forbid allocation).  Same arguments, results and errors as
 * uqc_fock_build for a closed-shell build, with these limits:
 *   - D, J, K, G are device pointers on the context's device (host pointers: UQC_E_ARG);
 *   - the scaled density, the J and K accumulators, the scalars, the per-task counters and the item counters of the
 *     class launches live in a fixed device array of the library (25.7 MB per device, held until the process ends)
 *     instead of the basis's workspace and plan, so
 *     the basis has at most 1024 basis functions (else UQC_E_ARG);
 *   - the screening plan for (opts->schwarz_tau, opts->precision, opts->fp64_bound, opts->fp64_boys_T) must
 *     already exist on this basis: an earlier uqc_fock_build with the same four options makes it (else UQC_E_ARG);
 *   - every class launch is queued on the context's stream (opts->streams is not used); opts->timing must be 0.
 * Every call on one device shares that device's array, so calls that overlap on one device (from two host threads,
 * or on two contexts' streams) race and give wrong results; calls in sequence on one stream are safe (each starts by
 * clearing what it accumulates into). */
uqc_status uqc_fock_build_noalloc(uqc_basis* b, const double* D, double* J, double* K, double* G,
                                  const uqc_fock_opts* opts, uqc_stats* stats);

/* Unrestricted Fock build (the paper's URHF, for open shells: the Pople-Nesbet equations of Szabo-Ostlund Sec. 3.8,
 * Eq. (12) applied per spin): for the spin densities Da, Db (nbf*nbf, row-major, symmetric; Da + Db is the total
 * density), J = J(Da + Db), Ka = K(Da), Kb = K(Db), Ga = J - x Ka, Gb = J - x Kb (x = opts->exchange_scale) and
 * stats->E2 = 1/2 sum (Da Ga + Db Gb).  Da and Db and the outputs
 * are all device pointers or all host pointers, as for uqc_fock_build; any of J, Ka, Kb, Ga, Gb may be NULL.  With
 * Da = Db = D/2 the result is that of uqc_fock_build for D (Ga = Gb = G).
 * Errors: UQC_E_ARG, UQC_E_NOT_SYMMETRIC, UQC_E_NOMEM, UQC_E_DEVICE. */
uqc_status uqc_fock_build_uhf(uqc_basis* b, const double* Da, const double* Db, double* J, double* Ka, double* Kb,
                              double* Ga, double* Gb, const uqc_fock_opts* opts, uqc_stats* stats);

/* One-electron integrals over the basis (paper, Eq. (2)-(4)): overlap S, kinetic T and attraction V to point nuclei
 * of charges Z[natom] at R[natom][3] (bohr; host arrays, natom >= 0), each nbf*nbf row-major.  S, T, V are all
 * device pointers or all host pointers; any may be NULL.  Same basis conventions as the ERIs.
 * Errors: UQC_E_ARG, UQC_E_NOMEM, UQC_E_DEVICE. */
uqc_status uqc_one_electron(uqc_basis* b, int natom, const double* Z, const double* R, double* S, double* T,
                            double* V);

/* Restricted closed-shell Hartree-Fock around the Fock build (the paper's HF method with Pulay DIIS acceleration,
 * Sec. "Implementation details", and the closed-shell equations of Szabo-Ostlund it follows): symmetric
 * orthogonalisation X = S^{-1/2}, core-Hamiltonian guess, F = H + J(P) - K(P)/2 with P = 2 C_occ C_occ^T,
 * E = 1/2 tr P (H + F) + E_nuc.  Every matrix stays on the device; eigendecompositions use rocSOLVER. */
typedef struct {
    int max_iter;          /* default 100 */
    double e_conv;         /* |E_k - E_(k-1)| in hartree, default 1e-10 */
    double d_conv;         /* max |F P S - S P F|, default 1e-8 */
    int diis_size;         /* DIIS subspace size (0: plain Roothaan iteration), default 8, at most 16 */
    uqc_fock_opts fock;    /* options of every Fock build (its progress callback is not used) */
    double guess_mix;      /* uqc_scf_uhf: angle theta (radians) by which the alpha core guess' highest occupied
                              (h) and lowest virtual (l) orbitals are rotated, h' = cos h + sin l,
                              l' = -sin h + cos l, to break the symmetry of a closed-shell start; default 0 */
} uqc_scf_opts;

typedef struct {
    double E_total, E_elec, E_nuc;
    int iterations;        /* Fock builds performed */
    int converged;         /* 1 if both criteria were met within max_iter */
    double error;          /* final max |F P S - S P F| */
    double ms;             /* wall time of the call */
    double fock_ms;        /* of which in Fock builds */
    long long quartets;    /* shell quartets of one Fock build */
    double s2;             /* <S^2> of the final determinant (0 for uqc_scf_rhf) */
} uqc_scf_result;

/* Fills *o with the defaults above (guess_mix = 0) and uqc_fock_opts_default() for the builds. */
void uqc_scf_opts_default(uqc_scf_opts* o);

/* Runs the SCF for nuclei Z[natom] at R[natom][3] (host arrays) with nocc doubly occupied orbitals (1 <= nocc <=
 * nbf).  P (host, nbf*nbf) and eps (host, nbf: orbital energies, ascending) receive the final density and orbital
 * energies if not NULL.  Not converging within max_iter is not an error (res->converged = 0).
 * Errors: UQC_E_ARG, UQC_E_NOMEM, UQC_E_DEVICE (also when S is numerically singular). */
uqc_status uqc_scf_rhf(uqc_basis* b, int natom, const double* Z, const double* R, int nocc, const uqc_scf_opts* o,
                       double* P, double* eps, uqc_scf_result* res);

/* Unrestricted Hartree-Fock (the paper's URHF; Pople-Nesbet equations, Szabo-Ostlund Sec. 3.8) with nalpha and
 * nbeta electrons (0 <= n <= nbf, nalpha + nbeta >= 1): core-Hamiltonian guess for both spins (the alpha one
 * rotated by opts->guess_mix), P^s = C^s_occ C^s_occ^T, F^s = H + G^s from uqc_fock_build_uhf,
 * E = sum (P^a + P^b) H + E2 + E_nuc, DIIS over the pair of errors F^s P^s S - S P^s F^s with one set of
 * coefficients for both spins; res->error is the larger spin's max |F P S - S P F| and res->s2 = <S^2>.
 * Pa, Pb (host, nbf*nbf) and eps_a, eps_b (host, nbf) receive the final spin densities and orbital energies if not
 * NULL.  Same options, stopping rule and errors as uqc_scf_rhf. */
uqc_status uqc_scf_uhf(uqc_basis* b, int natom, const double* Z, const double* R, int nalpha, int nbeta,
                       const uqc_scf_opts* o, double* Pa, double* Pb, double* eps_a, double* eps_b,
                       uqc_scf_result* res);

/* Closed-shell second-order Moller-Plesset correlation energy (the paper's MP2; spin-adapted form of Szabo-Ostlund
 * Sec. 6.5) for canonical orbitals C (host, nbf*nbf row-major: C[mu*nbf + p] is the coefficient of basis function
 * mu in orbital p) with energies eps (host, nbf, virtual ones above the occupied ones), nocc doubly occupied
 * orbitals of which the first nfrozen are left out (frozen core, 0 <= nfrozen < nocc <= nbf):
 *   E2 = sum_{ijab} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b),
 * i, j active occupied, a, b virtual.  The AO integrals are computed on the GPU (shell quartets with
 * Q_ab Q_cd >= tau; tau = 0: all) in batches of ket index pairs, each batch transformed over its first index at once
 * (the nbf^4 AO tensor is never held), then transformed to (ia|jb) by three more GEMMs; the call needs about
 * 8 (o nbf^3 + o v nbf^2) bytes of free device memory plus one batch (o active occupied, v virtual orbitals; e.g.
 * 14 GB at nbf = 440, o = 20) and fails with UQC_E_NOMEM otherwise.  batch_bytes > 0 caps the memory of one batch
 * (more, smaller batches; it must hold the widest ket shell pair's columns, up to 72, of nbf^2 + o nbf doubles
 * each, else UQC_E_NOMEM); 0: as much as free memory allows.  Every GEMM operand is kept below 2^31 doubles (one
 * batch at most that much); when o v nbf^2 or o v^2 nbf reaches 2^31 (about nbf = 450 for a lattice with
 * o = nbf / 22) the call fails with UQC_E_UNSUPPORTED.  `res` may be NULL.
 * Errors: UQC_E_ARG, UQC_E_NOMEM, UQC_E_UNSUPPORTED, UQC_E_DEVICE. */
typedef struct {
    double e2;               /* correlation energy (hartree) */
    double e_os, e_ss;       /* opposite-spin part sum (ia|jb)^2 / D and same-spin part, e2 = e_os + e_ss */
    long long quartets;      /* shell quartets evaluated for the AO integrals (over all batches) */
    double ao_ms, transform_ms, energy_ms, ms;   /* wall time of the stages and of the call */
    double transform_flops;  /* 2 (o nbf^4 + o v nbf^3 + o v^2 nbf^2 + o^2 v^2 nbf) */
    int batches;             /* ket-pair batches of the AO integrals */
} uqc_mp2_result;

uqc_status uqc_mp2(uqc_basis* b, const double* C, const double* eps, int nocc, int nfrozen, double tau,
                   size_t batch_bytes, uqc_mp2_result* res);

/* Device Boys function, for verification: F_0..F_mmax (mmax <= 8) at n arguments T (host arrays; out is
 * n*(mmax+1), row-major).  precision UQC_FP64: tabulated Taylor grid + downward recursion (asymptotic form with
 * upward recursion beyond the grid); UQC_MIXED: the FP32 evaluation used for T <= 30 in mixed mode. */
uqc_status uqc_boys(uqc_ctx* ctx, int precision, int mmax, int n, const double* T, double* out);

/* ------------------------------------------------------------------------------------------------------------
 * Serving: a request loop that admits Fock-build requests for molecules of different sizes as they arrive,
 * subject to an HBM budget and a slot limit, keeps each request's basis plan and density resident on the device
 * between iterations, and runs the quartet classes of all admitted requests together, one launch per class.
 * A step carries a bounded amount of work (about 1.5e12 algorithmic FLOPs when several requests are admitted):
 * the builds of small requests complete within a step, those of large ones are spread over several steps, so an
 * admitted small request is not held back by a large one.  The next step is queued while the current one runs.
 * Admission takes queued requests in arrival order; one that does not fit the remaining budget is passed over for
 * later ones that do, until it has waited 2 s, after which nothing more is admitted before it.
 *
 * A request runs n_iter builds.  Iteration t uses density D_t; after it, D_{t+1} = (1-eps) D_t + eps R_t R_t^T
 * rescaled to tr(D_0), with R_t an nbf x ncol matrix of standard normal numbers drawn on the device from a
 * counter-based generator keyed by (seed, t) (SplitMix64 finaliser, Box-Muller).
 * ------------------------------------------------------------------------------------------------------------ */
typedef struct {
    int nshell;
    const int* l;
    const int* nprim;
    const double* center;
    const double* alpha;
    const double* coef;
    const double* D0;           /* nbf*nbf host, symmetric */
    int n_iter;                 /* 1..64 */
    int ncol;                   /* columns of R_t (>= 1) */
    double eps;                 /* perturbation weight in [0, 1] */
    unsigned long long seed;
    uqc_fock_opts opts;         /* its progress callback is not used by the server; a step spreads its class
                                   launches over as many streams as any admitted request's opts.streams asks for */
    double arrival_ms;          /* arrival time stamp on the caller's clock (reported back; informational) */
} uqc_request;

#define UQC_MAX_ITER 64

typedef struct {
    int n_iter;
    int nbf;
    double E2[UQC_MAX_ITER];    /* E2 of every iteration */
    double submit_ms;           /* server clock (ms since server creation) at submit */
    double admit_ms;            /* ... when admitted to the device */
    double finish_ms;           /* ... when the last iteration completed */
    long long quartets;         /* shell quartets computed over all iterations */
    double* J;                  /* optional host outputs (nbf*nbf) of the LAST iteration: set to caller memory or */
    double* K;                  /* NULL before calling uqc_poll; filled when the request is done */
    double* G;
    double* D;                  /* density of the last iteration */
    long long device_bytes;     /* device memory the request held while admitted (what the HBM budget was charged) */
    int steps;                  /* server steps the request took part in (a build may span several) */
} uqc_result;

/* hbm_budget_bytes: device memory the server may hold for admitted requests; max_slots: admitted at once. */
uqc_status uqc_server_create(uqc_ctx* ctx, size_t hbm_budget_bytes, int max_slots, uqc_server** out);
/* Copies the request; returns a ticket.  UQC_E_NOMEM if the request alone exceeds the budget. */
uqc_status uqc_submit(uqc_server* s, const uqc_request* req, long long* ticket);
/* UQC_PENDING while queued or running; UQC_OK once finished (result filled, ticket released);
 * UQC_E_NOT_FOUND for an unknown or already collected ticket. */
uqc_status uqc_poll(uqc_server* s, long long ticket, uqc_result* res);
/* Runs the server loop on the calling thread until every submitted request is finished (for callers without a
 * background thread); returns immediately if the server has its own thread. */
uqc_status uqc_server_drain(uqc_server* s);
/* Stops accepting work, finishes outstanding requests, frees everything. */
uqc_status uqc_server_destroy(uqc_server* s);

#ifdef __cplusplus
}
#endif
#endif /* UQC_H */
