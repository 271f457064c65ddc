// Internal data layout shared by the host plan and the device kernels of libuqc.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace uqc {

constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kBlock = 256;            // threads per block of the quartet kernels (4 wavefronts)
constexpr int kMaxK = 16;              // maximum contraction depth
// A primitive pair e of a shell pair is dropped when Q_e * Q_max <= kPrimEps, where Q_e = sqrt(max (e|e)) over its
// Cartesian components and Q_max is the largest contracted pair bound of the basis.  By the Cauchy-Schwarz
// inequality every integral then changes by at most (dropped primitive pairs of bra and ket) * kPrimEps.
constexpr double kPrimEps = 1e-15;
constexpr int kMaxNbf = 65535;         // maximum basis size (N x N matrices indexed with 32-bit offsets)
constexpr int kBoysGridPerUnit = 8;    // Boys Taylor grid: T_g = g / 8 (exact in binary, same points in FP32/FP64)
constexpr int kBoysTmax = 60;          // grid covers [0, 60); asymptotic form beyond
constexpr int kBoysNg = kBoysTmax * kBoysGridPerUnit + 1;
constexpr int kBoysNm = 18;            // per grid point: F_0 .. F_16 (m <= 8 plus Taylor order 8), then exp(-T_g)
constexpr int kBoysExpCol = 17;
// Device layout of the FP64 table: one slice per highest order L = 0..8, each row holding the Taylor coefficients
// F_{L+k}(T_g) / k!, k = 0..8, and exp(-T_g) (10 doubles, 80 bytes, 16-byte aligned), so a Boys evaluation reads
// one row with five 16-byte loads.
constexpr int kBoysRow = 10;
constexpr int kBoysLmax = 8;
constexpr int kBoysTmax32 = 30;        // FP32 evaluation limit in mixed mode
constexpr int kNumClasses = 21;
constexpr int kTeamKets = 10;          // ket pairs per wavefront in the six-lane team kernels
constexpr int kGroupBras = 8;          // bra pairs per work item (one wavefront), 64-ket kernels
constexpr int kTeamGroupBras = 4;      // bra pairs per work item, team kernels
constexpr int kXcds = 8;               // accelerator complex dies; workgroups are dealt to them round-robin
constexpr long long kMaxItemsPerLaunch = 1LL << 20;  // work items per class-kernel launch (longer classes split)
constexpr int kQueueWords = 16;        // item counters of one class-kernel launch: one per die, padded to 64 bytes

// Primitive-pair fields, stored field-major: prim[field][k][np] (consecutive pairs contiguous; the ket side, one
// pair per lane), and again pair-major: rec[np][k][kRec] (the bra side, one pair per wavefront, scalar loads)
enum PrimField { F_Z = 0, F_PX, F_PY, F_PZ, F_PAX, F_PAY, F_PAZ, F_PREF, F_O2Z, kNumFields };
constexpr int kRec = 10;               // doubles per pair-major primitive record: the fields, then Q_e
constexpr int kRecQ = kNumFields;      // record slot of the primitive pair's bound Q_e
constexpr int kHdr = 8;                // doubles per pair header: A-B (3), sdeg, Q, {off_a, off_b} (two ints), pad

// One bin of shell pairs with the same (l_a, l_b, K_a, K_b).  Pairs are ordered by decade of their Schwarz bound
// (descending), then by their first shell, so that the ket range of any bra pair is a prefix at decade granularity
// and kets sharing their first shell are adjacent inside a wavefront.
struct BinDev {
    const double* prim;   // [kNumFields][K][np]
    const double* rec;    // [np][K][kRec] the same fields, pair-major
    const double* hdr;    // [np][kHdr] AB, sdeg, Q and the two offsets of every pair
    const double* AB;     // [3][np]  A - B
    const int* off_a;     // [np] first basis function of shell a (the higher-l shell)
    const int* off_b;     // [np]
    const double* sdeg;   // [np] 0.5 if a == b else 1
    const double* Q;      // [np] Schwarz bound of the pair
    const int* kp;        // [np] primitive pairs evaluated by the Fock build: the leading kp of the pair's K, which
                          // are ordered by decreasing bound (the rest fall under kPrimEps)
    const double* cq;     // [ceil(np / 64)][K] for each chunk of 64 consecutive pairs and each primitive position k,
                          // the largest bound Q_e of the chunk's k-th primitive pairs (non-increasing in k)
    int np;
    int K;                // primitive pairs per shell pair (K_a * K_b)
};

// One (bra bin, ket bin) block of the quartet work list of a Fock build.  The ket bin is cut into chunks of S
// consecutive ket pairs (S = 64, or 10 for the team kernels); a work item is one chunk and a group of up to
// kGroupBras (kTeamGroupBras) bra pairs whose ket ranges meet that chunk.  Items are ordered chunk by chunk, and
// inside a chunk the bra pairs are ordered by their first shell, so a wavefront keeps its kets (and their partial
// J_cd, K_ad, K_ac sums) across the group, and the items that share a chunk run on one die close in time.
struct TaskDev {
    BinDev bra, ket;
    const int* lo;             // [nbra] first ket index (in the ket bin)
    const int* hi;             // [nbra] one past the last ket index
    const int* blist;          // bra indices, chunk by chunk
    const int2* items;         // [nitems + 1] {first blist entry, chunk}; the group ends at the next item's entry
    long long item_begin;      // first work item of this task within its launch
    long long nitems;
    double tau;                // a quartet in the range is computed iff Q_ab Q_cd >= tau
    double lo_excl, hi_incl;   //   and lo_excl < Q_ab Q_cd <= hi_incl (precision routing)
    double boys_t;             // mixed tasks: primitive quartets with Boys argument T <= boys_t use the FP32 table
    unsigned long long* count; // quartets computed by this task (one atomic per wavefront)
    unsigned long long* pcount;  // primitive quartets computed by this task
    int nbra;
    int same;                  // bra bin == ket bin: the diagonal quartet (bra == ket) gets an extra 1/2
    const double* D;           // scaled density D' = f D f (nbf x nbf); spin builds: the alpha density, for K
    double* J;                 // J accumulator (nbf x nbf), symmetrised in the finalize step
    double* K;                 // K accumulator (spin builds: of the alpha density)
    const double* DJ;          // spin builds: the total density D'a + D'b, for J
    const double* D2;          // spin builds: the beta density, for K
    double* K2;                // spin builds: the beta K accumulator
    int nbf;
    int cidx;                  // index of this task's counters in its plan's counter array
};

// Closed-shell builds whose density, accumulators and counters live in a caller-chosen workspace instead of the
// ones the task descriptors name: when J is non-null, the kernels read D and accumulate into J and K given here,
// and count task t's quartets at count[cidx] and its primitive quartets at count[ncount + cidx].
struct WorkRedirect {
    const double* D;
    double* J;
    double* K;
    unsigned long long* count;
    int ncount;
};

// An explicit list of quartets (bra index, ket index) for block output or Schwarz bounds.
struct ListDev {
    BinDev bra, ket;
    const int* bra_idx;
    const int* ket_idx;
    int n;
    double* out;               // STORE: [n][NA*NB*NC*ND]; SCHWARZ: [n]; SCATTER: the nbf^4 tensor; BATCH: see Mode
    int nbf;                   // SCATTER and BATCH
    // BATCH: the quartets are implicit, every pair p of the physical bra bin times the nket ket pairs kpos[t] of the
    // physical ket bin (q = p nket + t, n = np nket), those with Q_p Q_kpos[t] >= tau computed and counted in
    // *count (bra_idx and ket_idx unused)
    const int* col;            // BATCH: [nket] first column of ket pair t in the batch
    int ncols;                 // BATCH: columns of the batch
    int swap;                  // BATCH: 1 if the kernel's bra pair is the physical ket pair (class order)
    const int* kpos;           // BATCH: [nket] positions of the batch's ket pairs in the physical ket bin
    int nket;
    double tau;
    unsigned long long* count;
};

// STORE: each quartet's block; SCHWARZ: sqrt of the largest diagonal element; SCATTER: every element of the block
// written to the dense tensor out[((i nbf + j) nbf + k) nbf + l] at its eight permutationally equivalent places;
// BATCH: every element (mu nu|lam sig) written to out[(mu nbf + nu) ncols + col(lam sig)] for both orders of the bra
// pair and both orders of the ket pair, where the ket pair's columns start at col[t]: (lam in c, sig in d) at
// col + k n_d + l, then, for c != d, (lam in d, sig in c) at col + n_c n_d + l n_c + k.
enum Mode { MODE_STORE = 0, MODE_SCHWARZ = 1, MODE_SCATTER = 2, MODE_BATCH = 3 };

// Host launchers of one angular-momentum class (defined in uqc_eri_class.hip, one object per class).
struct ClassLaunchers {
    hipError_t (*digest)(bool mixed, int nspin, const TaskDev* d_tasks, const long long* d_task_begin, int ntask,
                         long long item0, long long nitems, const double* boys64, const float* boys32,
                         const WorkRedirect& wr, unsigned* queue, hipStream_t s);
    hipError_t (*list)(bool mixed, int mode, const ListDev& list, const double* boys64, const float* boys32,
                       hipStream_t s);
    hipError_t (*list_rys)(const ListDev& list, const double* rystab, hipStream_t s);  // MODE_STORE by Rys quadrature
};

// Host-side launchers (defined in uqc_kernels.hip).
int class_index(int la, int lb, int lc, int ld);           // -1 if not canonical
void class_ls(int idx, int* la, int* lb, int* lc, int* ld);
// Work items [item0, item0 + nitems) of one (class, precision) launch group.
// nspin = 1: J and K of D; nspin = 2: J of DJ, K of D into K and of D2 into K2, each integral evaluated once.
// wr.J non-null (nspin = 1 only): D, J, K and the counters are taken from wr instead of the task descriptors.
// queue: kQueueWords device words the launch hands its items out from (one counter per die), cleared by this call
// on stream s; launches that can run at the same time need distinct queues.
hipError_t launch_digest(int cls, bool mixed, int nspin, const TaskDev* d_tasks, const long long* d_task_begin,
                         int ntask, long long item0, long long nitems, const double* boys64, const float* boys32,
                         const WorkRedirect& wr, unsigned* queue, hipStream_t s);
hipError_t launch_list(int cls, bool mixed, int mode, const ListDev& list, const double* boys64,
                       const float* boys32, hipStream_t s);
hipError_t launch_list_rys(int cls, const ListDev& list, const double* rystab, hipStream_t s);
hipError_t launch_prepare(const double* D, const double* f, double* Dp, int nbf, unsigned long long* maxbits,
                          hipStream_t s);
hipError_t launch_zero(double* p, size_t n, hipStream_t s);
hipError_t launch_add(const double* A, const double* B, double* C, size_t n, hipStream_t s);   // C = A + B
hipError_t launch_scale_cols(const double* U, const double* w, double* W, int N, hipStream_t s);  // W = U diag(w)
hipError_t launch_antisym(const double* M, double* E, int N, hipStream_t s);                  // E = M - M^T
hipError_t launch_finalize(const double* D, const double* Jacc, const double* Kacc, const double* f, double* J,
                           double* K, double* G, double xs, double* E2, int nbf, hipStream_t s);
// Spin densities: J = sym(Jacc), K^s = sym(K^s acc), G^s = J - xs K^s, E2 += 1/2 sum (Da Ga + Db Gb); any output
// may be null.
hipError_t launch_finalize_uhf(const double* Da, const double* Db, const double* Jacc, const double* Kaacc,
                               const double* Kbacc, const double* f, double xs, double* J, double* Ka, double* Kb,
                               double* Ga, double* Gb, double* E2, int nbf, hipStream_t s);
hipError_t launch_boys(int prec, int mmax, int n, const double* T, double* out, const double* boys64,
                       const float* boys32, hipStream_t s);
hipError_t launch_perturb(double* D, const double* R, int nbf, int ncol, double eps, double trace0, double* work,
                          hipStream_t s);
hipError_t launch_normal(double* R, long long n, unsigned long long seed, unsigned long long stream,
                         hipStream_t s);
hipError_t launch_trace(const double* D, int nbf, double* out, hipStream_t s);
double class_flops_prim(int cls);
int class_team(int cls);               // 1 if the class's Fock-build kernel is the six-lane team kernel
double class_flops_contr(int cls);

}  // namespace uqc
