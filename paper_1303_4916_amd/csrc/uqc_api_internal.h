// Host-side objects behind the opaque handles of include/uqc.h.
#pragma once
#include "uqc.h"
#include "uqc_internal.h"
#include "uqc_one.h"

#include <list>
#include <string>
#include <utility>
#include <vector>

uqc_status uqc_fail(uqc_status s, const std::string& msg);

#define UQC_HIP(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return uqc_fail(UQC_E_DEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

struct uqc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    double* boys64 = nullptr;
    float* boys32 = nullptr;
    double* rys = nullptr;   // Rys quadrature table (generated/rys_consts.h layout)
    std::vector<hipEvent_t> events;
    hipStream_t side[3] = {nullptr, nullptr, nullptr};  // extra streams of a build spread over several (lazy)
    hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
    void* blas = nullptr;  // rocblas_handle of the SCF driver, created on first use
};

void release_blas(uqc_ctx* c);  // destroys the rocBLAS handle if one was created

hipEvent_t ctx_event(uqc_ctx* c, size_t i);
// Stream i of a build spread over several: 0 is the context's stream, 1..3 the context's extra streams (created on
// first use, default priority).  nullptr if creation fails.
hipStream_t ctx_stream(uqc_ctx* c, int i);
// v[0], v[n-1], v[1], v[n-2], ...: launch order of classes sorted largest first
std::vector<size_t> interleave_ends(const std::vector<size_t>& v);

namespace uqc {

struct ShellH {
    int l = 0, K = 0, off = 0;
    double A[3] = {0, 0, 0};
    std::vector<double> alpha, c;  // exponents; coefficients with radial and contracted normalisation folded in
};

struct Bin {
    int la = 0, lb = 0, Ka = 0, Kb = 0, K = 0, np = 0;
    std::vector<double> prim, AB, sdeg, Q;
    std::vector<int> off_a, off_b, sa, sb;
    std::vector<int> kp;                       // [np] leading primitive pairs above the primitive bound
    std::vector<double> qprim;                 // [K][np] primitive-pair bounds Q_e, in the order of prim (empty
                                               // until the bounds are known)
    std::vector<int> bucket;                   // [np] decade of Q (floor(log10 Q)), non-increasing along the bin
    std::vector<std::pair<int, int>> bstart;   // (decade, first index) for every decade present, in bin order
    int first_below(int dec) const;            // first index whose decade is < dec (np if none)
    int first_at_or_below(int dec) const;      // first index whose decade is <= dec (np if none)
    void* d_mem = nullptr;
    size_t bytes = 0;                          // device bytes of d_mem
    BinDev dev{};
};

struct LaunchGroup {
    int cls = 0;
    int mixed = 0;
    int ntask = 0;
    int task0 = 0;                     // index of the group's first task counter in the plan's counter array
    long long nitems = 0, quartets = 0, prim_quartets = 0;  // counts of the last build
    double flops = 0;
    const TaskDev* d_tasks = nullptr;
    const long long* d_begin = nullptr;
    std::vector<TaskDev> host_tasks;   // copies (device pointers inside), used to batch several bases
    std::vector<long long> host_begin;
};

struct PlanKey {
    double tau;
    int prec;
    double bound;
    double boys_t;  // mixed plans: the FP32 Boys evaluation covers T <= boys_t
};

struct Plan {
    std::vector<LaunchGroup> groups;
    long long canonical = 0;                       // canonical shell quartets of the basis
    long long quartets = 0, screened = 0, prim_quartets = 0, fp64_quartets = 0;  // counts of the last build
    double flops = 0;
    int ntasks = 0;
    unsigned long long* d_count = nullptr;         // [2 ntasks] per-task quartet, then primitive-quartet counters
    unsigned* d_queue = nullptr;                   // [groups][kQueueWords] item counters of each group's launches
    std::vector<unsigned long long> h_count;
    void* d_mem = nullptr;
    size_t bytes = 0;                              // device bytes of d_mem
};

// Counts of the last build, from the per-task counters (h_count must hold the device values).
void plan_account(Plan& p);

void free_plan(Plan& p);

}  // namespace uqc

struct uqc_basis {
    uqc_ctx* ctx = nullptr;
    int nshell = 0, nbf = 0;
    std::vector<uqc::ShellH> shells;
    std::vector<double> fcomp;
    std::vector<uqc::Bin> bins;
    std::vector<int> pair_bin, pair_pos, pair_first;  // [a * nshell + b]
    std::vector<double> Qfull;
    double qmax = 0;
    std::list<std::pair<uqc::PlanKey, uqc::Plan>> plans;  // list: plan pointers stay valid
    void* d_work = nullptr;
    size_t work_bytes = 0;
    double *d_f = nullptr, *d_Dp = nullptr, *d_J = nullptr, *d_K = nullptr, *d_scal = nullptr, *d_io = nullptr;
    double *d_Dp2 = nullptr, *d_K2 = nullptr;  // second spin density D' and K accumulator (spin-density builds)
    double* d_Dp3 = nullptr;                     // spin-density builds: D'a + D'b, the density of the J pass
    double* d_uio = nullptr;                     // host-pointer staging of spin-density builds (7 nbf^2, on first use)
    // one-electron integrals: shell table and per-pair-class shell-pair lists (uploaded on first use), nuclei
    void* d_shells = nullptr;
    uqc::ShellsDev shells_dev{};
    const int2* d_pairs[6] = {};
    int npairs[6] = {};
    double* d_nuc = nullptr;
    size_t nuc_cap = 0;
    size_t device_bytes() const;  // device memory held for Fock builds: pair bins, workspace and plans
    ~uqc_basis();
};

namespace uqc {
// Checks the options of a Fock build (tau, precision, fp64_bound, max_items_per_launch, exchange_scale, streams);
// UQC_E_ARG with a message naming `who` otherwise.
uqc_status check_fock_opts(const uqc_fock_opts& o, const std::string& who);
}

uqc::Plan* get_plan(uqc_basis* B, double tau, int prec, double bound, double boys_t, uqc_status* st);
// The plan already made for these options, or nullptr (never allocates).
uqc::Plan* find_plan(uqc_basis* B, double tau, int prec, double bound, double boys_t);

namespace uqc {
// A caller-chosen device workspace for a closed-shell Fock build: D' (nbf^2), the J and K accumulators (nbf^2 each),
// 8 scalars, 2 max_tasks counters and the kQueueWords item counters of the class launches (which run one after
// another).
struct FockWorkspace {
    double* Dp;
    double* J;
    double* K;
    double* scal;
    unsigned long long* count;
    int max_tasks;
    unsigned* queue;
};
// The Fock build behind uqc_fock_build (nspin = 1: Din = {D}, out = {J, K, G}) and uqc_fock_build_uhf (nspin = 2:
// Din = {Da, Db}, out = {J, Ka, Kb, Ga, Gb}).  ws == nullptr: the basis's workspace, the plan made on first use.
// ws != nullptr (closed shell, device pointers): everything the build writes besides its outputs goes to *ws, the
// plan must exist already, and every class launch is queued on the context's stream; nothing is allocated.
uqc_status fock_run(uqc_basis* B, int nspin, const double* const* Din, double* const* out, const uqc_fock_opts* opts,
                    uqc_stats* stats, const char* name, const FockWorkspace* ws);
// Takes, with `device` current, the device address of the fixed workspace of uqc_fock_build_noalloc.
uqc_status noalloc_setup(int device);
}  // namespace uqc

typedef struct _rocblas_handle* rocblas_handle;

namespace uqc {
bool is_device_ptr(const void* p);  // device or managed memory (false for host memory and null)
// The context's rocBLAS handle (created on first use), bound to the context's stream, host pointer mode.
uqc_status ensure_blas(uqc_ctx* ctx, rocblas_handle* out);
}
