// uqc_fock_build_noalloc: the closed-shell Fock build of uqc_fock_build with everything it writes besides its
// outputs (the scaled density D', the J and K accumulators, the scalars, the per-task quartet counters and the item
// counters of the class launches) in one fixed device array of this file instead of the basis's workspace, for
// callers that cannot allocate device memory.
// Each device the library runs on holds its own copy of the array until the process ends; its address on a device
// is taken once, by uqc_init, with that device current.
#include "uqc_api_internal.h"

#include <mutex>

namespace {

constexpr size_t kScratchMaxNbf = 1024;     // largest basis: 3 nbf^2 doubles of D', J and K accumulators
constexpr size_t kScratchMaxTasks = 32768;  // largest screening plan (tasks = pairs of pair bins and precisions)
constexpr size_t kScratchQueue = uqc::kQueueWords / 2;  // the item counters of a class launch, in doubles
constexpr size_t kScratchDoubles =
    3 * kScratchMaxNbf * kScratchMaxNbf + 8 + 2 * kScratchMaxTasks + kScratchQueue;  // 25.7 MB

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device (null until taken)

}  // namespace

uqc_status uqc::noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return uqc_fail(UQC_E_UNSUPPORTED, "uqc_init: device index too large");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return UQC_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return uqc_fail(UQC_E_DEVICE, std::string("uqc_init: hipGetSymbolAddress of the fixed workspace failed: ") +
                                          hipGetErrorString(e));
    g_scratch[device] = static_cast<double*>(p);
    return UQC_OK;
}

extern "C" uqc_status uqc_fock_build_noalloc(uqc_basis* B, const double* D, double* J, double* K, double* G,
                                             const uqc_fock_opts* opts, uqc_stats* stats) {
    if (!B || !D) return uqc_fail(UQC_E_ARG, "uqc_fock_build_noalloc: NULL basis or density");
    const size_t N = (size_t)B->nbf;
    if (N > kScratchMaxNbf)
        return uqc_fail(UQC_E_ARG, "uqc_fock_build_noalloc: more than " + std::to_string(kScratchMaxNbf) +
                                       " basis functions (the fixed workspace holds 3 nbf^2 doubles)");
    double* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        const int dev = B->ctx->device;
        if (dev >= 0 && dev < kMaxDevices) base = g_scratch[dev];
    }
    if (!base) return uqc_fail(UQC_E_DEVICE, "uqc_fock_build_noalloc: the fixed workspace was not set up");
    const size_t NN = N * N;
    uqc::FockWorkspace ws;
    ws.Dp = base;
    ws.J = base + NN;
    ws.K = base + 2 * NN;
    ws.scal = base + 3 * NN;
    ws.count = reinterpret_cast<unsigned long long*>(base + 3 * NN + 8);
    ws.max_tasks = (int)kScratchMaxTasks;
    ws.queue = reinterpret_cast<unsigned*>(base + 3 * NN + 8 + 2 * kScratchMaxTasks);
    const double* Din[1] = {D};
    double* out[3] = {J, K, G};
    return uqc::fock_run(B, 1, Din, out, opts, stats, "uqc_fock_build_noalloc", &ws);
}
