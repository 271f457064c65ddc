// One angular-momentum class of the quartet kernels: compiled once per class with
// -DUQC_CLASS_ID=n -DUQC_LA=.. -DUQC_LB=.. -DUQC_LC=.. -DUQC_LD=.. -DUQC_TEAM=0|1 so that the classes build in
// parallel; UQC_TEAM selects the six-lane team kernel for the Fock build.
#include "uqc_eri_impl.h"
#include "uqc_rys.h"
#if UQC_TEAM
#include "uqc_eri_team.h"
#endif

#if !defined(UQC_CLASS_ID) || !defined(UQC_LA) || !defined(UQC_LB) || !defined(UQC_LC) || !defined(UQC_LD)
#error "uqc_eri_class.hip needs UQC_CLASS_ID and UQC_LA..UQC_LD"
#endif

#define UQC_CAT2(a, b) a##b
#define UQC_CAT(a, b) UQC_CAT2(a, b)

namespace uqc {

// Workgroups of a digest kernel that fit on the current device at once (occupancy x compute units, rounded down to
// a multiple of the die count), found once per kernel; 0 if the runtime cannot tell.
static long long resident_blocks(const void* fn) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess)
        return 0;
    return (long long)cus * per_cu / kXcds * kXcds;
}

template <bool MIXED, int NSPIN>
static void launch_digest_one(long long nitems_blocks, const TaskDev* d_tasks, const long long* d_task_begin,
                              int ntask, long long item0, long long nitems, const double* b64, const float* b32,
                              const WorkRedirect& wr, unsigned* queue, hipStream_t s) {
#if UQC_TEAM
    const void* fn = reinterpret_cast<const void*>(&k_digest_team<UQC_LA, UQC_LB, UQC_LC, UQC_LD, MIXED, NSPIN>);
#else
    const void* fn = reinterpret_cast<const void*>(&k_digest<UQC_LA, UQC_LB, UQC_LC, UQC_LD, MIXED, NSPIN>);
#endif
    // one workgroup per four items, at most as many as are resident at once (the wavefronts then loop over items)
    static const long long resident = resident_blocks(fn);
    const long long nb = resident > 0 && nitems_blocks > resident ? resident : nitems_blocks;
#if UQC_TEAM
    hipLaunchKernelGGL((k_digest_team<UQC_LA, UQC_LB, UQC_LC, UQC_LD, MIXED, NSPIN>), dim3((unsigned)nb),
                       dim3(kBlock), 0, s, d_tasks, d_task_begin, ntask, item0, nitems, b64, b32, wr, queue);
#else
    hipLaunchKernelGGL((k_digest<UQC_LA, UQC_LB, UQC_LC, UQC_LD, MIXED, NSPIN>), dim3((unsigned)nb), dim3(kBlock), 0,
                       s, d_tasks, d_task_begin, ntask, item0, nitems, b64, b32, wr, queue);
#endif
}

static hipError_t launch_digest_cls(bool mixed, int nspin, const TaskDev* d_tasks, const long long* d_task_begin,
                                    int ntask, long long item0, long long nitems, const double* b64, const float* b32,
                                    const WorkRedirect& wr, unsigned* queue, hipStream_t s) {
    const long long waves_per_block = kBlock / kWave;
    const long long nblocks = (nitems + waves_per_block - 1) / waves_per_block;
    if (nblocks <= 0) return hipSuccess;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (nspin == 2) {
        if (mixed) launch_digest_one<true, 2>(nblocks, d_tasks, d_task_begin, ntask, item0, nitems, b64, b32, wr, queue,
                                               s);
        else launch_digest_one<false, 2>(nblocks, d_tasks, d_task_begin, ntask, item0, nitems, b64, b32, wr, queue,
                                          s);
    } else {
        if (mixed) launch_digest_one<true, 1>(nblocks, d_tasks, d_task_begin, ntask, item0, nitems, b64, b32, wr, queue,
                                               s);
        else launch_digest_one<false, 1>(nblocks, d_tasks, d_task_begin, ntask, item0, nitems, b64, b32, wr, queue,
                                          s);
    }
    return hipGetLastError();
}

#if UQC_TEAM
// The MP2 batch form of a team class: ten quartets per wavefront.
static void launch_team_batch(const ListDev& L, const double* b64, hipStream_t s) {
    const long long waves = ((long long)L.n + kTeamsPerWave - 1) / kTeamsPerWave;
    const unsigned nblocks = (unsigned)((waves + kBlock / kWave - 1) / (kBlock / kWave));
    hipLaunchKernelGGL((k_list_team_batch<UQC_LA, UQC_LB, UQC_LC, UQC_LD>), dim3(nblocks), dim3(kBlock), 0, s, L, b64);
}
#endif

static hipError_t launch_list_cls(bool mixed, int mode, const ListDev& L, const double* b64, const float* b32,
                                  hipStream_t s) {
    if (L.n <= 0) return hipSuccess;
#if UQC_TEAM
    if (mode == MODE_BATCH) {
        launch_team_batch(L, b64, s);
        return hipGetLastError();
    }
#endif
    const unsigned nblocks = (unsigned)((L.n + kBlock - 1) / kBlock);
    if (mode == MODE_SCHWARZ)
        hipLaunchKernelGGL((k_list<UQC_LA, UQC_LB, UQC_LC, UQC_LD, false, MODE_SCHWARZ>), dim3(nblocks),
                           dim3(kBlock), 0, s, L, b64, b32);
    else if (mode == MODE_SCATTER)
        hipLaunchKernelGGL((k_list<UQC_LA, UQC_LB, UQC_LC, UQC_LD, false, MODE_SCATTER>), dim3(nblocks),
                           dim3(kBlock), 0, s, L, b64, b32);
    else if (mode == MODE_BATCH)
        hipLaunchKernelGGL((k_list<UQC_LA, UQC_LB, UQC_LC, UQC_LD, false, MODE_BATCH>), dim3(nblocks),
                           dim3(kBlock), 0, s, L, b64, b32);
    else if (mixed)
        hipLaunchKernelGGL((k_list<UQC_LA, UQC_LB, UQC_LC, UQC_LD, true, MODE_STORE>), dim3(nblocks), dim3(kBlock), 0,
                           s, L, b64, b32);
    else
        hipLaunchKernelGGL((k_list<UQC_LA, UQC_LB, UQC_LC, UQC_LD, false, MODE_STORE>), dim3(nblocks), dim3(kBlock),
                           0, s, L, b64, b32);
    return hipGetLastError();
}

static hipError_t launch_list_rys_cls(const ListDev& L, const double* rystab, hipStream_t s) {
    if (L.n <= 0) return hipSuccess;
    const unsigned nblocks = (unsigned)((L.n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_list_rys<UQC_LA, UQC_LB, UQC_LC, UQC_LD>), dim3(nblocks), dim3(kBlock), 0, s, L, rystab);
    return hipGetLastError();
}

ClassLaunchers UQC_CAT(class_launchers_, UQC_CLASS_ID)() {
    return ClassLaunchers{&launch_digest_cls, &launch_list_cls, &launch_list_rys_cls};
}

}  // namespace uqc
