// Serving loop of libuqc: continuous batching of Fock-build requests.
//
// A background thread owns a private context (a non-blocking stream plus the extra streams of a build) and a second
// one for admission.  It
//   1. admits queued requests in arrival order while a slot is free and the request's device footprint fits the
//      remaining HBM budget; a request that does not fit is passed over for later ones that do until it has waited
//      kMaxSkipMs, after which nothing more is admitted before it (so none starves).  Admission (basis, screening
//      plan, density upload) runs on the admission context's stream, beside the steps already on the device, and
//      the budget is then charged what the request really holds;
//   2. queues one bounded step: every admitted request whose build has not started gets its density prepared and
//      its accumulators cleared; every admitted request contributes a slice of its remaining work items (all of
//      them when the build fits its share of the step's work); ONE launch per (angular-momentum class, precision)
//      covers the slices of all requests (each task carries its own request's density and J/K accumulators); the
//      requests whose build completes in the step are finalised, then perturbed to their next density (generated
//      on the device) or left for retirement;
//   3. keeps at most kInFlight steps queued: before queuing another it waits for the oldest, takes its energies and
//      counts, and retires the requests that finished in it (results copied out, device memory released, budget
//      returned).
// A request admitted while others are mid-way joins at the next step, so its work shares launches with theirs;
// the builds of small requests complete within a step while a large one's spreads over several.
#include "uqc_api_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

using namespace uqc;

namespace {

constexpr double kStepFlops = 1.5e12;     // algorithmic FLOPs of one step when several requests share it
constexpr double kSoloStepFlops = 6e12;   // ... when one request is admitted and none waits
constexpr double kMaxSkipMs = 2000.0;     // a request passed over by admission blocks the queue after this long
constexpr int kInFlight = 2;              // steps queued on the device at once
constexpr int kPinnedTasks = 16384;       // per-slot staging of a plan's task counters (larger plans: refused)

struct Req {
    long long ticket = 0;
    // owned copies of the request arrays
    std::vector<int> l, nprim;
    std::vector<double> center, alpha, coef, D0;
    int nshell = 0, nbf = 0, n_iter = 1, ncol = 1;
    double eps = 0;
    unsigned long long seed = 0;
    uqc_fock_opts opts{};
    size_t footprint = 0;      // estimate until admitted, then the device bytes held
    // device state
    uqc_basis* basis = nullptr;
    Plan* plan = nullptr;
    double* d_D = nullptr;     // current density (nbf*nbf), then R (nbf*ncol)
    double* d_R = nullptr;
    double trace0 = 0;
    int iter = 0;              // builds queued to completion
    int slot = -1;             // pinned staging slot
    std::vector<long long> pos;  // per plan group: work items of the current build already queued
    bool started = false;      // the current build's preparation is queued
    bool counted = false;      // the plan's counts have been read back (they are the same for every build)
    int steps = 0;
    // results
    uqc_status status = UQC_PENDING;
    std::string error;
    double E2[UQC_MAX_ITER] = {0};
    long long quartets = 0;
    double submit_ms = 0, admit_ms = 0, finish_ms = 0;
    std::vector<double> J, K, G, D;
};

// Device bytes a request will hold, estimated before its basis exists: the basis workspace (10 nbf^2 doubles), the
// density and perturbation, the pair bins (per primitive pair the field-major and pair-major records, per pair the
// header, AB, degeneracy, bound and three ints), and the work lists (both precisions).  The charge is replaced by
// the bytes really held once the request is admitted.
size_t estimate_footprint(const Req& r) {
    const size_t N = r.nbf, NN = N * N;
    size_t prim_pairs = 0, pairs = 0;
    for (int a = 0; a < r.nshell; ++a)
        for (int b = 0; b <= a; ++b) {
            prim_pairs += (size_t)r.nprim[a] * r.nprim[b];
            ++pairs;
        }
    size_t bytes = (N + 8 + 10 * NN) * sizeof(double);           // basis workspace
    bytes += NN * sizeof(double) + N * r.ncol * sizeof(double);  // density + perturbation
    bytes += prim_pairs * (kNumFields + kRec) * sizeof(double) + pairs * ((kHdr + 6) * sizeof(double) + 3 * sizeof(int));
    bytes += pairs * 2 * (2 * sizeof(int) + sizeof(long long)) + 64 * 1024;  // screened work lists (both precisions)
    return bytes;
}

// Static FLOPs per work item of a task before any build of the request has been counted: half of every quartet
// of the item's kets and bras surviving, each with all its primitive quartets.
double item_flops_estimate(int cls, const TaskDev& t) {
    const double kets = class_team(cls) ? kTeamKets : kWave, bras = kGroupBras;
    return 0.5 * kets * bras * ((double)t.bra.K * t.ket.K * class_flops_prim(cls) + class_flops_contr(cls));
}

}  // namespace

struct uqc_server {
    uqc_ctx* ctx = nullptr;   // steps: private non-blocking stream (+ the extra streams), own Boys tables
    uqc_ctx* actx = nullptr;  // admission: basis creation and uploads
    hipStream_t own_stream = nullptr;
    size_t budget = 0;
    int max_slots = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> queue;
    std::vector<Req*> active;
    std::map<long long, Req*> table;
    size_t used = 0;
    bool stop = false;
    long long next_ticket = 1;
    std::thread worker;
    std::chrono::steady_clock::time_point t0;
    // staging: pinned host memory per admitted slot (energies, counters), per in-flight step the task lists
    double* pinned = nullptr;
    std::vector<int> free_slots;
    struct Step {
        hipEvent_t ev = nullptr;
        std::vector<std::pair<Req*, int>> done;  // (request, index of the build completed by this step)
        std::vector<Req*> retiring;              // requests whose last build completed in this step
        void* d_tasks = nullptr;
        size_t d_bytes = 0;
        char* h_tasks = nullptr;  // pinned
        size_t h_bytes = 0;
    };
    Step ring[kInFlight];
    std::deque<int> inflight;  // ring indices, oldest first
    int next_ring = 0;

    static size_t slot_doubles() { return UQC_MAX_ITER + 2 * (size_t)kPinnedTasks; }
    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    void loop();
    bool admit_one(Req* r);
    void retire(Req* r, uqc_status st, const std::string& msg);
    bool queue_step(Step& f);
    void complete(Step& f);
    void fail_everything(const char* msg);
};

void uqc_server::retire(Req* r, uqc_status st, const std::string& msg) {
    if (r->d_D) (void)hipFree(r->d_D);
    r->d_D = r->d_R = nullptr;
    if (r->basis) uqc_basis_destroy(r->basis);
    r->basis = nullptr;
    r->plan = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    used -= r->footprint;
    if (r->slot >= 0) free_slots.push_back(r->slot);
    r->slot = -1;
    r->status = st;
    r->error = msg;
    r->finish_ms = now_ms();
    cv_done.notify_all();
}

bool uqc_server::admit_one(Req* r) {
    uqc_status st = uqc_basis_create(actx, r->nshell, r->l.data(), r->nprim.data(), r->center.data(),
                                     r->alpha.data(), r->coef.data(), &r->basis);
    if (st != UQC_OK) {
        retire(r, st, uqc_last_error());
        return false;
    }
    r->plan = get_plan(r->basis, r->opts.schwarz_tau, r->opts.precision, r->opts.fp64_bound, r->opts.fp64_boys_T,
                       &st);
    const size_t NN = (size_t)r->nbf * r->nbf;
    if (!r->plan) {
        retire(r, st, uqc_last_error());
        return false;
    }
    if (r->plan->ntasks > kPinnedTasks) {
        retire(r, UQC_E_UNSUPPORTED, "server: screening plan has more than 16384 tasks");
        return false;
    }
    const size_t dbytes = (NN + (size_t)r->nbf * r->ncol) * sizeof(double);
    if (hipMalloc(&r->d_D, dbytes) != hipSuccess) {
        r->d_D = nullptr;
        retire(r, UQC_E_NOMEM, "server: density allocation failed");
        return false;
    }
    r->d_R = r->d_D + NN;
    if (hipMemcpy(r->d_D, r->D0.data(), NN * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        retire(r, UQC_E_DEVICE, "server: density upload failed");
        return false;
    }
    r->trace0 = 0;
    for (int i = 0; i < r->nbf; ++i) r->trace0 += r->D0[(size_t)i * r->nbf + i];
    const size_t held = r->basis->device_bytes() + dbytes;
    {
        std::lock_guard<std::mutex> lk(mu);
        used = used - r->footprint + held;  // charge what the request really holds
        r->footprint = held;
        r->slot = free_slots.back();
        free_slots.pop_back();
    }
    r->pos.assign(r->plan->groups.size(), 0);
    r->admit_ms = now_ms();
    return true;
}

void uqc_server::fail_everything(const char* msg) {
    if (ctx) (void)hipStreamSynchronize(ctx->stream);
    for (int ri : inflight)
        for (Req* r : ring[ri].retiring) retire(r, UQC_E_DEVICE, msg);
    for (int ri : inflight) {
        ring[ri].done.clear();
        ring[ri].retiring.clear();
    }
    inflight.clear();
    for (Req* r : active) retire(r, UQC_E_DEVICE, msg);
    active.clear();
}

// Queues one bounded step for the admitted requests (no host wait); false on a launch failure.
bool uqc_server::queue_step(Step& f) {
    hipStream_t s = ctx->stream;
    std::vector<Req*> act = active;
    f.done.clear();
    f.retiring.clear();
    for (Req* r : act) {
        ++r->steps;
        if (r->started) continue;
        uqc_basis* B = r->basis;
        const size_t NN = (size_t)B->nbf * B->nbf;
        if ((r->plan->ntasks && launch_zero((double*)r->plan->d_count, 2 * (size_t)r->plan->ntasks, s) != hipSuccess) ||
            launch_zero(B->d_scal, 8, s) != hipSuccess ||
            launch_prepare(r->d_D, B->d_f, B->d_Dp, B->nbf, (unsigned long long*)(B->d_scal + 1), s) != hipSuccess ||
            launch_zero(B->d_J, 2 * NN, s) != hipSuccess)
            return false;
        std::fill(r->pos.begin(), r->pos.end(), 0LL);
        r->started = true;
    }
    // work left in each request's build: per group the items not yet queued times the FLOPs per item (the last
    // build's, else the static estimate)
    const size_t na = act.size();
    std::vector<double> rem(na, 0.0);
    std::vector<std::vector<double>> per_item(na);
    for (size_t i = 0; i < na; ++i) {
        const Plan& P = *act[i]->plan;
        per_item[i].resize(P.groups.size());
        for (size_t g = 0; g < P.groups.size(); ++g) {
            const LaunchGroup& G = P.groups[g];
            double fi = 0;
            if (act[i]->counted && G.nitems > 0) {
                fi = G.flops / (double)G.nitems;
            } else if (!G.host_tasks.empty()) {
                for (const TaskDev& t : G.host_tasks) fi += item_flops_estimate(G.cls, t) * (double)t.nitems;
                fi /= (double)std::max(1LL, G.nitems);
            }
            per_item[i][g] = std::max(fi, 1.0);
            rem[i] += per_item[i][g] * (double)(G.nitems - act[i]->pos[g]);
        }
    }
    // shares of the step's work: the smallest builds first, each at most an equal share of what is left
    bool waiting;
    {
        std::lock_guard<std::mutex> lk(mu);
        waiting = !queue.empty();
    }
    double left = (na == 1 && !waiting) ? kSoloStepFlops : kStepFlops;
    std::vector<size_t> ord(na);
    for (size_t i = 0; i < na; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return rem[x] < rem[y]; });
    std::vector<double> frac(na, 1.0);
    for (size_t k = 0; k < na; ++k) {
        const size_t i = ord[k];
        const double share = left / (double)(na - k);
        const double take = std::min(rem[i], share);
        frac[i] = rem[i] > 0 ? take / rem[i] : 1.0;
        left -= take;
    }
    // slices: the same fraction of every group's remaining items (at least one), concatenated per (class,
    // precision) over the requests as task descriptors whose item lists start at the slice
    struct Grp {
        int cls, mixed;
        std::vector<TaskDev> tasks;
        std::vector<long long> begin;
        long long items = 0;
        double flops = 0;
    };
    std::vector<Grp> groups;
    for (size_t i = 0; i < na; ++i) {
        Req* r = act[i];
        const Plan& P = *r->plan;
        for (size_t g = 0; g < P.groups.size(); ++g) {
            const LaunchGroup& G = P.groups[g];
            const long long remaining = G.nitems - r->pos[g];
            if (remaining <= 0) continue;
            long long n = frac[i] >= 1.0 ? remaining : (long long)std::ceil(frac[i] * (double)remaining);
            n = std::max(1LL, std::min(n, remaining));
            const long long a = r->pos[g], b = a + n;
            r->pos[g] = b;
            Grp* dst = nullptr;
            for (auto& x : groups)
                if (x.cls == G.cls && x.mixed == G.mixed) dst = &x;
            if (!dst) {
                groups.push_back(Grp{G.cls, G.mixed, {}, {}, 0, 0.0});
                dst = &groups.back();
            }
            dst->flops += per_item[i][g] * (double)n;
            for (size_t t = 0; t < G.host_tasks.size(); ++t) {
                const long long tb = G.host_begin[t], te = tb + G.host_tasks[t].nitems;
                const long long lo = std::max(a, tb), hi = std::min(b, te);
                if (lo >= hi) continue;
                TaskDev td = G.host_tasks[t];
                td.items += (lo - tb);
                td.nitems = hi - lo;
                td.item_begin = dst->items;
                dst->begin.push_back(dst->items);
                dst->items += td.nitems;
                dst->tasks.push_back(td);
            }
        }
    }
    size_t bytes = 0;
    for (auto& g : groups) bytes += g.tasks.size() * (sizeof(TaskDev) + sizeof(long long)) + 512 + 256;
    if (bytes > f.d_bytes) {
        if (f.d_tasks) (void)hipFree(f.d_tasks);
        if (f.h_tasks) (void)hipHostFree(f.h_tasks);
        f.d_tasks = nullptr;
        f.h_tasks = nullptr;
        f.d_bytes = f.h_bytes = 0;
        if (hipMalloc(&f.d_tasks, bytes * 2) != hipSuccess) return false;
        if (hipHostMalloc((void**)&f.h_tasks, bytes * 2) != hipSuccess) return false;
        f.d_bytes = f.h_bytes = bytes * 2;
    }
    std::vector<std::pair<const TaskDev*, const long long*>> ptrs;
    size_t pos = 0;
    for (auto& g : groups) {
        pos = (pos + 255) & ~(size_t)255;
        std::memcpy(f.h_tasks + pos, g.tasks.data(), g.tasks.size() * sizeof(TaskDev));
        const TaskDev* dt = (const TaskDev*)((char*)f.d_tasks + pos);
        pos += g.tasks.size() * sizeof(TaskDev);
        std::memcpy(f.h_tasks + pos, g.begin.data(), g.begin.size() * sizeof(long long));
        const long long* db = (const long long*)((char*)f.d_tasks + pos);
        pos += g.begin.size() * sizeof(long long);
        ptrs.push_back({dt, db});
    }
    // item counters of each group's launches (device only: cleared by each launch), after the uploaded part
    pos = (pos + 255) & ~(size_t)255;
    unsigned* d_queue = (unsigned*)((char*)f.d_tasks + pos);
    static_assert(kQueueWords * sizeof(unsigned) <= 256, "a group's item counters fit its 256 reserved bytes");
    if (pos && hipMemcpyAsync(f.d_tasks, f.h_tasks, pos, hipMemcpyHostToDevice, s) != hipSuccess) return false;
    pos += groups.size() * kQueueWords * sizeof(unsigned);
    // classes side by side on several streams, as in a single build (the most any admitted request asks for):
    // largest first, each to the least-loaded stream, queued alternately from the large and the small end
    int kStreams = 1;
    for (Req* r : act) kStreams = std::max(kStreams, r->opts.streams);
    hipStream_t S[4] = {s, nullptr, nullptr, nullptr};
    for (int k = 1; k < kStreams; ++k)
        if (!(S[k] = ctx_stream(ctx, k))) return false;
    std::vector<size_t> order(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) order[gi] = gi;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return groups[x].flops > groups[y].flops; });
    if (kStreams > 1 && hipEventRecord(ctx->fork, s) != hipSuccess) return false;
    for (int k = 1; k < kStreams; ++k)
        if (hipStreamWaitEvent(S[k], ctx->fork, 0) != hipSuccess) return false;
    double load[4] = {0, 0, 0, 0};
    std::vector<int> gstream(groups.size(), 0);
    for (size_t gi : order) {
        const int k = (int)(std::min_element(load, load + kStreams) - load);
        load[k] += groups[gi].flops;
        gstream[gi] = k;
    }
    for (size_t gi : interleave_ends(order)) {
        const int k = gstream[gi];
        for (long long i0 = 0; i0 < groups[gi].items; i0 += kMaxItemsPerLaunch)
            if (launch_digest(groups[gi].cls, groups[gi].mixed, 1, ptrs[gi].first, ptrs[gi].second,
                              (int)groups[gi].tasks.size(), i0, std::min(kMaxItemsPerLaunch, groups[gi].items - i0),
                              ctx->boys64, ctx->boys32, WorkRedirect{}, d_queue + gi * kQueueWords, S[k]) !=
                hipSuccess)
                return false;
    }
    for (int k = 1; k < kStreams; ++k)
        if (hipEventRecord(ctx->join[k - 1], S[k]) != hipSuccess || hipStreamWaitEvent(s, ctx->join[k - 1], 0) !=
                                                                         hipSuccess)
            return false;
    // builds completed by this step: finalise, read back energy (and counts once), next density or retirement
    std::vector<Req*> keep;
    for (Req* r : act) {
        bool complete = true;
        for (size_t g = 0; g < r->plan->groups.size(); ++g) complete = complete && r->pos[g] >= r->plan->groups[g].nitems;
        if (!complete) {
            keep.push_back(r);
            continue;
        }
        uqc_basis* B = r->basis;
        const size_t N = B->nbf, NN = N * N;
        double* stage = pinned + (size_t)r->slot * slot_doubles();
        const int it = r->iter;
        if (launch_finalize(r->d_D, B->d_J, B->d_K, B->d_f, B->d_io + NN, B->d_io + 2 * NN, B->d_io + 3 * NN,
                            r->opts.exchange_scale, B->d_scal, B->nbf, s) != hipSuccess ||
            hipMemcpyAsync(stage + it, B->d_scal, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
            return false;
        if (!r->counted && r->plan->ntasks &&
            hipMemcpyAsync(stage + UQC_MAX_ITER, r->plan->d_count, 2 * r->plan->ntasks * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s) != hipSuccess)
            return false;
        r->started = false;
        ++r->iter;
        f.done.push_back({r, it});
        if (r->iter >= r->n_iter) {
            f.retiring.push_back(r);
            continue;
        }
        if (launch_normal(r->d_R, (long long)N * r->ncol, r->seed, (unsigned long long)it, s) != hipSuccess ||
            launch_perturb(r->d_D, r->d_R, (int)N, r->ncol, r->eps, r->trace0, B->d_scal + 3, s) != hipSuccess)
            return false;
        keep.push_back(r);
    }
    if (hipEventRecord(f.ev, s) != hipSuccess) return false;
    active.swap(keep);
    return true;
}

// Host side of a finished step: energies and counts of the builds it completed, retirement of finished requests.
void uqc_server::complete(Step& f) {
    for (auto& d : f.done) {
        Req* r = d.first;
        const double* stage = pinned + (size_t)r->slot * slot_doubles();
        r->E2[d.second] = stage[d.second];
        if (!r->counted) {
            std::memcpy(r->plan->h_count.data(), stage + UQC_MAX_ITER,
                        2 * r->plan->ntasks * sizeof(unsigned long long));
            plan_account(*r->plan);
            r->counted = true;
        }
        r->quartets += r->plan->quartets;
    }
    for (Req* r : f.retiring) {
        uqc_basis* B = r->basis;
        const size_t NN = (size_t)B->nbf * B->nbf;
        r->J.resize(NN);
        r->K.resize(NN);
        r->G.resize(NN);
        r->D.resize(NN);
        const bool ok = hipMemcpy(r->J.data(), B->d_io + NN, NN * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess &&
                        hipMemcpy(r->K.data(), B->d_io + 2 * NN, NN * sizeof(double), hipMemcpyDeviceToHost) ==
                            hipSuccess &&
                        hipMemcpy(r->G.data(), B->d_io + 3 * NN, NN * sizeof(double), hipMemcpyDeviceToHost) ==
                            hipSuccess &&
                        hipMemcpy(r->D.data(), r->d_D, NN * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess;
        retire(r, ok ? UQC_OK : UQC_E_DEVICE, ok ? "" : "server: result copy failed");
    }
    f.done.clear();
    f.retiring.clear();
}

void uqc_server::loop() {
    (void)hipSetDevice(ctx->device);
    for (;;) {
        std::vector<Req*> admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty() || !inflight.empty(); });
            if (stop && queue.empty() && active.empty() && inflight.empty()) return;
            // arrival order; a request that does not fit is passed over until it has waited kMaxSkipMs
            const double now = now_ms();
            // (a slot stays taken until its request has retired, which can be a step after its last build)
            for (auto it = queue.begin(); it != queue.end() && admit.size() < free_slots.size();) {
                Req* r = *it;
                if (used + r->footprint <= budget) {
                    used += r->footprint;
                    admit.push_back(r);
                    it = queue.erase(it);
                    continue;
                }
                if (now - r->submit_ms > kMaxSkipMs) break;
                ++it;
            }
        }
        for (Req* r : admit)
            if (admit_one(r)) active.push_back(r);
        if (!active.empty()) {
            if ((int)inflight.size() >= kInFlight) {  // make room: wait for the oldest step
                Step& old = ring[inflight.front()];
                if (hipEventSynchronize(old.ev) != hipSuccess) {
                    fail_everything("server: step failed on the device");
                    continue;
                }
                inflight.pop_front();
                complete(old);
            }
            Step& f = ring[next_ring];
            if (!queue_step(f)) {
                fail_everything("server: step launch failed");
                continue;
            }
            inflight.push_back(next_ring);
            next_ring = (next_ring + 1) % kInFlight;
        } else if (!inflight.empty()) {  // nothing more to queue: finish what is on the device
            Step& old = ring[inflight.front()];
            if (hipEventSynchronize(old.ev) != hipSuccess) {
                fail_everything("server: step failed on the device");
                continue;
            }
            inflight.pop_front();
            complete(old);
        }
    }
}

uqc_status uqc_server_create(uqc_ctx* ctx, size_t hbm_budget_bytes, int max_slots, uqc_server** out) {
    if (!ctx || !out) return uqc_fail(UQC_E_ARG, "uqc_server_create: NULL argument");
    if (max_slots < 1 || max_slots > 1024 || hbm_budget_bytes == 0)
        return uqc_fail(UQC_E_ARG, "uqc_server_create: bad budget or slots (1..1024)");
    *out = nullptr;
    uqc_server* s = new uqc_server();
    UQC_HIP(hipSetDevice(ctx->device));
    // a non-blocking stream, so that the admission context's synchronous copies do not wait for queued steps
    if (hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return uqc_fail(UQC_E_DEVICE, "uqc_server_create: stream creation failed");
    }
    uqc_status st = uqc_init(ctx->device, s->own_stream, &s->ctx);
    if (st == UQC_OK) st = uqc_init(ctx->device, nullptr, &s->actx);
    bool ok = st == UQC_OK;
    for (int i = 0; ok && i < kInFlight; ++i)
        ok = hipEventCreateWithFlags(&s->ring[i].ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s->pinned, (size_t)max_slots * uqc_server::slot_doubles() * sizeof(double)) ==
                   hipSuccess;
    if (!ok) {
        for (auto& f : s->ring)
            if (f.ev) (void)hipEventDestroy(f.ev);
        if (s->pinned) (void)hipHostFree(s->pinned);
        if (s->actx) uqc_finalize(s->actx);
        if (s->ctx) uqc_finalize(s->ctx);
        (void)hipStreamDestroy(s->own_stream);
        delete s;
        return st != UQC_OK ? st : uqc_fail(UQC_E_NOMEM, "uqc_server_create: staging allocation failed");
    }
    for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->t0 = std::chrono::steady_clock::now();
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return UQC_OK;
}

uqc_status uqc_submit(uqc_server* s, const uqc_request* q, long long* ticket) {
    if (!s || !q || !ticket) return uqc_fail(UQC_E_ARG, "uqc_submit: NULL argument");
    if (q->nshell <= 0 || !q->l || !q->nprim || !q->center || !q->alpha || !q->coef || !q->D0)
        return uqc_fail(UQC_E_ARG, "uqc_submit: incomplete request");
    if (q->n_iter < 1 || q->n_iter > UQC_MAX_ITER || q->ncol < 1 || !(q->eps >= 0 && q->eps <= 1))
        return uqc_fail(UQC_E_ARG, "uqc_submit: n_iter must be 1..64, ncol >= 1, eps in [0, 1]");
    Req* r = new Req();
    r->nshell = q->nshell;
    r->l.assign(q->l, q->l + q->nshell);
    r->nprim.assign(q->nprim, q->nprim + q->nshell);
    size_t np = 0;
    int nbf = 0;
    for (int i = 0; i < q->nshell; ++i) {
        if (r->l[i] < 0 || r->l[i] > 2 || r->nprim[i] < 1 || r->nprim[i] > kMaxK) {
            const uqc_status e = (r->l[i] > 2 || r->nprim[i] > kMaxK) ? UQC_E_UNSUPPORTED : UQC_E_ARG;
            delete r;
            return uqc_fail(e, "uqc_submit: l must be 0..2 and nprim 1..16");
        }
        np += r->nprim[i];
        nbf += (r->l[i] + 1) * (r->l[i] + 2) / 2;
    }
    r->center.assign(q->center, q->center + 3 * (size_t)q->nshell);
    r->alpha.assign(q->alpha, q->alpha + np);
    r->coef.assign(q->coef, q->coef + np);
    r->nbf = nbf;
    r->D0.assign(q->D0, q->D0 + (size_t)nbf * nbf);
    double md = 0, ma = 0;
    for (int i = 0; i < nbf; ++i)
        for (int j = 0; j < nbf; ++j) {
            const double v = r->D0[(size_t)i * nbf + j];
            if (!std::isfinite(v)) md = INFINITY;
            md = std::max(md, std::fabs(v - r->D0[(size_t)j * nbf + i]));
            ma = std::max(ma, std::fabs(v));
        }
    if (!(md <= 1e-12 * ma)) {
        delete r;
        return uqc_fail(UQC_E_NOT_SYMMETRIC, "uqc_submit: D0 is not symmetric (or not finite)");
    }
    r->n_iter = q->n_iter;
    r->ncol = q->ncol;
    r->eps = q->eps;
    r->seed = q->seed;
    r->opts = q->opts;
    if (const uqc_status e = check_fock_opts(r->opts, "uqc_submit")) {
        delete r;
        return e;
    }
    r->footprint = estimate_footprint(*r);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        delete r;
        return uqc_fail(UQC_E_BUSY, "uqc_submit: server is shutting down");
    }
    if (r->footprint > s->budget) {
        delete r;
        return uqc_fail(UQC_E_NOMEM, "uqc_submit: request exceeds the whole HBM budget");
    }
    r->ticket = s->next_ticket++;
    r->submit_ms = s->now_ms();
    s->table[r->ticket] = r;
    s->queue.push_back(r);
    *ticket = r->ticket;
    s->cv_work.notify_all();
    return UQC_OK;
}

uqc_status uqc_poll(uqc_server* s, long long ticket, uqc_result* res) {
    if (!s) return uqc_fail(UQC_E_ARG, "uqc_poll: NULL server");
    Req* r = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->table.find(ticket);
        if (it == s->table.end()) return uqc_fail(UQC_E_NOT_FOUND, "uqc_poll: unknown ticket");
        r = it->second;
        if (r->status == UQC_PENDING) return UQC_PENDING;
        s->table.erase(it);
    }
    const uqc_status st = r->status;
    if (res) {
        res->n_iter = r->iter;
        res->nbf = r->nbf;
        for (int i = 0; i < UQC_MAX_ITER; ++i) res->E2[i] = i < r->iter ? r->E2[i] : 0.0;
        res->submit_ms = r->submit_ms;
        res->admit_ms = r->admit_ms;
        res->finish_ms = r->finish_ms;
        res->quartets = r->quartets;
        res->device_bytes = (long long)r->footprint;
        res->steps = r->steps;
        const size_t NN = (size_t)r->nbf * r->nbf;
        if (st == UQC_OK) {
            if (res->J) std::memcpy(res->J, r->J.data(), NN * sizeof(double));
            if (res->K) std::memcpy(res->K, r->K.data(), NN * sizeof(double));
            if (res->G) std::memcpy(res->G, r->G.data(), NN * sizeof(double));
            if (res->D) std::memcpy(res->D, r->D.data(), NN * sizeof(double));
        }
    }
    std::string msg = r->error;
    delete r;
    if (st != UQC_OK) return uqc_fail(st, "uqc_poll: request failed: " + msg);
    return UQC_OK;
}

uqc_status uqc_server_drain(uqc_server* s) {
    if (!s) return uqc_fail(UQC_E_ARG, "uqc_server_drain: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] {
        if (!s->queue.empty()) return false;
        for (auto& kv : s->table)
            if (kv.second->status == UQC_PENDING) return false;
        return true;
    });
    return UQC_OK;
}

uqc_status uqc_server_destroy(uqc_server* s) {
    if (!s) return uqc_fail(UQC_E_ARG, "uqc_server_destroy: NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->table) delete kv.second;
    for (auto& f : s->ring) {
        if (f.d_tasks) (void)hipFree(f.d_tasks);
        if (f.h_tasks) (void)hipHostFree(f.h_tasks);
        if (f.ev) (void)hipEventDestroy(f.ev);
    }
    if (s->pinned) (void)hipHostFree(s->pinned);
    uqc_finalize(s->actx);
    uqc_finalize(s->ctx);
    (void)hipStreamDestroy(s->own_stream);
    delete s;
    return UQC_OK;
}
