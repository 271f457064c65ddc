// Serving loop of libuqc: continuous batching of Fock-build requests.
//
// A background thread owns a private context (its own stream).  Each step it
//   1. admits queued requests in arrival order while a slot is free and the request's device footprint fits the
//      remaining HBM budget (first-in first-out: a request that does not fit blocks the ones behind it, so none
//      starves);
//   2. runs one Fock build for every admitted request at once: per-request density preparation, then ONE launch
//      per (angular-momentum class, precision) whose work list concatenates the quartet tasks of all admitted
//      requests (each task carries its own request's density and J/K accumulators), then per-request finalisation;
//   3. advances every request to its next density, generated on the device, or retires it (results copied to the
//      host, device memory released, budget returned).
// Requests admitted while others are mid-way join at the next step, so their work shares launches with the
// requests already on the device.
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

struct Req {
    long long ticket = 0;
    // owned copies of the request arrays
    std::vector<int> l, nprim;
    std::vector<double> center, alpha, coef, D0;
    int nshell = 0, nbf = 0, n_iter = 1, ncol = 1;
    double eps = 0;
    unsigned long long seed = 0;
    uqc_fock_opts opts{};
    size_t footprint = 0;
    // device state
    uqc_basis* basis = nullptr;
    Plan* plan = nullptr;
    double* d_D = nullptr;   // current density (nbf*nbf), then R (nbf*ncol)
    double* d_R = nullptr;
    double trace0 = 0;
    int iter = 0;
    // results
    uqc_status status = UQC_PENDING;
    std::string error;
    double E2[UQC_MAX_ITER] = {0};
    long long quartets = 0;
    double submit_ms = 0, admit_ms = 0, finish_ms = 0;
    std::vector<double> J, K, G, D;
};

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
    bytes += prim_pairs * kNumFields * sizeof(double) + pairs * (4 * sizeof(double) + 2 * sizeof(int));
    bytes += pairs * 2 * (2 * sizeof(int) + sizeof(long long)) + 64 * 1024;  // screened work lists (both precisions)
    return bytes;
}

}  // namespace

struct uqc_server {
    uqc_ctx* ctx = nullptr;  // private context: own stream, own Boys tables
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
    // per-step device buffer for the concatenated task lists
    void* d_tasks = nullptr;
    size_t d_tasks_bytes = 0;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    void loop();
    bool admit_one(Req* r);
    void retire(Req* r, uqc_status st, const std::string& msg);
    bool step();
};

void uqc_server::retire(Req* r, uqc_status st, const std::string& msg) {
    if (r->d_D) (void)hipFree(r->d_D);
    r->d_D = r->d_R = nullptr;
    if (r->basis) uqc_basis_destroy(r->basis);
    r->basis = nullptr;
    r->plan = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    used -= r->footprint;
    r->status = st;
    r->error = msg;
    r->finish_ms = now_ms();
    cv_done.notify_all();
}

bool uqc_server::admit_one(Req* r) {
    uqc_status st = uqc_basis_create(ctx, r->nshell, r->l.data(), r->nprim.data(), r->center.data(),
                                     r->alpha.data(), r->coef.data(), &r->basis);
    if (st != UQC_OK) {
        retire(r, st, uqc_last_error());
        return false;
    }
    r->plan = get_plan(r->basis, r->opts.schwarz_tau, r->opts.precision, r->opts.fp64_bound, &st);
    const size_t NN = (size_t)r->nbf * r->nbf;
    if (!r->plan) {
        retire(r, st, uqc_last_error());
        return false;
    }
    if (hipMalloc(&r->d_D, (NN + (size_t)r->nbf * r->ncol) * sizeof(double)) != hipSuccess) {
        r->d_D = nullptr;
        retire(r, UQC_E_NOMEM, "server: density allocation failed");
        return false;
    }
    r->d_R = r->d_D + NN;
    if (hipMemcpyAsync(r->d_D, r->D0.data(), NN * sizeof(double), hipMemcpyHostToDevice, ctx->stream) !=
        hipSuccess) {
        retire(r, UQC_E_DEVICE, "server: density upload failed");
        return false;
    }
    r->trace0 = 0;
    for (int i = 0; i < r->nbf; ++i) r->trace0 += r->D0[(size_t)i * r->nbf + i];
    r->admit_ms = now_ms();
    return true;
}

// One build for every admitted request; returns false on a device failure (all active requests are failed).
bool uqc_server::step() {
    hipStream_t s = ctx->stream;
    std::vector<Req*> act = active;
    auto fail_all = [&](const char* msg) {
        for (Req* r : act) retire(r, UQC_E_DEVICE, msg);
        active.clear();
        return false;
    };
    for (Req* r : act) {
        uqc_basis* B = r->basis;
        const size_t NN = (size_t)B->nbf * B->nbf;
        if ((r->plan->ntasks && launch_zero((double*)r->plan->d_count, 2 * (size_t)r->plan->ntasks, s) != hipSuccess) ||
            launch_zero(B->d_scal, 8, s) != hipSuccess ||
            launch_prepare(r->d_D, B->d_f, B->d_Dp, B->nbf, (unsigned long long*)(B->d_scal + 1), s) != hipSuccess ||
            launch_zero(B->d_J, 2 * NN, s) != hipSuccess)
            return fail_all("server: preparation launch failed");
    }
    // concatenate the tasks of all requests per (class, precision)
    struct G {
        int cls, mixed;
        std::vector<TaskDev> tasks;
        std::vector<long long> begin;
        long long items = 0;
        double flops = 0;  // of the requests' previous builds (0 before the first)
    };
    std::vector<G> groups;
    for (Req* r : act)
        for (auto& g : r->plan->groups) {
            G* dst = nullptr;
            for (auto& x : groups)
                if (x.cls == g.cls && x.mixed == g.mixed) dst = &x;
            if (!dst) {
                groups.push_back(G{g.cls, g.mixed, {}, {}, 0, 0.0});
                dst = &groups.back();
            }
            dst->flops += g.flops;
            for (TaskDev t : g.host_tasks) {
                t.item_begin = dst->items;
                dst->begin.push_back(dst->items);
                dst->items += t.nitems;
                dst->tasks.push_back(t);
            }
        }
    std::sort(groups.begin(), groups.end(), [](const G& a, const G& b) {
        return a.cls != b.cls ? a.cls > b.cls : a.mixed < b.mixed;  // heavy classes first
    });
    size_t bytes = 0;
    for (auto& g : groups) bytes += g.tasks.size() * (sizeof(TaskDev) + sizeof(long long)) + 512;
    if (bytes > d_tasks_bytes) {
        if (d_tasks) (void)hipFree(d_tasks);
        d_tasks = nullptr;
        d_tasks_bytes = 0;
        if (hipMalloc(&d_tasks, bytes * 2) != hipSuccess) return fail_all("server: task buffer allocation failed");
        d_tasks_bytes = bytes * 2;
    }
    std::vector<char> host(bytes);
    std::vector<std::pair<const TaskDev*, const long long*>> ptrs;
    size_t pos = 0;
    for (auto& g : groups) {
        pos = (pos + 255) & ~(size_t)255;
        std::memcpy(host.data() + pos, g.tasks.data(), g.tasks.size() * sizeof(TaskDev));
        const TaskDev* dt = (const TaskDev*)((char*)d_tasks + pos);
        pos += g.tasks.size() * sizeof(TaskDev);
        std::memcpy(host.data() + pos, g.begin.data(), g.begin.size() * sizeof(long long));
        const long long* db = (const long long*)((char*)d_tasks + pos);
        pos += g.begin.size() * sizeof(long long);
        ptrs.push_back({dt, db});
    }
    if (pos && hipMemcpyAsync(d_tasks, host.data(), pos, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail_all("server: task upload failed");
    // classes side by side on several streams, as in a single build (the most any admitted request asks for):
    // largest first, each to the least-loaded stream (weights: FLOPs of the previous step when every group has
    // them, else work items), queued alternately from the large and the small end
    int kStreams = 1;
    for (Req* r : act) kStreams = std::max(kStreams, r->opts.streams);
    hipStream_t S[4] = {s, nullptr, nullptr, nullptr};
    for (int k = 1; k < kStreams; ++k)
        if (!(S[k] = ctx_stream(ctx, k))) return fail_all("server: stream creation failed");
    bool have_flops = true;
    for (auto& g : groups) have_flops = have_flops && g.flops > 0;
    std::vector<size_t> order(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) order[gi] = gi;
    auto weight = [&](size_t gi) { return have_flops ? groups[gi].flops : (double)groups[gi].items; };
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return weight(x) > weight(y); });
    if (kStreams > 1 && hipEventRecord(ctx->fork, s) != hipSuccess) return fail_all("server: event record failed");
    for (int k = 1; k < kStreams; ++k)
        if (hipStreamWaitEvent(S[k], ctx->fork, 0) != hipSuccess) return fail_all("server: stream wait failed");
    double load[4] = {0, 0, 0, 0};
    std::vector<int> gstream(groups.size(), 0);
    for (size_t gi : order) {
        const int k = (int)(std::min_element(load, load + kStreams) - load);
        load[k] += weight(gi);
        gstream[gi] = k;
    }
    for (size_t gi : interleave_ends(order)) {
        const int k = gstream[gi];
        for (long long i0 = 0; i0 < groups[gi].items; i0 += kMaxItemsPerLaunch)
            if (launch_digest(groups[gi].cls, groups[gi].mixed, 1, ptrs[gi].first, ptrs[gi].second,
                              (int)groups[gi].tasks.size(), i0, std::min(kMaxItemsPerLaunch, groups[gi].items - i0),
                              ctx->boys64, ctx->boys32, WorkRedirect{}, S[k]) != hipSuccess)
                return fail_all("server: class launch failed");
    }
    for (int k = 1; k < kStreams; ++k)
        if (hipEventRecord(ctx->join[k - 1], S[k]) != hipSuccess || hipStreamWaitEvent(s, ctx->join[k - 1], 0) !=
                                                                         hipSuccess)
            return fail_all("server: stream join failed");
    std::vector<double> e2(act.size());
    for (size_t i = 0; i < act.size(); ++i) {
        uqc_basis* B = act[i]->basis;
        const size_t NN = (size_t)B->nbf * B->nbf;
        if (launch_finalize(act[i]->d_D, B->d_J, B->d_K, B->d_f, B->d_io + NN, B->d_io + 2 * NN, B->d_io + 3 * NN,
                            act[i]->opts.exchange_scale, B->d_scal, B->nbf, s) != hipSuccess ||
            hipMemcpyAsync(&e2[i], B->d_scal, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            (act[i]->plan->ntasks &&
             hipMemcpyAsync(act[i]->plan->h_count.data(), act[i]->plan->d_count,
                            2 * act[i]->plan->ntasks * sizeof(unsigned long long), hipMemcpyDeviceToHost, s) !=
                                hipSuccess))
            return fail_all("server: finalize failed");
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail_all("server: step failed on the device");
    std::vector<Req*> keep;
    for (size_t i = 0; i < act.size(); ++i) {
        Req* r = act[i];
        r->E2[r->iter] = e2[i];
        plan_account(*r->plan);
        r->quartets += r->plan->quartets;
        ++r->iter;
        uqc_basis* B = r->basis;
        const size_t N = B->nbf, NN = N * N;
        if (r->iter >= r->n_iter) {
            r->J.resize(NN);
            r->K.resize(NN);
            r->G.resize(NN);
            r->D.resize(NN);
            bool ok = hipMemcpyAsync(r->J.data(), B->d_io + NN, NN * sizeof(double), hipMemcpyDeviceToHost, s) ==
                          hipSuccess &&
                      hipMemcpyAsync(r->K.data(), B->d_io + 2 * NN, NN * sizeof(double), hipMemcpyDeviceToHost, s) ==
                          hipSuccess &&
                      hipMemcpyAsync(r->G.data(), B->d_io + 3 * NN, NN * sizeof(double), hipMemcpyDeviceToHost, s) ==
                          hipSuccess &&
                      hipMemcpyAsync(r->D.data(), r->d_D, NN * sizeof(double), hipMemcpyDeviceToHost, s) ==
                          hipSuccess &&
                      hipStreamSynchronize(s) == hipSuccess;
            retire(r, ok ? UQC_OK : UQC_E_DEVICE, ok ? "" : "server: result copy failed");
        } else {
            if (launch_normal(r->d_R, (long long)N * r->ncol, r->seed, (unsigned long long)r->iter - 1, s) !=
                    hipSuccess ||
                launch_perturb(r->d_D, r->d_R, (int)N, r->ncol, r->eps, r->trace0, B->d_scal + 3, s) != hipSuccess) {
                retire(r, UQC_E_DEVICE, "server: perturbation launch failed");
                continue;
            }
            keep.push_back(r);
        }
    }
    active.swap(keep);
    return true;
}

void uqc_server::loop() {
    (void)hipSetDevice(ctx->device);
    for (;;) {
        std::vector<Req*> admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
            if (stop && queue.empty() && active.empty()) return;
            while (!queue.empty() && (int)(active.size() + admit.size()) < max_slots) {
                Req* r = queue.front();
                if (used + r->footprint > budget) break;  // FIFO: wait for memory to free up
                used += r->footprint;
                queue.pop_front();
                admit.push_back(r);
            }
        }
        for (Req* r : admit)
            if (admit_one(r)) active.push_back(r);
        if (!active.empty()) step();
    }
}

uqc_status uqc_server_create(uqc_ctx* ctx, size_t hbm_budget_bytes, int max_slots, uqc_server** out) {
    if (!ctx || !out) return uqc_fail(UQC_E_ARG, "uqc_server_create: NULL argument");
    if (max_slots < 1 || hbm_budget_bytes == 0) return uqc_fail(UQC_E_ARG, "uqc_server_create: bad budget or slots");
    *out = nullptr;
    uqc_server* s = new uqc_server();
    uqc_status st = uqc_init(ctx->device, nullptr, &s->ctx);
    if (st != UQC_OK) {
        delete s;
        return st;
    }
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
    if (!std::isfinite(r->opts.exchange_scale)) {
        delete r;
        return uqc_fail(UQC_E_ARG, "uqc_submit: exchange_scale is not finite");
    }
    if (r->opts.streams < 0 || r->opts.streams > 4) {
        delete r;
        return uqc_fail(UQC_E_ARG, "uqc_submit: streams must be in 0..4");
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
    if (s->d_tasks) (void)hipFree(s->d_tasks);
    uqc_finalize(s->ctx);
    delete s;
    return UQC_OK;
}
