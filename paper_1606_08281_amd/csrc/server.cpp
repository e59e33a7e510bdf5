// server.cpp -- continuous-batching likelihood server.
//
// One worker thread drives one HIP stream.  Each iteration it (1) admits
// queued requests, first come first served, while filter slots, device arena
// memory and pinned staging memory are free (inputs are staged through
// pinned memory and copied asynchronously, then k_admit fills the request's
// filter slots); (2) runs one engine iteration: every resident filter,
// whatever its request, network, particle count or trajectory length,
// advances by one observation interval in shared launches (one propagation
// launch per (network, precision) group, one weighting launch); (3) for each
// request whose longest trajectory just finished, enqueues its per-theta
// reduction and the copy of its results into pinned memory, followed by an
// event.  Requests are complete when their event has passed; their slots and
// memory are then released.  At most `max_inflight` iterations are enqueued
// ahead of the GPU, which bounds how long a new request waits to join.
// A request withdrawn while queued (lik_server_cancel, or its own time limit)
// leaves the queue at once; one withdrawn while resident has its slots
// stopped by a kernel enqueued behind the iterations already in flight, and
// its slots and memory are released once that kernel has passed, so no
// later request can be placed in memory an earlier iteration still uses.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.hpp"

using namespace lik;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit range allocator over [0, size) in units of `align`.
class RangeAlloc {
   public:
    void init(size_t size, size_t align) {
        align_ = align;
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t *off) {
        n = (n + align_ - 1) / align_ * align_;
        if (n == 0) n = align_;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_[*off] = n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t n = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    size_t high_water() const {  // end of the last used range
        return used_.empty() ? 0 : used_.rbegin()->first + used_.rbegin()->second;
    }

   private:
    size_t align_ = 1;
    std::map<size_t, size_t> free_, used_;
};

struct Request {
    uint64_t ticket;
    lik_network *net;
    lik_obs_model obs;
    int32_t precision, n_theta, M, H, Hp, t_max;
    uint64_t seed, event_cap;
    std::vector<double> theta, t_obs, y, t0;
    std::vector<uint32_t> ids;
    std::vector<int32_t> offsets, x0, x0_hi;  // x0_hi empty: fixed initial counts
    Clock::time_point submitted;
    bool has_deadline = false;  // its own time limit (lik_request.timeout_us)
    Clock::time_point deadline;
    // withdrawal (cancel or time limit): the status every theta reports
    bool withdraw = false;
    int32_t withdraw_status = LIK_STATUS_OK;
    // placement, once admitted
    int group = -1;
    size_t slot = 0, dev_off = 0, pin_off = 0;
    int iterations_left = 0;
    hipEvent_t done_event = nullptr;
    bool finishing = false;
    // results
    bool done = false;
    std::vector<double> loglik;
    std::vector<int32_t> status;

    size_t F() const { return (size_t)n_theta * M; }
    size_t input_bytes() const {
        return align256(theta.size() * 8) + align256(ids.size() * 4) +
               align256(offsets.size() * 4) + align256(t_obs.size() * 8) + align256(y.size() * 8) +
               align256(t0.size() * 8) + align256(x0.size() * 4) + align256(x0_hi.size() * 4);
    }
    size_t device_bytes() const {
        return input_bytes() + align256(request_state_bytes((int64_t)F(), net->U, Hp));
    }
};

struct Group {
    lik_network *net = nullptr;
    int precision = 0;
    int residents = 0;
    GroupLaunch launch;
};

}  // namespace

struct lik_server {
    lik_server_opts opts;
    int device = 0;
    bool persistent = false;  // persistent propagation kernels for small networks
    hipStream_t stream = nullptr;
    char *dev_base = nullptr;       // engine table + arena
    char *arena = nullptr;
    size_t arena_bytes = 0;
    char *pinned = nullptr;         // staging for inputs, then results
    double *res_loglik = nullptr;   // pinned [max_filters]
    int32_t *res_status = nullptr;  // pinned [max_filters]
    double *dev_loglik = nullptr;   // device [max_filters]
    int32_t *dev_status = nullptr;  // device [max_filters]
    FilterDesc *desc = nullptr;
    EngineArgs e;
    RangeAlloc slots, dmem, pmem;
    Group groups[kMaxGroups];

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::vector<std::shared_ptr<Request>> resident;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
    std::deque<hipEvent_t> inflight;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::thread worker;

    // statistics
    uint64_t n_submitted = 0, n_completed = 0, n_evals = 0, n_iterations = 0, n_cancelled = 0;
    std::vector<double> latencies_us;
    double busy_s = 0.0;
    bool busy = false;
    std::chrono::steady_clock::time_point busy_since;
    std::string worker_error;
};

namespace {

int validate_request(const lik_server *srv, const lik_request *q) {
    if (!q) return fail(LIK_EINVAL, "request is NULL");
    if (q->reserved != 0) return fail(LIK_EINVAL, "reserved must be 0");
    if (q->timeout_us < 0) return fail(LIK_EINVAL, "timeout_us must be >= 0");
    lik_eval_opts o = {q->precision, LIK_KERNEL_AUTO, q->event_cap, q->theta_ids, 0, 0};
    int rc = check_common(q->net, &q->obs, &o, q->n_theta, q->data.n_traj, q->n_particles);
    if (rc) return rc;
    int t_max = 0;
    int64_t total = 0;
    rc = check_offsets(q->data.obs_offsets, q->data.n_traj, &t_max, &total);
    if (rc) return rc;
    if (q->n_theta < 1) return fail(LIK_EINVAL, "a request needs at least one theta");
    if (!q->theta || !q->data.t_obs || !q->data.y || !q->data.t0 || !q->data.x0)
        return fail(LIK_EINVAL, "NULL input pointer");
    rc = check_host_data(q->net, &q->obs, &q->data, q->n_theta, q->theta_ids);
    if (rc) return rc;
    if ((int64_t)q->n_theta * q->data.n_traj > srv->opts.max_filters)
        return fail(LIK_EINVAL, "request has more filters than the server has slots");
    return LIK_OK;
}

// Copies inputs to pinned staging, then to the arena; fills the slots.
hipError_t admit(lik_server *S, Request &r) {
    char *pin = S->pinned + r.pin_off;
    char *dev = S->arena + r.dev_off;
    size_t off = 0;
    auto put = [&](const void *src, size_t bytes) -> void * {
        void *d = dev + off;
        if (bytes) memcpy(pin + off, src, bytes);
        off += align256(bytes);
        return bytes ? d : nullptr;
    };
    RequestArgs a;
    memset(&a, 0, sizeof(a));
    a.theta = (const double *)put(r.theta.data(), r.theta.size() * 8);
    a.theta_ids = (const uint32_t *)put(r.ids.data(), r.ids.size() * 4);
    a.obs_offsets = (const int32_t *)put(r.offsets.data(), r.offsets.size() * 4);
    a.t_obs = (const double *)put(r.t_obs.data(), r.t_obs.size() * 8);
    a.y = (const double *)put(r.y.data(), r.y.size() * 8);
    a.t0 = (const double *)put(r.t0.data(), r.t0.size() * 8);
    a.x0 = (const int32_t *)put(r.x0.data(), r.x0.size() * 4);
    a.x0_hi = (const int32_t *)put(r.x0_hi.data(), r.x0_hi.size() * 4);
    hipError_t err = hipMemcpyAsync(dev, pin, off, hipMemcpyHostToDevice, S->stream);
    if (err != hipSuccess) return err;
    a.state = (int32_t *)(dev + off);
    a.n_theta = r.n_theta;
    a.M = r.M;
    a.H = r.H;
    a.Hp = r.Hp;
    a.U = r.net->U;
    a.R = r.net->R;
    a.P = r.obs.n_observed;
    a.obs_kind = r.obs.kind;
    a.group = r.group;
    a.precision = r.precision;
    for (int k = 0; k < LIK_MAX_OBSERVED; ++k) a.obs_species[k] = r.obs.species[k];
    a.sigma = r.obs.sigma;
    a.gain = r.obs.gain;
    a.bg_mean = r.obs.bg_mean;
    a.bg_sd = r.obs.bg_sd;
    a.seed = r.seed;
    a.event_cap = (uint32_t)(r.event_cap ? r.event_cap : LIK_DEFAULT_EVENT_CAP);
    a.base = (int32_t)r.slot;
    fill_reactant_tables(a, r.net->kind, r.net->s1, r.net->s2, r.net->R);
    err = launch_admit(S->desc, S->e, a, S->stream);
    if (err == hipSuccess && a.x0_hi)
        err = launch_init_start(S->desc, (int32_t)r.slot, (int32_t)r.F(), S->stream);
    return err;
}

int find_group(lik_server *S, lik_network *net, int precision) {
    int free_g = -1;
    for (int g = 0; g < kMaxGroups; ++g) {
        if (S->groups[g].residents > 0 && S->groups[g].net == net &&
            S->groups[g].precision == precision)
            return g;
        if (S->groups[g].residents == 0 && free_g < 0) free_g = g;
    }
    return free_g;
}

// Tries to place the queue head; false if it does not fit yet.
bool try_place(lik_server *S, Request &r, std::string *err) {
    const int g = find_group(S, r.net, r.precision);
    if (g < 0) return false;
    size_t slot, doff, poff;
    if (!S->slots.alloc(r.F(), &slot)) return false;
    if (!S->dmem.alloc(r.device_bytes(), &doff)) {
        S->slots.release(slot);
        return false;
    }
    if (!S->pmem.alloc(r.input_bytes(), &poff)) {
        S->slots.release(slot);
        S->dmem.release(doff);
        return false;
    }
    Group &G = S->groups[g];
    if (G.residents == 0) {
        G.net = r.net;
        G.precision = r.precision;
        G.launch = GroupLaunch();
        G.launch.netargs = generic_netargs(*r.net);
        G.launch.umax = r.net->umax;
        G.launch.rmax = r.net->rmax;
        G.launch.precision = r.precision;
        G.launch.persistent = S->persistent && r.net->R <= kPersistentMaxR;
        G.launch.persistent_waves = persistent_waves();
        if (S->opts.kernel != LIK_KERNEL_GENERIC) {
            G.launch.spec = specialized_kernel(*r.net, r.precision, err);
            if (G.launch.spec && G.launch.persistent)
                G.launch.spec_p = specialized_kernel(*r.net, r.precision, err, kSpecPersistent);
            // an unavailable specialisation leaves the group on the generic kernel
        }
    }
    G.residents += 1;
    r.group = g;
    r.slot = slot;
    r.dev_off = doff;
    r.pin_off = poff;
    r.iterations_left = r.t_max;
    return true;
}

void release(lik_server *S, Request &r) {
    S->slots.release(r.slot);
    S->dmem.release(r.dev_off);
    S->pmem.release(r.pin_off);
    S->groups[r.group].residents -= 1;
}

// Results of a withdrawn request: NaN log-likelihoods and its status.
void complete_withdrawn(lik_server *S, Request &r) {
    r.loglik.assign((size_t)r.n_theta, __builtin_nan(""));
    r.status.assign((size_t)r.n_theta, r.withdraw_status);
    r.done = true;
    S->n_cancelled += 1;
    S->cv_done.notify_all();
}

// Withdraws a request (caller holds the lock): a queued one leaves the queue
// and completes now; a resident one is stopped by the worker.  A request
// already finishing (results on their way) is left alone.
void withdraw(lik_server *S, const std::shared_ptr<Request> &r, int32_t status) {
    if (r->done || r->finishing || r->withdraw) return;
    r->withdraw = true;
    r->withdraw_status = status;
    if (r->group < 0) {
        auto it = std::find(S->queue.begin(), S->queue.end(), r);
        if (it != S->queue.end()) S->queue.erase(it);
        complete_withdrawn(S, *r);
    }
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const size_t k = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
    return v[k];
}

void worker_main(lik_server *S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // requests past their own time limit are withdrawn
        const Clock::time_point now = Clock::now();
        std::vector<std::shared_ptr<Request>> expired;
        for (auto &q : S->queue)
            if (q->has_deadline && now >= q->deadline) expired.push_back(q);
        for (auto &q : expired) withdraw(S, q, LIK_STATUS_TIMED_OUT);  // leaves the queue
        for (auto &r : S->resident)
            if (r->has_deadline && now >= r->deadline) withdraw(S, r, LIK_STATUS_TIMED_OUT);
        // withdrawn resident requests: their slots stop behind the iterations
        // already enqueued; slots and memory are released when that has passed
        for (auto &r : S->resident) {
            if (!r->withdraw || r->finishing) continue;
            if (launch_stop(S->e, (int32_t)r->slot, (int32_t)r->F(), S->stream) != hipSuccess)
                S->worker_error = "stop launch failed";
            (void)hipEventCreateWithFlags(&r->done_event, hipEventDisableTiming);
            (void)hipEventRecord(r->done_event, S->stream);
            r->finishing = true;
            r->iterations_left = 0;
        }
        // completions whose results have reached pinned memory
        for (auto it = S->resident.begin(); it != S->resident.end();) {
            Request &r = **it;
            if (r.finishing && hipEventQuery(r.done_event) == hipSuccess) {
                (void)hipEventDestroy(r.done_event);
                r.done_event = nullptr;
                release(S, r);
                if (r.withdraw) {
                    complete_withdrawn(S, r);
                } else {
                    r.loglik.assign(S->res_loglik + r.slot, S->res_loglik + r.slot + r.n_theta);
                    r.status.assign(S->res_status + r.slot, S->res_status + r.slot + r.n_theta);
                    r.done = true;
                    S->n_completed += 1;
                    S->n_evals += (uint64_t)r.n_theta;
                    S->latencies_us.push_back(
                        std::chrono::duration<double, std::micro>(Clock::now() - r.submitted)
                            .count());
                }
                it = S->resident.erase(it);
                S->cv_done.notify_all();
                if (S->resident.empty() && S->busy) {
                    S->busy = false;
                    S->busy_s += std::chrono::duration<double>(Clock::now() - S->busy_since).count();
                }
            } else {
                ++it;
            }
        }
        // admission, first come first served
        std::string err;
        while (!S->queue.empty() && try_place(S, *S->queue.front(), &err)) {
            std::shared_ptr<Request> r = S->queue.front();
            S->queue.pop_front();
            if (admit(S, *r) != hipSuccess) S->worker_error = "admission failed";
            if (!S->busy) {
                S->busy = true;
                S->busy_since = Clock::now();
            }
            S->resident.push_back(r);
        }
        bool active = false;
        for (auto &r : S->resident)
            if (r->iterations_left > 0) active = true;
        if (!active) {
            if (S->stopping && S->queue.empty() && S->resident.empty()) break;
            if (!S->resident.empty()) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            }
            continue;
        }
        // bound the iterations enqueued ahead of the GPU
        while ((int)S->inflight.size() >= S->opts.max_inflight) {
            hipEvent_t ev = S->inflight.front();
            S->inflight.pop_front();
            lk.unlock();
            (void)hipEventSynchronize(ev);
            lk.lock();
            (void)hipEventDestroy(ev);
        }
        // one iteration over every resident filter
        GroupLaunch launches[kMaxGroups];
        unsigned need[kMaxGroups] = {0};
        int32_t h_max = 1;
        for (auto &r : S->resident)
            if (r->iterations_left > 0) {
                need[r->group] += (unsigned)(r->F() * (r->Hp / 64));
                h_max = std::max(h_max, r->H);
            }
        S->e.h_max = h_max;
        unsigned off = 0;
        for (int g = 0; g < kMaxGroups; ++g) {
            launches[g] = S->groups[g].launch;
            launches[g].max_items = need[g];
            S->e.group_off[g] = off;
            off += need[g];
        }
        S->e.f_lo = 0;
        S->e.f_hi = (int32_t)S->slots.high_water();
        S->e.pool_chunks = off;  // groups of 64 particles of the slots still running
        if (engine_iteration(S->e, launches, kMaxGroups, S->stream) != hipSuccess)
            S->worker_error = "iteration launch failed";
        S->n_iterations += 1;
        for (auto &r : S->resident) {
            if (r->iterations_left <= 0) continue;
            r->iterations_left -= 1;
            if (r->iterations_left == 0) {
                if (launch_finish(S->e, (int32_t)r->slot, r->n_theta, r->M,
                                  S->dev_loglik + r->slot, S->dev_status + r->slot, nullptr,
                                  S->stream) != hipSuccess)
                    S->worker_error = "finish launch failed";
                (void)hipMemcpyAsync(S->res_loglik + r->slot, S->dev_loglik + r->slot,
                                     (size_t)r->n_theta * 8, hipMemcpyDeviceToHost, S->stream);
                (void)hipMemcpyAsync(S->res_status + r->slot, S->dev_status + r->slot,
                                     (size_t)r->n_theta * 4, hipMemcpyDeviceToHost, S->stream);
                (void)hipEventCreateWithFlags(&r->done_event, hipEventDisableTiming);
                (void)hipEventRecord(r->done_event, S->stream);
                r->finishing = true;
            }
        }
        hipEvent_t ev = nullptr;
        (void)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        (void)hipEventRecord(ev, S->stream);
        S->inflight.push_back(ev);
    }
    for (hipEvent_t ev : S->inflight) {
        (void)hipEventSynchronize(ev);
        (void)hipEventDestroy(ev);
    }
    S->inflight.clear();
}

}  // namespace

extern "C" {

int lik_server_create(const lik_server_opts *opts, lik_server_t *out) {
    if (!out) return fail(LIK_EINVAL, "out is NULL");
    *out = nullptr;
    lik_server_opts o = opts ? *opts : lik_server_opts{0, 0, 0, 0, 0, 0};
    if (o.reserved != 0) return fail(LIK_EINVAL, "reserved must be 0");
    if (o.tuning && !tuning_valid(*o.tuning)) return fail(LIK_EINVAL, tuning_rule());
    if (o.kernel != 0 && o.kernel != LIK_KERNEL_GENERIC && o.kernel != LIK_KERNEL_SPECIALIZED)
        return fail(LIK_EINVAL, "unknown kernel variant");
    if (o.arena_bytes == 0) o.arena_bytes = (size_t)1 << 30;
    if (o.staging_bytes == 0) o.staging_bytes = (size_t)64 << 20;
    if (o.max_filters <= 0) o.max_filters = 65536;
    if (o.max_filters > (1 << 24)) return fail(LIK_EINVAL, "max_filters above 2^24");
    if (o.max_inflight <= 0) o.max_inflight = 2;
    std::unique_ptr<lik_server> S(new (std::nothrow) lik_server());
    if (!S) return fail(LIK_ENOMEM, "out of host memory");
    S->opts = o;
    if (hipGetDevice(&S->device) != hipSuccess) return fail(LIK_EDEVICE, "no current device");
    const size_t slots = (size_t)o.max_filters;
    const size_t table = align256(slots * sizeof(FilterDesc)) + 4 * align256(slots * 4) +
                         align256(slots) +
                         2 * align256(slots * 8) + align256(slots * 64 * 4) +
                         2 * align256(kMaxGroups * 4) + align256(slots * 8) +
                         align256(slots * 4) + 2 * align256(kMaxGroups * kCostKeys * 4) +
                         align256(2 * 4);
    hipError_t err = hipMalloc((void **)&S->dev_base, table + o.arena_bytes + 256);
    if (err != hipSuccess) return fail(LIK_ENOMEM, "device arena allocation failed");
    const size_t pinned_bytes = o.staging_bytes + slots * 12 + 512;
    err = hipHostMalloc((void **)&S->pinned, pinned_bytes, hipHostMallocDefault);
    if (err != hipSuccess) {
        (void)hipFree(S->dev_base);
        return fail(LIK_ENOMEM, "pinned staging allocation failed");
    }
    char *p = S->dev_base;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += align256(bytes);
        return q;
    };
    memset(&S->e, 0, sizeof(S->e));
    S->desc = (FilterDesc *)take(slots * sizeof(FilterDesc));
    S->e.desc = S->desc;
    S->e.tcur = (int32_t *)take(slots * 4);
    S->e.fstatus = (int32_t *)take(slots * 4);
    S->e.fflags = (uint32_t *)take(slots * 4);
    S->e.cost = (uint32_t *)take(slots * 4);
    S->e.pool = (uint8_t *)take(slots);
    S->e.fll = (double *)take(slots * 8);
    S->e.fevents = (uint64_t *)take(slots * 8);
    S->e.items = (uint32_t *)take(slots * 64 * 4);
    S->e.item_count = (uint32_t *)take(kMaxGroups * 4);
    S->e.item_cursor = (uint32_t *)take(kMaxGroups * 4);
    S->e.order_count = (uint32_t *)take(kMaxGroups * kCostKeys * 4);
    S->e.order_pos = (uint32_t *)take(kMaxGroups * kCostKeys * 4);
    S->e.order_ctl = (uint32_t *)take(2 * 4);
    S->dev_loglik = (double *)take(slots * 8);
    S->dev_status = (int32_t *)take(slots * 4);
    S->arena = p;
    S->arena_bytes = o.arena_bytes;
    S->res_loglik = (double *)(S->pinned + align256(o.staging_bytes));
    S->res_status = (int32_t *)((char *)S->res_loglik + align256(slots * 8));
    S->slots.init(slots, 1);
    S->dmem.init(o.arena_bytes, 256);
    const lik_tuning tu = o.tuning ? *o.tuning : kDefaultTuning;
    S->e.pool_min = tu.pool_min;
    S->e.pool_max = tu.pool_max;
    S->e.pool_events = tu.pool_events;
    S->e.pool_first = tu.pool_first;
    S->e.refill_min = tu.refill_min;
    S->e.priority = tu.priority;
    S->e.pool_min_items = (uint32_t)tu.items_per_cu * compute_units();
    S->persistent = tu.persistent != 0;
    S->pmem.init(o.staging_bytes, 256);
    // every slot starts inactive (stopped), so stale slots are never ordered
    std::vector<uint32_t> stopped(slots, kFlagStopped);
    // the ordering passes' counts start at zero (each iteration leaves them so)
    std::vector<uint32_t> zeros(kMaxGroups * kCostKeys + 2, 0u);
    if (hipStreamCreate(&S->stream) != hipSuccess ||
        hipMemcpy(S->e.fflags, stopped.data(), slots * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S->e.order_count, zeros.data(), kMaxGroups * kCostKeys * 4,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S->e.order_ctl, zeros.data(), 2 * 4, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipHostFree(S->pinned);
        (void)hipFree(S->dev_base);
        return fail(LIK_EDEVICE, "stream or slot initialisation failed");
    }
    lik_server *raw = S.release();
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
    return LIK_OK;
}

int lik_server_submit(lik_server_t S, const lik_request *q, uint64_t *ticket) {
    if (!S || !ticket) return fail(LIK_EINVAL, "server or ticket is NULL");
    int rc = validate_request(S, q);
    if (rc) return rc;
    auto r = std::make_shared<Request>();
    r->net = q->net;
    r->obs = q->obs;
    r->precision = q->precision;
    r->n_theta = q->n_theta;
    r->M = q->data.n_traj;
    r->H = q->n_particles;
    r->Hp = (q->n_particles + 63) / 64 * 64;
    r->seed = q->seed;
    r->event_cap = q->event_cap;
    const int U = q->net->U, R = q->net->R, P = q->obs.n_observed, M = r->M;
    const int total = q->data.obs_offsets[M];
    r->theta.assign(q->theta, q->theta + (size_t)q->n_theta * R);
    if (q->theta_ids) r->ids.assign(q->theta_ids, q->theta_ids + q->n_theta);
    r->offsets.assign(q->data.obs_offsets, q->data.obs_offsets + M + 1);
    r->t_obs.assign(q->data.t_obs, q->data.t_obs + total);
    r->y.assign(q->data.y, q->data.y + (size_t)total * P);
    r->t0.assign(q->data.t0, q->data.t0 + M);
    r->x0.assign(q->data.x0, q->data.x0 + (size_t)M * U);
    if (q->data.x0_hi) r->x0_hi.assign(q->data.x0_hi, q->data.x0_hi + (size_t)M * U);
    r->t_max = 0;
    for (int m = 0; m < M; ++m) r->t_max = std::max(r->t_max, r->offsets[m + 1] - r->offsets[m]);
    if (r->device_bytes() > S->arena_bytes || r->input_bytes() > S->opts.staging_bytes)
        return fail(LIK_EINVAL, "request larger than the server's arena or staging memory");
    r->submitted = Clock::now();
    if (q->timeout_us > 0) {
        r->has_deadline = true;
        r->deadline = r->submitted + std::chrono::microseconds(q->timeout_us);
    }
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stopping) return fail(LIK_EINVAL, "server is shutting down");
    r->ticket = S->next_ticket++;
    S->tickets[r->ticket] = r;
    S->queue.push_back(r);
    S->n_submitted += 1;
    *ticket = r->ticket;
    S->cv_work.notify_one();
    return LIK_OK;
}

int lik_server_wait(lik_server_t S, uint64_t ticket, double *loglik_out, int32_t *status_out,
                    int64_t timeout_us) {
    if (!S) return fail(LIK_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(LIK_EINVAL, "unknown ticket");
    std::shared_ptr<Request> r = it->second;
    auto ready = [&] { return r->done || !S->worker_error.empty(); };
    if (timeout_us < 0) {
        S->cv_done.wait(lk, ready);
    } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return fail(LIK_ETIMEOUT, "request not finished yet");
    }
    if (!r->done) return fail(LIK_EDEVICE, S->worker_error);
    if (loglik_out) memcpy(loglik_out, r->loglik.data(), r->loglik.size() * 8);
    if (status_out) memcpy(status_out, r->status.data(), r->status.size() * 4);
    S->tickets.erase(ticket);
    return LIK_OK;
}

int lik_server_cancel(lik_server_t S, uint64_t ticket) {
    if (!S) return fail(LIK_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return fail(LIK_EINVAL, "unknown ticket");
    withdraw(S, it->second, LIK_STATUS_CANCELLED);
    S->cv_work.notify_one();
    return LIK_OK;
}

int lik_server_stats_get(lik_server_t S, lik_server_stats *out) {
    if (!S || !out) return fail(LIK_EINVAL, "server or out is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    out->submitted = S->n_submitted;
    out->completed = S->n_completed;
    out->evals = S->n_evals;
    out->iterations = S->n_iterations;
    out->cancelled = S->n_cancelled;
    out->p50_latency_us = percentile(S->latencies_us, 0.50);
    out->p99_latency_us = percentile(S->latencies_us, 0.99);
    out->busy_s = S->busy_s + (S->busy ? std::chrono::duration<double>(Clock::now() -
                                                                       S->busy_since).count()
                                       : 0.0);
    return LIK_OK;
}

int lik_server_destroy(lik_server_t S) {
    if (!S) return LIK_OK;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stopping = true;
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    (void)hipStreamSynchronize(S->stream);
    (void)hipStreamDestroy(S->stream);
    (void)hipHostFree(S->pinned);
    (void)hipFree(S->dev_base);
    delete S;
    return LIK_OK;
}

}  // extern "C"
