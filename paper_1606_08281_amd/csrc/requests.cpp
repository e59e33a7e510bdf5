// requests.cpp -- many requests, of several networks, particle counts and
// trajectory lengths, evaluated together: one admission launch for all of
// them, one persistent flow launch that runs every interval of every filter
// (each work item with its own network's propagation body), one finishing
// launch.  Results are those of each request evaluated alone (the random
// streams are keyed by each request's seed and theta ids, the weighing is
// per filter).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "host.hpp"

using namespace lik;

namespace {

int check_request(const lik_request *q) {
    if (q->reserved != 0) return fail(LIK_EINVAL, "reserved must be 0");
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
    return check_host_data(q->net, &q->obs, &q->data, q->n_theta, q->theta_ids);
}

// Byte layout of one allocation.
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    }
};

struct ReqPlan {
    int32_t M, H, Hp, t_max, total, group;
    int64_t F;
    size_t in_theta, in_ids, in_offs, in_t, in_y, in_t0, in_x0, in_x0h, state;  // offsets
};

}  // namespace

extern "C" {

int lik_eval_requests(const lik_request *reqs, int32_t n_req, const lik_tuning *tuning,
                      int32_t kernel, double *loglik_out, int32_t *status_out, double *done_ms) {
    if (n_req < 0 || (n_req > 0 && !reqs)) return fail(LIK_EINVAL, "requests missing");
    if (n_req == 0) return LIK_OK;
    if (!loglik_out) return fail(LIK_EINVAL, "loglik_out is NULL");
    if (kernel < LIK_KERNEL_AUTO || kernel > LIK_KERNEL_SPECIALIZED)
        return fail(LIK_EINVAL, "unknown kernel variant");
    const lik_tuning tu = tuning ? *tuning : kDefaultTuning;
    if (!tuning_valid(tu)) return fail(LIK_EINVAL, tuning_rule());
    const int precision = reqs[0].precision;

    // validation, networks (one group each), sizes
    std::vector<lik_network *> nets;
    std::vector<ReqPlan> plan((size_t)n_req);
    std::vector<int32_t> fstart((size_t)n_req + 1), outoff((size_t)n_req + 1);
    int64_t F = 0, chunks = 0, items_max = 0, n_out = 0;
    double work = 0.0;
    int h_max = 1, t_max = 0, umax = 4, rmax = 8;
    for (int k = 0; k < n_req; ++k) {
        const lik_request &q = reqs[k];
        int rc = check_request(&q);
        if (rc) return fail(rc, "request " + std::to_string(k) + ": " + lik_last_error());
        if (q.precision != precision)
            return fail(LIK_EINVAL, "every request of one call must have the same precision");
        int g = (int)(std::find(nets.begin(), nets.end(), q.net) - nets.begin());
        if (g == (int)nets.size()) {
            if ((int)nets.size() == kMaxGroups)
                return fail(LIK_EUNSUPPORTED, "at most 16 networks in one call");
            nets.push_back(q.net);
        }
        ReqPlan &p = plan[(size_t)k];
        p.group = g;
        p.M = q.data.n_traj;
        p.H = q.n_particles;
        p.Hp = (p.H + 63) / 64 * 64;
        p.total = q.data.obs_offsets[p.M];
        p.t_max = 0;
        for (int m = 0; m < p.M; ++m)
            p.t_max = std::max(p.t_max, q.data.obs_offsets[m + 1] - q.data.obs_offsets[m]);
        p.F = (int64_t)q.n_theta * p.M;
        fstart[(size_t)k] = (int32_t)F;
        outoff[(size_t)k] = (int32_t)n_out;
        F += p.F;
        n_out += q.n_theta;
        chunks += p.F * (p.Hp / 64);
        items_max += (int64_t)q.n_theta * p.total * (p.Hp / 64);
        work += (double)p.F * p.H * p.t_max;
        h_max = std::max(h_max, p.H);
        t_max = std::max(t_max, p.t_max);
        umax = std::max(umax, q.net->umax);
        rmax = std::max(rmax, q.net->rmax);
        if (F >= ((int64_t)1 << 26) || n_out >= ((int64_t)1 << 31))
            return fail(LIK_EINVAL, "too many filters in one call (at most 2^26)");
    }
    fstart[(size_t)n_req] = (int32_t)F;
    outoff[(size_t)n_req] = (int32_t)n_out;

    // one allocation: engine, flow rings, tables and inputs (staged from one
    // host copy), particle state
    const uint32_t ring_cap = flow_ring_capacity((size_t)chunks, 1);
    Carve c;
    const size_t o_desc = c.take((size_t)F * sizeof(FilterDesc));
    const size_t o_tcur = c.take((size_t)F * 4), o_fst = c.take((size_t)F * 4);
    const size_t o_ffl = c.take((size_t)F * 4), o_cost = c.take((size_t)F * 4);
    const size_t o_pool = c.take((size_t)F), o_fll = c.take((size_t)F * 8);
    const size_t o_fev = c.take((size_t)F * 8), o_items = c.take((size_t)chunks * 4);
    const size_t o_icount = c.take(kMaxGroups * 4), o_icur = c.take(kMaxGroups * 4);
    const size_t o_ocount = c.take(kMaxGroups * kCostKeys * 4);
    const size_t o_opos = c.take(kMaxGroups * kCostKeys * 4), o_octl = c.take(2 * 4);
    const size_t o_ring = c.take((size_t)ring_cap * 8 * kFlowRings);
    const size_t o_rem = c.take((size_t)F * 4), o_ctl = c.take(kCtlWords * 4);
    const size_t o_fdone = c.take((size_t)F * 8), o_start = c.take(8);
    const size_t o_ll = c.take((size_t)n_out * 8), o_st = c.take((size_t)n_out * 4);
    // staged region: tables, then every request's inputs
    const size_t o_stage = c.off;
    const size_t o_reqs = c.take((size_t)n_req * sizeof(RequestArgs));
    const size_t o_fstart = c.take(((size_t)n_req + 1) * 4);
    const size_t o_spans = c.take((size_t)n_req * sizeof(ReqSpan));
    const size_t o_nets = c.take(kMaxGroups * sizeof(Net8x16));
    for (int k = 0; k < n_req; ++k) {
        const lik_request &q = reqs[k];
        ReqPlan &p = plan[(size_t)k];
        p.in_theta = c.take((size_t)q.n_theta * q.net->R * 8);
        p.in_ids = c.take(q.theta_ids ? (size_t)q.n_theta * 4 : 0);
        p.in_offs = c.take(((size_t)p.M + 1) * 4);
        p.in_t = c.take((size_t)p.total * 8);
        p.in_y = c.take((size_t)p.total * q.obs.n_observed * 8);
        p.in_t0 = c.take((size_t)p.M * 8);
        p.in_x0 = c.take((size_t)p.M * q.net->U * 4);
        p.in_x0h = c.take(q.data.x0_hi ? (size_t)p.M * q.net->U * 4 : 0);
    }
    const size_t stage_bytes = c.off - o_stage;
    for (int k = 0; k < n_req; ++k) {
        ReqPlan &p = plan[(size_t)k];
        p.state = c.take(request_state_bytes(p.F, reqs[k].net->U, p.Hp));
    }
    char *dev = nullptr;
    hipError_t err = hipMalloc((void **)&dev, c.off + 256);
    if (err != hipSuccess) return fail(LIK_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(err));
    std::vector<char> host(stage_bytes, 0);
    auto put = [&](size_t off, const void *src, size_t bytes) {
        if (bytes) memcpy(host.data() + (off - o_stage), src, bytes);
    };
    RequestArgs *ra = reinterpret_cast<RequestArgs *>(host.data() + (o_reqs - o_stage));
    ReqSpan *spans = reinterpret_cast<ReqSpan *>(host.data() + (o_spans - o_stage));
    Net8x16 *nt = reinterpret_cast<Net8x16 *>(host.data() + (o_nets - o_stage));
    Net4x8 *nt4 = reinterpret_cast<Net4x8 *>(host.data() + (o_nets - o_stage));
    for (size_t g = 0; g < nets.size(); ++g) {
        if (umax == 4 && rmax == 8)
            nt4[g] = nets[g]->n4;
        else
            nt[g] = nets[g]->n8;
    }
    put(o_fstart, fstart.data(), ((size_t)n_req + 1) * 4);
    bool any_random_start = false;
    for (int k = 0; k < n_req; ++k) {
        const lik_request &q = reqs[k];
        const ReqPlan &p = plan[(size_t)k];
        const int U = q.net->U, R = q.net->R, P = q.obs.n_observed;
        put(p.in_theta, q.theta, (size_t)q.n_theta * R * 8);
        if (q.theta_ids) put(p.in_ids, q.theta_ids, (size_t)q.n_theta * 4);
        put(p.in_offs, q.data.obs_offsets, ((size_t)p.M + 1) * 4);
        put(p.in_t, q.data.t_obs, (size_t)p.total * 8);
        put(p.in_y, q.data.y, (size_t)p.total * P * 8);
        put(p.in_t0, q.data.t0, (size_t)p.M * 8);
        put(p.in_x0, q.data.x0, (size_t)p.M * U * 4);
        if (q.data.x0_hi) put(p.in_x0h, q.data.x0_hi, (size_t)p.M * U * 4);
        RequestArgs a;
        memset(&a, 0, sizeof(a));
        a.theta = (const double *)(dev + p.in_theta);
        a.theta_ids = q.theta_ids ? (const uint32_t *)(dev + p.in_ids) : nullptr;
        a.obs_offsets = (const int32_t *)(dev + p.in_offs);
        a.t_obs = (const double *)(dev + p.in_t);
        a.y = (const double *)(dev + p.in_y);
        a.t0 = (const double *)(dev + p.in_t0);
        a.x0 = (const int32_t *)(dev + p.in_x0);
        a.x0_hi = q.data.x0_hi ? (const int32_t *)(dev + p.in_x0h) : nullptr;
        any_random_start = any_random_start || q.data.x0_hi != nullptr;
        a.state = (int32_t *)(dev + p.state);
        a.n_theta = q.n_theta;
        a.M = p.M;
        a.H = p.H;
        a.Hp = p.Hp;
        a.U = U;
        a.R = R;
        a.P = P;
        a.obs_kind = q.obs.kind;
        a.group = p.group;
        a.precision = precision;
        for (int j = 0; j < LIK_MAX_OBSERVED; ++j) a.obs_species[j] = j < P ? q.obs.species[j] : 0;
        a.sigma = q.obs.sigma;
        a.gain = q.obs.gain;
        a.bg_mean = q.obs.bg_mean;
        a.bg_sd = q.obs.bg_sd;
        a.seed = q.seed;
        a.event_cap = (uint32_t)(q.event_cap ? q.event_cap : LIK_DEFAULT_EVENT_CAP);
        a.base = fstart[(size_t)k];
        fill_reactant_tables(a, q.net->kind, q.net->s1, q.net->s2, R);
        ra[k] = a;
        spans[k] = ReqSpan{fstart[(size_t)k], q.n_theta, p.M, outoff[(size_t)k]};
    }

    // the engine over every slot
    EngineArgs e;
    memset(&e, 0, sizeof(e));
    FilterDesc *desc = (FilterDesc *)(dev + o_desc);
    e.desc = desc;
    e.tcur = (int32_t *)(dev + o_tcur);
    e.fstatus = (int32_t *)(dev + o_fst);
    e.fflags = (uint32_t *)(dev + o_ffl);
    e.cost = (uint32_t *)(dev + o_cost);
    e.pool = (uint8_t *)(dev + o_pool);
    e.fll = (double *)(dev + o_fll);
    e.fevents = (uint64_t *)(dev + o_fev);
    e.items = (uint32_t *)(dev + o_items);
    e.item_count = (uint32_t *)(dev + o_icount);
    e.item_cursor = (uint32_t *)(dev + o_icur);
    e.order_count = (uint32_t *)(dev + o_ocount);
    e.order_pos = (uint32_t *)(dev + o_opos);
    e.order_ctl = (uint32_t *)(dev + o_octl);
    e.fdone = (uint64_t *)(dev + o_fdone);
    e.f_lo = 0;
    e.f_hi = (int32_t)F;
    e.pool_min = tu.pool_min;
    e.pool_max = tu.pool_max;
    e.pool_events = tu.pool_events;
    e.pool_first = tu.pool_first;
    e.refill_min = tu.refill_min;
    e.priority = tu.priority;
    e.pool_min_items = (uint32_t)tu.items_per_cu * compute_units();
    e.h_max = h_max;
    e.pool_chunks = (uint32_t)std::min<int64_t>(chunks, 0xFFFFFFFFll);

    // schedule and kernels
    std::string msg;
    bool flow = tu.schedule == 1 && items_max < ((int64_t)1 << 26);
    hipFunction_t spec_multi = nullptr;
    if (flow) {
        int per_cu = 0;
        const bool want_spec = kernel == LIK_KERNEL_SPECIALIZED ||
                               (kernel == LIK_KERNEL_AUTO && work >= 4194304.0);
        if (want_spec) {
            spec_multi = specialized_multi_kernel(nets, precision, &msg);
            if (!spec_multi && kernel == LIK_KERNEL_SPECIALIZED) {
                (void)hipFree(dev);
                return fail(LIK_EDEVICE, "specialised multi-network kernel unavailable: " + msg);
            }
            if (spec_multi &&
                hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, spec_multi, kPropBlock,
                                                                   0) != hipSuccess)
                per_cu = 0;
        }
        if (!spec_multi) per_cu = flow_multi_blocks_per_cu(umax, rmax, precision);
        flow = per_cu >= kFlowMinWavesPerCu;
    }
    FlowArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.ring = (uint64_t *)(dev + o_ring);
    fa.remaining = (uint32_t *)(dev + o_rem);
    fa.ctl = (uint32_t *)(dev + o_ctl);
    fa.mask = ring_cap - 1;
    fa.n_slots = (int32_t)F;
    fa.g_par = (int32_t)std::max<int64_t>(1, chunks / std::max<uint32_t>(e.pool_min_items, 1u));
    fa.urgent_events = tu.urgent_events;
    fa.backlog = std::max(compute_units(), 1u) * tu.backlog_per_cu;
    int dev_id = 0, khz = 0;
    if (hipGetDevice(&dev_id) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev_id) != hipSuccess ||
        khz <= 0)
        khz = 100000;
    const char *stall_us = getenv("LIK_FLOW_STALL_US");
    const uint64_t us = (stall_us && *stall_us) ? strtoull(stall_us, nullptr, 10) : 60000000ull;
    fa.stall_ticks = (uint64_t)khz * us / 1000ull;
    // per-interval launches: one propagation launch per network group
    GroupLaunch groups[kMaxGroups];
    if (!flow) {
        std::vector<int64_t> need(nets.size(), 0);
        for (int k = 0; k < n_req; ++k)
            need[(size_t)plan[(size_t)k].group] += plan[(size_t)k].F * (plan[(size_t)k].Hp / 64);
        uint32_t off = 0;
        for (size_t g = 0; g < nets.size(); ++g) {
            GroupLaunch &G = groups[g];
            G.netargs = generic_netargs(*nets[g]);
            G.umax = nets[g]->umax;
            G.rmax = nets[g]->rmax;
            G.precision = precision;
            G.max_items = (unsigned)need[g];
            if (!choose_specialized(*nets[g], precision, kernel, work, &G.spec, &msg)) {
                (void)hipFree(dev);
                return fail(LIK_EDEVICE, "specialised kernel unavailable: " + msg);
            }
            G.persistent = tu.persistent != 0 && nets[g]->R <= kPersistentMaxR;
            G.persistent_waves = persistent_waves();
            if (G.spec && G.persistent)
                G.spec_p = specialized_kernel(*nets[g], precision, &msg, kSpecPersistent);
            e.group_off[g] = off;
            off += (uint32_t)need[g];
        }
    }

    hipStream_t s = nullptr;
    int rc = LIK_OK;
    std::vector<uint64_t> fdone((size_t)F, 0);
    uint64_t start_tick = 0;
    do {
        if ((err = hipStreamCreate(&s)) != hipSuccess) { rc = hip_fail(err, "hipStreamCreate"); break; }
        if ((err = hipMemcpyAsync(dev + o_stage, host.data(), stage_bytes, hipMemcpyHostToDevice,
                                  s)) != hipSuccess) {
            rc = hip_fail(err, "copy to device");
            break;
        }
        err = launch_admit_requests(desc, e, (const RequestArgs *)(dev + o_reqs),
                                    (const int32_t *)(dev + o_fstart), n_req, (int32_t)F,
                                    (uint64_t *)(dev + o_start), s);
        if (err != hipSuccess) { rc = hip_fail(err, "admit launch"); break; }
        if (any_random_start && (err = launch_init_start(desc, 0, (int32_t)F, s)) != hipSuccess) {
            rc = hip_fail(err, "initial-count launch");
            break;
        }
        if (flow) {
            if ((err = launch_flow_setup(e, fa, s)) != hipSuccess) { rc = hip_fail(err, "flow setup"); break; }
            const unsigned waves = (unsigned)std::max<int64_t>(items_max, 1);
            hipEvent_t t0 = timing_begin(s);
            if (spec_multi) {
                EngineArgs ea = e;
                const FlowArgs *fb = flow_args_copy(fa.ctl);  // written by k_flow_init
                void *params[] = {(void *)&ea, (void *)&fb};
                err = hipModuleLaunchKernel(spec_multi, waves, 1, 1, kPropBlock, 1, 1, 0, s, params,
                                            nullptr);
            } else {
                err = launch_flow_multi(e, fa, waves, dev + o_nets, umax, rmax, precision, s);
            }
            if (err != hipSuccess) { rc = hip_fail(err, "flow launch"); break; }
            timing_end_propagate(t0, s);
            if ((err = launch_flow_check(e, fa, s)) != hipSuccess) { rc = hip_fail(err, "flow check"); break; }
        } else {
            if ((err = launch_order_reset(e, s)) != hipSuccess) { rc = hip_fail(err, "order reset"); break; }
            for (int t = 0; t < t_max && err == hipSuccess; ++t)
                err = engine_iteration(e, groups, (int)nets.size(), s);
            if (err != hipSuccess) { rc = hip_fail(err, "iteration launch"); break; }
        }
        err = launch_finish_requests(e, (const ReqSpan *)(dev + o_spans), n_req,
                                     (double *)(dev + o_ll), (int32_t *)(dev + o_st), s);
        if (err != hipSuccess) { rc = hip_fail(err, "finish launch"); break; }
        if ((err = hipMemcpyAsync(loglik_out, dev + o_ll, (size_t)n_out * 8,
                                  hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (status_out && (err = hipMemcpyAsync(status_out, dev + o_st, (size_t)n_out * 4,
                                                 hipMemcpyDeviceToHost, s)) != hipSuccess) ||
            (done_ms && ((err = hipMemcpyAsync(fdone.data(), dev + o_fdone, (size_t)F * 8,
                                               hipMemcpyDeviceToHost, s)) != hipSuccess ||
                         (err = hipMemcpyAsync(&start_tick, dev + o_start, 8,
                                               hipMemcpyDeviceToHost, s)) != hipSuccess))) {
            rc = hip_fail(err, "copy to host");
            break;
        }
        if ((err = hipStreamSynchronize(s)) != hipSuccess) { rc = hip_fail(err, "synchronize"); break; }
    } while (0);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(dev);
    if (rc == LIK_OK && done_ms) {
        // completion of a request: its last filter's finish on the device
        // clock, from the admission launch (0 if no filter ran)
        for (int k = 0; k < n_req; ++k) {
            uint64_t last = 0;
            for (int64_t f = fstart[(size_t)k]; f < fstart[(size_t)k + 1]; ++f)
                last = std::max(last, fdone[(size_t)f]);
            done_ms[k] = last > start_tick ? (double)(last - start_tick) / (double)khz : 0.0;
        }
    }
    return rc;
}

int lik_precompile_requests(const lik_network_t *nets, int32_t n_nets, int32_t precision) {
    if (!nets || n_nets < 1 || n_nets > kMaxGroups)
        return fail(LIK_EINVAL, "1 to 16 networks are needed");
    if (precision != LIK_FP64 && precision != LIK_FP32_MIXED)
        return fail(LIK_EINVAL, "unknown precision");
    std::vector<lik_network *> v(nets, nets + n_nets);
    for (lik_network *n : v)
        if (!n) return fail(LIK_EINVAL, "network is NULL");
    std::string err;
    if (!precompile_multi(v, precision, &err)) return fail(LIK_EDEVICE, err);
    return LIK_OK;
}

int lik_autotune_requests(const lik_request *reqs, int32_t n_req, int32_t kernel,
                          lik_tuning *chosen) {
    if (!chosen) return fail(LIK_EINVAL, "chosen is NULL");
    int n_cands = 0;
    const lik_tuning *cands = autotune_candidates(&n_cands);
    int64_t n_out = 0;
    for (int k = 0; k < n_req && reqs; ++k) n_out += reqs[k].n_theta;
    std::vector<double> ll((size_t)std::max<int64_t>(n_out, 1));
    // one untimed run loads kernels and warms caches
    int rc = lik_eval_requests(reqs, n_req, &cands[0], kernel, ll.data(), nullptr, nullptr);
    if (rc) return rc;
    // each candidate timed over one whole (synchronous) call
    double best = -1.0;
    for (int ci = 0; ci < n_cands; ++ci) {
        const auto t0 = std::chrono::steady_clock::now();
        rc = lik_eval_requests(reqs, n_req, &cands[ci], kernel, ll.data(), nullptr, nullptr);
        const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (rc) return rc;
        if (best < 0.0 || s < best) {
            best = s;
            *chosen = cands[ci];
        }
    }
    return LIK_OK;
}

}  // extern "C"
