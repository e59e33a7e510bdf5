// api.cpp -- C ABI of liblik.so: validation, workspace layout, launch order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lik.h"
#include "host.hpp"
#include "lik_internal.hpp"

using namespace lik;

namespace {
thread_local std::string g_err;
}  // namespace

int lik::fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int lik::hip_fail(hipError_t e, const char *where) {
    return fail(LIK_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool lik::tuning_valid(const lik_tuning &v) {
    return v.pool_min >= 1 && v.pool_max >= v.pool_min && v.pool_max <= 64 &&
           v.pool_first >= 1 && v.pool_first <= 64 && v.refill_min >= 1 && v.refill_min <= 64 &&
           (v.priority == 0 || v.priority == 1) && v.items_per_cu >= 0 &&
           v.items_per_cu <= (1 << 20) && (v.persistent == 0 || v.persistent == 1) &&
           (v.schedule == 0 || v.schedule == 1) && v.backlog_per_cu >= 1 &&
           v.backlog_per_cu <= (1u << 16);
}

const char *lik::tuning_rule() {
    return "tuning must satisfy 1 <= pool_min <= pool_max <= 64, 1 <= pool_first <= 64, "
           "1 <= refill_min <= 64, priority 0 or 1, 0 <= items_per_cu <= 2^20, "
           "persistent 0 or 1, schedule 0 or 1, 1 <= backlog_per_cu <= 65536";
}

unsigned lik::persistent_waves() { return compute_units() * 32u; }

uint32_t lik::compute_units() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return (uint32_t)cus;
}

namespace {

// Kernel timing (lik_timing_enable / lik_timing_read).
struct TimedLaunches {
    bool enabled = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prop, weigh;
};
TimedLaunches g_timing;

hipEvent_t timing_mark(hipStream_t s) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    if (hipEventRecord(e, s) != hipSuccess) {
        (void)hipEventDestroy(e);
        return nullptr;
    }
    return e;
}

}  // namespace

hipEvent_t lik::timing_begin(hipStream_t s) { return g_timing.enabled ? timing_mark(s) : nullptr; }

void lik::timing_end_propagate(hipEvent_t begin, hipStream_t s) {
    if (g_timing.enabled && begin) g_timing.prop.push_back({begin, timing_mark(s)});
}

const lik_tuning *lik::autotune_candidates(int *n) {
    static const lik_tuning cands[] = {
        {1, 6, 1536, 1, 1, 0, 160, 0, 1, 16000, 60},  // default: flow schedule
        {1, 6, 1536, 1, 1, 0, 160, 0, 1, 16000, 30},  // flow, shorter queue
        {1, 6, 1536, 1, 1, 0, 160, 0, 1, 32000, 60},
        {1, 6, 1536, 1, 1, 0, 160, 0, 1, 0, 60},      // flow, first come first served
        {1, 4, 1024, 1, 1, 0, 160, 0, 1, 16000, 60},
        {1, 6, 1536, 1, 1, 0, 160, 0, 0, 16000, 60},  // one launch sequence per interval
        {1, 4, 1024, 1, 1, 0, 160, 0, 0, 16000, 60},
        {2, 6, 2048, 1, 1, 0, 160, 0, 0, 16000, 60},
        {1, 1, 0, 1, 1, 0, 0, 0, 0, 16000, 60},       // one group of 64 particles per wavefront
        {1, 1, 0, 1, 1, 0, 0, 1, 0, 16000, 60},       // persistent wavefronts (R <= 16)
    };
    *n = (int)(sizeof(cands) / sizeof(cands[0]));
    return cands;
}

template <int RMAX, int W>
static void fill_net(const lik_network &src, NetArgs<RMAX, W> &dst) {
    memset(&dst, 0, sizeof(dst));
    dst.U = src.U;
    dst.R = src.R;
    for (int r = 0; r < src.R && r < RMAX; ++r) {
        dst.kind[r] = src.kind[r];
        dst.s1[r] = src.s1[r];
        dst.s2[r] = src.s2[r];
        for (int w = 0; w < W; ++w) dst.nu[r][w] = src.nu[r][w];
    }
}

extern "C" {

const char *lik_last_error(void) { return g_err.c_str(); }

int lik_timing_enable(int enable) {
    g_timing.enabled = enable != 0;
    return LIK_OK;
}

int lik_timing_read(lik_timing *out) {
    if (!out) return fail(LIK_EINVAL, "out is NULL");
    memset(out, 0, sizeof(*out));
    int rc = LIK_OK;
    auto drain = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>> &v, double *ms, int64_t *n) {
        for (auto &pr : v) {
            float dt = 0.0f;
            if (pr.first && pr.second && hipEventSynchronize(pr.second) == hipSuccess &&
                hipEventElapsedTime(&dt, pr.first, pr.second) == hipSuccess) {
                *ms += dt;
                *n += 1;
            } else {
                rc = fail(LIK_EDEVICE, "a timing event could not be read");
            }
        }
        // an event may close one launch and open the next: destroy each once
        std::vector<hipEvent_t> all;
        for (auto &pr : v) { all.push_back(pr.first); all.push_back(pr.second); }
        v.clear();
        return all;
    };
    std::vector<hipEvent_t> all = drain(g_timing.prop, &out->propagate_ms, &out->propagate_launches);
    std::vector<hipEvent_t> w = drain(g_timing.weigh, &out->weigh_ms, &out->weigh_launches);
    all.insert(all.end(), w.begin(), w.end());
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    for (hipEvent_t e : all)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

const char *lik_version(void) { return "lik 0.1 (gfx950)"; }

int lik_create_network(int32_t n_species, int32_t n_reactions, const int32_t *reactant_orders,
                       const int32_t *stoichiometry, lik_network_t *out) {
    if (!out) return fail(LIK_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_species < 1 || n_species > LIK_MAX_SPECIES)
        return fail(LIK_EINVAL, "n_species must be in [1, 32]");
    if (n_reactions < 1 || n_reactions > LIK_MAX_REACTIONS)
        return fail(LIK_EINVAL, "n_reactions must be in [1, 64]");
    if (!reactant_orders || !stoichiometry) return fail(LIK_EINVAL, "NULL network table");
    lik_network *n = new (std::nothrow) lik_network();
    if (!n) return fail(LIK_ENOMEM, "out of host memory");
    const int U = n_species, R = n_reactions;
    n->U = U;
    n->R = R;
    n->orders.assign(reactant_orders, reactant_orders + (size_t)R * U);
    n->stoich.assign(stoichiometry, stoichiometry + (size_t)R * U);
    memset(n->nu, 0, sizeof(n->nu));
    for (int r = 0; r < R; ++r) {
        int total = 0, first = -1, second = -1, homo = -1;
        for (int u = 0; u < U; ++u) {
            const int p = reactant_orders[r * U + u];
            const int v = stoichiometry[r * U + u];
            if (p < 0) { delete n; return fail(LIK_EINVAL, "negative reactant order"); }
            total += p;
            if (total > 2) { delete n; return fail(LIK_EINVAL, "reaction order above 2"); }
            if (p == 2) homo = u;
            if (p == 1) (first < 0 ? first : second) = u;
            if (v < -p) { delete n; return fail(LIK_EINVAL, "net change consumes an unused reactant"); }
            if (v < -7 || v > 7) { delete n; return fail(LIK_EUNSUPPORTED, "|net change| above 7"); }
            if (nu_bytes(U))
                n->nu[r][0] |= ((uint32_t)v & 0xFFu) << (8 * u);
            else
                n->nu[r][u >> 3] |= ((uint32_t)v & 0xFu) << (4 * (u & 7));
        }
        if (homo >= 0) { n->kind[r] = kOrder2Homo; n->s1[r] = homo; n->s2[r] = homo; }
        else if (second >= 0) { n->kind[r] = kOrder2Hetero; n->s1[r] = first; n->s2[r] = second; }
        else if (first >= 0) { n->kind[r] = kOrder1; n->s1[r] = first; n->s2[r] = first; }
        else { n->kind[r] = kOrder0; n->s1[r] = 0; n->s2[r] = 0; }
    }
    if (U <= 4 && R <= 8) { n->umax = 4; n->rmax = 8; }
    else if (U <= 8 && R <= 16) { n->umax = 8; n->rmax = 16; }
    else { n->umax = 32; n->rmax = 64; }
    fill_net(*n, n->n4);
    fill_net(*n, n->n8);
    fill_net(*n, n->n32);
    *out = n;
    return LIK_OK;
}

int lik_network_set_tuning(lik_network_t net, const lik_tuning *t) {
    if (!net) return fail(LIK_EINVAL, "network is NULL");
    lik_tuning v = t ? *t : kDefaultTuning;
    if (!tuning_valid(v)) return fail(LIK_EINVAL, tuning_rule());
    net->tuning = v;
    return LIK_OK;
}

int lik_network_get_tuning(lik_network_t net, lik_tuning *out) {
    if (!net || !out) return fail(LIK_EINVAL, "network or out is NULL");
    *out = net->tuning;
    return LIK_OK;
}

int lik_autotune_device(lik_network_t net, const lik_obs_model *obs, const lik_eval_opts *opts,
                        int32_t n_theta, const double *theta, const lik_data *data,
                        const int32_t *obs_offsets_host, int32_t n_particles, uint64_t seed,
                        double *loglik_out, int32_t *status_out, void *workspace,
                        size_t workspace_bytes, void *stream, lik_tuning *chosen) {
    if (!net) return fail(LIK_EINVAL, "network is NULL");
    int n_cands = 0;
    const lik_tuning *cands = autotune_candidates(&n_cands);
    const lik_tuning saved = net->tuning;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return fail(LIK_EDEVICE, "hipEventCreate failed");
    float best_ms = -1.0f;
    lik_tuning best = saved;
    int rc = LIK_OK;
    lik_eval_opts o = opts ? *opts : lik_eval_opts{LIK_FP64, LIK_KERNEL_AUTO, 0, nullptr, 0, 0};
    o.flags &= ~LIK_FLAG_GRAPH;
    // one untimed run loads kernels and warms caches
    rc = lik_eval_batch_device(net, obs, &o, n_theta, theta, data, obs_offsets_host, n_particles,
                               seed, loglik_out, status_out, nullptr, workspace, workspace_bytes,
                               stream);
    for (int ci = 0; ci < n_cands; ++ci) {
        const lik_tuning &c = cands[ci];
        if (rc != LIK_OK) break;
        net->tuning = c;
        (void)hipEventRecord(a, s);
        rc = lik_eval_batch_device(net, obs, &o, n_theta, theta, data, obs_offsets_host,
                                   n_particles, seed, loglik_out, status_out, nullptr, workspace,
                                   workspace_bytes, stream);
        (void)hipEventRecord(b, s);
        if (rc != LIK_OK) break;
        float ms = 0.0f;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) {
            rc = fail(LIK_EDEVICE, "timing failed");
            break;
        }
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    net->tuning = rc == LIK_OK ? best : saved;
    if (rc == LIK_OK && chosen) *chosen = best;
    return rc;
}

int lik_network_precompile(lik_network_t net, int32_t precision) {
    if (!net) return fail(LIK_EINVAL, "network is NULL");
    if (precision != LIK_FP64 && precision != LIK_FP32_MIXED)
        return fail(LIK_EINVAL, "unknown precision");
    std::string err;
    if (!precompile_specialized(*net, precision, &err)) return fail(LIK_EDEVICE, err);
    return LIK_OK;
}

int lik_destroy_network(lik_network_t net) {
    if (net) {
        release_graphs(*net);
        release_specialized(*net);
    }
    delete net;
    return LIK_OK;
}

}  // extern "C"

int lik::check_host_data(const lik_network *net, const lik_obs_model *obs, const lik_data *data,
                         int32_t n_theta, const uint32_t *theta_ids) {
    const int M = data->n_traj, U = net->U, P = obs->n_observed;
    for (int m = 0; m < M; ++m) {
        double prev = data->t0[m];
        if (!isfinite(prev)) return fail(LIK_EINVAL, "t0 must be finite");
        for (int k = data->obs_offsets[m]; k < data->obs_offsets[m + 1]; ++k) {
            if (!(data->t_obs[k] > prev) || !isfinite(data->t_obs[k]))
                return fail(LIK_EINVAL, "observation times must increase strictly from t0");
            prev = data->t_obs[k];
            for (int q = 0; q < P; ++q) {
                const double v = data->y[(size_t)k * P + q];
                if (!isfinite(v)) return fail(LIK_EINVAL, "observations must be finite");
                if (obs->kind == LIK_OBS_LOGNORMAL && !(v > 0.0))
                    return fail(LIK_EINVAL, "log-normal observations must be > 0");
            }
        }
        for (int u = 0; u < U; ++u) {
            const int32_t v = data->x0[(size_t)m * U + u];
            if (v < 0 || v > kCountLimit) return fail(LIK_EINVAL, "x0 out of [0, 2^30]");
            if (data->x0_hi) {
                const int32_t h = data->x0_hi[(size_t)m * U + u];
                if (h < v || h > kCountLimit) return fail(LIK_EINVAL, "x0_hi out of [x0, 2^30]");
            }
        }
    }
    if (theta_ids)
        for (int i = 0; i < n_theta; ++i)
            if (theta_ids[i] >= (1u << 30)) return fail(LIK_EINVAL, "theta id >= 2^30");

    return LIK_OK;
}

int lik::check_common(lik_network_t net, const lik_obs_model *obs, const lik_eval_opts *opts,
                        int32_t n_theta, int32_t n_traj, int32_t n_particles) {
    if (!net) return fail(LIK_EINVAL, "network is NULL");
    if (!obs) return fail(LIK_EINVAL, "observation model is NULL");
    if (obs->kind != LIK_OBS_GAUSSIAN && obs->kind != LIK_OBS_LOGNORMAL &&
        obs->kind != LIK_OBS_FLUORESCENCE)
        return fail(LIK_EINVAL, "unknown observation kind");
    if (obs->n_observed < 1 || obs->n_observed > LIK_MAX_OBSERVED)
        return fail(LIK_EINVAL, "n_observed must be in [1, 8]");
    for (int k = 0; k < obs->n_observed; ++k)
        if (obs->species[k] < 0 || obs->species[k] >= net->U)
            return fail(LIK_EINVAL, "observed species out of range");
    if (obs->kind == LIK_OBS_FLUORESCENCE) {
        if (!(obs->sigma >= 0.0) || isinf(obs->sigma))
            return fail(LIK_EINVAL, "fluorescence: sigma must be finite and >= 0");
        if (!isfinite(obs->gain) || !isfinite(obs->bg_mean))
            return fail(LIK_EINVAL, "fluorescence: gain and bg_mean must be finite");
        if (!(obs->bg_sd > 0.0) || isinf(obs->bg_sd))
            return fail(LIK_EINVAL, "fluorescence: bg_sd must be finite and > 0");
    } else if (!(obs->sigma > 0.0) || isinf(obs->sigma)) {
        return fail(LIK_EINVAL, "sigma must be > 0");
    }
    if (n_theta < 0) return fail(LIK_EINVAL, "n_theta < 0");
    if (n_theta >= (1 << 30)) return fail(LIK_EINVAL, "n_theta too large");
    if (n_traj < 1 || n_traj > LIK_MAX_TRAJ) return fail(LIK_EINVAL, "n_traj out of range");
    if ((int64_t)n_theta * n_traj * ((n_particles + 63) / 64) > (int64_t)0x7FFFFFFF)
        return fail(LIK_EINVAL, "too many filters in one batch");
    if (n_particles < 1 || n_particles > LIK_MAX_PARTICLES)
        return fail(LIK_EINVAL, "n_particles must be in [1, 4096]");
    if (opts) {
        if (opts->precision != LIK_FP64 && opts->precision != LIK_FP32_MIXED)
            return fail(LIK_EINVAL, "unknown precision");
        if (opts->kernel < LIK_KERNEL_AUTO || opts->kernel > LIK_KERNEL_SPECIALIZED)
            return fail(LIK_EINVAL, "unknown kernel variant");
        if ((opts->flags & ~LIK_FLAG_GRAPH) != 0 || opts->reserved != 0)
            return fail(LIK_EINVAL, "unknown flags or nonzero reserved field");
        if (opts->event_cap > LIK_MAX_EVENT_CAP) return fail(LIK_EINVAL, "event_cap above 2^27");
    }
    return LIK_OK;
}

int lik::check_offsets(const int32_t *offs, int32_t M, int *t_max, int64_t *total) {
    if (!offs) return fail(LIK_EINVAL, "obs_offsets is NULL");
    if (offs[0] != 0) return fail(LIK_EINVAL, "obs_offsets[0] must be 0");
    int tm = 0;
    for (int m = 0; m < M; ++m) {
        const int T = offs[m + 1] - offs[m];
        if (T < 1 || T > LIK_MAX_OBS_PER_TRAJ)
            return fail(LIK_EINVAL, "every trajectory needs 1..65535 observations");
        tm = std::max(tm, T);
    }
    *t_max = tm;
    *total = offs[M];
    return LIK_OK;
}

extern "C" {

size_t lik_workspace_size(lik_network_t net, int32_t n_theta, int32_t n_traj,
                          int32_t n_particles) {
    if (!net || n_theta < 0 || n_traj < 1 || n_particles < 1) return 0;
    const size_t F = (size_t)n_theta * n_traj;
    const int Hp = (n_particles + 63) / 64 * 64;
    size_t b = 0;
    b += align256(F * sizeof(FilterDesc));
    b += align256(F * 4) * 4;                 // tcur, fstatus, fflags, cost
    b += align256(F);                         // pool
    b += align256(F * 8) * 2;                 // fll, fevents
    b += align256(F * (Hp / 64) * 4);         // items
    b += align256(kMaxGroups * 4);            // item_count
    b += align256(kMaxGroups * 4);            // item_cursor
    b += 2 * align256(kMaxGroups * kCostKeys * 4) + align256(2 * 4);  // ordering passes
    b += align256((size_t)flow_ring_capacity(F, Hp / 64) * 8 * kFlowRings);  // flow rings
    b += align256(F * 4);                     // flow: items left per slot
    b += align256(kCtlWords * 4);             // flow: control words
    b += align256(request_state_bytes((int64_t)F, net->U, Hp));
    return b + 256;
}

}  // extern "C"

void lik::release_graphs(lik_network &net) {
    std::lock_guard<std::mutex> g(net.graph_lock);
    for (auto &kv : net.graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    net.graphs.clear();
}

namespace {

// Slices an engine's device memory (filter table, state, work items) out of
// one buffer, for `slots` filters with at most `items` work items.
struct EngineLayout {
    FilterDesc *desc;
    EngineArgs e;
    FlowArgs fa;
    int32_t *state;
};

EngineLayout carve_engine(char *p, size_t slots, size_t items, size_t state_bytes,
                          uint32_t ring_capacity) {
    auto take = [&](size_t bytes) {
        char *q = p;
        p += align256(bytes);
        return q;
    };
    EngineLayout L;
    memset(&L.e, 0, sizeof(L.e));
    L.desc = (FilterDesc *)take(slots * sizeof(FilterDesc));
    L.e.desc = L.desc;
    L.e.tcur = (int32_t *)take(slots * 4);
    L.e.fstatus = (int32_t *)take(slots * 4);
    L.e.fflags = (uint32_t *)take(slots * 4);
    L.e.cost = (uint32_t *)take(slots * 4);
    L.e.pool = (uint8_t *)take(slots);
    L.e.fll = (double *)take(slots * 8);
    L.e.fevents = (uint64_t *)take(slots * 8);
    L.e.items = (uint32_t *)take(items * 4);
    L.e.item_count = (uint32_t *)take(kMaxGroups * 4);
    L.e.item_cursor = (uint32_t *)take(kMaxGroups * 4);
    L.e.order_count = (uint32_t *)take(kMaxGroups * kCostKeys * 4);
    L.e.order_pos = (uint32_t *)take(kMaxGroups * kCostKeys * 4);
    L.e.order_ctl = (uint32_t *)take(2 * 4);
    memset(&L.fa, 0, sizeof(L.fa));
    L.fa.ring = (uint64_t *)take((size_t)ring_capacity * 8 * kFlowRings);
    L.fa.remaining = (uint32_t *)take(slots * 4);
    L.fa.ctl = (uint32_t *)take(kCtlWords * 4);
    L.fa.mask = ring_capacity - 1;
    L.fa.n_slots = (int32_t)slots;
    L.state = (int32_t *)take(state_bytes);
    return L;
}

}  // namespace

hipError_t lik::engine_iteration(const EngineArgs &e, const GroupLaunch *groups, int n_groups,
                                 hipStream_t s, bool timed) {
    timed = timed && g_timing.enabled;
    hipError_t err = launch_order(e, s);
    if (err != hipSuccess) return err;
    for (int g = 0; g < n_groups; ++g) {
        const GroupLaunch &G = groups[g];
        if (G.max_items == 0) continue;
        hipEvent_t e0 = timed ? timing_mark(s) : nullptr;
        const bool pers = G.persistent && (G.spec ? G.spec_p != nullptr : G.rmax <= 16);
        const unsigned grid = pers ? std::min(G.max_items, G.persistent_waves) : G.max_items;
        if (G.spec) {
            int group = g;
            void *params[] = {(void *)&e, (void *)&group};
            err = hipModuleLaunchKernel(pers ? G.spec_p : G.spec, grid, 1, 1, kPropBlock, 1, 1, 0,
                                        s, params, nullptr);
        } else {
            err = launch_propagate(e, g, grid, G.netargs, G.umax, G.rmax, G.precision, pers, s);
        }
        if (err != hipSuccess) return err;
        if (timed) g_timing.prop.push_back({e0, timing_mark(s)});
    }
    hipEvent_t w0 = timed ? timing_mark(s) : nullptr;
    err = launch_weigh(e, s);
    if (err == hipSuccess && timed) g_timing.weigh.push_back({w0, timing_mark(s)});
    return err;
}

bool lik::choose_specialized(lik_network &net, int precision, int variant, double work,
                             hipFunction_t *fn, std::string *err) {
    *fn = nullptr;
    // Specialise when the work is large enough to amortise a compile (or a
    // cache read): >= 2^22 particle-intervals.
    if (variant == LIK_KERNEL_SPECIALIZED ||
        (variant == LIK_KERNEL_AUTO && work >= 4194304.0)) {
        *fn = specialized_kernel(net, precision, err);
        if (!*fn && variant == LIK_KERNEL_SPECIALIZED) return false;
    }
    return true;
}

const void *lik::generic_netargs(const lik_network &net) {
    return net.umax == 4 ? (const void *)&net.n4
           : net.umax == 8 ? (const void *)&net.n8
                           : (const void *)&net.n32;
}

// Scratch of lik_eval_batch_device_noalloc: that entry point's workspace, in
// a file-scope device array (every GPU the library runs on holds its own
// copy, at its own address, until the process ends).  In host code the
// array's name is a host-side stand-in, never a device address: host code
// uses only the address hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) unsigned char scratch[LIK_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];  // device address of each device's copy (null: not yet taken)

// The current device's copy of `scratch`: taken once per device, with that
// device current, on the first no-allocation call there.
int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(LIK_EUNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return LIK_OK;
}

// Body of the device-pointer entry points.  no_alloc: the caller cannot
// allocate, so nothing here may -- no graph capture or instantiation, no
// timing events, no compile or load of a specialised kernel (one already
// loaded on this device by an earlier call is used).
int eval_device(lik_network_t net, const lik_obs_model *obs, const lik_eval_opts *opts,
                int32_t n_theta, const double *theta, const lik_data *data,
                const int32_t *obs_offsets_host, int32_t n_particles, uint64_t seed,
                double *loglik_out, int32_t *status_out, const lik_aux *aux, void *workspace,
                size_t workspace_bytes, void *stream, bool no_alloc) {
    if (!data) return fail(LIK_EINVAL, "data is NULL");
    int rc = check_common(net, obs, opts, n_theta, data->n_traj, n_particles);
    if (rc) return rc;
    int t_max = 0;
    int64_t total = 0;
    rc = check_offsets(obs_offsets_host, data->n_traj, &t_max, &total);
    if (rc) return rc;
    if (n_theta == 0) return LIK_OK;
    if (!theta || !loglik_out || !data->obs_offsets || !data->t_obs || !data->y || !data->t0 ||
        !data->x0)
        return fail(LIK_EINVAL, "NULL input or output pointer");
    const size_t need = lik_workspace_size(net, n_theta, data->n_traj, n_particles);
    if (no_alloc && opts && (opts->flags & LIK_FLAG_GRAPH))
        return fail(LIK_EINVAL, "LIK_FLAG_GRAPH needs allocation (graph capture)");
    if (no_alloc && need > workspace_bytes)
        return fail(LIK_EINVAL, "batch needs " + std::to_string(need) +
                                    " bytes of workspace, above the no-allocation entry point's "
                                    "maximum of LIK_NOALLOC_SCRATCH_BYTES");
    if (!workspace || workspace_bytes < need)
        return fail(LIK_EINVAL, "workspace too small (see lik_workspace_size)");
    const bool timed = g_timing.enabled && !no_alloc;

    const int M = data->n_traj;
    const size_t F = (size_t)n_theta * M;
    const int H = n_particles;
    const int Hp = (H + 63) / 64 * 64;
    const int nchunk = Hp / 64;
    char *p = (char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    // the flow schedule launches one wavefront per possible work item (every
    // interval of every filter in groups of 64); beyond 2^26 of them the batch
    // takes the per-interval schedule, with the same results
    const size_t items_max = (size_t)n_theta * (size_t)total * (size_t)nchunk;
    bool flow = net->tuning.schedule == 1 && items_max < ((size_t)1 << 26);
    EngineLayout L = carve_engine(p, F, F * nchunk, request_state_bytes((int64_t)F, net->U, Hp),
                                  flow_ring_capacity(F, nchunk));
    L.e.f_lo = 0;
    L.e.f_hi = (int32_t)F;
    L.e.pool_min = net->tuning.pool_min;
    L.e.pool_max = net->tuning.pool_max;
    L.e.pool_events = net->tuning.pool_events;
    L.e.pool_first = net->tuning.pool_first;
    L.e.refill_min = net->tuning.refill_min;
    L.e.priority = net->tuning.priority;
    L.e.pool_min_items = (uint32_t)net->tuning.items_per_cu * compute_units();
    L.e.h_max = H;
    L.e.pool_chunks = (uint32_t)std::min<size_t>(F * nchunk, 0xFFFFFFFFu);

    const int precision = opts ? opts->precision : LIK_FP64;
    const int variant = opts ? opts->kernel : LIK_KERNEL_AUTO;
    GroupLaunch G;
    G.max_items = (unsigned)(F * nchunk);
    G.netargs = generic_netargs(*net);
    G.umax = net->umax;
    G.rmax = net->rmax;
    G.precision = precision;
    std::string err;
    if (no_alloc) {
        if (variant != LIK_KERNEL_GENERIC) G.spec = loaded_specialized_kernel(*net, precision);
        if (!G.spec && variant == LIK_KERNEL_SPECIALIZED)
            return fail(LIK_EINVAL, "the specialised kernel is not loaded on this device yet "
                                    "(an earlier call of another entry point loads it)");
    } else if (!choose_specialized(*net, precision, variant, (double)F * H * t_max, &G.spec,
                                   &err)) {
        return fail(LIK_EDEVICE, "specialised kernel unavailable: " + err);
    }
    G.persistent = net->tuning.persistent != 0 && net->R <= kPersistentMaxR;
    G.persistent_waves = persistent_waves();
    if (G.spec && G.persistent)
        G.spec_p = no_alloc ? loaded_specialized_kernel(*net, precision, kSpecPersistent)
                            : specialized_kernel(*net, precision, &err, kSpecPersistent);

    // flow schedule: its kernel and one wavefront per work item the batch can
    // have (every interval of every filter in groups of 64)
    hipFunction_t flow_spec = nullptr;
    unsigned flow_waves = 0;
    if (flow) {
        // ... and only where its kernel keeps enough wavefronts resident
        int per_cu = 0;
        if (G.spec) {
            flow_spec = no_alloc ? loaded_specialized_kernel(*net, precision, kSpecFlow)
                                 : specialized_kernel(*net, precision, &err, kSpecFlow);
            if (!flow_spec) return fail(LIK_EDEVICE, "specialised flow kernel unavailable: " + err);
            if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, flow_spec, kPropBlock,
                                                                    0) != hipSuccess)
                per_cu = 0;
        } else {
            per_cu = flow_blocks_per_cu(net->umax, net->rmax, precision);
        }
        flow = per_cu >= kFlowMinWavesPerCu;
    }
    if (flow) {
        flow_waves = (unsigned)std::max<size_t>(items_max, 1);
        L.fa.g_par = (int32_t)std::max<size_t>(
            1, F * nchunk / std::max<uint32_t>(L.e.pool_min_items, 1u));
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
            khz <= 0)
            khz = 100000;
        // one minute; LIK_FLOW_STALL_US overrides it (tests of the give-up path)
        const char *stall_us = getenv("LIK_FLOW_STALL_US");
        const uint64_t us = (stall_us && *stall_us) ? strtoull(stall_us, nullptr, 10) : 60000000ull;
        L.fa.stall_ticks = (uint64_t)khz * us / 1000ull;
        L.fa.urgent_events = net->tuning.urgent_events;
        L.fa.backlog = std::max(compute_units(), 1u) * net->tuning.backlog_per_cu;
    }

    RequestArgs r;
    memset(&r, 0, sizeof(r));
    r.theta = theta;
    r.theta_ids = opts ? opts->theta_ids : nullptr;
    r.obs_offsets = data->obs_offsets;
    r.t_obs = data->t_obs;
    r.y = data->y;
    r.t0 = data->t0;
    r.x0 = data->x0;
    r.x0_hi = data->x0_hi;
    r.state = L.state;
    r.n_theta = n_theta;
    r.M = M;
    r.H = H;
    r.Hp = Hp;
    r.U = net->U;
    r.R = net->R;
    r.P = obs->n_observed;
    r.obs_kind = obs->kind;
    r.group = 0;
    r.precision = precision;
    for (int k = 0; k < LIK_MAX_OBSERVED; ++k) r.obs_species[k] = k < r.P ? obs->species[k] : 0;
    r.sigma = obs->sigma;
    r.gain = obs->gain;
    r.bg_mean = obs->bg_mean;
    r.bg_sd = obs->bg_sd;
    r.seed = seed;
    r.event_cap = (uint32_t)((opts && opts->event_cap) ? opts->event_cap : LIK_DEFAULT_EVENT_CAP);
    r.base = 0;
    fill_reactant_tables(r, net->kind, net->s1, net->s2, net->R);

    hipStream_t s = (hipStream_t)stream;
    auto enqueue = [&](hipStream_t st) -> int {
        hipError_t e = launch_admit(L.desc, L.e, r, st);
        if (e != hipSuccess) return hip_fail(e, "admit launch");
        if (r.x0_hi && (e = launch_init_start(L.desc, 0, (int32_t)F, st)) != hipSuccess)
            return hip_fail(e, "initial-count launch");
        if (flow) {
            e = launch_flow_setup(L.e, L.fa, st);
            if (e != hipSuccess) return hip_fail(e, "flow setup launch");
            hipEvent_t e0 = timed ? timing_mark(st) : nullptr;
            if (flow_spec) {
                EngineArgs ea = L.e;
                const FlowArgs *fb = flow_args_copy(L.fa.ctl);  // written by k_flow_init
                void *params[] = {(void *)&ea, (void *)&fb};
                e = hipModuleLaunchKernel(flow_spec, flow_waves, 1, 1, kPropBlock, 1, 1, 0, st,
                                          params, nullptr);
            } else {
                e = launch_flow(L.e, L.fa, flow_waves, G.netargs, G.umax, G.rmax, precision, st);
            }
            if (e != hipSuccess) return hip_fail(e, "flow launch");
            if (timed) g_timing.prop.push_back({e0, timing_mark(st)});
            e = launch_flow_check(L.e, L.fa, st);
            if (e != hipSuccess) return hip_fail(e, "flow check launch");
        } else {
            e = launch_order_reset(L.e, st);
            if (e != hipSuccess) return hip_fail(e, "order reset launch");
            for (int t = 0; t < t_max; ++t) {
                e = engine_iteration(L.e, &G, 1, st, timed);
                if (e != hipSuccess) return hip_fail(e, "iteration launch");
            }
        }
        e = launch_finish(L.e, 0, n_theta, M, loglik_out, status_out, aux, st);
        if (e != hipSuccess) return hip_fail(e, "finish launch");
        return LIK_OK;
    };
    if (!(opts && (opts->flags & LIK_FLAG_GRAPH))) return enqueue(s);

    // Graph path: everything but the seed is fixed by the key below.
    std::string key;
    auto add = [&](const void *v, size_t n) { key.append((const char *)v, n); };
    const void *ptrs[] = {theta, r.theta_ids, data->obs_offsets, data->t_obs, data->y, data->t0,
                          data->x0, data->x0_hi, loglik_out, status_out,
                          aux ? aux->filter_events : nullptr,
                          aux ? aux->filter_loglik : nullptr, aux ? aux->final_state : nullptr,
                          workspace, (const void *)G.spec};
    add(ptrs, sizeof(ptrs));
    const int32_t ints[] = {n_theta, M, H, precision, r.P, r.obs_kind, t_max};
    add(ints, sizeof(ints));
    add(obs_offsets_host, (size_t)(M + 1) * 4);
    add(r.obs_species, sizeof(r.obs_species));
    add(&r.sigma, 8);
    add(&r.gain, 8);
    add(&r.bg_mean, 8);
    add(&r.bg_sd, 8);
    add(&r.event_cap, 4);
    add(&net->tuning, sizeof(lik_tuning));
    int dev = 0;
    (void)hipGetDevice(&dev);
    add(&dev, 4);
    std::lock_guard<std::mutex> lock(net->graph_lock);
    auto it = net->graphs.find(key);
    if (it == net->graphs.end()) {
        lik_network::Graph g;
        // Capture only records the launches, on a private stream (the
        // caller's may be the legacy default stream, which cannot capture);
        // the graph is launched on the caller's stream below.
        hipStream_t cs = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cs);
            return hip_fail(e, "hipStreamBeginCapture");
        }
        const bool timing = g_timing.enabled;
        g_timing.enabled = false;  // no timing events inside a captured graph
        int rc2 = enqueue(cs);
        g_timing.enabled = timing;
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        (void)hipStreamDestroy(cs);
        if (rc2 != LIK_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc2;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        // the admission kernel node: its arguments carry the seed
        size_t n = 0;
        (void)hipGraphGetNodes(graph, nullptr, &n);
        std::vector<hipGraphNode_t> nodes(n);
        (void)hipGraphGetNodes(graph, nodes.data(), &n);
        for (hipGraphNode_t nd : nodes) {
            hipGraphNodeType ty;
            if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
            hipKernelNodeParams kp;
            if (hipGraphKernelNodeGetParams(nd, &kp) == hipSuccess && kp.func == admit_kernel()) {
                g.admit = nd;
                g.admit_blocks = kp.gridDim.x;
            }
        }
        if (!g.admit) {
            (void)hipGraphDestroy(graph);
            return fail(LIK_EDEVICE, "captured graph has no admission node");
        }
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(e, "hipGraphInstantiate");
        }
        g.graph = graph;
        g.desc = L.desc;
        g.e = L.e;
        g.r = r;
        it = net->graphs.emplace(key, g).first;
    }
    lik_network::Graph &g = it->second;
    RequestArgs rr = g.r;
    rr.seed = seed;
    FilterDesc *dsc = g.desc;
    EngineArgs ee = g.e;
    void *args[] = {(void *)&dsc, (void *)&ee, (void *)&rr};
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof(kp));
    kp.func = (void *)admit_kernel();
    kp.gridDim = dim3(g.admit_blocks);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipError_t e = hipGraphExecKernelNodeSetParams(g.exec, g.admit, &kp);
    if (e != hipSuccess) return hip_fail(e, "hipGraphExecKernelNodeSetParams");
    e = hipGraphLaunch(g.exec, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return LIK_OK;
}

}  // namespace

extern "C" {

int lik_eval_batch_device(lik_network_t net, const lik_obs_model *obs, const lik_eval_opts *opts,
                          int32_t n_theta, const double *theta, const lik_data *data,
                          const int32_t *obs_offsets_host, int32_t n_particles, uint64_t seed,
                          double *loglik_out, int32_t *status_out, const lik_aux *aux,
                          void *workspace, size_t workspace_bytes, void *stream) {
    return eval_device(net, obs, opts, n_theta, theta, data, obs_offsets_host, n_particles, seed,
                       loglik_out, status_out, aux, workspace, workspace_bytes, stream, false);
}

int lik_eval_batch_device_noalloc(lik_network_t net, const lik_obs_model *obs,
                                  const lik_eval_opts *opts, int32_t n_theta, const double *theta,
                                  const lik_data *data, const int32_t *obs_offsets_host,
                                  int32_t n_particles, uint64_t seed, double *loglik_out,
                                  int32_t *status_out, const lik_aux *aux, void *stream) {
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc) return rc;
    return eval_device(net, obs, opts, n_theta, theta, data, obs_offsets_host, n_particles, seed,
                       loglik_out, status_out, aux, ws, LIK_NOALLOC_SCRATCH_BYTES, stream, true);
}

int lik_eval_batch(lik_network_t net, const lik_obs_model *obs, const lik_eval_opts *opts,
                   int32_t n_theta, const double *theta, const lik_data *data,
                   int32_t n_particles, uint64_t seed, double *loglik_out, int32_t *status_out,
                   const lik_aux *aux) {
    if (!data) return fail(LIK_EINVAL, "data is NULL");
    int rc = check_common(net, obs, opts, n_theta, data->n_traj, n_particles);
    if (rc) return rc;
    int t_max = 0;
    int64_t total = 0;
    rc = check_offsets(data->obs_offsets, data->n_traj, &t_max, &total);
    if (rc) return rc;
    const int M = data->n_traj, U = net->U, P = obs->n_observed;
    if (n_theta == 0) return LIK_OK;
    if (!theta || !loglik_out || !data->t_obs || !data->y || !data->t0 || !data->x0)
        return fail(LIK_EINVAL, "NULL input or output pointer");
    rc = check_host_data(net, obs, data, n_theta, opts ? opts->theta_ids : nullptr);
    if (rc) return rc;

    const size_t F = (size_t)n_theta * M;
    const size_t ws = lik_workspace_size(net, n_theta, M, n_particles);
    const size_t sz_theta = (size_t)n_theta * net->R * 8;
    const size_t sz_ids = (opts && opts->theta_ids) ? (size_t)n_theta * 4 : 0;
    const size_t sz_off = (size_t)(M + 1) * 4, sz_t = (size_t)total * 8;
    const size_t sz_y = (size_t)total * P * 8, sz_t0 = (size_t)M * 8, sz_x0 = (size_t)M * U * 4;
    const size_t sz_x0h = data->x0_hi ? sz_x0 : 0;
    const size_t sz_ll = (size_t)n_theta * 8, sz_st = (size_t)n_theta * 4;
    const size_t sz_ev = (aux && aux->filter_events) ? F * 8 : 0;
    const size_t sz_fl = (aux && aux->filter_loglik) ? F * 8 : 0;
    const size_t sz_fs = (aux && aux->final_state) ? F * U * n_particles * 4 : 0;
    const size_t sizes[] = {sz_theta, sz_ids, sz_off, sz_t, sz_y, sz_t0, sz_x0, sz_x0h,
                            sz_ll, sz_st, sz_ev, sz_fl, sz_fs, ws};
    size_t total_bytes = 0;
    for (size_t v : sizes) total_bytes += align256(v);
    char *dev = nullptr;
    hipError_t e = hipMalloc((void **)&dev, total_bytes + 256);
    if (e != hipSuccess) return fail(LIK_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    char *p = dev;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += align256(bytes);
        return q;
    };
    double *d_theta = (double *)take(sz_theta);
    uint32_t *d_ids = (uint32_t *)take(sz_ids);
    int32_t *d_off = (int32_t *)take(sz_off);
    double *d_t = (double *)take(sz_t);
    double *d_y = (double *)take(sz_y);
    double *d_t0 = (double *)take(sz_t0);
    int32_t *d_x0 = (int32_t *)take(sz_x0);
    int32_t *d_x0h = (int32_t *)take(sz_x0h);
    double *d_ll = (double *)take(sz_ll);
    int32_t *d_st = (int32_t *)take(sz_st);
    uint64_t *d_ev = (uint64_t *)take(sz_ev);
    double *d_fl = (double *)take(sz_fl);
    int32_t *d_fs = (int32_t *)take(sz_fs);
    void *d_ws = take(ws);

    hipStream_t s = nullptr;
    rc = LIK_OK;
    do {
        if ((e = hipStreamCreate(&s)) != hipSuccess) { rc = hip_fail(e, "hipStreamCreate"); break; }
        struct { void *d; const void *h; size_t n; } up[] = {
            {d_theta, theta, sz_theta}, {d_ids, opts ? opts->theta_ids : nullptr, sz_ids},
            {d_off, data->obs_offsets, sz_off}, {d_t, data->t_obs, sz_t}, {d_y, data->y, sz_y},
            {d_t0, data->t0, sz_t0}, {d_x0, data->x0, sz_x0}, {d_x0h, data->x0_hi, sz_x0h}};
        for (auto &u : up) {
            if (!u.n) continue;
            if ((e = hipMemcpyAsync(u.d, u.h, u.n, hipMemcpyHostToDevice, s)) != hipSuccess) break;
        }
        if (e != hipSuccess) { rc = hip_fail(e, "copy to device"); break; }
        lik_eval_opts o = opts ? *opts : lik_eval_opts{LIK_FP64, LIK_KERNEL_AUTO, 0, nullptr, 0, 0};
        o.theta_ids = sz_ids ? d_ids : nullptr;
        lik_data dd = {M, d_off, d_t, d_y, d_t0, d_x0, sz_x0h ? d_x0h : nullptr};
        lik_aux da = {sz_ev ? d_ev : nullptr, sz_fl ? d_fl : nullptr, sz_fs ? d_fs : nullptr};
        rc = lik_eval_batch_device(net, obs, &o, n_theta, d_theta, &dd, data->obs_offsets,
                                   n_particles, seed, d_ll, d_st, aux ? &da : nullptr, d_ws, ws, s);
        if (rc) break;
        struct { void *h; const void *d; size_t n; } down[] = {
            {loglik_out, d_ll, sz_ll}, {status_out, d_st, status_out ? sz_st : 0},
            {aux ? aux->filter_events : nullptr, d_ev, sz_ev},
            {aux ? aux->filter_loglik : nullptr, d_fl, sz_fl},
            {aux ? aux->final_state : nullptr, d_fs, sz_fs}};
        for (auto &d : down) {
            if (!d.n) continue;
            if ((e = hipMemcpyAsync(d.h, d.d, d.n, hipMemcpyDeviceToHost, s)) != hipSuccess) break;
        }
        if (e != hipSuccess) { rc = hip_fail(e, "copy to host"); break; }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = hip_fail(e, "synchronize"); break; }
    } while (0);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(dev);
    return rc;
}

}  // extern "C"
