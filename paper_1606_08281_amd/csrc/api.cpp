// api.cpp -- C ABI of liblik.so: validation, workspace layout, launch order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/lik.h"
#include "lik_internal.hpp"

using namespace lik;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where) {
    return fail(LIK_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

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

struct lik_network {
    int32_t U, R;
    int32_t umax, rmax;  // kernel size bucket
    std::vector<int32_t> orders, stoich;
    int32_t kind[LIK_MAX_REACTIONS];
    int32_t s1[LIK_MAX_REACTIONS], s2[LIK_MAX_REACTIONS];
    uint32_t nu[LIK_MAX_REACTIONS][4];
    Net4x8 n4;
    Net8x16 n8;
    Net32x64 n32;
};

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

int lik_destroy_network(lik_network_t net) {
    delete net;
    return LIK_OK;
}

static int check_common(lik_network_t net, const lik_obs_model *obs, const lik_eval_opts *opts,
                        int32_t n_theta, int32_t n_traj, int32_t n_particles) {
    if (!net) return fail(LIK_EINVAL, "network is NULL");
    if (!obs) return fail(LIK_EINVAL, "observation model is NULL");
    if (obs->kind != LIK_OBS_GAUSSIAN && obs->kind != LIK_OBS_LOGNORMAL)
        return fail(LIK_EINVAL, "unknown observation kind");
    if (obs->n_observed < 1 || obs->n_observed > LIK_MAX_OBSERVED)
        return fail(LIK_EINVAL, "n_observed must be in [1, 8]");
    for (int k = 0; k < obs->n_observed; ++k)
        if (obs->species[k] < 0 || obs->species[k] >= net->U)
            return fail(LIK_EINVAL, "observed species out of range");
    if (!(obs->sigma > 0.0) || isinf(obs->sigma)) return fail(LIK_EINVAL, "sigma must be > 0");
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
        if (opts->reserved != 0) return fail(LIK_EINVAL, "reserved must be 0");
        if (opts->event_cap > LIK_MAX_EVENT_CAP) return fail(LIK_EINVAL, "event_cap above 2^27");
    }
    return LIK_OK;
}

static int check_offsets(const int32_t *offs, int32_t M, int *t_max, int64_t *total) {
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

size_t lik_workspace_size(lik_network_t net, int32_t n_theta, int32_t n_traj,
                          int32_t n_particles) {
    if (!net || n_theta < 0 || n_traj < 1 || n_particles < 1) return 0;
    const size_t F = (size_t)n_theta * n_traj;
    const size_t Hp = (size_t)((n_particles + 63) / 64) * 64;
    size_t b = 0;
    b += align256(F * net->U * Hp * 4) * 2;  // xa, xb
    b += align256(F * Hp * 8);               // lw
    b += align256(F * Hp * 4);               // anc
    b += align256(F * 8);                    // fll
    b += align256(F * 4) * 2;                // fstatus, fflags
    b += align256(F * 8);                    // fevents
    b += align256(F * 4) * 3;                // fsteps, order, cost
    return b + 256;
}

int lik_eval_batch_device(lik_network_t net, const lik_obs_model *obs, const lik_eval_opts *opts,
                          int32_t n_theta, const double *theta, const lik_data *data,
                          const int32_t *obs_offsets_host, int32_t n_particles, uint64_t seed,
                          double *loglik_out, int32_t *status_out, const lik_aux *aux,
                          void *workspace, size_t workspace_bytes, void *stream) {
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
    if (!workspace || workspace_bytes < need)
        return fail(LIK_EINVAL, "workspace too small (see lik_workspace_size)");

    const int M = data->n_traj;
    const size_t F = (size_t)n_theta * M;
    const int H = n_particles;
    const int Hp = (H + 63) / 64 * 64;
    EvalArgs a;
    memset(&a, 0, sizeof(a));
    a.theta = theta;
    a.theta_ids = opts ? opts->theta_ids : nullptr;
    a.obs_offsets = data->obs_offsets;
    a.t_obs = data->t_obs;
    a.y = data->y;
    a.t0 = data->t0;
    a.x0 = data->x0;
    a.n_theta = n_theta;
    a.M = M;
    a.H = H;
    a.Hp = Hp;
    a.U = net->U;
    a.R = net->R;
    a.P = obs->n_observed;
    a.nchunk = (H + kPropBlock - 1) / kPropBlock;
    a.obs_kind = obs->kind;
    for (int k = 0; k < LIK_MAX_OBSERVED; ++k) a.obs_species[k] = k < a.P ? obs->species[k] : 0;
    a.sigma = obs->sigma;
    a.seed = seed;
    a.event_cap = (uint32_t)((opts && opts->event_cap) ? opts->event_cap : LIK_DEFAULT_EVENT_CAP);

    char *p = (char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    auto take = [&](size_t bytes) {
        char *q = p;
        p += align256(bytes);
        return q;
    };
    a.xa = (int32_t *)take(F * a.U * Hp * 4);
    a.xb = (int32_t *)take(F * a.U * Hp * 4);
    a.lw = (double *)take(F * Hp * 8);
    a.anc = (int32_t *)take(F * Hp * 4);
    a.fll = (double *)take(F * 8);
    a.fstatus = (int32_t *)take(F * 4);
    a.fflags = (uint32_t *)take(F * 4);
    a.fevents = (uint64_t *)take(F * 8);
    a.fsteps = (int32_t *)take(F * 4);
    a.order = (uint32_t *)take(F * 4);
    a.cost = (uint32_t *)take(F * 4);

    const void *netargs = net->umax == 4 ? (const void *)&net->n4
                          : net->umax == 8 ? (const void *)&net->n8
                                           : (const void *)&net->n32;
    const int precision = opts ? opts->precision : LIK_FP64;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_init(a, s);
    if (e != hipSuccess) return hip_fail(e, "init launch");
    for (int t = 0; t < t_max; ++t) {
        if (t > 0) {
            e = launch_order(a, t, s);
            if (e != hipSuccess) return hip_fail(e, "order launch");
        }
        hipEvent_t e0 = g_timing.enabled ? timing_mark(s) : nullptr;
        e = launch_propagate(a, netargs, net->umax, net->rmax, precision, t, s);
        if (e != hipSuccess) return hip_fail(e, "propagate launch");
        hipEvent_t e1 = g_timing.enabled ? timing_mark(s) : nullptr;
        e = launch_weigh(a, t, s);
        if (e != hipSuccess) return hip_fail(e, "weigh launch");
        if (g_timing.enabled) {
            hipEvent_t e2 = timing_mark(s);
            g_timing.prop.push_back({e0, e1});
            g_timing.weigh.push_back({e1, e2});
        }
    }
    e = launch_finish(a, loglik_out, status_out, aux, s);
    if (e != hipSuccess) return hip_fail(e, "finish launch");
    return LIK_OK;
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
    // host-side checks of the observations
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
        }
    }
    if (opts && opts->theta_ids)
        for (int i = 0; i < n_theta; ++i)
            if (opts->theta_ids[i] >= (1u << 30)) return fail(LIK_EINVAL, "theta id >= 2^30");

    const size_t F = (size_t)n_theta * M;
    const size_t ws = lik_workspace_size(net, n_theta, M, n_particles);
    const size_t sz_theta = (size_t)n_theta * net->R * 8;
    const size_t sz_ids = (opts && opts->theta_ids) ? (size_t)n_theta * 4 : 0;
    const size_t sz_off = (size_t)(M + 1) * 4, sz_t = (size_t)total * 8;
    const size_t sz_y = (size_t)total * P * 8, sz_t0 = (size_t)M * 8, sz_x0 = (size_t)M * U * 4;
    const size_t sz_ll = (size_t)n_theta * 8, sz_st = (size_t)n_theta * 4;
    const size_t sz_ev = (aux && aux->filter_events) ? F * 8 : 0;
    const size_t sz_fl = (aux && aux->filter_loglik) ? F * 8 : 0;
    const size_t sz_fs = (aux && aux->final_state) ? F * U * n_particles * 4 : 0;
    const size_t sizes[] = {sz_theta, sz_ids, sz_off, sz_t, sz_y, sz_t0, sz_x0,
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
            {d_t0, data->t0, sz_t0}, {d_x0, data->x0, sz_x0}};
        for (auto &u : up) {
            if (!u.n) continue;
            if ((e = hipMemcpyAsync(u.d, u.h, u.n, hipMemcpyHostToDevice, s)) != hipSuccess) break;
        }
        if (e != hipSuccess) { rc = hip_fail(e, "copy to device"); break; }
        lik_eval_opts o = opts ? *opts : lik_eval_opts{LIK_FP64, 0, 0, nullptr};
        o.theta_ids = sz_ids ? d_ids : nullptr;
        lik_data dd = {M, d_off, d_t, d_y, d_t0, d_x0};
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
