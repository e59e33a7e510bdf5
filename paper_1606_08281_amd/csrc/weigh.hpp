// weigh.hpp -- the per-filter arithmetic of the weighing step, shared by the
// per-interval engine (k_weigh, one workgroup per filter) and the flow
// engine (one wavefront per filter, flow.hpp), so that both compute every
// log-weight, the log-likelihood increment and the resampling offset with
// the same operations in the same order.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "devmath.hpp"
#include "lik_internal.hpp"

namespace lik {

// ---------------------------------------------------------------------------
// wavefront reductions (butterflies: every lane ends with the same value;
// lane = lane_id())
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v, int lane) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, lane_read(v, lane ^ off));
    return v;
}

__device__ __forceinline__ double wave_sum(double v, int lane) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += lane_read(v, lane ^ off);
    return v;
}

__device__ __forceinline__ float wave_sum_f32(float v, int lane) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += lane_read(v, lane ^ off);
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v, int lane) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += lane_read(v, lane ^ off);
    return v;
}

// inclusive prefix sum over the 64 lanes of a wavefront
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t o = lane_read(v, lane >= off ? lane - off : lane);
        if (lane >= off) v += o;
    }
    return v;
}

__device__ __forceinline__ bool slot_active(const EngineArgs &e, int f) {
    return !(e.fflags[f] & kFlagStopped) && e.tcur[f] < e.desc[f].T;
}

// Pool size G of slot f for its coming interval (c: expected events of the
// slot), at most g_par, the LDS budget and the slot's groups of 64.
__device__ __forceinline__ int pool_size(const EngineArgs &e, int f, uint32_t c, int g_par) {
    const int nchunk = e.desc[f].Hp >> 6;
    int g;
    if (e.tcur[f] == 0 && c == 0) {
        g = e.pool_first;  // no estimate
    } else {
        const uint32_t per = c / (uint32_t)e.desc[f].H;  // expected events per particle
        const uint32_t want = e.pool_events / (per > 0 ? per : 1u);
        g = (int)min(want, (uint32_t)e.pool_max);
        g = max(g, e.pool_min);
    }
    const int lds_cap = pool_lds_cap(e.desc[f].U);  // pool fits in LDS
    g = min(min(g, lds_cap), g_par);
    return min(max(g, 1), nchunk);
}

// log p(y_t | x_j) without its particle-independent part (the "Compute
// l_t^i" step): a sum over the observed components of -z^2/2, with z the
// standardised residual of y (Gaussian) or of log y (log-normal, where a
// count <= 0 has density zero); for the fluorescence model, whose variance
// v = sigma^2 x + bg_sd^2 depends on the count, -r^2/(2v) - log(v)/2 with
// r = y - (gain x + bg_mean).  logy[k] = log y_k for the log-normal model.
// obs_term adds component k's term to l; false (l = -inf, later components
// skipped) for a log-normal observation of a count <= 0.
// The observation model's parameters of one filter, read once into scalar
// registers (every lane of a wavefront weighs particles of the same filter).
struct ObsParams {
    int kind;
    double sigma, gain, bg_mean, s2, b2;
};
__device__ __forceinline__ ObsParams obs_params(const FilterDesc &d) {
    return ObsParams{wave_uniform(d.obs_kind), wave_uniform(d.sigma), wave_uniform(d.gain),
                     wave_uniform(d.bg_mean), wave_uniform(d.obs_s2), wave_uniform(d.bg_s2)};
}

// FLUO false: the caller has excluded the fluorescence model (a shorter body).
template <bool FLUO = true>
__device__ __forceinline__ bool obs_term(const ObsParams &o, int k, int cnt, const double *logy,
                                         const double *yt, double &l) {
    if (FLUO && o.kind == LIK_OBS_FLUORESCENCE) {
        const double x = (double)cnt;
        const double v = o.s2 * x + o.b2;
        const double r = yt[k] - (o.gain * x + o.bg_mean);
        l = l - 0.5 * ((r * r) / v);
        l = l - 0.5 * dlog(v);
    } else if (o.kind == LIK_OBS_LOGNORMAL) {
        if (cnt <= 0) {
            l = -__builtin_inf();
            return false;
        }
        const double z = (logy[k] - dlog((double)cnt)) / o.sigma;
        l = l - 0.5 * (z * z);
    } else {
        const double z = (yt[k] - (double)cnt) / o.sigma;
        l = l - 0.5 * (z * z);
    }
    return true;
}

__device__ __forceinline__ double obs_logweight(const FilterDesc &d, const ObsParams &o,
                                                const int32_t *xs, int j, const double *logy,
                                                const double *yt) {
    double l = 0.0;
    for (int k = 0; k < d.P; ++k)
        if (!obs_term(o, k, xs[(size_t)d.obs_species[k] * d.Hp + j], logy, yt, l)) break;
    return l;
}

// Log of the mean weight plus the particle-independent part of the
// observation density: the interval's factor of the likelihood estimate.
// mx: largest log-weight, S: sum of exp(l_j - mx).
__device__ __forceinline__ double loglik_increment(const FilterDesc &d, double mx, double S,
                                                   const double *yt) {
    const double half_log_2pi = 0.5 * dlog(2.0 * 3.141592653589793);
    const double per_comp =
        d.obs_kind == LIK_OBS_FLUORESCENCE ? half_log_2pi : dlog(d.sigma) + half_log_2pi;
    double cst = -((double)d.P * per_comp);
    if (d.obs_kind == LIK_OBS_LOGNORMAL)
        for (int k = 0; k < d.P; ++k) cst = cst - dlog(yt[k]);
    return ((mx + dlog(S)) - dlog((double)d.H)) + cst;
}

// The 64-bit uniform word of the systematic resampling before interval
// t + 1 (stream purpose 1).
__device__ __forceinline__ uint64_t resample_word(const FilterDesc &d, int t) {
    const Block4 b = philox4x32_10(0u, 0u, (d.traj << 16) | (uint32_t)(t + 1),
                                   (d.theta_id << 2) | 1u, (uint32_t)d.seed,
                                   (uint32_t)(d.seed >> 32));
    return ((uint64_t)b.w1 << 32) | b.w0;
}

// Expected events of the next interval (a scheduling estimate): the summed
// total propensities of the resampled particles' states times its length.
__device__ __forceinline__ uint32_t cost_estimate(const FilterDesc &d, int t, double tot) {
    const double expect = tot * (d.t_obs[t + 1] - d.t_obs[t]);
    return expect >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)expect;
}

}  // namespace lik
