// propagate.hpp -- one propagation work item: 64 particles of one filter.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "devmath.hpp"
#include "lik_internal.hpp"

namespace lik {

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Propensities a_r = c_r h_r(x) and their running sums S_r in reaction
// order (h_r = prod_u C(x_u, p_ru)); returns S_{R-1}.  Real is double for the
// binary64 step; for the binary32 step the factor h_r (exact in binary64) is
// rounded to binary32 and multiplied by the binary32 rate.
template <class NetT, int RMAX, class Real>
__device__ __forceinline__ Real running_sums(const NetT &net, const Real *c, const int *x,
                                             Real *S) {
    Real s = (Real)0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        if (r < net.R) {
            double h;
            const int kind = net.kind[r];
            if (kind == kOrder0) {
                h = 1.0;
            } else if (kind == kOrder1) {
                h = (double)x[net.s1[r]];
            } else if (kind == kOrder2Homo) {
                const int v = x[net.s1[r]];
                h = 0.5 * ((double)v * (double)(v - 1));
            } else {
                h = (double)x[net.s1[r]] * (double)x[net.s2[r]];
            }
            s = s + c[r] * (Real)h;
            S[r] = s;
        }
    }
    return s;
}

// Packed net change of r* = min{r : S_r > target}.  S_{R-1} > target always:
// target = fl(u2 S_{R-1}) with u2 <= 1 - 2^-53 (binary32: 1 - 2^-24) stays
// below S_{R-1}, and a zero propensity repeats the previous sum, so r* has
// a_r* > 0.
template <class NetT, int RMAX, int W, class Real>
__device__ __forceinline__ void select_reaction(const NetT &net, const Real *S, Real target,
                                                uint32_t *sel) {
#pragma unroll
    for (int w = 0; w < W; ++w) sel[w] = net.nu[net.R - 1][w];
#pragma unroll
    for (int r = RMAX - 2; r >= 0; --r) {
        if (r < net.R - 1) {
            const bool hit = S[r] > target;
#pragma unroll
            for (int w = 0; w < W; ++w) sel[w] = hit ? net.nu[r][w] : sel[w];
        }
    }
}

template <int UMAX, int W>
__device__ __forceinline__ void apply_change(int U, const uint32_t *sel, int *x) {
#pragma unroll
    for (int u = 0; u < UMAX; ++u)
        if (u < U) x[u] += __builtin_amdgcn_sbfe(sel[u >> 3], 4 * (u & 7), 4);
}

// ---------------------------------------------------------------------------
// propagate: resample-gather, direct-method SSA to the next observation time,
// particle log-weight.
// ---------------------------------------------------------------------------
// NetT provides U, R, kind[], s1[], s2[], nu[][W] either as kernel-argument
// data (generic kernels) or as compile-time constants (network-specialised
// kernels); the arithmetic is the same in both.
template <class NetT, int UMAX, int RMAX, int W, int PREC>
__device__ __forceinline__ void propagate_item(const EngineArgs &e, const NetT &net, int group) {
    if (blockIdx.x >= e.item_count[group]) return;
    const uint32_t item = e.items[e.group_off[group] + blockIdx.x];
    const int f = (int)(item >> 6);
    const int chunk = (int)(item & 63u);
    const FilterDesc &d = e.desc[f];
    const int t = e.tcur[f];

    const int U = net.U;
    const int R = net.R;
    const int H = d.H;
    const int Hp = d.Hp;
    const int j = chunk * kPropBlock + (int)threadIdx.x;
    const bool active = j < H;
    const double t_start = (t == 0) ? d.t0 : d.t_obs[t - 1];
    const double t_end = d.t_obs[t];
    const uint32_t c2 = (d.traj << 16) | (uint32_t)t;
    const uint32_t c3 = d.theta_id << 2;  // purpose 0: reaction events
    const uint32_t k0 = (uint32_t)d.seed, k1 = (uint32_t)(d.seed >> 32);

    double c[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) c[r] = (r < R) ? d.theta[r] : 0.0;

    int x[UMAX];
    if (t == 0) {
#pragma unroll
        for (int u = 0; u < UMAX; ++u) x[u] = (u < U) ? d.x0[u] : 0;
    } else {
        const int32_t *src = (t & 1) ? d.xb : d.xa;
        const int anc = active ? d.anc[j] : 0;
#pragma unroll
        for (int u = 0; u < UMAX; ++u) x[u] = (u < U) ? src[(size_t)u * Hp + anc] : 0;
    }

    uint32_t n = 0;
    int st = LIK_STATUS_OK;
    if (active) {
        double clock = t_start;
        if (PREC == LIK_FP32_MIXED) {
            float cf[RMAX];
#pragma unroll
            for (int r = 0; r < RMAX; ++r) cf[r] = (float)c[r];
            // Event n uses words 2(n&1), 2(n&1)+1 of block n>>1: both events
            // of a pair sit in one iteration, so every lane enters it at an
            // even n and one block serves two events.
            float Sf[RMAX];
            auto fire = [&](uint32_t wa, uint32_t wb, float sf) -> bool {
                const float u1 = (float)((wa >> 8) + 1u) * 0x1p-24f;
                const float u2 = (float)(wb >> 8) * 0x1p-24f;
                const float tau = -flog(u1) / sf;
                const double tau_d = (double)tau;
                if (clock + tau_d > t_end) return false;  // the pending event is discarded
                uint32_t sel[W];
                select_reaction<NetT, RMAX, W, float>(net, Sf, u2 * sf, sel);
                apply_change<UMAX, W>(U, sel, x);
                clock = clock + tau_d;
                n = n + 1;
                return true;
            };
            for (;;) {
                float sf = running_sums<NetT, RMAX, float>(net, cf, x, Sf);
                if (!(sf > 0.0f)) break;
                if (n >= d.event_cap) { st = LIK_STATUS_EVENT_CAP; break; }
                const Block4 b = philox4x32_10(n >> 1, (uint32_t)j, c2, c3, k0, k1);
                if (!fire(b.w0, b.w1, sf)) break;
                sf = running_sums<NetT, RMAX, float>(net, cf, x, Sf);
                if (!(sf > 0.0f)) break;
                if (n >= d.event_cap) { st = LIK_STATUS_EVENT_CAP; break; }
                if (!fire(b.w2, b.w3, sf)) break;
            }
        } else {
            double S[RMAX];
            for (;;) {
                const double s = running_sums<NetT, RMAX, double>(net, c, x, S);
                if (!(s > 0.0)) break;
                if (n >= d.event_cap) { st = LIK_STATUS_EVENT_CAP; break; }
                const Block4 b = philox4x32_10(n, (uint32_t)j, c2, c3, k0, k1);
                const uint64_t z1 = ((((uint64_t)b.w1) << 32) | b.w0) >> 11;
                const uint64_t z2 = ((((uint64_t)b.w3) << 32) | b.w2) >> 11;
                const double u1 = (double)(z1 + 1) * 0x1p-53;  // (0, 1]
                const double u2 = (double)z2 * 0x1p-53;        // [0, 1)
                const double tau = -dlog(u1) / s;
                if (clock + tau > t_end) break;  // the pending event is discarded
                uint32_t sel[W];
                select_reaction<NetT, RMAX, W, double>(net, S, u2 * s, sel);
                apply_change<UMAX, W>(U, sel, x);
                clock = clock + tau;
                n = n + 1;
            }
        }
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < U && x[u] > kCountLimit) st = st > LIK_STATUS_COUNT_OVERFLOW ? st : LIK_STATUS_COUNT_OVERFLOW;

        // Particle-dependent part of log p(y_t | x).
        const double *yt = d.y + (size_t)t * d.P;
        double lw = 0.0;
        for (int k = 0; k < d.P; ++k) {
            const int cnt = x[d.obs_species[k]];
            if (d.obs_kind == LIK_OBS_LOGNORMAL) {
                if (cnt <= 0) {
                    lw = -__builtin_inf();
                    break;
                }
                const double z = (dlog(yt[k]) - dlog((double)cnt)) / d.sigma;
                lw = lw - 0.5 * (z * z);
            } else {
                const double z = (yt[k] - (double)cnt) / d.sigma;
                lw = lw - 0.5 * (z * z);
            }
        }
        int32_t *dst = (t & 1) ? d.xa : d.xb;
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < U) dst[(size_t)u * Hp + j] = x[u];
        d.lw[j] = lw;
        if (st != LIK_STATUS_OK) atomicMax(&e.fstatus[f], st);
    }
    const uint64_t ev = wave_sum_u64((uint64_t)n);
    if (threadIdx.x == 0 && ev) {
        atomicAdd((unsigned long long *)&e.fevents[f], (unsigned long long)ev);
        atomicAdd(&e.cost[f], (uint32_t)(ev > 0xFFFFFFFFull ? 0xFFFFFFFFu : ev));
    }
}

}  // namespace lik
