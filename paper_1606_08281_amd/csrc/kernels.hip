// kernels.hip -- gfx950 kernels of the particle-filter likelihood engine.
//
// One engine iteration advances every active filter slot by one observation
// interval:
//   k_order: the work list.  Active slots, grouped by (network, precision),
//     heaviest first by the events their particles are expected to need;
//     each slot contributes one item per pool of G * 64 particles.
//   k_propagate (body in propagate.hpp): one wavefront per item, a pool of
//     particles of one slot.  Gathers each particle's ancestor state and runs
//     Gillespie's direct method from the previous observation time to the
//     next one (Supplementary I, Algorithm "Likelihood Approximation using
//     particle filter", the "Simulate" step).
//   k_weigh: one workgroup per slot.  The particles' log-weights (the
//     "Compute l_t^i" step), their log-sum-exp into the running
//     log-likelihood (multiplying p(y_{t-1}|theta) by the mean weight), then
//     systematic resampling with integer weights for the next interval (the
//     "Sample H indices according to weights" step).
// k_admit fills the slots of a request; k_finish sums its log-likelihoods
// over trajectories.
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#endif

#include "devmath.hpp"
#include "lik_internal.hpp"
#include "flow.hpp"
#include "propagate.hpp"
#include "weigh.hpp"

namespace lik {

// ---------------------------------------------------------------------------
// admit: fill the slots of one request.  Rates that are negative, infinite or
// NaN -- and, for the binary32 step, beyond the binary32 range (they would
// round to infinity, and infinity times a zero mass-action factor is NaN) --
// mark every slot of that theta BAD_THETA before any simulation.
// ---------------------------------------------------------------------------
// Filter k of request r (theta k / M against trajectory k % M) into its slot.
__device__ __forceinline__ void admit_one(FilterDesc *desc, const EngineArgs &e,
                                          const RequestArgs &r, int k) {
    const int i = k / r.M;
    const int m = k - i * r.M;
    const int f = r.base + k;
    const int off = r.obs_offsets[m];
    FilterDesc d;
    d.theta = r.theta + (size_t)i * r.R;
    d.t_obs = r.t_obs + off;
    d.y = r.y + (size_t)off * r.P;
    d.x0 = r.x0 + (size_t)m * r.U;
    d.x0_hi = r.x0_hi ? r.x0_hi + (size_t)m * r.U : nullptr;
    const size_t per = (size_t)r.U * r.Hp;
    int32_t *st = r.state + (size_t)k * (2 * per + 5 * (size_t)r.Hp);
    d.xa = st;
    d.xb = st + per;
    d.lw = (double *)(st + 2 * per);  // 8-byte aligned: per and Hp are multiples of 64
    d.anc = st + 2 * per + 2 * (size_t)r.Hp;
    d.pev = (uint32_t *)(st + 2 * per + 3 * (size_t)r.Hp);
    d.pa0 = (float *)(st + 2 * per + 4 * (size_t)r.Hp);
    d.t0 = r.t0[m];
    d.sigma = r.sigma;
    d.gain = r.gain;
    d.bg_mean = r.bg_mean;
    d.obs_s2 = r.sigma * r.sigma;
    d.bg_s2 = r.bg_sd * r.bg_sd;
    d.seed = r.seed;
    d.theta_id = r.theta_ids ? r.theta_ids[i] : (uint32_t)i;
    d.traj = (uint32_t)m;
    d.H = r.H;
    d.Hp = r.Hp;
    d.T = r.obs_offsets[m + 1] - off;
    d.U = r.U;
    d.R = r.R;
    d.P = r.P;
    d.obs_kind = r.obs_kind;
    d.group = r.group;
    d.event_cap = r.event_cap;
    d.pad = 0;
    for (int q = 0; q < LIK_MAX_OBSERVED; ++q) d.obs_species[q] = r.obs_species[q];
    desc[f] = d;
    bool bad = false;
    for (int q = 0; q < r.R; ++q) {
        const double c = d.theta[q];
        if (!(c >= 0.0) || isinf(c)) bad = true;
        if (r.precision == LIK_FP32_MIXED && isinf((float)c)) bad = true;
    }
    e.tcur[f] = 0;
    if (e.fdone) e.fdone[f] = 0;
    e.fll[f] = bad ? __builtin_nan("") : 0.0;
    e.fstatus[f] = bad ? LIK_STATUS_BAD_THETA : LIK_STATUS_OK;
    e.fflags[f] = bad ? kFlagStopped : 0u;
    e.fevents[f] = 0;
    // expected events of the first interval (a scheduling estimate):
    // H x total propensity at x0 x the interval's length
    double a0 = 0.0;
    if (!bad) {
        for (int q = 0; q < r.R; ++q) {
            const int k = r.kind[q];
            double h = 1.0;
            if (k == kOrder1) {
                h = (double)d.x0[r.s1[q]];
            } else if (k == kOrder2Homo) {
                const double v = (double)d.x0[r.s1[q]];
                h = 0.5 * v * (v - 1.0);
            } else if (k == kOrder2Hetero) {
                h = (double)d.x0[r.s1[q]] * (double)d.x0[r.s2[q]];
            }
            a0 += d.theta[q] * h;
        }
    }
    const double expect = (double)r.H * a0 * (d.t_obs[0] - d.t0);
    e.cost[f] = !(expect > 0.0) ? 0u : expect >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)expect;
}

__global__ void k_admit(FilterDesc *desc, EngineArgs e, RequestArgs r) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < r.n_theta * r.M) admit_one(desc, e, r, k);
}

// Every request of a multi-request batch: thread g admits the g-th filter
// overall, of the request q with fstart[q] <= g < fstart[q + 1] (its first
// slot is fstart[q]); thread 0 also records the batch's start time.
__global__ void k_admit_requests(FilterDesc *desc, EngineArgs e, const RequestArgs *reqs,
                                 const int32_t *fstart, int32_t n_req, uint64_t *start_tick) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) *start_tick = wall_clock64();
    if (g >= fstart[n_req]) return;
    int lo = 0, hi = n_req - 1;  // the last q with fstart[q] <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fstart[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    admit_one(desc, e, reqs[lo], g - fstart[lo]);
}

// Random initial counts (stream purpose 2): one workgroup per slot; particle
// j of a slot with bounds draws species u from Philox block (u / 4, j,
// traj << 16, theta id << 2 | 2), word u % 4, as x0 + floor(w (x0_hi - x0 + 1)
// / 2^32), into the buffer the first interval reads, with ancestor j.
__global__ void k_init_start(const FilterDesc *desc, int32_t base) {
    const FilterDesc &d = desc[base + (int)blockIdx.x];
    if (!d.x0_hi) return;
    const uint32_t k0 = (uint32_t)d.seed, k1 = (uint32_t)(d.seed >> 32);
    const uint32_t c2 = d.traj << 16, c3 = (d.theta_id << 2) | 2u;
    for (int j = threadIdx.x; j < d.H; j += blockDim.x) {
        for (int u4 = 0; u4 < d.U; u4 += 4) {
            const Block4 b = philox4x32_10((uint32_t)(u4 >> 2), (uint32_t)j, c2, c3, k0, k1);
            const uint32_t w[4] = {b.w0, b.w1, b.w2, b.w3};
            for (int q = 0; q < 4 && u4 + q < d.U; ++q) {
                const int u = u4 + q;
                const uint64_t span = (uint64_t)(d.x0_hi[u] - d.x0[u]) + 1u;
                d.xa[(size_t)u * d.Hp + j] = d.x0[u] + (int32_t)(((uint64_t)w[q] * span) >> 32);
            }
        }
        d.anc[j] = j;
    }
}

void fill_reactant_tables(RequestArgs &r, const int32_t *kind, const int32_t *s1,
                          const int32_t *s2, int R) {
    for (int q = 0; q < LIK_MAX_REACTIONS; ++q) {
        r.kind[q] = q < R ? (int8_t)kind[q] : (int8_t)0;
        r.s1[q] = q < R ? (int8_t)s1[q] : (int8_t)0;
        r.s2[q] = q < R ? (int8_t)s2[q] : (int8_t)0;
    }
}

// ---------------------------------------------------------------------------
// order: the pool size of each slot, and a counting sort of the active slots
// over (group, duration key): the expected events per lane of the slot's
// work items (expected events per particle times the groups per pool), in
// quarter octaves, longest first.  Order inside a key is arbitrary (atomics
// decide it): it only changes which wavefront starts first, never a result.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int duration_key(uint64_t c) {
    if (c == 0) return kCostKeys - 1;
    if (c > 0xFFFFFFFFull) c = 0xFFFFFFFFull;
    const uint32_t v = (uint32_t)c;
    const int b = 32 - __clz(v);  // bit length, 1..32
    const int frac = b >= 3 ? (int)((v >> (b - 3)) & 3u) : (int)((v << (3 - b)) & 3u);
    return 4 * (32 - b) + (3 - frac);  // 0 = longest
}

// Three passes over the slots, each a grid of kOrderBlock-slot blocks:
// count (items per (group, key) and the most expected events per particle),
// scan (one block: first positions of every (group, key), per-group totals),
// place (each slot takes its positions with one atomic and writes its items).
// Pool sizes are capped by g_par = pool_chunks / pool_min_items, with
// pool_chunks the host's count of groups of 64 particles over the slots that
// may be active, so that a small iteration still spreads its particles over
// as many wavefronts as it can.
__device__ __forceinline__ int order_gpar(const EngineArgs &e) {
    return (int)max(1u, e.pool_chunks / max(e.pool_min_items, 1u));
}

__global__ __launch_bounds__(kOrderBlock) void k_order_count(EngineArgs e) {
    __shared__ uint32_t hist[kMaxGroups * kCostKeys];
    __shared__ uint32_t max_per;
    for (int k = threadIdx.x; k < kMaxGroups * kCostKeys; k += blockDim.x) hist[k] = 0;
    if (threadIdx.x == 0) max_per = 0;
    __syncthreads();
    const int f = e.f_lo + (int)(blockIdx.x * kOrderBlock + threadIdx.x);
    if (f < e.f_hi && slot_active(e, f)) {
        const uint32_t c = e.cost[f];
        const int nchunk = e.desc[f].Hp >> 6;
        const int g = pool_size(e, f, c, order_gpar(e));
        const int key = duration_key((uint64_t)(c / (uint32_t)e.desc[f].H) * (uint64_t)g);
        atomicAdd(&hist[e.desc[f].group * kCostKeys + key], (uint32_t)((nchunk + g - 1) / g));
        atomicMax(&max_per, c / (uint32_t)e.desc[f].H);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kMaxGroups * kCostKeys; k += blockDim.x)
        if (hist[k]) atomicAdd(&e.order_count[k], hist[k]);
    if (threadIdx.x == 0 && max_per) atomicMax(&e.order_ctl[0], max_per);
}

// One block, one wavefront per group: exclusive scan in key order (longest
// first) from the group's first item, 64 keys at a time with the running
// total carried; leaves the counts zero for the next iteration.
__global__ __launch_bounds__(64 * kMaxGroups) void k_order_scan(EngineArgs e) {
    const int g = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    uint64_t run = e.group_off[g];
    for (int k0 = 0; k0 < kCostKeys; k0 += 64) {
        const int k = k0 + lane;
        const uint32_t h = k < kCostKeys ? e.order_count[g * kCostKeys + k] : 0u;
        const uint64_t incl = wave_incl_scan_u64(h, lane);
        if (k < kCostKeys) {
            e.order_pos[g * kCostKeys + k] = (uint32_t)(run + incl - h);
            e.order_count[g * kCostKeys + k] = 0u;
        }
        run += lane_read(incl, 63);
    }
    if (lane == 0) {
        e.item_count[g] = (uint32_t)(run - e.group_off[g]);
        e.item_cursor[g] = 0;
    }
    if (threadIdx.x == 0) {
        e.order_ctl[1] = e.order_ctl[0];
        e.order_ctl[0] = 0u;
    }
}

// Positions are taken per block: the block's slots first reserve their items
// within the block (LDS atomics), then one global atomic per (group, key)
// reserves the block's share.
__global__ __launch_bounds__(kOrderBlock) void k_order_place(EngineArgs e) {
    __shared__ uint32_t lcount[kMaxGroups * kCostKeys];
    for (int k = threadIdx.x; k < kMaxGroups * kCostKeys; k += blockDim.x) lcount[k] = 0u;
    __syncthreads();
    const int f = e.f_lo + (int)(blockIdx.x * kOrderBlock + threadIdx.x);
    const bool on = f < e.f_hi && slot_active(e, f);
    uint32_t c = 0, n_items = 0, local = 0;
    int g = 1, gk = 0;
    if (on) {
        c = e.cost[f];
        const int nchunk = e.desc[f].Hp >> 6;
        g = pool_size(e, f, c, order_gpar(e));  // as in the counting pass
        const int key = duration_key((uint64_t)(c / (uint32_t)e.desc[f].H) * (uint64_t)g);
        gk = e.desc[f].group * kCostKeys + key;
        n_items = (uint32_t)((nchunk + g - 1) / g);
        local = atomicAdd(&lcount[gk], n_items);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kMaxGroups * kCostKeys; k += blockDim.x)
        if (lcount[k]) lcount[k] = atomicAdd(&e.order_pos[k], lcount[k]);  // the block's base
    __syncthreads();
    if (!on) return;
    const uint32_t pos = lcount[gk] + local;
    for (uint32_t q = 0; q < n_items; ++q) e.items[pos + q] = ((uint32_t)f << 6) | (q * g);
    // Wavefront priority: the slots whose particles are expected to need
    // the most events are the ones the iteration waits for; their
    // wavefronts issue first on a SIMD they share with lighter ones.
    const uint32_t max_per = e.order_ctl[1];
    const uint32_t per = c / (uint32_t)e.desc[f].H;
    int prio = 0;
    if (e.priority && per > 0)
        prio = (uint64_t)per * 4u >= max_per ? 3 : (uint64_t)per * 32u >= max_per ? 1 : 0;
    e.pool[f] = (uint8_t)((prio << 6) | (g - 1));
}

__global__ void k_order_reset(EngineArgs e) {
    for (int k = threadIdx.x; k < kMaxGroups * kCostKeys; k += blockDim.x) e.order_count[k] = 0u;
    if (threadIdx.x < 2) e.order_ctl[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// propagate (generic network tables; the network-specialised variant is
// compiled at run time from the same body)
// ---------------------------------------------------------------------------
template <int UMAX, int RMAX, int W, int PREC>
__global__ __launch_bounds__(kPropBlock) void k_propagate(EngineArgs e, int group,
                                                          NetArgs<RMAX, W> net) {
    propagate_item<NetArgs<RMAX, W>, UMAX, RMAX, W, PREC>(e, net, group);
}

template <int UMAX, int RMAX, int W, int PREC>
__global__ __launch_bounds__(kPropBlock) void k_propagate_p(EngineArgs e, int group,
                                                            NetArgs<RMAX, W> net) {
    propagate_persistent<NetArgs<RMAX, W>, UMAX, RMAX, W, PREC>(e, net, group);
}

// ---------------------------------------------------------------------------
// flow engine (flow.hpp): ring reset, the first interval's items, the
// persistent launch, and the check that it did not give up
// ---------------------------------------------------------------------------
__global__ void k_flow_init(FlowArgs fa) {
    const size_t cap = (size_t)fa.mask + 1;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap * kFlowRings;
         i += (size_t)gridDim.x * blockDim.x)
        fa.ring[i] = (uint64_t)(i & fa.mask) << 32;  // free for position i
    if (blockIdx.x == 0) {
        for (int w = threadIdx.x; w < kCtlArgs; w += blockDim.x) fa.ctl[w] = 0u;
        if (threadIdx.x == 0) *const_cast<FlowArgs *>(flow_args_copy(fa.ctl)) = fa;
    }
}

// The first interval's items: urgent filters first (pass 0), then the rest
// (pass 1), appended while the item ring holds fewer than `backlog` items
// and parked beyond.
__global__ void k_flow_seed(EngineArgs e, FlowArgs fa, int pass) {
    const int f = e.f_lo + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (f >= e.f_hi) return;
    if (!slot_active(e, f)) {
        if (pass == 0) atomicAdd(&fa.ctl[kCtlFinished], 1u);
        return;
    }
    const int G = pool_size(e, f, e.cost[f], fa.g_par);
    const bool urgent = flow_urgent(e, fa, f, e.cost[f], G);
    if (urgent != (pass == 0)) return;
    const int n_items = ((e.desc[f].Hp >> 6) + G - 1) / G;
    e.pool[f] = (uint8_t)(G - 1);
    fa.remaining[f] = (uint32_t)n_items;
    const bool park = !urgent && atomicAdd(&fa.ctl[kCtlSeedItems], (uint32_t)n_items) >= fa.backlog;
    const int r = park ? kRingParked : kRingItems;
    const int n = park ? 1 : n_items;
    const uint32_t base = atomicAdd(&fa.ctl[kCtlTail + 64 * r], (uint32_t)n);
    uint64_t *ring = fa.ring + (size_t)r * (fa.mask + 1);
    for (int k = 0; k < n; ++k) {
        const uint32_t pos = base + (uint32_t)k;
        const uint32_t entry = park ? (uint32_t)f : (((uint32_t)f << 6) | (uint32_t)(k * G));
        ring[pos & fa.mask] = ((uint64_t)(pos + 1u) << 32) | entry;
    }
}

// e must stay the first argument: flow_run reads it again from offset 0 of
// the kernel-argument segment.
template <int UMAX, int RMAX, int W, int PREC>
__global__ __launch_bounds__(kPropBlock) void k_flow(EngineArgs e, const FlowArgs *fa,
                                                     NetArgs<RMAX, W> net) {
    flow_run<NetArgs<RMAX, W>, UMAX, RMAX, W, PREC>(e, *fa, net);
}

// One flow launch over filters of several networks (generic tables): each
// work item's network tables, nets[group of its filter], are read into
// scalar registers before its pool runs.
template <int UMAX, int RMAX, int W, int PREC>
__global__ __launch_bounds__(kPropBlock) void k_flow_multi(EngineArgs e, const FlowArgs *fa,
                                                           const NetArgs<RMAX, W> *nets) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[item_lds_words<UMAX, RMAX, PREC>()];
    flow_run_with(e, *fa, [&](uint32_t item) {
        const int g = __builtin_amdgcn_readfirstlane(e.desc[item >> 6].group);
        const NetArgs<RMAX, W> &src = nets[g];
        NetArgs<RMAX, W> net;
        net.U = __builtin_amdgcn_readfirstlane(src.U);
        net.R = __builtin_amdgcn_readfirstlane(src.R);
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            net.kind[r] = __builtin_amdgcn_readfirstlane(src.kind[r]);
            net.s1[r] = __builtin_amdgcn_readfirstlane(src.s1[r]);
            net.s2[r] = __builtin_amdgcn_readfirstlane(src.s2[r]);
#pragma unroll
            for (int w = 0; w < W; ++w) net.nu[r][w] = __builtin_amdgcn_readfirstlane(src.nu[r][w]);
        }
        run_item<NetArgs<RMAX, W>, UMAX, RMAX, W, PREC>(e, net, item, lds);
    });
}

__global__ void k_flow_check(EngineArgs e, FlowArgs fa) {
    if (fa.ctl[kCtlAbort] == 0u) return;
    const int f = e.f_lo + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (f >= e.f_hi || !slot_active(e, f)) return;
    e.fstatus[f] = LIK_STATUS_SCHEDULER;
    e.fll[f] = __builtin_nan("");
    e.fflags[f] |= kFlagStopped;
}

// ---------------------------------------------------------------------------
// weigh: log-sum-exp into the running log-likelihood, then systematic
// resampling with q_j = floor(e_j 2^32), integer prefix sums C, one offset
// rho = floor(w64 Q / 2^64) and ancestors a_j = min{i : H C_{i+1} > j Q + rho}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWeighBlock) void k_weigh(EngineArgs e) {
    extern __shared__ uint64_t Cs[];  // [h_max]: Cs[k] = C_{k+1}
    __shared__ double red[kWeighBlock / 64];
    __shared__ double logy[LIK_MAX_OBSERVED];
    __shared__ uint64_t redu[kWeighBlock / 64];
    __shared__ double bcast;
    __shared__ uint64_t bcast_u;

    const int f = e.f_lo + (int)blockIdx.x;
    if (!slot_active(e, f)) return;
    const FilterDesc &d = e.desc[f];
    const int t = e.tcur[f];
    const int T = d.T;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int H = d.H;
    // events of the interval into the filter's total
    {
        uint64_t evs = 0;
        for (int j = tid; j < H; j += kWeighBlock) evs += d.pev[j];
        evs = wave_sum_u64(evs, lane);
        if (lane == 0) redu[wave] = evs;
        __syncthreads();
        if (tid == 0) {
            uint64_t tot = 0;
            for (int w = 0; w < kWeighBlock / 64; ++w) tot += redu[w];
            e.fevents[f] += tot;
        }
    }
    __syncthreads();  // every thread has read tcur and redu before thread 0 moves on
    if (e.fstatus[f] != LIK_STATUS_OK) {
        if (tid == 0) {
            e.tcur[f] = t + 1;
            e.fll[f] = __builtin_nan("");
            e.fflags[f] |= kFlagStopped;
            if (e.fdone) e.fdone[f] = wall_clock64();
        }
        return;
    }
    double *lw = d.lw;
    const int per = (H + kWeighBlock - 1) / kWeighBlock;
    const int j0 = tid * per;
    const int j1 = min(j0 + per, H);
    const int32_t *xs = (t & 1) ? d.xa : d.xb;  // counts at the observation time
    const double *yt = d.y + (size_t)t * d.P;
    if (tid < d.P) logy[tid] = d.obs_kind == LIK_OBS_LOGNORMAL ? dlog(yt[tid]) : 0.0;
    __syncthreads();

    // particle-dependent part of log p(y_t | x_j) (the "Compute l_t^i" step),
    // kept in lw for this thread's second pass; and the maximum
    double mx = -__builtin_inf();
    const ObsParams op = obs_params(d);
    for (int j = j0; j < j1; ++j) {
        const double l = obs_logweight(d, op, xs, j, logy, yt);
        lw[j] = l;
        mx = fmax(mx, l);
    }
    mx = wave_max(mx, lane);
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    if (tid == 0) {
        double v = red[0];
        for (int w = 1; w < kWeighBlock / 64; ++w) v = fmax(v, red[w]);
        bcast = v;
    }
    __syncthreads();
    mx = bcast;
    if (mx == -__builtin_inf()) {
        if (tid == 0) {
            e.tcur[f] = t + 1;
            e.fll[f] = -__builtin_inf();
            e.fflags[f] |= kFlagStopped;
            if (e.fdone) e.fdone[f] = wall_clock64();
        }
        return;
    }

    // e_j (kept in lw) and integer weights q_j (kept in Cs until the scan)
    uint64_t qsum = 0;
    for (int j = j0; j < j1; ++j) {
        const double ej = dexp_nonpos(lw[j] - mx);
        lw[j] = ej;
        const uint64_t q = (uint64_t)(ej * 4294967296.0);
        Cs[j] = q;
        qsum += q;
    }
    __syncthreads();  // every e_j, and red[] reuse
    // S = sum of e_j in a fixed order: lane-wise sums over j = lane + 64 k in
    // increasing k, then one butterfly (the order the flow schedule's
    // one-wavefront weighing takes as well)
    if (wave == 0) {
        double s = 0.0;
        for (int j = lane; j < H; j += 64) s += lw[j];
        s = wave_sum(s, lane);
        if (lane == 0) red[0] = s;
    }

    // exclusive scan of the per-thread sums (thread order = particle order)
    const uint64_t incl = wave_incl_scan_u64(qsum, lane);
    if (lane == 63) redu[wave] = incl;
    __syncthreads();
    uint64_t base = incl - qsum;
    for (int w = 0; w < wave; ++w) base += redu[w];
    uint64_t run = base;
    for (int j = j0; j < j1; ++j) {
        run += Cs[j];
        Cs[j] = run;
    }
    if (tid == 0) {
        const double S = red[0];
        // running log-likelihood
        e.fll[f] = e.fll[f] + loglik_increment(d, mx, S, yt);
        e.tcur[f] = t + 1;
        if (t + 1 < T) bcast_u = resample_word(d, t);
        else if (e.fdone) e.fdone[f] = wall_clock64();
    }
    if (t + 1 >= T) return;
    __syncthreads();
    const uint64_t Q = Cs[H - 1];
    const uint64_t rho = __umul64hi(bcast_u, Q);
    const uint64_t Hu = (uint64_t)H;
    float pred = 0.0f;  // sum of the ancestors' total propensities
    for (int jj = tid; jj < H; jj += kWeighBlock) {
        const uint64_t point = (uint64_t)jj * Q + rho;
        int lo = 0, hi = H - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (Hu * Cs[mid] > point) hi = mid;
            else lo = mid + 1;
        }
        d.anc[jj] = lo;
        pred += d.pa0[lo];
    }
    // Ordering cost of the next interval: the events its particles are
    // expected to need, total propensity of their starting states times the
    // interval's length (a scheduling estimate only).
    pred = wave_sum_f32(pred, lane);
    __syncthreads();  // red[] reuse
    if (lane == 0) red[wave] = (double)pred;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int w = 0; w < kWeighBlock / 64; ++w) tot += red[w];
        e.cost[f] = cost_estimate(d, t, tot);
    }
}

// stop: the slots of a withdrawn request take no further interval
__global__ void k_stop(EngineArgs e, int32_t base, int32_t F) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < F) e.fflags[base + k] |= kFlagStopped;
}

// ---------------------------------------------------------------------------
// finish: per-theta sum over trajectories in trajectory order, status, aux.
// ---------------------------------------------------------------------------
__global__ void k_finish(EngineArgs e, int32_t base, int32_t n_theta, int32_t M, double *loglik,
                         int32_t *status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_theta) return;
    double s = 0.0;
    int32_t st = LIK_STATUS_OK;
    for (int m = 0; m < M; ++m) {
        const int f = base + i * M + m;
        if (st == LIK_STATUS_OK && e.fstatus[f] != LIK_STATUS_OK) st = e.fstatus[f];
        s = s + e.fll[f];
    }
    loglik[i] = st == LIK_STATUS_OK ? s : __builtin_nan("");
    if (status) status[i] = st;
}

// Per-theta results of every request of a multi-request batch: block q sums
// request q's filters over its trajectories, in trajectory order.
__global__ void k_finish_requests(EngineArgs e, const ReqSpan *spans, double *loglik,
                                  int32_t *status) {
    const ReqSpan sp = spans[blockIdx.x];
    for (int i = threadIdx.x; i < sp.n_theta; i += blockDim.x) {
        double s = 0.0;
        int32_t st = LIK_STATUS_OK;
        for (int m = 0; m < sp.M; ++m) {
            const int f = sp.base + i * sp.M + m;
            if (st == LIK_STATUS_OK && e.fstatus[f] != LIK_STATUS_OK) st = e.fstatus[f];
            s = s + e.fll[f];
        }
        loglik[sp.out + i] = st == LIK_STATUS_OK ? s : __builtin_nan("");
        if (status) status[sp.out + i] = st;
    }
}

__global__ void k_aux_filters(EngineArgs e, int32_t base, int32_t F, uint64_t *events,
                              double *fll) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= F) return;
    if (events) events[k] = e.fevents[base + k];
    if (fll) fll[k] = e.fll[base + k];
}

// counts after the last interval each slot ran ([F][U][H])
__global__ void k_aux_state(EngineArgs e, int32_t base, int32_t F, int32_t *out) {
    const FilterDesc &d0 = e.desc[base];
    const size_t per = (size_t)d0.U * d0.H;
    const size_t total = (size_t)F * per;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (size_t)gridDim.x * blockDim.x) {
        const int f = base + (int)(k / per);
        const size_t rem = k - (size_t)(f - base) * per;
        const FilterDesc &d = e.desc[f];
        const int u = (int)(rem / d.H), j = (int)(rem % d.H);
        const int steps = e.tcur[f];
        const int32_t *src = (steps & 1) ? d.xb : d.xa;
        out[k] = (steps == 0 && !d.x0_hi) ? d.x0[u] : src[(size_t)u * d.Hp + j];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t request_state_bytes(int64_t F, int32_t U, int32_t Hp) {
    return (size_t)F * (2 * (size_t)U * Hp + 5 * (size_t)Hp) * sizeof(int32_t);
}

hipError_t launch_admit(FilterDesc *desc, const EngineArgs &e, const RequestArgs &r,
                        hipStream_t s) {
    const int F = r.n_theta * r.M;
    if (F == 0) return hipSuccess;
    hipLaunchKernelGGL(k_admit, dim3((F + 255) / 256), dim3(256), 0, s, desc, e, r);
    return hipGetLastError();
}

const void *admit_kernel() { return (const void *)k_admit; }

hipError_t launch_init_start(const FilterDesc *desc, int32_t base, int32_t F, hipStream_t s) {
    if (F <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_start, dim3((unsigned)F), dim3(256), 0, s, desc, base);
    return hipGetLastError();
}

hipError_t launch_admit_requests(FilterDesc *desc, const EngineArgs &e, const RequestArgs *reqs,
                                 const int32_t *fstart, int32_t n_req, int32_t n_filters,
                                 uint64_t *start_tick, hipStream_t s) {
    const unsigned blocks = (unsigned)std::max(1, (n_filters + 255) / 256);
    hipLaunchKernelGGL(k_admit_requests, dim3(blocks), dim3(256), 0, s, desc, e, reqs, fstart,
                       n_req, start_tick);
    return hipGetLastError();
}

hipError_t launch_finish_requests(const EngineArgs &e, const ReqSpan *spans, int32_t n_req,
                                  double *loglik, int32_t *status, hipStream_t s) {
    if (n_req > 0)
        hipLaunchKernelGGL(k_finish_requests, dim3((unsigned)n_req), dim3(64), 0, s, e, spans,
                           loglik, status);
    return hipGetLastError();
}

hipError_t launch_stop(const EngineArgs &e, int32_t base, int32_t F, hipStream_t s) {
    if (F <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stop, dim3((F + 255) / 256), dim3(256), 0, s, e, base, F);
    return hipGetLastError();
}

hipError_t launch_order(const EngineArgs &e, hipStream_t s) {
    const int F = e.f_hi - e.f_lo;
    const unsigned blocks = (unsigned)((F + kOrderBlock - 1) / kOrderBlock);
    if (blocks) hipLaunchKernelGGL(k_order_count, dim3(blocks), dim3(kOrderBlock), 0, s, e);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64 * kMaxGroups), 0, s, e);
    if (blocks) hipLaunchKernelGGL(k_order_place, dim3(blocks), dim3(kOrderBlock), 0, s, e);
    return hipGetLastError();
}

hipError_t launch_order_reset(const EngineArgs &e, hipStream_t s) {
    hipLaunchKernelGGL(k_order_reset, dim3(1), dim3(256), 0, s, e);
    return hipGetLastError();
}

template <int UMAX, int RMAX, int W>
static hipError_t launch_prop_t(const EngineArgs &e, int group, unsigned n_items,
                                const void *net, int precision, hipStream_t s) {
    const NetArgs<RMAX, W> &n = *static_cast<const NetArgs<RMAX, W> *>(net);
    if (precision == LIK_FP32_MIXED)
        hipLaunchKernelGGL((k_propagate<UMAX, RMAX, W, LIK_FP32_MIXED>), dim3(n_items),
                           dim3(kPropBlock), 0, s, e, group, n);
    else
        hipLaunchKernelGGL((k_propagate<UMAX, RMAX, W, LIK_FP64>), dim3(n_items),
                           dim3(kPropBlock), 0, s, e, group, n);
    return hipGetLastError();
}

// persistent variant: n_waves wavefronts take the group's items from its counter
template <int UMAX, int RMAX, int W>
static hipError_t launch_prop_p(const EngineArgs &e, int group, unsigned n_waves,
                                const void *net, int precision, hipStream_t s) {
    const NetArgs<RMAX, W> &n = *static_cast<const NetArgs<RMAX, W> *>(net);
    if (precision == LIK_FP32_MIXED)
        hipLaunchKernelGGL((k_propagate_p<UMAX, RMAX, W, LIK_FP32_MIXED>), dim3(n_waves),
                           dim3(kPropBlock), 0, s, e, group, n);
    else
        hipLaunchKernelGGL((k_propagate_p<UMAX, RMAX, W, LIK_FP64>), dim3(n_waves),
                           dim3(kPropBlock), 0, s, e, group, n);
    return hipGetLastError();
}

hipError_t launch_propagate(const EngineArgs &e, int group, unsigned n_items, const void *net,
                            int umax, int rmax, int precision, bool persistent, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    if (persistent && umax == 4 && rmax == 8)
        return launch_prop_p<4, 8, 1>(e, group, n_items, net, precision, s);
    if (persistent && umax == 8 && rmax == 16)
        return launch_prop_p<8, 16, 1>(e, group, n_items, net, precision, s);
    if (umax == 4 && rmax == 8)
        return launch_prop_t<4, 8, 1>(e, group, n_items, net, precision, s);
    if (umax == 8 && rmax == 16)
        return launch_prop_t<8, 16, 1>(e, group, n_items, net, precision, s);
    if (umax == 32 && rmax == 64)
        return launch_prop_t<32, 64, 4>(e, group, n_items, net, precision, s);
    return hipErrorInvalidValue;
}

hipError_t launch_flow_setup(const EngineArgs &e, const FlowArgs &fa, hipStream_t s) {
    hipLaunchKernelGGL(k_flow_init, dim3(1024), dim3(256), 0, s, fa);
    const int F = e.f_hi - e.f_lo;
    for (int pass = 0; pass < 2 && F > 0; ++pass)
        hipLaunchKernelGGL(k_flow_seed, dim3((F + 255) / 256), dim3(256), 0, s, e, fa, pass);
    return hipGetLastError();
}

hipError_t launch_flow_check(const EngineArgs &e, const FlowArgs &fa, hipStream_t s) {
    const int F = e.f_hi - e.f_lo;
    if (F > 0) hipLaunchKernelGGL(k_flow_check, dim3((F + 255) / 256), dim3(256), 0, s, e, fa);
    return hipGetLastError();
}

template <int UMAX, int RMAX, int W>
static const void *flow_fn(int precision) {
    return precision == LIK_FP32_MIXED ? (const void *)k_flow<UMAX, RMAX, W, LIK_FP32_MIXED>
                                       : (const void *)k_flow<UMAX, RMAX, W, LIK_FP64>;
}

static const void *flow_kernel(int umax, int rmax, int precision) {
    if (umax == 4 && rmax == 8) return flow_fn<4, 8, 1>(precision);
    if (umax == 8 && rmax == 16) return flow_fn<8, 16, 1>(precision);
    if (umax == 32 && rmax == 64) return flow_fn<32, 64, 4>(precision);
    return nullptr;
}

template <int UMAX, int RMAX, int W>
static const void *flow_multi_fn(int precision) {
    return precision == LIK_FP32_MIXED ? (const void *)k_flow_multi<UMAX, RMAX, W, LIK_FP32_MIXED>
                                       : (const void *)k_flow_multi<UMAX, RMAX, W, LIK_FP64>;
}

// the multi-network flow kernel exists for the small buckets (networks whose
// tables fit scalar registers)
static const void *flow_multi_kernel(int umax, int rmax, int precision) {
    if (umax == 4 && rmax == 8) return flow_multi_fn<4, 8, 1>(precision);
    if (umax == 8 && rmax == 16) return flow_multi_fn<8, 16, 1>(precision);
    return nullptr;
}

int flow_multi_blocks_per_cu(int umax, int rmax, int precision) {
    const void *fn = flow_multi_kernel(umax, rmax, precision);
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kPropBlock, 0) != hipSuccess)
        return 0;
    return n;
}

hipError_t launch_flow_multi(const EngineArgs &e, const FlowArgs &fa, unsigned n_waves,
                             const void *nets_dev, int umax, int rmax, int precision,
                             hipStream_t s) {
    const void *fn = flow_multi_kernel(umax, rmax, precision);
    if (!fn || n_waves == 0) return hipErrorInvalidValue;
    EngineArgs ea = e;
    const FlowArgs *fb = flow_args_copy(fa.ctl);  // written by k_flow_init
    const void *nd = nets_dev;
    void *args[] = {(void *)&ea, (void *)&fb, (void *)&nd};
    return hipLaunchKernel(fn, dim3(n_waves), dim3(kPropBlock), args, 0, s);
}

int flow_blocks_per_cu(int umax, int rmax, int precision) {
    const void *fn = flow_kernel(umax, rmax, precision);
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kPropBlock, 0) != hipSuccess)
        return 0;
    return n;
}

hipError_t launch_flow(const EngineArgs &e, const FlowArgs &fa, unsigned n_waves, const void *net,
                       int umax, int rmax, int precision, hipStream_t s) {
    const void *fn = flow_kernel(umax, rmax, precision);
    if (!fn || n_waves == 0) return hipErrorInvalidValue;
    EngineArgs ea = e;
    const FlowArgs *fb = flow_args_copy(fa.ctl);  // written by k_flow_init
    void *args[] = {(void *)&ea, (void *)&fb, const_cast<void *>(net)};
    return hipLaunchKernel(fn, dim3(n_waves), dim3(kPropBlock), args, 0, s);
}

hipError_t launch_weigh(const EngineArgs &e, hipStream_t s) {
    if (e.f_hi <= e.f_lo) return hipSuccess;
    if (e.h_max < 1 || e.h_max > LIK_MAX_PARTICLES) return hipErrorInvalidValue;
    const size_t lds = (size_t)e.h_max * sizeof(uint64_t);  // the prefix sums C
    hipLaunchKernelGGL(k_weigh, dim3((unsigned)(e.f_hi - e.f_lo)), dim3(kWeighBlock), lds, s, e);
    return hipGetLastError();
}

hipError_t launch_finish(const EngineArgs &e, int32_t base, int32_t n_theta, int32_t M,
                         double *loglik, int32_t *status, const lik_aux *aux, hipStream_t s) {
    if (n_theta > 0)
        hipLaunchKernelGGL(k_finish, dim3((n_theta + 255) / 256), dim3(256), 0, s, e, base,
                           n_theta, M, loglik, status);
    const int F = n_theta * M;
    if (aux && F > 0) {
        if (aux->filter_events || aux->filter_loglik)
            hipLaunchKernelGGL(k_aux_filters, dim3((F + 255) / 256), dim3(256), 0, s, e, base, F,
                               aux->filter_events, aux->filter_loglik);
        if (aux->final_state)
            hipLaunchKernelGGL(k_aux_state, dim3(4096), dim3(256), 0, s, e, base, F,
                               aux->final_state);
    }
    return hipGetLastError();
}

}  // namespace lik
