// flow.hpp -- the flow engine: one persistent launch runs every observation
// interval of a batch of filters.
//
// The per-interval engine advances all filters together: a launch per
// interval, so every filter waits at each observation time for the slowest
// wavefront of that interval, and the compute units idle through each
// launch's tail.  Here a filter advances as soon as its own particles are
// weighed.  Wavefronts take work items -- pools of particles of one filter
// over one interval, exactly those of the per-interval engine -- from a
// ring in arrival order, one item each.  The wavefront
// that finishes a filter's last item of an interval weighs that filter
// (log-weights, log-sum-exp, systematic resampling; the same arithmetic in
// the same order as k_weigh, so results are bit-identical) and writes the
// items of its next interval to the ring.  Wavefronts left without an item
// leave once every filter is done.
//
// Ring protocol (a bounded multi-producer multi-consumer queue with one
// sequence word per slot): a consumer claims position p from the head
// counter and waits until slot p & mask holds sequence p + 1, takes the
// item and marks the slot free for position p + capacity; a producer
// claims p from the tail counter, waits until the slot holds sequence p
// (free for p) and writes (p + 1, item).  At most one interval of items per
// filter is outstanding, so at most sum(groups of 64) <= capacity / 2 items
// sit in the ring and a producer never waits for a slot that no wavefront
// has claimed.  Hand-offs between wavefronts (item results before the
// weighing, the weighing's state before the next items) are agent-scope
// release/acquire pairs.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "propagate.hpp"
#include "weigh.hpp"

namespace lik {

__device__ __forceinline__ uint32_t ctl_load(const FlowArgs &fa, int w) {
    return __hip_atomic_load(&fa.ctl[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until ring slot `pos` holds sequence `want` (its entry in *entry).
// False if the batch is done (when `until_done`) or the flow has given up:
// a wavefront that sees no work item finish for stall_ticks sets the abort
// word, which every waiting wavefront then sees.
__device__ __forceinline__ bool ring_wait(const FlowArgs &fa, uint32_t pos, uint32_t want,
                                          uint64_t *entry, bool until_done) {
    uint64_t since = wall_clock64();
    uint32_t seen = ctl_load(fa, kCtlProgress);
    for (;;) {
        const uint64_t v =
            __hip_atomic_load(&fa.ring[pos & fa.mask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == want) {
            *entry = v;
            return true;
        }
        if (until_done && (int)ctl_load(fa, kCtlFinished) >= fa.n_slots) return false;
        if (ctl_load(fa, kCtlAbort) != 0u) return false;
        const uint32_t prog = ctl_load(fa, kCtlProgress);
        const uint64_t now = wall_clock64();
        if (prog != seen) {
            seen = prog;
            since = now;
        } else if (now - since > fa.stall_ticks) {
            __hip_atomic_store(&fa.ctl[kCtlAbort], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

// Weighing of filter f after its interval tcur[f] (one wavefront; the
// arithmetic of k_weigh with its 256 threads emulated as 4 x 64 lanes: thread
// v = 64 w + lane owns particles [v per, (v + 1) per), per = ceil(H / 256)).
// The log-weights and then the integer prefix sums live in the slot's lw
// array (8 bytes per particle).  Returns true when the filter goes on to
// another interval; *cost receives its expected events.
__device__ __forceinline__ bool flow_weigh(const EngineArgs &e, int f, double *logy,
                                           uint32_t *cost) {
    const FilterDesc &d = e.desc[f];
    const int lane = lane_id();
    const int t = e.tcur[f];
    const int H = d.H;
    {
        uint64_t evs = 0;
        for (int j = lane; j < H; j += 64) evs += d.pev[j];
        evs = wave_sum_u64(evs, lane);
        if (lane == 0) e.fevents[f] += evs;
    }
    if (e.fstatus[f] != LIK_STATUS_OK) {
        if (lane == 0) {
            e.tcur[f] = t + 1;
            e.fll[f] = __builtin_nan("");
            e.fflags[f] |= kFlagStopped;
        }
        return false;
    }
    const int32_t *xs = (t & 1) ? d.xa : d.xb;  // counts at the observation time
    const double *yt = d.y + (size_t)t * d.P;
    if (lane < d.P) logy[lane] = d.obs_kind == LIK_OBS_LOGNORMAL ? dlog(yt[lane]) : 0.0;
    __syncthreads();
    uint64_t *cw = reinterpret_cast<uint64_t *>(d.lw);
    constexpr int kVirt = kWeighBlock / 64;  // emulated wavefronts
    const int per = (H + kWeighBlock - 1) / kWeighBlock;

    double mx = -__builtin_inf();
#pragma unroll 1
    for (int w = 0; w < kVirt; ++w) {
        const int j0 = (w * 64 + lane) * per;
        const int j1 = min(j0 + per, H);
#pragma unroll 1
        for (int j = j0; j < j1; ++j) {
            const double l = obs_logweight(d, xs, j, logy, yt);
            cw[j] = (uint64_t)__double_as_longlong(l);
            mx = fmax(mx, l);
        }
    }
    mx = wave_max(mx, lane);
    if (mx == -__builtin_inf()) {
        if (lane == 0) {
            e.tcur[f] = t + 1;
            e.fll[f] = -__builtin_inf();
            e.fflags[f] |= kFlagStopped;
        }
        return false;
    }

    // per emulated wavefront w: e_j and its threads' sums s (S adds the
    // wavefront sums in wavefront order), q_j = floor(e_j 2^32), then the
    // inclusive prefix sums C_{j+1} in place (thread order = particle order)
    double S = 0.0;
    uint64_t before = 0;  // q of the emulated wavefronts before w
#pragma unroll 1
    for (int w = 0; w < kVirt; ++w) {
        const int j0 = (w * 64 + lane) * per;
        const int j1 = min(j0 + per, H);
        double s = 0.0;
        uint64_t qsum = 0;
#pragma unroll 1
        for (int j = j0; j < j1; ++j) {
            const double ej = dexp_nonpos(__longlong_as_double((long long)cw[j]) - mx);
            s += ej;
            const uint64_t q = (uint64_t)(ej * 4294967296.0);
            cw[j] = q;
            qsum += q;
        }
        const double r = wave_sum(s, lane);
        S = (w == 0) ? r : S + r;
        const uint64_t incl = wave_incl_scan_u64(qsum, lane);
        uint64_t run = before + incl - qsum;
#pragma unroll 1
        for (int j = j0; j < j1; ++j) {
            run += cw[j];
            cw[j] = run;
        }
        before += lane_read(incl, 63);
    }
    if (lane == 0) {
        e.fll[f] = e.fll[f] + loglik_increment(d, mx, S, yt);
        e.tcur[f] = t + 1;
    }
    if (t + 1 >= d.T) return false;
    __syncthreads();  // every lane's prefix sums before any lane searches them

    // a_j = min{i : H C_{i+1} > j Q + rho}; nondecreasing in j, so each lane
    // searches the first of its consecutive outputs and walks on from there
    const uint64_t Q = cw[H - 1];
    const uint64_t rho = __umul64hi(resample_word(d, t), Q);
    const uint64_t Hu = (uint64_t)H;
    const int per64 = (H + 63) / 64;
    const int a0 = lane * per64;
    const int a1 = min(a0 + per64, H);
    float pred = 0.0f;  // sum of the ancestors' total propensities
    if (a0 < a1) {
        const uint64_t point0 = (uint64_t)a0 * Q + rho;
        int lo = 0, hi = H - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (Hu * cw[mid] > point0) hi = mid;
            else lo = mid + 1;
        }
        int a = lo;
#pragma unroll 1
        for (int jj = a0; jj < a1; ++jj) {
            const uint64_t point = (uint64_t)jj * Q + rho;
            while (!(Hu * cw[a] > point)) ++a;
            d.anc[jj] = a;
            pred += d.pa0[a];
        }
    }
    pred = wave_sum_f32(pred, lane);
    *cost = cost_estimate(d, t, (double)pred);
    return true;
}

// Writes the items of filter f's next interval to the ring.
__device__ __forceinline__ void flow_push(const EngineArgs &e, const FlowArgs &fa, int f,
                                          uint32_t cost) {
    const int lane = lane_id();
    __syncthreads();  // the weighing's state (tcur, ancestors) from every lane
    const int G = pool_size(e, f, cost, fa.g_par);
    const int nchunk = e.desc[f].Hp >> 6;
    const int n_items = (nchunk + G - 1) / G;
    if (lane == 0) {
        e.cost[f] = cost;
        e.pool[f] = (uint8_t)(G - 1);
        __hip_atomic_store(&fa.remaining[f], (uint32_t)n_items, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    // release: everything above before the items become visible
    __threadfence();
    __syncthreads();
    uint32_t base = 0;
    if (lane == 0)
        base = __hip_atomic_fetch_add(&fa.ctl[kCtlTail], (uint32_t)n_items, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    base = __builtin_amdgcn_readfirstlane(base);  // lane 0's: every lane is active
    if (lane < n_items) {  // n_items <= 64: one lane per item
        const uint32_t pos = base + (uint32_t)lane;
        const uint32_t item = ((uint32_t)f << 6) | (uint32_t)(lane * G);
        uint64_t ent;
        if (ring_wait(fa, pos, pos, &ent, false))
            __hip_atomic_store(&fa.ring[pos & fa.mask], ((uint64_t)(pos + 1u) << 32) | item,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One work item per wavefront (a grid of at least as many wavefronts as the
// batch has work items; the hardware starts each as a slot frees): claim the
// next ring position, run its item, and if it was its filter's last of the
// interval, weigh the filter and write its next items.  A wavefront whose
// position is never filled leaves when every filter is done.  One item per
// wavefront, rather than a loop over items, keeps the event loop's register
// allocation that of the per-interval kernel.
template <class NetT, int UMAX, int RMAX, int W, int PREC>
__device__ __forceinline__ void flow_run(const EngineArgs &e, const FlowArgs &fa,
                                         const NetT &net) {
    __shared__ double logy[LIK_MAX_OBSERVED];
    // the wavefronts beyond the batch's last item start after it is done
    if ((int)__builtin_amdgcn_readfirstlane(ctl_load(fa, kCtlFinished)) >= fa.n_slots) return;
    uint32_t pos = 0;
    uint64_t ent = 0;
    int ok = 0;
    if (lane_id() == 0) {
        pos = __hip_atomic_fetch_add(&fa.ctl[kCtlHead], 1u, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        ok = ring_wait(fa, pos, pos + 1u, &ent, true) ? 1 : 0;
        if (ok)  // the slot is free for its next lap
            __hip_atomic_store(&fa.ring[pos & fa.mask], (uint64_t)(pos + fa.mask + 1u) << 32,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    ok = __builtin_amdgcn_readfirstlane(ok);  // lane 0's: every lane is active
    if (!ok) return;  // every filter is done (or the flow gave up)
    // acquire: the filter's state written before the item was published
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const uint32_t item = __builtin_amdgcn_readfirstlane((uint32_t)ent);
    const int f = (int)(item >> 6);
    run_item<NetT, UMAX, RMAX, W, PREC>(e, net, item);

    // release: this item's results before the filter's count goes down
    __threadfence();
    __syncthreads();
    uint32_t left = 0;
    if (lane_id() == 0) {
        left = __hip_atomic_fetch_sub(&fa.remaining[f], 1u, __ATOMIC_ACQ_REL,
                                      __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&fa.ctl[kCtlProgress], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    left = __builtin_amdgcn_readfirstlane(left);
    if (left != 1u) return;
    // the last item of the interval: weigh the filter with every item's results
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    uint32_t cost = 0;
    if (flow_weigh(e, f, logy, &cost)) {
        flow_push(e, fa, f, cost);
    } else {
        __threadfence();
        __syncthreads();
        if (lane_id() == 0)
            __hip_atomic_fetch_add(&fa.ctl[kCtlFinished], 1u, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace lik
