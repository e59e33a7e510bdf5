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
// Ring protocol (bounded multi-producer multi-consumer queues with one
// sequence word per slot): a producer reserves position p from a ring's
// tail counter, waits until slot p & mask holds sequence p (free for p) and
// writes (p + 1, entry); a consumer takes p from the head counter, waits
// until the slot holds p + 1, takes the entry and marks the slot free for
// position p + capacity.  Every wavefront claims its item with one
// fetch-and-add, so thousands of waiting wavefronts never contend on a
// compare-and-swap.
//
// Priority without a second claim path: first come, first served would let
// a filter wait at every interval behind a whole generation of other
// filters' items, and the filters with the longest chains (many intervals
// left times long items) would set the end of the run.  So the item ring is
// kept short: a filter that is not urgent and finds `backlog` items already
// waiting is parked (its id goes to a second ring) instead of appending its
// items; every wavefront that finishes an item takes one parked filter and
// appends its items while fewer than `backlog` wait.  Urgent filters always
// append, and so wait only behind a short ring.  No deadlock: a filter is
// parked only while items wait, and the last of them to finish un-parks.
// At most one interval of items per filter is outstanding, so at most
// sum(groups of 64) <= capacity / 2 entries sit in a ring and a producer
// never waits for a slot that no wavefront has claimed.  Hand-offs between wavefronts (item results before the
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

// Gives up (sets the abort word, which every waiting wavefront then sees)
// once no work item has finished for stall_ticks.  `seen` and `since` carry
// the wait's last progress count and its time.
__device__ __forceinline__ bool flow_stalled(const FlowArgs &fa, uint32_t &seen,
                                             uint64_t &since) {
    if (ctl_load(fa, kCtlAbort) != 0u) return true;
    const uint32_t prog = ctl_load(fa, kCtlProgress);
    const uint64_t now = wall_clock64();
    if (prog != seen) {
        seen = prog;
        since = now;
    } else if (now - since > fa.stall_ticks) {
        __hip_atomic_store(&fa.ctl[kCtlAbort], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    return false;
}

__device__ __forceinline__ uint64_t *ring_slot(const FlowArgs &fa, int r, uint32_t pos) {
    return fa.ring + (size_t)r * (fa.mask + 1) + (pos & fa.mask);
}

// Waits until slot `pos` of ring r holds sequence `want` (its entry in
// *entry); false if the flow has given up, or (when `until_done`) once
// every filter is done.
__device__ __forceinline__ bool ring_wait(const FlowArgs &fa, int r, uint32_t pos, uint32_t want,
                                          uint64_t *entry, bool until_done) {
    uint64_t since = wall_clock64();
    uint32_t seen = ctl_load(fa, kCtlProgress);
    for (;;) {
        const uint64_t v =
            __hip_atomic_load(ring_slot(fa, r, pos), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == want) {
            *entry = v;
            return true;
        }
        if (until_done && (int)ctl_load(fa, kCtlFinished) >= fa.n_slots) return false;
        if (flow_stalled(fa, seen, since)) return false;
        __builtin_amdgcn_s_sleep(8);
    }
}

// Reserves n positions of ring r and writes one entry per lane below n (a
// lane waits until its slot is free for the position).  The caller has
// released what the entries' readers need.
__device__ __forceinline__ void ring_put(const FlowArgs &fa, int r, int n, uint32_t entry_of_lane,
                                         int lane) {
    uint32_t base = 0;
    if (lane == 0)
        base = __hip_atomic_fetch_add(&fa.ctl[kCtlTail + 64 * r], (uint32_t)n, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    base = __builtin_amdgcn_readfirstlane(base);  // lane 0's: every lane is active
    if (lane < n) {
        const uint32_t pos = base + (uint32_t)lane;
        uint64_t ent;
        if (ring_wait(fa, r, pos, pos, &ent, false))
            __hip_atomic_store(ring_slot(fa, r, pos), ((uint64_t)(pos + 1u) << 32) | entry_of_lane,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Takes the slot's entry of position pos and frees the slot for its next lap.
__device__ __forceinline__ void ring_take(const FlowArgs &fa, int r, uint32_t pos) {
    __hip_atomic_store(ring_slot(fa, r, pos), (uint64_t)(pos + fa.mask + 1u) << 32,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A filter is urgent (its items never wait in the parked ring) when its
// intervals left times the expected events per lane of its items (events
// per particle times the G particles a lane takes) reach urgent_events.
__device__ __forceinline__ bool flow_urgent(const EngineArgs &e, const FlowArgs &fa, int f,
                                            uint32_t cost, int G) {
    if (fa.urgent_events == 0u) return true;  // no parking: first come, first served
    const FilterDesc &d = e.desc[f];
    const uint64_t per_lane = (uint64_t)(cost / (uint32_t)d.H) * (uint64_t)G;
    const uint64_t left = (uint64_t)(d.T - e.tcur[f]);
    return per_lane * left >= (uint64_t)fa.urgent_events;
}

// Items waiting in the item ring; negative when wavefronts wait for items
// (they take positions ahead of the tail).
__device__ __forceinline__ int32_t item_backlog(const FlowArgs &fa) {
    return (int32_t)(ctl_load(fa, kCtlTail + 64 * kRingItems) -
                     ctl_load(fa, kCtlHead + 64 * kRingItems));
}

// Writes the work items of filter f (pool size G, state already released)
// to the item ring.
__device__ __forceinline__ void emit_items(const EngineArgs &e, const FlowArgs &fa, int f, int G,
                                           int lane) {
    const int n_items = ((e.desc[f].Hp >> 6) + G - 1) / G;  // <= 64: one lane per item
    ring_put(fa, kRingItems, n_items, ((uint32_t)f << 6) | (uint32_t)(lane * G), lane);
}

// While the item ring is short and filters are parked, takes one parked
// filter and writes its items; false if it took none.  Called by every
// wavefront that finishes an item, and by the wavefront first in line for
// the next item while it waits, so that parked filters move as soon as
// there is room.
__device__ __forceinline__ bool flow_unpark(const EngineArgs &e, const FlowArgs &fa, int lane) {
    int f = -1;
    if (lane == 0 && item_backlog(fa) < (int32_t)fa.backlog) {
        uint32_t h = ctl_load(fa, kCtlHead + 64 * kRingParked);
        const uint32_t tl = ctl_load(fa, kCtlTail + 64 * kRingParked);
        if ((int32_t)(tl - h) > 0 &&
            __hip_atomic_compare_exchange_strong(&fa.ctl[kCtlHead + 64 * kRingParked], &h, h + 1u,
                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
            uint64_t ent;
            if (ring_wait(fa, kRingParked, h, h + 1u, &ent, false)) {
                ring_take(fa, kRingParked, h);
                f = (int)(uint32_t)ent;
            }
        }
    }
    f = __builtin_amdgcn_readfirstlane(f);
    if (f < 0) return false;
    // acquire the parked filter's state; release it again to the items' takers
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int G = (int)e.pool[f] + 1;
    __threadfence();
    __syncthreads();
    emit_items(e, fa, f, G, lane);
    return true;
}

// After an item: takes parked filters (at most kUnparkPerItem) while the
// item ring is short.
constexpr int kUnparkPerItem = 4;
__device__ __forceinline__ void flow_unpark_some(const EngineArgs &e, const FlowArgs &fa,
                                                 int lane) {
    for (int k = 0; k < kUnparkPerItem; ++k)
        if (!flow_unpark(e, fa, lane)) break;
}

// Waits (lane 0) for the item of position pos of the item ring: 1 with the
// entry in *entry; 2 when this wavefront is first in line (no producer has
// reserved pos yet) and filters are parked -- the caller un-parks one and
// waits again; 0 once every filter is done or the flow has given up.
__device__ __forceinline__ int item_wait(const FlowArgs &fa, uint32_t pos, uint64_t *entry) {
    uint64_t since = wall_clock64();
    uint32_t seen = ctl_load(fa, kCtlProgress);
    for (;;) {
        const uint64_t v = __hip_atomic_load(ring_slot(fa, kRingItems, pos), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == pos + 1u) {
            *entry = v;
            return 1;
        }
        if (ctl_load(fa, kCtlTail + 64 * kRingItems) == pos &&
            (int32_t)(ctl_load(fa, kCtlTail + 64 * kRingParked) -
                      ctl_load(fa, kCtlHead + 64 * kRingParked)) > 0)
            return 2;
        if ((int)ctl_load(fa, kCtlFinished) >= fa.n_slots) return 0;
        if (flow_stalled(fa, seen, since)) return 0;
        __builtin_amdgcn_s_sleep(8);
    }
}

// Number of resampling points j*Q + rho (j = 0, 1, ...) below x:
// ceil((x - rho) / Q) for x > rho.  The quotient (at most H) is estimated in
// binary64 and then made exact with integer products (x < 2^57, Q < 2^45).
__device__ __forceinline__ uint64_t points_below(uint64_t x, uint64_t rho, uint64_t Q) {
    if (x <= rho) return 0;
    const uint64_t y = x - rho - 1;  // n = floor(y / Q) + 1
    uint64_t m = (uint64_t)((double)y / (double)Q);
    while (m > 0 && m * Q > y) --m;
    while ((m + 1) * Q <= y) ++m;
    return m + 1;
}

// Weighing of filter f after its interval tcur[f], by one wavefront, with
// k_weigh's results bit for bit.  Per-particle steps (log-weights, e_j, q_j)
// run over particles lane-strided, so every lane's loads are independent.
// The one order-dependent sum, S = sum e_j, follows k_weigh's order: each
// lane adds its particles j = lane + 64 k in increasing k, then one
// butterfly over the lanes.  The slot's lw array holds l_j, then e_j.  Resampling is taken from the particles' side: with
// J(x) = #{j >= 0 : j Q + rho < x}, particle i is the ancestor of exactly
// the j in [J(H C_i), J(H C_{i+1})) -- the same a_j = min{i : H C_{i+1} >
// j Q + rho} as the search over j, found without dependent loads.
// Returns true when the filter goes on to another interval; *cost receives
// its expected events.
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
    double *w = d.lw;
    const ObsParams op = obs_params(d);

    // Per-particle passes take kB particles per lane at a time, their loads
    // issued together (a load cannot move above an earlier iteration's store
    // to another array, so one particle at a time waits on each load).
    constexpr int kB = 2;
    // log-weights and their maximum
    double mx = -__builtin_inf();
    // counts of the first observed component: the next pair's are loaded
    // before this pair's log-weights are stored
    const int32_t *x0s = xs + (size_t)d.obs_species[0] * d.Hp;
    int c0[kB];
#pragma unroll
    for (int k = 0; k < kB; ++k) c0[k] = lane + 64 * k < H ? x0s[lane + 64 * k] : 0;
    if (op.kind == LIK_OBS_FLUORESCENCE) {
        // one particle at a time: its count-dependent variance makes the term
        // longer, and pairs would raise the kernel's register count
        for (int j = lane; j < H; j += 64) {
            const double l = obs_logweight(d, op, xs, j, logy, yt);
            w[j] = l;
            mx = fmax(mx, l);
        }
    } else
    for (int base = lane; base < H; base += 64 * kB) {
        double l[kB];
        bool on[kB];
        int n0[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            l[k] = 0.0;
            on[k] = base + 64 * k < H;
            const int jn = base + 64 * (kB + k);
            n0[k] = jn < H ? x0s[jn] : 0;
        }
        for (int o = 0; o < d.P; ++o) {
            const int32_t *xo = xs + (size_t)d.obs_species[o] * d.Hp;
            int cnt[kB];
#pragma unroll
            for (int k = 0; k < kB; ++k) cnt[k] = o == 0 ? c0[k] : on[k] ? xo[base + 64 * k] : 0;
#pragma unroll
            for (int k = 0; k < kB; ++k)
                if (on[k]) on[k] = obs_term<false>(op, o, cnt[k], logy, yt, l[k]);
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) c0[k] = n0[k];
#pragma unroll
        for (int k = 0; k < kB; ++k)
            if (base + 64 * k < H) {
                w[base + 64 * k] = l[k];
                mx = fmax(mx, l[k]);
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
    // e_j = exp(l_j - mx) in place, and S = sum e_j in k_weigh's order: each
    // lane's particles in increasing j, then one butterfly; the next pair's
    // loads are issued before this pair's stores
    double s = 0.0;
    {
        double v[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) v[k] = lane + 64 * k < H ? w[lane + 64 * k] : 0.0;
        for (int base = lane; base < H; base += 64 * kB) {
            double nx[kB];
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                const int jn = base + 64 * (kB + k);
                nx[k] = jn < H ? w[jn] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < kB; ++k)
                if (base + 64 * k < H) {
                    const double ej = dexp_nonpos(v[k] - mx);
                    w[base + 64 * k] = ej;
                    s += ej;
                }
#pragma unroll
            for (int k = 0; k < kB; ++k) v[k] = nx[k];
        }
    }
    const double S = wave_sum(s, lane);
    if (lane == 0) {
        e.fll[f] = e.fll[f] + loglik_increment(d, mx, S, yt);
        e.tcur[f] = t + 1;
    }
    if (t + 1 >= d.T) return false;

    // q_j = floor(e_j 2^32) and their total Q
    uint64_t Q = 0;
    for (int j = lane; j < H; j += 64) Q += (uint64_t)(w[j] * 4294967296.0);
    Q = wave_sum_u64(Q, lane);
    const uint64_t rho = __umul64hi(resample_word(d, t), Q);
    const uint64_t Hu = (uint64_t)H;
    // each group of 64 particles: prefix sums C_i, C_{i+1} (carried over
    // groups), then every particle writes the outputs it is the ancestor of
    float pred = 0.0f;  // sum of the ancestors' total propensities
    uint64_t carry = 0;    // C at the group's first particle
    uint64_t carry_j = 0;  // J(H C) there
    double v[kB];
    float a0[kB];
#pragma unroll
    for (int k = 0; k < kB; ++k) {
        const int i = 64 * k + lane;
        v[k] = i < H ? w[i] : 0.0;
        a0[k] = i < H ? d.pa0[i] : 0.0f;
    }
    for (int b0 = 0; b0 < H; b0 += 64 * kB) {
        // the next groups' weights, loaded before this group's stores
        double nv[kB];
        float na[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int i = b0 + 64 * (kB + k) + lane;
            nv[k] = i < H ? w[i] : 0.0;
            na[k] = i < H ? d.pa0[i] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int i = b0 + 64 * k + lane;
            const uint64_t q = i < H ? (uint64_t)(v[k] * 4294967296.0) : 0;
            const uint64_t incl = carry + wave_incl_scan_u64(q, lane);  // C_{i+1}
            // J(H C_{i+1}); J(H C_i) is the previous particle's
            const uint64_t j_hi = i < H ? min(points_below(Hu * incl, rho, Q), Hu) : Hu;
            const uint64_t prev = lane_read(j_hi, lane > 0 ? lane - 1 : 0);
            const uint64_t j_lo = lane > 0 ? prev : carry_j;
            if (i < H) {
                for (uint64_t j = j_lo; j < j_hi; ++j) d.anc[j] = i;
                pred += (float)(j_hi - j_lo) * a0[k];
            }
            carry = lane_read(incl, 63);
            carry_j = lane_read(j_hi, 63);
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            v[k] = nv[k];
            a0[k] = na[k];
        }
    }
    pred = wave_sum_f32(pred, lane);
    *cost = cost_estimate(d, t, (double)pred);
    return true;
}

// Sets up filter f's next interval and writes its items to the item ring,
// or parks the filter when the ring already holds `backlog` items and the
// filter is not urgent.
__device__ __forceinline__ void flow_push(const EngineArgs &e, const FlowArgs &fa, int f,
                                          uint32_t cost) {
    const int lane = lane_id();
    __syncthreads();  // the weighing's state (tcur, ancestors) from every lane
    // lane 0 wrote tcur: its reading decides, for every lane
    const int G = __builtin_amdgcn_readfirstlane(pool_size(e, f, cost, fa.g_par));
    const int nchunk = e.desc[f].Hp >> 6;
    const int n_items = (nchunk + G - 1) / G;
    const int park = __builtin_amdgcn_readfirstlane(
        (int)(!flow_urgent(e, fa, f, cost, G) && item_backlog(fa) >= (int32_t)fa.backlog));
    if (lane == 0) {
        e.cost[f] = cost;
        e.pool[f] = (uint8_t)(G - 1);
        __hip_atomic_store(&fa.remaining[f], (uint32_t)n_items, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    // release: everything above before the items (or the parked entry) are visible
    __threadfence();
    __syncthreads();
    if (park)
        ring_put(fa, kRingParked, 1, (uint32_t)f, lane);
    else
        emit_items(e, fa, f, G, lane);
}

// One work item per wavefront (a grid of at least as many wavefronts as the
// batch has work items; the hardware starts each as a slot frees): claim the
// next ring position, run its item, and if it was its filter's last of the
// interval, weigh the filter and write its next items.  A wavefront whose
// position is never filled leaves when every filter is done.  One item per
// wavefront, rather than a loop over items, keeps the event loop's register
// allocation that of the per-interval kernel.
// The kernel's first argument, its EngineArgs, read from the kernel-argument
// segment (constant memory: scalar loads) behind an empty asm statement, so
// the compiler issues new loads at the uses instead of keeping the values
// loaded at the kernel's start.  Every kernel that calls flow_run takes its
// EngineArgs by value as its first argument (offset 0 of the segment).
__device__ __forceinline__ const EngineArgs &reload_engine_args() {
    auto p = __builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return *(const EngineArgs *)p;
}

// run(item) runs one work item (the propagation of its pool); a launch over
// several networks picks the item's network inside it.
template <class RunItem>
__device__ __forceinline__ void flow_run_with(const EngineArgs &e, const FlowArgs &fa,
                                              RunItem &&run) {
    __shared__ double logy[LIK_MAX_OBSERVED];
    // the wavefronts beyond the batch's last item start after it is done
    if ((int)__builtin_amdgcn_readfirstlane(ctl_load(fa, kCtlFinished)) >= fa.n_slots) return;
    uint64_t ent = 0;
    uint32_t pos = 0;
    if (lane_id() == 0)
        pos = __hip_atomic_fetch_add(&fa.ctl[kCtlHead + 64 * kRingItems], 1u, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    int ok = 0;
    for (;;) {
        int st = 0;
        if (lane_id() == 0) st = item_wait(fa, pos, &ent);
        st = __builtin_amdgcn_readfirstlane(st);  // lane 0's: every lane is active
        if (st != 2) {
            ok = st;
            break;
        }
        flow_unpark(e, fa, lane_id());
    }
    if (ok && lane_id() == 0) ring_take(fa, kRingItems, pos);
    if (!ok) return;  // every filter is done (or the flow gave up)
    // acquire: the filter's state written before the item was published
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const uint32_t item = __builtin_amdgcn_readfirstlane((uint32_t)ent);
    const int f = (int)(item >> 6);
    run(item);

    // release: this item's results before the filter's count goes down
    __threadfence();
    __syncthreads();
    // From here on the engine's arguments are read again from the kernel's
    // argument segment, where used (the fields loaded at the kernel's start
    // would otherwise stay in scalar registers through the event loop).
    const EngineArgs &ec = reload_engine_args();
    uint32_t left = 0;
    if (lane_id() == 0) {
        left = __hip_atomic_fetch_sub(&fa.remaining[f], 1u, __ATOMIC_ACQ_REL,
                                      __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&fa.ctl[kCtlProgress], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    left = __builtin_amdgcn_readfirstlane(left);
    if (left != 1u) {
        flow_unpark_some(ec, fa, lane_id());
        return;
    }
    // the last item of the interval: weigh the filter with every item's results
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    uint32_t cost = 0;
    if (flow_weigh(ec, f, logy, &cost)) {
        flow_push(ec, fa, f, cost);
        flow_unpark_some(ec, fa, lane_id());
    } else {
        __threadfence();
        __syncthreads();
        if (lane_id() == 0) {
            if (ec.fdone) ec.fdone[f] = wall_clock64();
            __hip_atomic_fetch_add(&fa.ctl[kCtlFinished], 1u, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        flow_unpark_some(ec, fa, lane_id());
    }
}

template <class NetT, int UMAX, int RMAX, int W, int PREC>
__device__ __forceinline__ void flow_run(const EngineArgs &e, const FlowArgs &fa,
                                         const NetT &net) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[item_lds_words<UMAX, RMAX, PREC>()];
    flow_run_with(e, fa,
                  [&](uint32_t item) { run_item<NetT, UMAX, RMAX, W, PREC>(e, net, item, lds); });
}

}  // namespace lik
