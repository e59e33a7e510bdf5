// propagate.hpp -- one propagation work item: a pool of particles of one
// filter run over one observation interval by one wavefront.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "devmath.hpp"
#include "lik_internal.hpp"

namespace lik {

// Propensities a_r = c_r h_r(x) and their running sums S_r in reaction
// order (h_r = prod_u C(x_u, p_ru)); returns S_{R-1}.  Real is double for the
// binary64 step; for the binary32 step the factor h_r (exact in binary64) is
// rounded to binary32 and multiplied by the binary32 rate.  S_0 = a_0: a sum
// started from zero would differ only in the sign of an all-zero sum, which
// no comparison, division or result depends on.
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
            const Real a = c[r] * (Real)h;
            s = (r == 0) ? a : s + a;
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

// Networks of more than kRegRatesMax reactions keep their rates and net
// changes in the wavefront's LDS instead of registers: 40 binary64 rates
// would overflow the scalar registers (each spilled rate costs a vector
// read-back per event).  The rates are read at a wave-uniform address at
// every event; the reaction that fires is found as an index (the number of
// running sums not above the target) and its net changes are read from a
// table of signed bytes, ceil(U / 4) words per reaction padded to whole
// 16-byte rows.
constexpr int kRegRatesMax = 16;
template <int RMAX>
struct LdsNet {
    static constexpr bool on = RMAX > kRegRatesMax;
};
template <int UMAX>
__host__ __device__ constexpr int nu_row_words() {
    return ((UMAX + 3) / 4 + 3) / 4 * 4;
}

// LDS words a work item uses (the caller's buffer, 16-byte aligned): the
// pool's staged counts and processing order, the pool sort's buckets, and
// for a large network its rates and net-change table.
template <int UMAX, int RMAX, int PREC>
__host__ __device__ constexpr int item_lds_words() {
    return kPoolLdsWords + kSortBuckets +
           (LdsNet<RMAX>::on ? ((PREC == LIK_FP32_MIXED ? RMAX : 2 * RMAX) + 3) / 4 * 4 +
                                   RMAX * nu_row_words<UMAX>()
                             : 0);
}

// Index of the reaction that fires, r* = min{r : S_r > target}, else R - 1
// (no sum above a NaN or infinite target), as select_reaction picks it.
template <class NetT, int RMAX, class Real>
__device__ __forceinline__ int select_index(const NetT &net, const Real *S, Real target) {
    int rs = net.R - 1;
#pragma unroll
    for (int r = RMAX - 2; r >= 0; --r)
        if (r < net.R - 1) rs = (S[r] > target) ? r : rs;
    return rs;
}

// x += the net changes of reaction rs, read from its row of the byte table.
template <int UMAX>
__device__ __forceinline__ void apply_row(int U, const uint32_t *tab, int rs, int *x) {
    constexpr int kRow = nu_row_words<UMAX>();
    const uint4 *row = reinterpret_cast<const uint4 *>(tab + rs * kRow);
#pragma unroll
    for (int q = 0; q < kRow / 4; ++q) {
        const uint4 v = row[q];
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int u = 16 * q + k;
            if (u < UMAX && u < U) x[u] += (int)(signed char)(w4[k >> 2] >> (8 * (k & 3)));
        }
    }
}

template <int UMAX, int W>
__device__ __forceinline__ void apply_change(int U, const uint32_t *sel, int *x) {
    if (nu_bytes(U)) {
#pragma unroll
        for (int u = 0; u < (UMAX < 4 ? UMAX : 4); ++u)
            if (u < U) x[u] += (int)(signed char)(sel[0] >> (8 * u));
    } else {
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < U) x[u] += __builtin_amdgcn_sbfe(sel[u >> 3], 4 * (u & 7), 4);
    }
}


// base[i] = v through the global address space (base: device memory), with
// the byte offset formed in 32 bits: a wave-uniform base stays in scalar
// registers and the store takes the offset from one vector register.
template <class T>
__device__ __forceinline__ void store_global(T *base, uint32_t i, T v) {
    typedef __attribute__((address_space(1))) char gchar;
    typedef __attribute__((address_space(1))) T gT;
    *(gT *)((gchar *)base + i * (uint32_t)sizeof(T)) = v;
}

template <bool B, class T, class F>
struct pick_type {
    using type = T;
};
template <class T, class F>
struct pick_type<false, T, F> {
    using type = F;
};

// What an event takes from its random numbers (Supplementary I, the
// "Simulate" step): nl = -log u1 (the waiting time times the total
// propensity) and u2 (the reaction's share of the total), in the precision of
// the event arithmetic.  A function of the event's stream counter (n, j)
// alone, so any lane may compute it for any particle.  FP32-mixed draws two
// events at once from one Philox block (events n and n + 1, n even): nl1 and
// u21 are the second event's.
template <int PREC>
struct EventDraw {
    using Real = double;
    Real nl, u2;
};
template <>
struct EventDraw<LIK_FP32_MIXED> {
    using Real = float;
    Real nl, u2, nl1, u21;
};

// A 53-bit integer as binary64, exactly: hi 2^32 + lo < 2^53 is representable,
// so the one rounding of the fused multiply-add leaves it unchanged.
__device__ __forceinline__ double u53_to_f64(uint64_t z) {
    return __builtin_fma((double)(uint32_t)(z >> 32), 0x1p32, (double)(uint32_t)z);
}

template <int PREC>
__device__ __forceinline__ EventDraw<PREC> draw_from_block(const Block4 &b) {
    using Real = typename EventDraw<PREC>::Real;
    EventDraw<PREC> r;
    // u1 = (z + 1) 2^-k in (0, 1] and u2 = z' 2^-k in [0, 1), each formed
    // exactly (every intermediate value is representable)
    if constexpr (PREC == LIK_FP32_MIXED) {
        // the leading 24 bits of words 0, 1 (event n) and 2, 3 (event n + 1)
        const float u1 = __builtin_fmaf((float)(b.w0 >> 8), 0x1p-24f, 0x1p-24f);
        r.nl = -flog_pos(u1);
        r.u2 = (float)(b.w1 >> 8) * 0x1p-24f;
        const float u1b = __builtin_fmaf((float)(b.w2 >> 8), 0x1p-24f, 0x1p-24f);
        r.nl1 = -flog_pos(u1b);
        r.u21 = (float)(b.w3 >> 8) * 0x1p-24f;
    } else {
        const uint64_t z1 = ((((uint64_t)b.w1) << 32) | b.w0) >> 11;
        const uint64_t z2 = ((((uint64_t)b.w3) << 32) | b.w2) >> 11;
        const double u1 = fma_f64_s(u53_to_f64(z1), 0x1p-53);
        r.nl = (Real)(-dlog_pos(u1));
        r.u2 = (Real)(u53_to_f64(z2) * 0x1p-53);
    }
    return r;
}

// The Philox block of event n: n itself in FP64, n / 2 in FP32-mixed (whose
// events n and n + 1 share a block).
template <int PREC>
__device__ __forceinline__ uint32_t event_block(uint32_t n) {
    return PREC == LIK_FP32_MIXED ? n >> 1 : n;
}

// The draw of event n of particle j (any counter words; n even in
// FP32-mixed, where it is the draw of events n and n + 1).
template <int PREC>
__device__ __forceinline__ EventDraw<PREC> event_draw(uint32_t n, uint32_t j, uint32_t c2,
                                                      uint32_t c3, uint32_t k0, uint32_t k1) {
    return draw_from_block<PREC>(philox4x32_10(event_block<PREC>(n), j, c2, c3, k0, k1));
}

// The same where c2, c3 and the key are wave-uniform (one work item's
// particles): the generator's uniform parts go to scalar registers.
template <int PREC>
__device__ __forceinline__ EventDraw<PREC> event_draw_uniform(uint32_t n, uint32_t j,
                                                              uint32_t c2, uint32_t c3,
                                                              uint32_t k0, uint32_t k1) {
    return draw_from_block<PREC>(philox4x32_10_event(event_block<PREC>(n), j, c2, c3, k0, k1));
}

// One direct-method event of one particle (Supplementary I, the "Simulate"
// step; the SSA of Gillespie 1977): total propensity, then either the end of
// the particle's interval (no reaction possible, the event cap, or the next
// event beyond the observation time -- it is discarded) or one event; in
// FP32-mixed the same again for the block's second draw (two events per
// call, n even on entry).  draw() gives the EventDraw of the particle's
// current n.
// a0_end keeps the last total propensity (a scheduling estimate, stored as
// binary32 when the particle is).
// nu_tab: the byte table of net changes in LDS (large networks), else null.
template <class NetT, int UMAX, int RMAX, int W, int PREC, class Real, class DrawFn>
__device__ __forceinline__ void ssa_event(const NetT &net, const Real *c, int *x, Real *S,
                                          double t_end, uint32_t event_cap, double &clock,
                                          uint32_t &n, int &st, Real &a0_end, bool &have,
                                          const uint32_t *nu_tab, DrawFn &&draw) {
    // the total propensity after the last change (large networks: the rates
    // are read from LDS again at every event, the compiler would otherwise
    // keep all of them in vector registers)
    auto total = [&]() -> Real {
        if (LdsNet<RMAX>::on) asm volatile("" ::: "memory");
        const Real s = running_sums<NetT, RMAX, Real>(net, c, x, S);
        a0_end = s;
        return s;
    };
    // whether an event may be drawn: some reaction can fire, and the cap
    auto may_fire = [&](Real s) -> bool {
        if (!(s > (Real)0)) {
            have = false;  // no reaction can fire before the observation
            return false;
        }
        if (n >= event_cap) {
            st = st > LIK_STATUS_EVENT_CAP ? st : LIK_STATUS_EVENT_CAP;
            have = false;
            return false;
        }
        return true;
    };
    // the event of draw (nl, u2), or the end of the interval
    auto fire = [&](Real s, Real nl, Real u2) {
        double tau;
        Real target;
        if constexpr (PREC == LIK_FP32_MIXED) {
            tau = (double)((float)nl / (float)s);
            target = (Real)((float)u2 * (float)s);
        } else {
            tau = (double)nl / (double)s;
            target = (Real)((double)u2 * (double)s);
        }
        if (clock + tau > t_end) {
            have = false;  // the pending event is discarded
            return;
        }
        if (LdsNet<RMAX>::on) {
            apply_row<UMAX>(net.U, nu_tab, select_index<NetT, RMAX, Real>(net, S, target), x);
        } else {
            uint32_t sel[W];
            select_reaction<NetT, RMAX, W, Real>(net, S, target, sel);
            apply_change<UMAX, W>(net.U, sel, x);
        }
        clock = clock + tau;
        n = n + 1;
    };
    Real s = total();
    if (!may_fire(s)) return;
    const EventDraw<PREC> dr = draw();
    fire(s, dr.nl, dr.u2);
    if constexpr (PREC == LIK_FP32_MIXED) {
        // the second event of the block (n was even)
        if (!have) return;
        s = total();
        if (!may_fire(s)) return;
        fire(s, dr.nl1, dr.u21);
    }
}

// ---------------------------------------------------------------------------
// propagate: for every particle of the item's pool, gather its ancestor's
// counts, run Gillespie's direct method from the previous observation time
// to the next one, and store its counts (the weights are taken from them by
// k_weigh).
//
// A work item is a pool of G * 64 consecutive particles of one filter (G set
// per filter by k_order).  Each lane runs one event per loop iteration; a lane
// whose particle has reached the observation time finishes it and takes the
// next particle of the pool (ballot + rank among the idle lanes), so lanes are
// not held up by the slowest particle of a fixed group of 64.  Which lane runs
// a particle never changes its arithmetic or its random stream.
//
// NetT provides U, R, kind[], s1[], s2[], nu[][W] either as kernel-argument
// data (generic kernels) or as compile-time constants (network-specialised
// kernels).
// ---------------------------------------------------------------------------
// lds: the workgroup's buffer of at least item_lds_words<UMAX, RMAX, PREC>()
// words, 16-byte aligned (declared by the kernel, so that a kernel running
// the items of several networks holds one buffer for all of them).
template <class NetT, int UMAX, int RMAX, int W, int PREC>
__device__ __forceinline__ void run_item(const EngineArgs &e, const NetT &net, uint32_t item,
                                         uint32_t *lds) {
    // Every value of the item's context is the same on all lanes: moved to
    // scalar registers (a persistent caller loads them with vector loads,
    // after stores of earlier items, and would otherwise keep them in
    // vector registers through the event loop).
    item = wave_uniform(item);
    const int f = (int)(item >> 6);
    const FilterDesc &d = e.desc[f];
    const int t = wave_uniform(e.tcur[f]);

    const int U = net.U;
    const int R = net.R;
    const int H = wave_uniform(d.H);
    const int Hp = wave_uniform(d.Hp);
    const int lane = lane_id();
    const int p0 = (int)(item & 63u) * kPropBlock;
    const int pool = wave_uniform((int)e.pool[f]);  // (priority << 6) | (G - 1)
    const int p1 = min(p0 + ((pool & 63) + 1) * kPropBlock, H);

    const double t_start = wave_uniform((t == 0) ? d.t0 : d.t_obs[t - 1]);
    const double t_end = wave_uniform(d.t_obs[t]);
    const uint32_t c2 = wave_uniform((d.traj << 16) | (uint32_t)t);
    const uint32_t c3 = wave_uniform(d.theta_id << 2);  // purpose 0: reaction events
    const uint64_t seed = wave_uniform(d.seed);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int32_t *src = wave_uniform((t & 1) ? d.xb : d.xa);
    int32_t *dst = wave_uniform((t & 1) ? d.xa : d.xb);
    // Descriptor fields the event loop uses, read once: the loop's stores
    // could alias the descriptor as far as the compiler knows.
    const uint32_t event_cap = wave_uniform(d.event_cap);
    uint32_t *pev_p = wave_uniform(d.pev);
    float *pa0_p = wave_uniform(d.pa0);
    const int32_t *anc_p = wave_uniform(d.anc);
    const int32_t *x0_p = wave_uniform(d.x0);
    // every particle starts at x0 (fixed initial counts, first interval);
    // random initial counts were drawn into src with identity ancestors
    const bool fixed_start = t == 0 && wave_uniform(d.x0_hi) == nullptr;
    const int refill_min = e.refill_min;

    using Real = typename pick_type<PREC == LIK_FP32_MIXED, float, double>::type;
    // Rates are the same for the whole wavefront: kept in scalar registers,
    // or for a large network in LDS with its net-change table.
    constexpr bool kLds = LdsNet<RMAX>::on;
    constexpr int kRow = nu_row_words<UMAX>();
    int32_t *pool_x = reinterpret_cast<int32_t *>(lds);  // [U][npool], then order[npool] (uint16)
    uint32_t *bucket = lds + kPoolLdsWords;              // [kSortBuckets]
    Real *c_lds = reinterpret_cast<Real *>(lds + kPoolLdsWords + kSortBuckets);
    uint32_t *nu_lds = lds + kPoolLdsWords + kSortBuckets +
                       ((PREC == LIK_FP32_MIXED ? RMAX : 2 * RMAX) + 3) / 4 * 4;
    Real c_reg[kLds ? 1 : RMAX];
    if (kLds) {
        for (int r = lane; r < R; r += kPropBlock) c_lds[r] = (Real)d.theta[r];
        // net changes as signed bytes, from the network's packed fields
        for (int q = lane; q < R * kRow; q += kPropBlock) {
            const int r = q / kRow, w = q - r * kRow;
            uint32_t word = 0u;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int u = 4 * w + k;
                int v = 0;
                if (u < U)
                    v = nu_bytes(U) ? (int)(signed char)(net.nu[r][0] >> (8 * u))
                                    : __builtin_amdgcn_sbfe(net.nu[r][u >> 3], 4 * (u & 7), 4);
                word |= ((uint32_t)v & 0xFFu) << (8 * k);
            }
            nu_lds[q] = word;
        }
        __syncthreads();  // the workgroup is this one wavefront
    } else {
#pragma unroll
        for (int r = 0; r < RMAX; ++r)
            c_reg[r] = (r < R) ? wave_uniform((Real)d.theta[r]) : (Real)0;
    }
    const Real *c = kLds ? c_lds : c_reg;
    const uint32_t *nu_tab = kLds ? nu_lds : nullptr;

    // A pool of more than 64 particles first stages its ancestors' counts in
    // LDS ([u][particle - p0]); a lane taking a new particle reads them from
    // there, so the event loop never waits on a global load (a finished
    // particle's results are stored straight to global memory: stores do
    // not stall).  A pool of at most 64 particles has one per lane and
    // reads its counts directly.
    //
    // Lanes take the pool's particles heaviest first (longest processing
    // time first): a pool's length is set by the particles taken last, and
    // heavy particles taken last leave most lanes idle while they finish.
    // The weight of a particle is the total propensity of its starting
    // counts (its expected events over the interval, up to the common
    // interval length), bucketed by half octave below the pool's heaviest;
    // order[s] is the pool offset of the s-th particle taken.
    // Which lane runs a particle, and when, never changes its result.
    const int npool = p1 - p0;
    const bool staged = npool > kPropBlock;
    const bool ordered = staged && !fixed_start && npool <= kSortPerLane * kPropBlock &&
                         U * npool + (npool + 1) / 2 <= kPoolLdsWords;
    uint16_t *order = reinterpret_cast<uint16_t *>(pool_x + U * npool);
    if (ordered) {
        bucket[lane] = 0u;
        int a[kSortPerLane];
        uint32_t key[kSortPerLane];
        uint32_t kmax = 0u;
#pragma unroll
        for (int k = 0; k < kSortPerLane; ++k) {
            const int q = lane + k * kPropBlock;
            a[k] = (q < npool) ? anc_p[p0 + q] : 0;
        }
#pragma unroll
        for (int k = 0; k < kSortPerLane; ++k) {
            const int q = lane + k * kPropBlock;
            int xs[UMAX];
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                xs[u] = (u < U && q < npool) ? src[(size_t)u * Hp + a[k]] : 0;
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                if (u < U && q < npool) pool_x[u * npool + q] = xs[u];
            Real Sk[RMAX];
            const float w = (float)running_sums<NetT, RMAX, Real>(net, c, xs, Sk);
            // binary32 bits of a non-negative weight, shifted to sign,
            // exponent and leading fraction bit: half octaves, in order
            key[k] = (q < npool) ? (__float_as_uint(w) >> 22) : 0u;
            kmax = max(kmax, key[k]);
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) kmax = max(kmax, lane_read(kmax, lane ^ m));
        __syncthreads();  // the workgroup is this one wavefront
#pragma unroll
        for (int k = 0; k < kSortPerLane; ++k) {
            const int q = lane + k * kPropBlock;
            key[k] = min(kmax - key[k], (uint32_t)(kSortBuckets - 1));
            if (q < npool) atomicAdd(&bucket[key[k]], 1u);
        }
        __syncthreads();
        {  // exclusive prefix sum over the buckets, heaviest first
            const uint32_t v = bucket[lane];
            uint32_t incl = v;
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) {
                const uint32_t o = lane_read(incl, lane >= m ? lane - m : lane);
                if (lane >= m) incl += o;
            }
            bucket[lane] = incl - v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSortPerLane; ++k) {
            const int q = lane + k * kPropBlock;
            if (q < npool) order[atomicAdd(&bucket[key[k]], 1u)] = (uint16_t)q;
        }
        __syncthreads();
    } else if (staged) {
#pragma unroll 1
        for (int q = lane; q < npool; q += kPropBlock) {
            if (fixed_start) {
#pragma unroll
                for (int u = 0; u < UMAX; ++u)
                    if (u < U) pool_x[u * npool + q] = x0_p[u];
            } else {
                const int a = anc_p[p0 + q];
#pragma unroll
                for (int u = 0; u < UMAX; ++u)
                    if (u < U) pool_x[u * npool + q] = src[(size_t)u * Hp + a];
            }
        }
        __syncthreads();  // the workgroup is this one wavefront
    }

    int x[UMAX];
    double clock = t_start;
    uint32_t n = 0;
    int j = p0 + lane;  // the lane's particle
    bool have = j < p1;
    // the s-th particle taken from the pool: its index and starting counts
    auto load_lds = [&](int s) {
        const int q = ordered ? (int)order[s] : s;
        j = p0 + q;
#pragma unroll
        for (int u = 0; u < UMAX; ++u) x[u] = (u < U) ? pool_x[u * npool + q] : 0;
        clock = t_start;
        n = 0;
    };
    if (have) {
        if (staged) {
            load_lds(lane);
        } else if (fixed_start) {
#pragma unroll
            for (int u = 0; u < UMAX; ++u) x[u] = (u < U) ? x0_p[u] : 0;
        } else {
            const int a = anc_p[j];
#pragma unroll
            for (int u = 0; u < UMAX; ++u) x[u] = (u < U) ? src[(size_t)u * Hp + a] : 0;
        }
    }
    int next = p0 + kPropBlock;  // first particle of the pool no lane has taken (uniform)
    bool pend = have;            // the lane holds a particle not stored yet
    int st = LIK_STATUS_OK;
    Real S[RMAX];
    Real a0_end = (Real)0;  // total propensity at the particle's last state
    // a finished particle: overflow check, and its counts, events and final
    // total propensity into the pool's LDS slot (staged) or straight to
    // global memory
    // (global-memory stores at a wave-uniform base plus the particle's 32-bit
    // offset: one address operation per particle instead of one per array)
    auto retire = [&]() {
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < U && x[u] > kCountLimit)
                st = st > LIK_STATUS_COUNT_OVERFLOW ? st : LIK_STATUS_COUNT_OVERFLOW;
        const uint32_t jo = (uint32_t)j;
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < U) store_global(dst + (size_t)u * Hp, jo, x[u]);
        store_global(pev_p, jo, n);
        store_global(pa0_p, jo, (float)a0_end);
    };

    if ((pool >> 6) == 3) {
        __builtin_amdgcn_s_setprio(3);
    } else if ((pool >> 6) == 1) {
        __builtin_amdgcn_s_setprio(1);
    }
    for (;;) {
        if (have)
            ssa_event<NetT, UMAX, RMAX, W, PREC, Real>(
                net, c, x, S, t_end, event_cap, clock, n, st, a0_end, have, nu_tab,
                [&] { return event_draw_uniform<PREC>(n, (uint32_t)j, c2, c3, k0, k1); });
        // Once at least refill_min lanes are idle (or all are), the idle
        // lanes store what they hold and take the next particles of the
        // pool, in lane order.
        if (staged && next < p1) {
            const uint64_t idle = __ballot(!have);
            const int n_idle = (int)__popcll(idle);
            if (n_idle >= refill_min || idle == ~0ull) {
                if (!have) {
                    if (pend) retire();
                    pend = false;
                    // rank among the idle lanes: idle lanes below this one
                    const int nj = next + (int)__builtin_amdgcn_mbcnt_hi(
                                              (uint32_t)(idle >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                    if (nj < p1) {
                        have = true;
                        pend = true;
                        load_lds(nj - p0);
                    }
                }
                next += n_idle;
            }
        }
        const uint64_t busy = __ballot(have);
        if (busy == 0ull) break;
        if (!(staged && next < p1) && __popcll(busy) <= kPropBlock / 2) break;
    }

    // The pool's last particles.  Once every particle of the pool has been
    // taken and at most half of the lanes still run one, the idle lanes draw
    // the running lanes' coming events ahead of time: with k running lanes
    // and D = floor(64 / k), lane l computes the draw of event n + (l mod D)
    // of the running lane of rank floor(l / D), into LDS (the pool's staging
    // area, no longer read); each running lane then takes its next D draws
    // from there (in FP32-mixed a draw serves two events: lane l computes
    // the block of events n + 2 (l mod D) and n + 2 (l mod D) + 1).  A draw
    // depends on (n, j) only, so every event uses the numbers it would have
    // drawn itself; draws beyond a particle's end are left unused.
    using Draw = EventDraw<PREC>;
    Draw *dbuf = reinterpret_cast<Draw *>(pool_x);                    // [64]
    uint32_t *xn = reinterpret_cast<uint32_t *>(dbuf + kPropBlock);  // [32]: running lanes' n
    int32_t *xj = reinterpret_cast<int32_t *>(xn + kPropBlock / 2);  // [32]: and particles
    static_assert(sizeof(Draw) * kPropBlock + 4 * kPropBlock <= 4 * kPoolLdsWords,
                  "drain buffers fit the pool's LDS");
    __syncthreads();  // every read of the staged counts is done
    for (;;) {
        const uint64_t busy = __ballot(have);
        if (busy == 0ull) break;
        const int k = (int)__popcll(busy);  // <= 32
        const int D = kPropBlock / k;       // >= 2
        // floor(l / D) as (l * ceil(2^16 / D)) >> 16: the product exceeds
        // l * 2^16 / D by less than l <= 63 < 2^16 / D, too little to reach
        // the next multiple of 2^16 / D
        const int m = (0x10000 + D - 1) / D;
        const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(busy >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)busy, 0u));
        if (have) {
            xn[rank] = n;
            xj[rank] = j;
        }
        __syncthreads();
        const int r = (lane * m) >> 16;
        if (r < k)
            dbuf[lane] = event_draw_uniform<PREC>(
                xn[r] + (uint32_t)((lane - r * D) * (PREC == LIK_FP32_MIXED ? 2 : 1)),
                (uint32_t)xj[r], c2, c3, k0, k1);
        __syncthreads();
        const int slot = rank * D;
#pragma unroll 1
        for (int i = 0; i < D; ++i) {
            if (have)
                ssa_event<NetT, UMAX, RMAX, W, PREC, Real>(net, c, x, S, t_end, event_cap, clock,
                                                           n, st, a0_end, have, nu_tab,
                                                           [&] { return dbuf[slot + i]; });
            if (__ballot(have) == 0ull) break;
        }
        __syncthreads();  // the draws are read before the next round writes
    }
    if (pend) retire();
    if (st != LIK_STATUS_OK) atomicMax(&e.fstatus[f], st);
}

// One wavefront per work item of the iteration's list.
template <class NetT, int UMAX, int RMAX, int W, int PREC>
__device__ __forceinline__ void propagate_item(const EngineArgs &e, const NetT &net, int group) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[item_lds_words<UMAX, RMAX, PREC>()];
    if (blockIdx.x >= e.item_count[group]) return;
    run_item<NetT, UMAX, RMAX, W, PREC>(e, net, e.items[e.group_off[group] + blockIdx.x], lds);
}

// ---------------------------------------------------------------------------
// propagate_persistent: the same particles, streams and arithmetic as
// propagate_item, scheduled across work items.  A grid of wavefronts takes
// work items of the group from a counter in list order (longest first).  A
// lane whose particle reaches its observation time stores it and takes the
// next particle of the wavefront's current pool; once the pool is exhausted
// the wavefront takes the next item, stages its ancestors' counts in LDS and
// goes on filling idle lanes, while lanes still running particles of earlier
// items finish them.  Lanes therefore carry their particle's filter context
// (rates, observation time, stream ids, output pointers).  The Philox key
// stays wave-uniform: a pool whose filter has another seed waits until every
// lane is idle.  Used for networks of at most 16 reactions (the rates live
// in registers per lane).
// ---------------------------------------------------------------------------
template <class NetT, int UMAX, int RMAX, int W, int PREC>
__device__ __forceinline__ void propagate_persistent(const EngineArgs &e, const NetT &net,
                                                     int group) {
    using Real = typename pick_type<PREC == LIK_FP32_MIXED, float, double>::type;
    const int U = net.U;
    const int R = net.R;
    const int lane = (int)threadIdx.x;
    const uint32_t n_items = e.item_count[group];
    const uint32_t *items = e.items + e.group_off[group];
    const int refill_min = e.refill_min;
    __shared__ int32_t pool_x[kPoolLdsWords];  // [U][npool]: ancestors' counts of the pool

    // the current pool (wave-uniform)
    int p0 = 0, p1 = 0, next = 0, npool = 0;
    bool more = true;  // items may remain
    int pf = 0;        // its filter
    double p_t0 = 0.0, p_t1 = 0.0;
    uint32_t p_c2 = 0, p_c3 = 0, p_cap = 0;
    uint64_t p_seed = 0;
    int32_t *p_dst = nullptr;
    uint32_t *p_pev = nullptr;
    float *p_pa0 = nullptr;
    int p_hp = 0;
    Real p_c[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) p_c[r] = (Real)0;
    // the wavefront's Philox key
    uint32_t k0 = 0, k1 = 0;

    // the lane's particle and its filter context
    bool have = false, pend = false;
    int j = 0, fl = 0, hp = 0;
    int x[UMAX];
#pragma unroll
    for (int u = 0; u < UMAX; ++u) x[u] = 0;
    Real c[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) c[r] = (Real)0;
    double clock = 0.0, t_end = 0.0;
    uint32_t n = 0, c2 = 0, c3 = 0, cap = 0;
    int32_t *dst = nullptr;
    uint32_t *pev = nullptr;
    float *pa0 = nullptr;
    int st = LIK_STATUS_OK;
    Real a0_end = (Real)0;
    Real S[RMAX];

    auto retire = [&]() {
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < U && x[u] > kCountLimit)
                st = st > LIK_STATUS_COUNT_OVERFLOW ? st : LIK_STATUS_COUNT_OVERFLOW;
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < U) dst[(size_t)u * hp + j] = x[u];
        pev[j] = n;
        pa0[j] = (float)a0_end;
        if (st != LIK_STATUS_OK) atomicMax(&e.fstatus[fl], st);
        st = LIK_STATUS_OK;
    };

    for (;;) {
        if (have)
            ssa_event<NetT, UMAX, RMAX, W, PREC, Real>(
                net, c, x, S, t_end, cap, clock, n, st, a0_end, have,
                static_cast<const uint32_t *>(nullptr),
                [&] { return event_draw<PREC>(n, (uint32_t)j, c2, c3, k0, k1); });
        uint64_t idle = __ballot(!have);
        const int n_idle = (int)__popcll(idle);
        if (n_idle > 0 && (next < p1 || more) && (n_idle >= refill_min || idle == ~0ull)) {
            if (!have && pend) {
                retire();
                pend = false;
            }
            for (;;) {
                if (idle == 0ull) break;
                if (next >= p1) {
                    if (!more) break;
                    uint32_t idx = 0;
                    if (lane == 0) idx = atomicAdd(&e.item_cursor[group], 1u);
                    idx = __builtin_amdgcn_readfirstlane(__shfl(idx, 0, 64));
                    if (idx >= n_items) {
                        more = false;
                        break;
                    }
                    const uint32_t item = __builtin_amdgcn_readfirstlane(items[idx]);
                    pf = (int)(item >> 6);
                    const FilterDesc &d = e.desc[pf];
                    const int t = __builtin_amdgcn_readfirstlane(e.tcur[pf]);
                    const int H = __builtin_amdgcn_readfirstlane(d.H);
                    p_hp = __builtin_amdgcn_readfirstlane(d.Hp);
                    p0 = (int)(item & 63u) * kPropBlock;
                    const int g = (int)(__builtin_amdgcn_readfirstlane(e.pool[pf]) & 63u) + 1;
                    p1 = min(p0 + g * kPropBlock, H);
                    next = p0;
                    npool = p1 - p0;
                    p_t0 = wave_uniform((t == 0) ? d.t0 : d.t_obs[t - 1]);
                    p_t1 = wave_uniform(d.t_obs[t]);
                    p_c2 = __builtin_amdgcn_readfirstlane((d.traj << 16) | (uint32_t)t);
                    p_c3 = __builtin_amdgcn_readfirstlane(d.theta_id << 2);
                    p_cap = __builtin_amdgcn_readfirstlane(d.event_cap);
                    p_seed = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(d.seed >> 32))
                              << 32) |
                             __builtin_amdgcn_readfirstlane((uint32_t)d.seed);
                    const int32_t *src = (t & 1) ? d.xb : d.xa;
                    p_dst = (t & 1) ? d.xa : d.xb;
                    p_pev = d.pev;
                    p_pa0 = d.pa0;
#pragma unroll
                    for (int r = 0; r < RMAX; ++r)
                        p_c[r] = (r < R) ? wave_uniform((Real)d.theta[r]) : (Real)0;
                    // stage the pool's ancestors' counts (every lane has read
                    // the previous pool's entries it needed)
                    const int32_t *anc = d.anc;
                    const int32_t *x0 = d.x0;
                    const bool fixed0 = t == 0 && d.x0_hi == nullptr;
#pragma unroll 1
                    for (int q = lane; q < npool; q += kPropBlock) {
                        if (fixed0) {
#pragma unroll
                            for (int u = 0; u < UMAX; ++u)
                                if (u < U) pool_x[u * npool + q] = x0[u];
                        } else {
                            const int a = anc[p0 + q];
#pragma unroll
                            for (int u = 0; u < UMAX; ++u)
                                if (u < U) pool_x[u * npool + q] = src[(size_t)u * p_hp + a];
                        }
                    }
                    __syncthreads();  // the workgroup is this one wavefront
                }
                // a pool with another key waits until every lane is idle
                const uint32_t pk0 = (uint32_t)p_seed, pk1 = (uint32_t)(p_seed >> 32);
                if (pk0 != k0 || pk1 != k1) {
                    if (idle != ~0ull) break;
                    k0 = pk0;
                    k1 = pk1;
                }
                const int avail = p1 - next;
                if (!have) {
                    const int rank = (int)__builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                    if (rank < avail) {
                        j = next + rank;
#pragma unroll
                        for (int u = 0; u < UMAX; ++u)
                            x[u] = (u < U) ? pool_x[u * npool + (j - p0)] : 0;
#pragma unroll
                        for (int r = 0; r < RMAX; ++r) c[r] = p_c[r];
                        clock = p_t0;
                        t_end = p_t1;
                        n = 0;
                        c2 = p_c2;
                        c3 = p_c3;
                        cap = p_cap;
                        dst = p_dst;
                        pev = p_pev;
                        pa0 = p_pa0;
                        hp = p_hp;
                        fl = pf;
                        have = true;
                        pend = true;
                    }
                }
                next += min((int)__popcll(idle), avail);
                idle = __ballot(!have);
            }
        }
        if (__ballot(have) == 0ull && next >= p1 && !more) break;
    }
    if (pend) retire();
}

}  // namespace lik
