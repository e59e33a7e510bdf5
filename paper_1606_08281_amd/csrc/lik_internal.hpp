// lik_internal.hpp -- structures shared by the host engine and the kernels.
//
// Every filter (one rate vector against one observed trajectory) lives in a
// slot of a filter table: an immutable descriptor (where its inputs and its
// particle state are, its sizes, its random-stream ids) plus mutable
// per-slot state (next interval, log-likelihood, status).  One engine
// iteration advances every active slot by one observation interval, whatever
// request, network, particle count or trajectory length it belongs to.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "../../include/lik.h"

namespace lik {

constexpr int kPropBlock = 64;    // one wavefront per propagation work item
constexpr int kWeighBlock = 256;  // one workgroup per filter for weights/resampling
constexpr int kMaxGroups = 16;    // (network, precision) groups per iteration
constexpr int kCostKeys = 129;    // quarter octaves of expected events per lane, and zero
constexpr uint32_t kFlagStopped = 1u;
constexpr int32_t kCountLimit = 1 << 30;
// LDS that stages a pool's starting counts, per wavefront (6 KiB: 26
// wavefronts per CU fit in its 160 KiB).  A pool takes U words per particle
// for the counts and half a word for its processing order (16-bit indexes),
// so G <= kPoolLdsWords / (64 U + 32).
constexpr int kPoolLdsWords = 1536;
__host__ __device__ constexpr int pool_lds_cap(int U) { return kPoolLdsWords / (64 * U + 32); }
// Pools of up to 64 * kSortPerLane particles are taken heaviest first.
constexpr int kSortPerLane = 6;
constexpr int kSortBuckets = 64;  // half octaves of the expected cost, below the heaviest

// Reaction kinds after validation of the reactant orders.
enum : int32_t { kOrder0 = 0, kOrder1 = 1, kOrder2Homo = 2, kOrder2Hetero = 3 };

// Network tables in kernel-argument (scalar) memory.  Net change of reaction
// r for species u, two's complement: for at most four species a byte, bits
// [8u, 8u+8) of nu[r][0] (a byte field is added with its sign extension in
// one instruction); otherwise bits [4(u%8), 4(u%8)+4) of nu[r][u/8].
__host__ __device__ constexpr bool nu_bytes(int U) { return U <= 4; }
template <int RMAX, int W>
struct NetArgs {
    int32_t U, R;
    int32_t kind[RMAX];
    int32_t s1[RMAX];
    int32_t s2[RMAX];
    uint32_t nu[RMAX][W];
};

// Immutable description of one filter slot.
struct FilterDesc {
    const double *theta;   // [R] rate constants
    const double *t_obs;   // [T] observation times
    const double *y;       // [T * P] observations
    const int32_t *x0;     // [U] initial counts (lower bounds when x0_hi is set)
    const int32_t *x0_hi;  // [U] upper bounds of random initial counts, or null
    int32_t *xa;           // [U][Hp] counts after even-numbered intervals
    int32_t *xb;           // [U][Hp] counts after odd-numbered intervals
    double *lw;            // [Hp] particle log-weights (particle-dependent part)
    int32_t *anc;          // [Hp] ancestors for the next interval
    uint32_t *pev;         // [Hp] events of each particle in the last interval
    float *pa0;            // [Hp] total propensity at each particle's state at the
                           //      last observation time (cost prediction)
    double t0;             // start time
    double sigma;          // observation noise scale
    double gain, bg_mean;  // fluorescence model: mean gain * x + bg_mean ...
    double obs_s2, bg_s2;  // ... variance obs_s2 * x + bg_s2 (sigma^2, bg_sd^2)
    uint64_t seed;         // Philox key
    uint32_t theta_id;     // random-stream id of the rate vector
    uint32_t traj;         // trajectory index within its request
    int32_t H, Hp, T, U, R, P;
    int32_t obs_kind;
    int32_t group;         // (network, precision) group of this slot
    uint32_t event_cap;
    int32_t pad;
    int32_t obs_species[LIK_MAX_OBSERVED];
};

// Everything an iteration's kernels need: the filter table, its mutable
// state and the grouped work items.
struct EngineArgs {
    const FilterDesc *desc;   // [slots]
    int32_t *tcur;            // [slots] next interval to propagate
    double *fll;              // [slots] running log-likelihood
    int32_t *fstatus;         // [slots]
    uint32_t *fflags;         // [slots]
    uint64_t *fevents;        // [slots] SSA events applied
    uint32_t *cost;           // [slots] expected events of the next interval (ordering key)
    uint8_t *pool;            // [slots] (wave priority << 6) | (particles per item / 64 - 1)
    uint32_t *items;          // propagation work items (slot << 6 | chunk), grouped
    uint32_t *item_count;     // [kMaxGroups] items written per group
    uint32_t *item_cursor;    // [kMaxGroups] next item to take (persistent kernels)
    // Ordering of an iteration's work (three passes: count, scan, place).
    uint32_t *order_count;    // [kMaxGroups * kCostKeys] items per (group, duration key);
                              // zero between iterations
    uint32_t *order_pos;      // [kMaxGroups * kCostKeys] next position of each (group, key)
    uint32_t *order_ctl;      // [2]: most expected events per particle of any slot (zero
                              // between iterations), and its copy for the placing pass
    uint32_t pool_chunks;     // groups of 64 particles over the slots that may be active
    uint64_t *fdone;          // [slots] device wall clock when the slot's filter finished, or
                              // null (not recorded)
    int32_t f_lo, f_hi;       // slot range that may hold active filters
    // Pool size G per slot: G = clamp(pool_events / (events per particle in
    // the last interval), pool_min, pool_max); pool_first for the first one.
    uint32_t pool_events;
    int32_t pool_min, pool_max, pool_first;
    int32_t refill_min;       // idle lanes that trigger a refill from the pool
    int32_t priority;         // raise the wave priority of the heaviest slots
    uint32_t pool_min_items;  // work items an iteration keeps before pools grow
    int32_t h_max;            // most particles of any active slot (LDS of k_weigh)
    uint32_t group_off[kMaxGroups];  // first item of each group
};

// Flow engine (one launch runs every interval of a batch; flow.hpp).  Ring
// kRingItems holds work items, ring kRingParked the ids of filters whose
// items wait for room.  Control words sit 128 bytes apart in ctl.
constexpr int kFlowRings = 2;
enum : int { kRingItems = 0, kRingParked = 1 };
enum : int {
    kCtlHead = 0,         // + 64 r: next position of ring r a wavefront claims
    kCtlTail = 32,        // + 64 r: next position of ring r an entry is written to
    kCtlFinished = 128,   // slots that need no further interval
    kCtlAbort = 160,      // nonzero: a wavefront saw no progress for stall_ticks
    kCtlProgress = 192,   // work items finished
    kCtlSeedItems = 224,  // items of the first interval placed in the item ring
    kCtlArgs = 256,       // a copy of the launch's FlowArgs (16 words)
    kCtlWords = 272
};
struct FlowArgs {
    // ring r at ring + r (mask + 1): slot pos & mask holds (pos + 1) << 32 |
    // item once the item of position pos is written, pos << 32 while it is
    // free for position pos
    uint64_t *ring;
    uint32_t *remaining;   // [slots] work items of the slot's interval not finished
    uint32_t *ctl;         // [kCtlWords]
    uint32_t mask;         // ring capacity - 1: a power of two, at least twice the
                           // slots' groups of 64 (items outstanding at any time)
    int32_t n_slots;       // the batch is done when this many slots have finished
    int32_t g_par;         // largest pool (groups of 64) of a work item
    uint32_t urgent_events;  // a filter whose intervals left times the expected events
                             // per lane of its items reach this is never parked (0: no
                             // parking at all)
    uint32_t backlog;        // items waiting in the item ring above which a filter that
                             // is not urgent is parked
    uint32_t pad;
    uint64_t stall_ticks;  // wall-clock ticks without a finished item before a
                           // waiting wavefront gives up (a scheduler fault)
};
static_assert(sizeof(FlowArgs) <= 4 * (kCtlWords - kCtlArgs), "FlowArgs copy fits");
// The flow kernel reads its FlowArgs from the copy in device memory: its
// fields are loaded where they are used (the hand-off after the event loop
// reloads them) instead of being held in scalar registers through the event
// loop, as kernel arguments are.
__host__ __device__ inline const FlowArgs *flow_args_copy(uint32_t *ctl) {
    return reinterpret_cast<const FlowArgs *>(ctl + kCtlArgs);
}

#ifndef __HIPCC_RTC__
// Host-side launchers (kernels.hip).
hipError_t launch_order(const EngineArgs &e, hipStream_t s);
hipError_t launch_order_reset(const EngineArgs &e, hipStream_t s);  // before a batch's first
constexpr int kOrderBlock = 256;  // slots per block of the ordering passes
hipError_t launch_propagate(const EngineArgs &e, int group, unsigned n_items, const void *net,
                            int umax, int rmax, int precision, bool persistent, hipStream_t s);
constexpr int kPersistentMaxR = 16;  // rates per lane in registers: small networks only
hipError_t launch_weigh(const EngineArgs &e, hipStream_t s);
// Flow engine: ring reset and first items; the launch (generic network
// tables; n_waves wavefronts, one work item each); the scheduler-fault check.
hipError_t launch_flow_setup(const EngineArgs &e, const FlowArgs &fa, hipStream_t s);
hipError_t launch_flow(const EngineArgs &e, const FlowArgs &fa, unsigned n_waves, const void *net,
                       int umax, int rmax, int precision, hipStream_t s);
hipError_t launch_flow_check(const EngineArgs &e, const FlowArgs &fa, hipStream_t s);
int flow_blocks_per_cu(int umax, int rmax, int precision);  // resident flow wavefronts per CU
// The flow schedule hides each hand-off's latency behind other resident
// wavefronts: below this many per CU it is slower than the per-interval one.
constexpr int kFlowMinWavesPerCu = 16;
// Ring capacity for F slots of nchunk groups of 64 particles.
inline uint32_t flow_ring_capacity(size_t F, int nchunk) {
    const size_t need = 2 * F * (size_t)nchunk;
    uint32_t c = 1024;
    while ((size_t)c < need && c < (1u << 31)) c <<= 1;
    return c;
}

// Per-request setup / results.  A request is n_theta rate vectors against M
// trajectories, occupying slots base .. base + n_theta*M - 1.
struct RequestArgs {
    const double *theta;        // [n_theta * R]
    const uint32_t *theta_ids;  // [n_theta] or null
    const int32_t *obs_offsets; // [M + 1]
    const double *t_obs;
    const double *y;
    const double *t0;           // [M]
    const int32_t *x0;          // [M * U]
    const int32_t *x0_hi;       // [M * U] upper bounds of random initial counts, or null
    int32_t *state;             // particle state arena of the request
    int32_t n_theta, M, H, Hp, U, R, P, obs_kind, group;
    int32_t precision;          // LIK_FP64 or LIK_FP32_MIXED (rates checked for its range)
    int32_t obs_species[LIK_MAX_OBSERVED];
    double sigma, gain, bg_mean, bg_sd;
    uint64_t seed;
    uint32_t event_cap;
    int32_t base;               // first slot
    // reactant tables (kind, s1, s2 per reaction) for the first interval's
    // cost estimate: total propensity at x0 times the interval's length
    int8_t kind[LIK_MAX_REACTIONS], s1[LIK_MAX_REACTIONS], s2[LIK_MAX_REACTIONS];
};
void fill_reactant_tables(RequestArgs &r, const int32_t *kind, const int32_t *s1,
                          const int32_t *s2, int R);
size_t request_state_bytes(int64_t F, int32_t U, int32_t Hp);
// A request's place in a multi-request batch: first slot, sizes, and the
// offset of its per-theta results.
struct ReqSpan {
    int32_t base, n_theta, M, out;
};
// Random initial counts of the slots [base, base + F) that have them (the
// others are left alone): each particle's draw into the buffer its first
// interval reads, and identity ancestors.
hipError_t launch_init_start(const FilterDesc *desc, int32_t base, int32_t F, hipStream_t s);
hipError_t launch_admit_requests(FilterDesc *desc, const EngineArgs &e, const RequestArgs *reqs,
                                 const int32_t *fstart, int32_t n_req, int32_t n_filters,
                                 uint64_t *start_tick, hipStream_t s);
hipError_t launch_finish_requests(const EngineArgs &e, const ReqSpan *spans, int32_t n_req,
                                  double *loglik, int32_t *status, hipStream_t s);
// Flow launch over filters of several networks with the generic tables
// nets_dev[group] (NetArgs of the umax x rmax bucket, in device memory).
hipError_t launch_flow_multi(const EngineArgs &e, const FlowArgs &fa, unsigned n_waves,
                             const void *nets_dev, int umax, int rmax, int precision,
                             hipStream_t s);
int flow_multi_blocks_per_cu(int umax, int rmax, int precision);
hipError_t launch_admit(FilterDesc *desc, const EngineArgs &e, const RequestArgs &r,
                        hipStream_t s);
const void *admit_kernel();  // k_admit, for updating captured graph nodes
// Stops slots base .. base + F - 1 (a withdrawn request): later iterations skip them.
hipError_t launch_stop(const EngineArgs &e, int32_t base, int32_t F, hipStream_t s);
hipError_t launch_finish(const EngineArgs &e, int32_t base, int32_t n_theta, int32_t M,
                         double *loglik, int32_t *status, const lik_aux *aux, hipStream_t s);
#endif  // __HIPCC_RTC__

// Size-bucketed network argument blocks the generic launchers accept.
using Net4x8 = NetArgs<8, 1>;    // U <= 4, R <= 8
using Net8x16 = NetArgs<16, 1>;  // U <= 8, R <= 16
using Net32x64 = NetArgs<64, 4>; // U <= 32, R <= 64

}  // namespace lik
