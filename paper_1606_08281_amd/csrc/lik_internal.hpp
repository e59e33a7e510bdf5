// lik_internal.hpp -- structures shared by the host API and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lik.h"

namespace lik {

constexpr int kPropBlock = 64;    // one wavefront per propagation work item
constexpr int kWeighBlock = 256;  // one workgroup per filter for weights/resampling
constexpr uint32_t kFlagStopped = 1u;
constexpr int32_t kCountLimit = 1 << 30;

// Reaction kinds after validation of the reactant orders.
enum : int32_t { kOrder0 = 0, kOrder1 = 1, kOrder2Homo = 2, kOrder2Hetero = 3 };

// Network tables in kernel-argument (scalar) memory.  Net change of reaction
// r for species u sits in bits [4(u%8), 4(u%8)+4) of nu[r][u/8], two's
// complement.
template <int RMAX, int W>
struct NetArgs {
    int32_t U, R;
    int32_t kind[RMAX];
    int32_t s1[RMAX];
    int32_t s2[RMAX];
    uint32_t nu[RMAX][W];
};

// Everything a launch needs besides the network: inputs, workspace, shape.
struct EvalArgs {
    // inputs (device)
    const double *theta;
    const uint32_t *theta_ids;
    const int32_t *obs_offsets;
    const double *t_obs;
    const double *y;
    const double *t0;
    const int32_t *x0;
    // shape
    int32_t n_theta, M, H, Hp, U, R, P, nchunk;
    int32_t obs_kind;
    int32_t obs_species[LIK_MAX_OBSERVED];
    double sigma;
    uint64_t seed;
    uint32_t event_cap;
    // workspace (device)
    int32_t *xa;        // [F][U][Hp] counts, state after even-numbered intervals
    int32_t *xb;        // [F][U][Hp] counts, state after odd-numbered intervals
    double *lw;         // [F][Hp] particle log-weights (particle-dependent part)
    int32_t *anc;       // [F][Hp] ancestors for the next interval
    double *fll;        // [F] running log-likelihood
    int32_t *fstatus;   // [F]
    uint32_t *fflags;   // [F]
    uint64_t *fevents;  // [F]
    int32_t *fsteps;    // [F] intervals propagated
    uint32_t *order;    // [F] filter processing order (heaviest first)
    uint32_t *cost;     // [F] cost key for ordering
};

// Host-side launchers (kernels.hip).
hipError_t launch_init(const EvalArgs &a, hipStream_t s);
hipError_t launch_order(const EvalArgs &a, int t, hipStream_t s);
hipError_t launch_propagate(const EvalArgs &a, const void *net, int umax, int rmax,
                            int precision, int t, hipStream_t s);
hipError_t launch_weigh(const EvalArgs &a, int t, hipStream_t s);
hipError_t launch_finish(const EvalArgs &a, double *loglik, int32_t *status,
                         const lik_aux *aux, hipStream_t s);

// Size-bucketed network argument blocks the launchers accept.
using Net4x8 = NetArgs<8, 1>;    // U <= 4, R <= 8
using Net8x16 = NetArgs<16, 1>;  // U <= 8, R <= 16
using Net32x64 = NetArgs<64, 4>; // U <= 32, R <= 64

}  // namespace lik
