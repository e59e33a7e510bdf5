// kernels.hip -- gfx950 kernels of the particle-filter likelihood.
//
// One observation interval of every filter (theta i, trajectory m) is
// advanced per pair of launches:
//   k_propagate: one lane per filter particle, one wavefront per work item
//     (64 consecutive particles of one filter).  Gathers the particle's
//     ancestor state, runs Gillespie's direct method from the previous
//     observation time to the next one (Supplementary I, Algorithm
//     "Likelihood Approximation using particle filter", the "Simulate" step),
//     then evaluates the particle's log-weight (the "Compute l_t^i" step).
//   k_weigh: one workgroup per filter.  Log-sum-exp of the weights into the
//     running log-likelihood (the step that multiplies p(y_{t-1}|theta) by
//     the mean weight), then systematic resampling with integer weights for
//     the next interval (the "Sample H indices according to weights" step).
// k_order sorts filters heaviest-first by the events of their last interval
// so the wavefronts of expensive filters are dispatched first.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "devmath.hpp"
#include "lik_internal.hpp"

namespace lik {

// ---------------------------------------------------------------------------
// wavefront / workgroup reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// inclusive prefix sum over the 64 lanes of a wavefront
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// ---------------------------------------------------------------------------
// init: per-filter bookkeeping; rates that are negative, infinite or NaN mark
// every filter of that theta BAD_THETA before any simulation.
// ---------------------------------------------------------------------------
__global__ void k_init(EvalArgs a) {
    const int F = a.n_theta * a.M;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int i = f / a.M;
    bool bad = false;
    for (int r = 0; r < a.R; ++r) {
        const double c = a.theta[(size_t)i * a.R + r];
        if (!(c >= 0.0) || isinf(c)) bad = true;
    }
    a.fll[f] = bad ? __builtin_nan("") : 0.0;
    a.fstatus[f] = bad ? LIK_STATUS_BAD_THETA : LIK_STATUS_OK;
    a.fflags[f] = bad ? kFlagStopped : 0u;
    a.fevents[f] = 0;
    a.fsteps[f] = 0;
    a.order[f] = (uint32_t)f;
    a.cost[f] = 0;
}

// ---------------------------------------------------------------------------
// order: filters sorted by decreasing bit length of the events their
// particles needed in the previous interval (a counting sort over 33 keys in
// one workgroup).  Order inside a key is arbitrary: it only changes which
// wavefront starts first, never a result.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_order(EvalArgs a) {
    __shared__ uint32_t hist[33];
    const int F = a.n_theta * a.M;
    if (threadIdx.x < 33) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int f = threadIdx.x; f < F; f += blockDim.x) {
        const uint32_t c = (a.fflags[f] & kFlagStopped) ? 0u : a.cost[f];
        const int key = 32 - (c == 0 ? 0 : 32 - __clz(c));  // 0 = heaviest
        atomicAdd(&hist[key], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int k = 0; k < 33; ++k) {
            const uint32_t h = hist[k];
            hist[k] = run;
            run += h;
        }
    }
    __syncthreads();
    for (int f = threadIdx.x; f < F; f += blockDim.x) {
        const uint32_t c = (a.fflags[f] & kFlagStopped) ? 0u : a.cost[f];
        const int key = 32 - (c == 0 ? 0 : 32 - __clz(c));
        const uint32_t pos = atomicAdd(&hist[key], 1u);
        a.order[pos] = (uint32_t)f;
        a.cost[f] = 0;  // re-accumulated by the next propagation
    }
}

// ---------------------------------------------------------------------------
// propagate: resample-gather, direct-method SSA to the next observation time,
// particle log-weight.
// ---------------------------------------------------------------------------
template <int UMAX, int RMAX, int W, int PREC>
__global__ __launch_bounds__(kPropBlock) void k_propagate(EvalArgs a, NetArgs<RMAX, W> net,
                                                          int t) {
    const int item = blockIdx.x;
    const int f = (int)a.order[item / a.nchunk];
    const int chunk = item % a.nchunk;
    if (a.fflags[f] & kFlagStopped) return;
    const int i = f / a.M;
    const int m = f - i * a.M;
    const int off = a.obs_offsets[m];
    const int T = a.obs_offsets[m + 1] - off;
    if (t >= T) return;

    const int U = net.U;
    const int R = net.R;
    const int H = a.H;
    const int j = chunk * kPropBlock + (int)threadIdx.x;
    const bool active = j < H;
    const double t_start = (t == 0) ? a.t0[m] : a.t_obs[off + t - 1];
    const double t_end = a.t_obs[off + t];
    const uint32_t tid = a.theta_ids ? a.theta_ids[i] : (uint32_t)i;
    const uint32_t c2 = ((uint32_t)m << 16) | (uint32_t)t;
    const uint32_t c3 = tid << 2;  // purpose 0: reaction events
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);

    double c[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) c[r] = (r < R) ? a.theta[(size_t)i * R + r] : 0.0;

    int x[UMAX];
    const size_t fbase = (size_t)f * U * a.Hp;
    if (t == 0) {
#pragma unroll
        for (int u = 0; u < UMAX; ++u) x[u] = (u < U) ? a.x0[(size_t)m * U + u] : 0;
    } else {
        const int32_t *src = (t & 1) ? a.xb : a.xa;
        const int anc = active ? a.anc[(size_t)f * a.Hp + j] : 0;
#pragma unroll
        for (int u = 0; u < UMAX; ++u) x[u] = (u < U) ? src[fbase + (size_t)u * a.Hp + anc] : 0;
    }

    uint32_t n = 0;
    int st = LIK_STATUS_OK;
    if (active) {
        double clock = t_start;
        for (;;) {
            // Propensities a_r = c_r h_r(x) and running sums S_r, in r order.
            double S[RMAX];
            float Sf[RMAX];
            double s = 0.0;
            float sf = 0.0f;
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (r < R) {
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
                    if (PREC == LIK_FP32_MIXED) {
                        sf = sf + (float)c[r] * (float)h;
                        Sf[r] = sf;
                    } else {
                        s = s + c[r] * h;
                        S[r] = s;
                    }
                }
            }
            uint32_t sel[W];
            double tau_d;
            if (PREC == LIK_FP32_MIXED) {
                if (!(sf > 0.0f)) break;
                if (n >= a.event_cap) { st = LIK_STATUS_EVENT_CAP; break; }
                const Block4 b = philox4x32_10(n >> 1, (uint32_t)j, c2, c3, k0, k1);
                const uint32_t wa = (n & 1) ? b.w2 : b.w0;
                const uint32_t wb = (n & 1) ? b.w3 : b.w1;
                const float u1 = (float)((wa >> 8) + 1u) * 0x1p-24f;
                const float u2 = (float)(wb >> 8) * 0x1p-24f;
                const float tau = -flog(u1) / sf;
                tau_d = (double)tau;
                if (clock + tau_d > t_end) break;
                const float target = u2 * sf;
                // r* = min{r : S_r > target}; S_{R-1} = sf > target always
                // (u2 <= 1 - 2^-24), and a zero-propensity reaction repeats
                // the previous sum, so r* always has a_r* > 0.
#pragma unroll
                for (int w = 0; w < W; ++w) sel[w] = net.nu[R - 1][w];
#pragma unroll
                for (int r = RMAX - 2; r >= 0; --r) {
                    if (r < R - 1) {
                        const bool hit = Sf[r] > target;
#pragma unroll
                        for (int w = 0; w < W; ++w) sel[w] = hit ? net.nu[r][w] : sel[w];
                    }
                }
            } else {
                if (!(s > 0.0)) break;
                if (n >= a.event_cap) { st = LIK_STATUS_EVENT_CAP; break; }
                const Block4 b = philox4x32_10(n, (uint32_t)j, c2, c3, k0, k1);
                const uint64_t z1 = ((((uint64_t)b.w1) << 32) | b.w0) >> 11;
                const uint64_t z2 = ((((uint64_t)b.w3) << 32) | b.w2) >> 11;
                const double u1 = (double)(z1 + 1) * 0x1p-53;  // (0, 1]
                const double u2 = (double)z2 * 0x1p-53;        // [0, 1)
                tau_d = -dlog(u1) / s;
                if (clock + tau_d > t_end) break;  // the pending event is discarded
                const double target = u2 * s;
                // r* = min{r : S_r > target}; see the binary32 branch for why
                // the last sum always exceeds the target.
#pragma unroll
                for (int w = 0; w < W; ++w) sel[w] = net.nu[R - 1][w];
#pragma unroll
                for (int r = RMAX - 2; r >= 0; --r) {
                    if (r < R - 1) {
                        const bool hit = S[r] > target;
#pragma unroll
                        for (int w = 0; w < W; ++w) sel[w] = hit ? net.nu[r][w] : sel[w];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                if (u < U) x[u] += __builtin_amdgcn_sbfe(sel[u >> 3], 4 * (u & 7), 4);
            clock = clock + tau_d;
            n = n + 1;
        }
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < U && x[u] > kCountLimit) st = st > LIK_STATUS_COUNT_OVERFLOW ? st : LIK_STATUS_COUNT_OVERFLOW;

        // Particle-dependent part of log p(y_t | x).
        const double *yt = a.y + (size_t)(off + t) * a.P;
        double lw = 0.0;
        for (int k = 0; k < a.P; ++k) {
            const int cnt = x[a.obs_species[k]];
            if (a.obs_kind == LIK_OBS_LOGNORMAL) {
                if (cnt <= 0) {
                    lw = -__builtin_inf();
                    break;
                }
                const double z = (dlog(yt[k]) - dlog((double)cnt)) / a.sigma;
                lw = lw - 0.5 * (z * z);
            } else {
                const double z = (yt[k] - (double)cnt) / a.sigma;
                lw = lw - 0.5 * (z * z);
            }
        }
        int32_t *dst = (t & 1) ? a.xa : a.xb;
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < U) dst[fbase + (size_t)u * a.Hp + j] = x[u];
        a.lw[(size_t)f * a.Hp + j] = lw;
        if (st != LIK_STATUS_OK) atomicMax(&a.fstatus[f], st);
    }
    const uint64_t ev = wave_sum_u64((uint64_t)n);
    if (threadIdx.x == 0 && ev) {
        atomicAdd((unsigned long long *)&a.fevents[f], (unsigned long long)ev);
        atomicAdd(&a.cost[f], (uint32_t)(ev > 0xFFFFFFFFull ? 0xFFFFFFFFu : ev));
    }
}

// ---------------------------------------------------------------------------
// weigh: log-sum-exp into the running log-likelihood, then systematic
// resampling with q_j = floor(e_j 2^32), integer prefix sums C, one offset
// rho = floor(w64 Q / 2^64) and ancestors a_j = min{i : H C_{i+1} > j Q + rho}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWeighBlock) void k_weigh(EvalArgs a, int t) {
    __shared__ uint64_t Cs[LIK_MAX_PARTICLES];  // Cs[k] = C_{k+1}
    __shared__ double red[kWeighBlock / 64];
    __shared__ uint64_t redu[kWeighBlock / 64];
    __shared__ double bcast;
    __shared__ uint64_t bcast_u;

    const int f = blockIdx.x;
    if (a.fflags[f] & kFlagStopped) return;
    const int i = f / a.M;
    const int m = f - i * a.M;
    const int off = a.obs_offsets[m];
    const int T = a.obs_offsets[m + 1] - off;
    if (t >= T) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int H = a.H;
    if (tid == 0) a.fsteps[f] = t + 1;
    if (a.fstatus[f] != LIK_STATUS_OK) {
        if (tid == 0) {
            a.fll[f] = __builtin_nan("");
            a.fflags[f] |= kFlagStopped;
        }
        return;
    }
    const double *lw = a.lw + (size_t)f * a.Hp;
    const int per = (H + kWeighBlock - 1) / kWeighBlock;
    const int j0 = tid * per;
    const int j1 = min(j0 + per, H);

    // max
    double mx = -__builtin_inf();
    for (int j = j0; j < j1; ++j) mx = fmax(mx, lw[j]);
    mx = wave_max(mx);
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
            a.fll[f] = -__builtin_inf();
            a.fflags[f] |= kFlagStopped;
        }
        return;
    }

    // e_j, their sum, integer weights q_j (kept in Cs until the scan)
    double s = 0.0;
    uint64_t qsum = 0;
    for (int j = j0; j < j1; ++j) {
        const double e = dexp_nonpos(lw[j] - mx);
        s += e;
        const uint64_t q = (uint64_t)(e * 4294967296.0);
        Cs[j] = q;
        qsum += q;
    }
    s = wave_sum(s);
    __syncthreads();  // red[] reuse
    if (lane == 0) red[wave] = s;

    // exclusive scan of the per-thread sums (thread order = particle order)
    const uint64_t incl = wave_incl_scan_u64(qsum);
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
        double S = red[0];
        for (int w = 1; w < kWeighBlock / 64; ++w) S += red[w];
        // running log-likelihood: log of the mean weight plus the
        // particle-independent part of the observation density
        const double *yt = a.y + (size_t)(off + t) * a.P;
        const double per_comp = dlog(a.sigma) + 0.5 * dlog(2.0 * 3.141592653589793);
        double cst = -((double)a.P * per_comp);
        if (a.obs_kind == LIK_OBS_LOGNORMAL)
            for (int k = 0; k < a.P; ++k) cst = cst - dlog(yt[k]);
        const double inc = ((mx + dlog(S)) - dlog((double)H)) + cst;
        a.fll[f] = a.fll[f] + inc;
        if (t + 1 < T) {
            const uint32_t tid_th = a.theta_ids ? a.theta_ids[i] : (uint32_t)i;
            const Block4 b = philox4x32_10(0u, 0u, ((uint32_t)m << 16) | (uint32_t)(t + 1),
                                           (tid_th << 2) | 1u, (uint32_t)a.seed,
                                           (uint32_t)(a.seed >> 32));
            bcast_u = ((uint64_t)b.w1 << 32) | b.w0;
        }
    }
    if (t + 1 >= T) return;
    __syncthreads();
    const uint64_t Q = Cs[H - 1];
    const uint64_t rho = __umul64hi(bcast_u, Q);
    const uint64_t Hu = (uint64_t)H;
    int32_t *anc = a.anc + (size_t)f * a.Hp;
    for (int jj = tid; jj < H; jj += kWeighBlock) {
        const uint64_t point = (uint64_t)jj * Q + rho;
        int lo = 0, hi = H - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (Hu * Cs[mid] > point) hi = mid;
            else lo = mid + 1;
        }
        anc[jj] = lo;
    }
}

// ---------------------------------------------------------------------------
// finish: per-theta sum over trajectories in trajectory order, status, aux.
// ---------------------------------------------------------------------------
__global__ void k_finish(EvalArgs a, double *loglik, int32_t *status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_theta) return;
    double s = 0.0;
    int32_t st = LIK_STATUS_OK;
    for (int m = 0; m < a.M; ++m) {
        const int f = i * a.M + m;
        if (st == LIK_STATUS_OK && a.fstatus[f] != LIK_STATUS_OK) st = a.fstatus[f];
        s = s + a.fll[f];
    }
    loglik[i] = st == LIK_STATUS_OK ? s : __builtin_nan("");
    if (status) status[i] = st;
}

__global__ void k_aux_filters(EvalArgs a, uint64_t *events, double *fll) {
    const int F = a.n_theta * a.M;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    if (events) events[f] = a.fevents[f];
    if (fll) fll[f] = a.fll[f];
}

__global__ void k_aux_state(EvalArgs a, int32_t *out) {
    const size_t per = (size_t)a.U * a.H;
    const size_t total = (size_t)a.n_theta * a.M * per;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (size_t)gridDim.x * blockDim.x) {
        const int f = (int)(k / per);
        const size_t rem = k - (size_t)f * per;
        const int u = (int)(rem / a.H), j = (int)(rem % a.H);
        const int steps = a.fsteps[f];
        const int32_t *src = (steps & 1) ? a.xb : a.xa;
        out[k] = steps == 0 ? a.x0[(size_t)(f % a.M) * a.U + u]
                            : src[((size_t)f * a.U + u) * a.Hp + j];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_init(const EvalArgs &a, hipStream_t s) {
    const int F = a.n_theta * a.M;
    hipLaunchKernelGGL(k_init, dim3((F + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_order(const EvalArgs &a, int t, hipStream_t s) {
    (void)t;
    hipLaunchKernelGGL(k_order, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

template <int UMAX, int RMAX, int W>
static hipError_t launch_prop_t(const EvalArgs &a, const void *net, int precision, int t,
                                hipStream_t s) {
    const NetArgs<RMAX, W> &n = *static_cast<const NetArgs<RMAX, W> *>(net);
    const dim3 grid((unsigned)(a.n_theta * a.M * a.nchunk));
    if (precision == LIK_FP32_MIXED)
        hipLaunchKernelGGL((k_propagate<UMAX, RMAX, W, LIK_FP32_MIXED>), grid, dim3(kPropBlock), 0,
                           s, a, n, t);
    else
        hipLaunchKernelGGL((k_propagate<UMAX, RMAX, W, LIK_FP64>), grid, dim3(kPropBlock), 0, s,
                           a, n, t);
    return hipGetLastError();
}

hipError_t launch_propagate(const EvalArgs &a, const void *net, int umax, int rmax,
                            int precision, int t, hipStream_t s) {
    if (umax == 4 && rmax == 8) return launch_prop_t<4, 8, 1>(a, net, precision, t, s);
    if (umax == 8 && rmax == 16) return launch_prop_t<8, 16, 1>(a, net, precision, t, s);
    if (umax == 32 && rmax == 64) return launch_prop_t<32, 64, 4>(a, net, precision, t, s);
    return hipErrorInvalidValue;
}

hipError_t launch_weigh(const EvalArgs &a, int t, hipStream_t s) {
    hipLaunchKernelGGL(k_weigh, dim3((unsigned)(a.n_theta * a.M)), dim3(kWeighBlock), 0, s, a,
                       t);
    return hipGetLastError();
}

hipError_t launch_finish(const EvalArgs &a, double *loglik, int32_t *status, const lik_aux *aux,
                         hipStream_t s) {
    if (a.n_theta > 0)
        hipLaunchKernelGGL(k_finish, dim3((a.n_theta + 255) / 256), dim3(256), 0, s, a, loglik,
                           status);
    const int F = a.n_theta * a.M;
    if (aux && F > 0) {
        if (aux->filter_events || aux->filter_loglik)
            hipLaunchKernelGGL(k_aux_filters, dim3((F + 255) / 256), dim3(256), 0, s, a,
                               aux->filter_events, aux->filter_loglik);
        if (aux->final_state)
            hipLaunchKernelGGL(k_aux_state, dim3(4096), dim3(256), 0, s, a, aux->final_state);
    }
    return hipGetLastError();
}

}  // namespace lik
