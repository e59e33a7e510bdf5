// ode.hpp -- the per-lane Dormand-Prince solver of the deterministic-model
// likelihood (Sec. "Chemical Reaction Networks": dX/dt = f(X, t, theta);
// Results: no particle filter, the ODE solution and the noise density of the
// observations around it).  Shared by the generic kernel (the model's flux
// terms read at run time) and by the model-specialised kernels compiled with
// hipRTC (the terms as code with constant indices, the lane's parameters in
// registers); both take the same operations in the same order.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "../../include/lik.h"
#include "devmath.hpp"

namespace lik {

struct OdeArgs {
    const lik_ode_term *terms;
    const int32_t *x0_param;
    int32_t U, V, n_terms, obs_kind, obs_species, obs_species2, sd_param;
    double sd_const;
    int32_t fret[5];
    const double *theta;
    int32_t n_theta, M;
    const int32_t *obs_offsets;
    const double *t_obs, *y, *t0, *x0;
    const int32_t *in_offsets;  // null: no input
    const double *t_in, *u_in;
    double rtol, atol;
    int32_t max_steps;
    double *tll;     // [F] per-trajectory log-likelihood
    int32_t *tst;    // [F] per-trajectory status
    int32_t *tsteps; // [F] step attempts
};

// The model interpreted at run time: terms from memory, every index
// wave-uniform, species picked by uniform selects, parameters read from the
// lane's theta in memory.
template <int UMAX>
struct OdeGeneric {
    static constexpr int U = UMAX;
    struct Params {
        const double *th;
        __device__ double operator[](int k) const { return th[k]; }
    };
    __device__ static Params load(const double *th) { return Params{th}; }
    __device__ static double obs(const OdeArgs &a, const Params &p, const double *x);
    __device__ static void rhs(const OdeArgs &a, const Params &p, double u, const double *x,
                               double *dx) {
#pragma unroll
        for (int s = 0; s < UMAX; ++s) dx[s] = 0.0;
        for (int k = 0; k < a.n_terms; ++k) {
            const lik_ode_term &T = a.terms[k];
            double v = T.rate_param >= 0 ? T.rate_scale * p[T.rate_param] : T.rate_scale;
            for (int f = 0; f < T.n_factors; ++f) {
                const int kind = T.kind[f];
                double phi;
                if (kind == LIK_ODE_INPUT) {
                    phi = u;
                } else {
                    const int sp = T.species[f];
                    double xs = 0.0;
#pragma unroll
                    for (int s = 0; s < UMAX; ++s) xs = (s == sp) ? x[s] : xs;
                    if (kind == LIK_ODE_SPECIES) {
                        phi = xs;
                    } else if (kind == LIK_ODE_SATURATING) {
                        phi = xs / (p[T.param[f]] + xs);
                    } else if (kind == LIK_ODE_HILL2) {
                        const double q = xs * xs;
                        phi = q / (p[T.param[f]] + q);
                    } else {
                        const double K = p[T.param[f]];
                        phi = K / (K + xs * xs);
                    }
                }
                v = v * phi;
            }
            const int from = T.from, to = T.to;
#pragma unroll
            for (int s = 0; s < UMAX; ++s) {
                if (s == from) dx[s] = dx[s] - v;
                if (s == to) dx[s] = dx[s] + v;
            }
        }
    }
};

// The observation mean: the observed species, or the FRET ratio
// lambda (E fAA x_a / ((x_b + (1 - E) x_a) fDD) + bg).
template <int UMAX, class Params>
__device__ __forceinline__ double ode_obs_mean(const OdeArgs &a, const Params &p,
                                               const double *x) {
    double xa = 0.0, xb = 0.0;
#pragma unroll
    for (int s = 0; s < UMAX; ++s) {
        xa = (s == a.obs_species) ? x[s] : xa;
        xb = (s == a.obs_species2) ? x[s] : xb;
    }
    if (a.obs_kind == LIK_ODE_OBS_SPECIES) return xa;
    const double lam = p[a.fret[0]], bg = p[a.fret[1]], E = p[a.fret[2]];
    const double fAA = p[a.fret[3]], fDD = p[a.fret[4]];
    const double num = (E * fAA) * xa;
    const double den = (xb + (1.0 - E) * xa) * fDD;
    return lam * (num / den + bg);
}

template <int UMAX>
__device__ double OdeGeneric<UMAX>::obs(const OdeArgs &a, const Params &p, const double *x) {
    return ode_obs_mean<UMAX>(a, p, x);
}

// min(5, max(0.2, 0.9 err^(-1/5))), the power through log and exp with
// non-positive exponents only
__device__ __forceinline__ double ode_step_factor(double err) {
    if (err == 0.0) return 5.0;
    double fac = err < 1.0 ? 0.9 / dexp_nonpos(0.2 * dlog(err))
                           : 0.9 * dexp_nonpos(-0.2 * dlog(err));
    fac = fac > 5.0 ? 5.0 : fac;
    return fac < 0.2 ? 0.2 : fac;
}

// One (theta, trajectory) pair per lane: f = i * M + m.
template <class Model>
__device__ __forceinline__ void ode_lane(const OdeArgs &a, int f) {
    constexpr int UMAX = Model::U;
    const int i = f / a.M, m = f - (f / a.M) * a.M;
    const int U = a.U;
    const double *th = a.theta + (size_t)i * a.V;
    // Dormand-Prince 5(4)
    constexpr double a21 = 1.0 / 5.0;
    constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
    constexpr double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
    constexpr double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0,
                     a53 = 64448.0 / 6561.0, a54 = -212.0 / 729.0;
    constexpr double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0,
                     a64 = 49.0 / 176.0, a65 = -5103.0 / 18656.0;
    constexpr double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0,
                     b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
    constexpr double e1 = 71.0 / 57600.0, e3 = -71.0 / 16695.0, e4 = 71.0 / 1920.0,
                     e5 = -17253.0 / 339200.0, e6 = 22.0 / 525.0, e7 = -1.0 / 40.0;

    bool bad = false;
    for (int v = 0; v < a.V; ++v)
        if (!(th[v] >= 0.0) || __builtin_isinf(th[v])) bad = true;
    const double sd = a.sd_param >= 0 ? th[a.sd_param] : a.sd_const;
    if (bad || !(sd > 0.0)) {
        a.tll[f] = __builtin_nan("");
        a.tst[f] = LIK_STATUS_BAD_THETA;
        a.tsteps[f] = 0;
        return;
    }
    const typename Model::Params p = Model::load(th);
    double x[UMAX], xn[UMAX], z[UMAX];
    double k1[UMAX], k2[UMAX], k3[UMAX], k4[UMAX], k5[UMAX], k6[UMAX], k7[UMAX];
#pragma unroll
    for (int s = 0; s < UMAX; ++s) {
        const int q = s < U ? a.x0_param[s] : -1;
        x[s] = s >= U ? 0.0 : q >= 0 ? th[q] : a.x0[(size_t)m * U + s];
    }
    const int o0 = a.obs_offsets[m], T = a.obs_offsets[m + 1] - o0;
    const int q0 = a.in_offsets ? a.in_offsets[m] : 0;
    const int nq = a.in_offsets ? a.in_offsets[m + 1] - q0 : 0;
    double t = a.t0[m];
    const double span = a.t_obs[o0 + T - 1] - t;
    double u = 0.0;
    int q = 0;
    while (q < nq && a.t_in[q0 + q] <= t) {
        u = a.u_in[q0 + q];
        ++q;
    }
    double h = 0.01 * (a.t_obs[o0] - t);
    Model::rhs(a, p, u, x, k1);
    int steps = 0, status = LIK_STATUS_OK;
    double ll = 0.0;
    const double per = dlog(sd) + 0.5 * dlog(2.0 * 3.141592653589793);
    for (int k = 0; k < T && status == LIK_STATUS_OK; ++k) {
        const double t_obs = a.t_obs[o0 + k];
        for (;;) {
            const bool brk = q < nq && a.t_in[q0 + q] < t_obs;
            const double stop = brk ? a.t_in[q0 + q] : t_obs;
            while (t < stop) {
                if (steps >= a.max_steps || h < 1e-12 * span) {
                    status = LIK_STATUS_STEP_LIMIT;
                    break;
                }
                const bool last = t + h >= stop;
                const double hs = last ? stop - t : h;
#pragma unroll
                for (int s = 0; s < UMAX; ++s) z[s] = x[s] + hs * (a21 * k1[s]);
                Model::rhs(a, p, u, z, k2);
#pragma unroll
                for (int s = 0; s < UMAX; ++s) z[s] = x[s] + hs * (a31 * k1[s] + a32 * k2[s]);
                Model::rhs(a, p, u, z, k3);
#pragma unroll
                for (int s = 0; s < UMAX; ++s)
                    z[s] = x[s] + hs * (a41 * k1[s] + a42 * k2[s] + a43 * k3[s]);
                Model::rhs(a, p, u, z, k4);
#pragma unroll
                for (int s = 0; s < UMAX; ++s)
                    z[s] = x[s] + hs * (a51 * k1[s] + a52 * k2[s] + a53 * k3[s] + a54 * k4[s]);
                Model::rhs(a, p, u, z, k5);
#pragma unroll
                for (int s = 0; s < UMAX; ++s)
                    z[s] = x[s] + hs * (a61 * k1[s] + a62 * k2[s] + a63 * k3[s] + a64 * k4[s] +
                                        a65 * k5[s]);
                Model::rhs(a, p, u, z, k6);
#pragma unroll
                for (int s = 0; s < UMAX; ++s)
                    xn[s] = x[s] + hs * (b1 * k1[s] + b3 * k3[s] + b4 * k4[s] + b5 * k5[s] +
                                         b6 * k6[s]);
                Model::rhs(a, p, u, xn, k7);
                double err = 0.0;
                bool nan_err = false;
#pragma unroll
                for (int s = 0; s < UMAX; ++s) {
                    if (s >= U) continue;
                    const double es = hs * (e1 * k1[s] + e3 * k3[s] + e4 * k4[s] + e5 * k5[s] +
                                            e6 * k6[s] + e7 * k7[s]);
                    const double ax = __builtin_fabs(x[s]), an = __builtin_fabs(xn[s]);
                    const double sc = a.atol + a.rtol * (ax > an ? ax : an);
                    const double r = __builtin_fabs(es) / sc;
                    if (__builtin_isnan(r)) nan_err = true;
                    else if (r > err) err = r;
                }
                steps = steps + 1;
                if (nan_err || __builtin_isinf(err)) {
                    status = LIK_STATUS_NONFINITE;
                    break;
                }
                const double fac = ode_step_factor(err);
                if (err <= 1.0) {
                    t = last ? stop : t + hs;
#pragma unroll
                    for (int s = 0; s < UMAX; ++s) {
                        x[s] = xn[s];
                        k1[s] = k7[s];
                    }
                }
                h = hs * fac;
            }
            if (status != LIK_STATUS_OK || !brk) break;
            u = a.u_in[q0 + q];  // the input switches: f changes, k1 is recomputed
            ++q;
            Model::rhs(a, p, u, x, k1);
        }
        if (status != LIK_STATUS_OK) break;
        bool fin = true;
#pragma unroll
        for (int s = 0; s < UMAX; ++s)
            if (s < U && !__builtin_isfinite(x[s])) fin = false;
        const double g = Model::obs(a, p, x);
        if (!fin || !__builtin_isfinite(g)) {
            status = LIK_STATUS_NONFINITE;
            break;
        }
        const double zz = (a.y[o0 + k] - g) / sd;
        double lp = -0.5 * (zz * zz);
        lp = lp - per;
        ll = ll + lp;
    }
    a.tll[f] = status == LIK_STATUS_OK ? ll : __builtin_nan("");
    a.tst[f] = status;
    a.tsteps[f] = steps;
}

}  // namespace lik
