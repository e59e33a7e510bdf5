// ode.hpp -- the per-lane Dormand-Prince solver of the deterministic-model
// likelihood (Sec. "Chemical Reaction Networks": dX/dt = f(X, t, theta);
// Results: no particle filter, the ODE solution and the noise density of the
// observations around it).  Shared by the generic kernel (the model's flux
// terms read at run time) and by the model-specialised kernels compiled with
// hipRTC (the terms as code with constant indices, the lane's parameters
// read from LDS); both take the same operations in the same order.
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
    unsigned int *next;  // the next pair to take (zero at launch)
    const int32_t *m_order;  // [M] trajectories in the order their pairs are taken
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
    __device__ static Params load(const OdeArgs &a, int i) {
        return Params{a.theta + (size_t)i * a.V};
    }
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

// v, opaque to the compiler (an empty asm with side effects): what is
// computed from it stays after this point of the program.
__device__ __forceinline__ double ode_pin(double v) {
    asm volatile("" : "+s"(v));
    return v;
}

// The step factor's logarithm (x > 0) and exponential (d <= 0): the same
// operations, in the same order, as dlog_pos and dexp_nonpos of devmath.hpp,
// with each constant pinned where it is used; otherwise the compiler holds
// the series' coefficients in vector registers across the whole step loop.
__device__ __forceinline__ double ode_log_pos(double x) {
    const double mant = __builtin_amdgcn_frexp_mant(x);
    int e = __builtin_amdgcn_frexp_exp(x);
    double m;
    if (mant > ode_pin(kHalfSqrt2)) {
        m = mant;
    } else {
        m = mant * 2.0;
        e = e - 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double q = ode_pin(1.0 / 21.0);
    q = __builtin_fma(q, z, ode_pin(1.0 / 19.0));
    q = __builtin_fma(q, z, ode_pin(1.0 / 17.0));
    q = __builtin_fma(q, z, ode_pin(1.0 / 15.0));
    q = __builtin_fma(q, z, ode_pin(1.0 / 13.0));
    q = __builtin_fma(q, z, ode_pin(1.0 / 11.0));
    q = __builtin_fma(q, z, ode_pin(1.0 / 9.0));
    q = __builtin_fma(q, z, ode_pin(1.0 / 7.0));
    q = __builtin_fma(q, z, ode_pin(1.0 / 5.0));
    q = __builtin_fma(q, z, ode_pin(1.0 / 3.0));
    const double t = 2.0 * s;
    const double w = t * z;
    const double lm = __builtin_fma(w, q, t);
    const double ed = (double)e;
    return ed * ode_pin(kLn2Hi) + (ed * ode_pin(kLn2Lo) + lm);
}

__device__ __forceinline__ double ode_exp_nonpos(double d) {
    if (!(d >= -708.0)) return 0.0;
    const double kd = __builtin_floor(d * ode_pin(kInvLn2) + 0.5);
    const double r = (d - kd * ode_pin(kLn2Hi)) - kd * ode_pin(kLn2Lo);
    double p = ode_pin(1.0 / 6227020800.0);
    p = __builtin_fma(p, r, ode_pin(1.0 / 479001600.0));
    p = __builtin_fma(p, r, ode_pin(1.0 / 39916800.0));
    p = __builtin_fma(p, r, ode_pin(1.0 / 3628800.0));
    p = __builtin_fma(p, r, ode_pin(1.0 / 362880.0));
    p = __builtin_fma(p, r, ode_pin(1.0 / 40320.0));
    p = __builtin_fma(p, r, ode_pin(1.0 / 5040.0));
    p = __builtin_fma(p, r, ode_pin(1.0 / 720.0));
    p = __builtin_fma(p, r, ode_pin(1.0 / 120.0));
    p = __builtin_fma(p, r, ode_pin(1.0 / 24.0));
    p = __builtin_fma(p, r, ode_pin(1.0 / 6.0));
    p = __builtin_fma(p, r, 1.0 / 2.0);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, (int)kd);
}

// min(5, max(0.2, 0.9 err^(-1/5))), the power through log and exp with
// non-positive exponents only (err > 0 finite here)
__device__ __forceinline__ double ode_step_factor(double err) {
    if (err == 0.0) return 5.0;
    double fac = err < 1.0 ? 0.9 / ode_exp_nonpos(0.2 * ode_log_pos(err))
                           : 0.9 * ode_exp_nonpos(-0.2 * ode_log_pos(err));
    fac = fac > 5.0 ? 5.0 : fac;
    return fac < 0.2 ? 0.2 : fac;
}

// Every lane of the launch runs this loop: it takes (theta, trajectory) pairs
// f = i * M + m from the shared counter a.next until none is left, and solves
// one at a time; the counter runs over trajectories in the order m_order
// (all theta of one trajectory, then the next).  The loop is flat, one step attempt per pass: a lane that
// reaches an input breakpoint or an observation handles it at the top of its
// next pass, and a lane whose trajectory ends writes its results and starts
// the next pair there, so the lanes of a wavefront keep stepping side by side
// however different their step counts.  Per pair the operations and their
// order are those of a loop over observations, breakpoints and steps.
template <class Model>
__device__ __forceinline__ void ode_run(const OdeArgs &a) {
    constexpr int UMAX = Model::U;
    const int U = a.U, F = a.n_theta * a.M;
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
    const double half_log_2pi = 0.5 * ode_log_pos(2.0 * 3.141592653589793);

    typename Model::Params p{};
    double x[UMAX], xn[UMAX], z[UMAX];
    double k1[UMAX], k2[UMAX], k3[UMAX], k4[UMAX], k5[UMAX], k6[UMAX], k7[UMAX];
    double t = 0.0, h = 0.0, span = 0.0, u = 0.0, sd = 1.0, per = 0.0, ll = 0.0, stop = 0.0;
    int m = 0, o0 = 0, T = 0, q0 = 0, nq = 0, q = 0, k = 0, steps = 0;
    int status = LIK_STATUS_OK;
    bool live = false;  // a pair in progress
    int idx = (int)atomicAdd(a.next, 1u), f = 0;
    for (;;) {
        if (!live) {
            // the next pair; one with bad parameters is finished at once
            if (idx >= F) break;
            const int r = idx / a.n_theta, i = idx - r * a.n_theta;
            m = a.m_order[r];
            f = i * a.M + m;
            const double *th = a.theta + (size_t)i * a.V;
            bool bad = false;
            for (int v = 0; v < a.V; ++v)
                if (!(th[v] >= 0.0) || __builtin_isinf(th[v])) bad = true;
            sd = a.sd_param >= 0 ? th[a.sd_param] : a.sd_const;
            if (bad || !(sd > 0.0)) {
                a.tll[f] = __builtin_nan("");
                a.tst[f] = LIK_STATUS_BAD_THETA;
                a.tsteps[f] = 0;
                idx = (int)atomicAdd(a.next, 1u);
                continue;
            }
            p = Model::load(a, i);
#pragma unroll
            for (int s = 0; s < UMAX; ++s) {
                const int qs = s < U ? a.x0_param[s] : -1;
                x[s] = s >= U ? 0.0 : qs >= 0 ? th[qs] : a.x0[(size_t)m * U + s];
            }
            o0 = a.obs_offsets[m];
            T = a.obs_offsets[m + 1] - o0;
            q0 = a.in_offsets ? a.in_offsets[m] : 0;
            nq = a.in_offsets ? a.in_offsets[m + 1] - q0 : 0;
            t = a.t0[m];
            span = a.t_obs[o0 + T - 1] - t;
            u = 0.0;
            q = 0;
            while (q < nq && a.t_in[q0 + q] <= t) {
                u = a.u_in[q0 + q];
                ++q;
            }
            h = 0.01 * (a.t_obs[o0] - t);
            Model::rhs(a, p, u, x, k1);
            steps = 0;
            status = LIK_STATUS_OK;
            ll = 0.0;
            per = ode_log_pos(sd) + half_log_2pi;
            k = 0;
            stop = t;  // the first pass looks for the first stop
            live = true;
        }
        // at a stop: input switches and observations at the lane's time
        while (status == LIK_STATUS_OK && !(t < stop) && k < T) {
            const double t_obs = a.t_obs[o0 + k];
            const bool brk = q < nq && a.t_in[q0 + q] < t_obs;
            stop = brk ? a.t_in[q0 + q] : t_obs;
            if (t < stop) break;
            if (brk) {
                u = a.u_in[q0 + q];  // the input switches: f changes, k1 is recomputed
                ++q;
                Model::rhs(a, p, u, x, k1);
                continue;
            }
            // the observation at t = t_obs
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
            ++k;
        }
        if (status != LIK_STATUS_OK || k == T) {
            a.tll[f] = status == LIK_STATUS_OK ? ll : __builtin_nan("");
            a.tst[f] = status;
            a.tsteps[f] = steps;
            live = false;
            idx = (int)atomicAdd(a.next, 1u);
            continue;
        }
        // one step attempt toward stop
        if (steps >= a.max_steps || h < 1e-12 * span) {
            status = LIK_STATUS_STEP_LIMIT;
            continue;
        }
        const bool last = t + h >= stop;
        const double hs = last ? stop - t : h;
        // Each stage takes its coefficients through ode_pin, so that
        // none of its products is computed before the stage begins:
        // left free, the compiler forms the products with k1 of every
        // later stage up front and keeps them all live at once.
        {
            const double c1 = ode_pin(a21);
#pragma unroll
            for (int s = 0; s < UMAX; ++s) z[s] = x[s] + hs * (c1 * k1[s]);
        }
        Model::rhs(a, p, u, z, k2);
        {
            const double c1 = ode_pin(a31), c2 = ode_pin(a32);
#pragma unroll
            for (int s = 0; s < UMAX; ++s) z[s] = x[s] + hs * (c1 * k1[s] + c2 * k2[s]);
        }
        Model::rhs(a, p, u, z, k3);
        {
            const double c1 = ode_pin(a41), c2 = ode_pin(a42), c3 = ode_pin(a43);
#pragma unroll
            for (int s = 0; s < UMAX; ++s)
                z[s] = x[s] + hs * (c1 * k1[s] + c2 * k2[s] + c3 * k3[s]);
        }
        Model::rhs(a, p, u, z, k4);
        {
            const double c1 = ode_pin(a51), c2 = ode_pin(a52), c3 = ode_pin(a53);
            const double c4 = ode_pin(a54);
#pragma unroll
            for (int s = 0; s < UMAX; ++s)
                z[s] = x[s] + hs * (c1 * k1[s] + c2 * k2[s] + c3 * k3[s] + c4 * k4[s]);
        }
        Model::rhs(a, p, u, z, k5);
        {
            const double c1 = ode_pin(a61), c2 = ode_pin(a62), c3 = ode_pin(a63);
            const double c4 = ode_pin(a64), c5 = ode_pin(a65);
#pragma unroll
            for (int s = 0; s < UMAX; ++s)
                z[s] = x[s] + hs * (c1 * k1[s] + c2 * k2[s] + c3 * k3[s] + c4 * k4[s] +
                                    c5 * k5[s]);
        }
        Model::rhs(a, p, u, z, k6);
        // the solution and the error sum's first five terms (left to
        // right, as written out in full); k3..k6 are dead before the
        // last right-hand side
        {
            const double c1 = ode_pin(b1), c3 = ode_pin(b3), c4 = ode_pin(b4);
            const double c5 = ode_pin(b5), c6 = ode_pin(b6);
            const double d1 = ode_pin(e1), d3 = ode_pin(e3), d4 = ode_pin(e4);
            const double d5 = ode_pin(e5), d6 = ode_pin(e6);
#pragma unroll
            for (int s = 0; s < UMAX; ++s) {
                xn[s] = x[s] + hs * (c1 * k1[s] + c3 * k3[s] + c4 * k4[s] + c5 * k5[s] +
                                     c6 * k6[s]);
                z[s] = d1 * k1[s] + d3 * k3[s] + d4 * k4[s] + d5 * k5[s] + d6 * k6[s];
            }
        }
        Model::rhs(a, p, u, xn, k7);
        double err = 0.0;
        bool nan_err = false;
        const double d7 = ode_pin(e7);
#pragma unroll
        for (int s = 0; s < UMAX; ++s) {
            // (species beyond U: x = 0 and k = 0, so r = 0)
            const double es = hs * (z[s] + d7 * k7[s]);
            const double ax = __builtin_fabs(x[s]), an = __builtin_fabs(xn[s]);
            const double sc = a.atol + a.rtol * (ax > an ? ax : an);
            const double r = __builtin_fabs(es) / sc;
            // selects, not branches: a branch per species would split
            // the step into blocks the compiler fills with re-computed
            // stage values, keeping every stage's parameters live
            nan_err = nan_err | __builtin_isnan(r);
            err = r > err ? r : err;
        }
        steps = steps + 1;
        if (nan_err || __builtin_isinf(err)) {
            status = LIK_STATUS_NONFINITE;
            continue;
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
}

}  // namespace lik
