/*
 * ode_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU implementation of the likelihood of a deterministic
 * model (Mikelson & Khammash, arXiv 1606.08281, Sec. "Chemical Reaction
 * Networks": the state follows dX/dt = f(X, t, theta); Results: for a
 * deterministic model the likelihood needs no particle filter, only the
 * solution of the ODE and the noise density of the observations around it;
 * Supplementary "Egf-Ras-Raf-Mek-Erk model": Michaelis-Menten and Hill rate
 * laws, a time-dependent input, and a normally perturbed FRET read-out).
 *
 * The paper names no ODE solver.  This file integrates with the
 * Dormand-Prince 5(4) embedded Runge-Kutta pair (Dormand & Prince, J. Comput.
 * Appl. Math. 6, 1980; the tableau in Hairer, Norsett & Wanner, "Solving
 * Ordinary Differential Equations I", Table II.5.2), advancing with the
 * fifth-order solution, under the step-size rule written out in the library
 * header, with the oracle's own log and exp.  Every floating-point operation
 * is one IEEE-754 binary64 operation in the order written (no contraction).
 * It shares no code with the GPU library.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

double orc_log(double x);
double orc_exp(double d);

#define ODE_OK 0
#define ODE_BAD_THETA 3
#define ODE_STEP_LIMIT 7
#define ODE_NONFINITE 8

#define F_SPECIES 0
#define F_SATURATING 1
#define F_HILL2 2
#define F_REPRESS2 3
#define F_INPUT 4

#define OBS_SPECIES 0
#define OBS_FRET 1

#define ODE_MAXU 32

typedef struct {
    int32_t from, to, rate_param, n_factors;
    double rate_scale;
    int32_t kind[3], species[3], param[3];
} orc_ode_term;

typedef struct {
    int32_t U, V, n_terms;
    const orc_ode_term *terms;
    const int32_t *x0_param;      /* [U] theta index or -1 */
    int32_t obs_kind, obs_species, obs_species2, sd_param;
    double sd_const;
    int32_t fret_param[5];        /* lambda, bg, E, fAA, fDD */
    int32_t n_theta;
    const double *theta;          /* [n_theta * V] */
    int32_t n_traj;
    const int32_t *obs_offsets;   /* [M+1] */
    const double *t_obs, *y, *t0, *x0;  /* x0 [M*U] */
    const int32_t *in_offsets;    /* [M+1] or NULL */
    const double *t_in, *u_in;
    double rtol, atol;
    int32_t max_steps;
} orc_ode_problem;

/* f(x): the sum of the fluxes, term by term in order (u: current input). */
static void rhs(const orc_ode_problem *P, const double *th, double u, const double *x, double *dx)
{
    for (int s = 0; s < P->U; ++s) dx[s] = 0.0;
    for (int k = 0; k < P->n_terms; ++k) {
        const orc_ode_term *T = &P->terms[k];
        double v = T->rate_param >= 0 ? T->rate_scale * th[T->rate_param] : T->rate_scale;
        for (int f = 0; f < T->n_factors; ++f) {
            double phi;
            if (T->kind[f] == F_INPUT) {
                phi = u;
            } else {
                double xs = x[T->species[f]];
                if (T->kind[f] == F_SPECIES) {
                    phi = xs;
                } else if (T->kind[f] == F_SATURATING) {
                    phi = xs / (th[T->param[f]] + xs);
                } else if (T->kind[f] == F_HILL2) {
                    double q = xs * xs;
                    phi = q / (th[T->param[f]] + q);
                } else {
                    double K = th[T->param[f]];
                    phi = K / (K + xs * xs);
                }
            }
            v = v * phi;
        }
        if (T->from >= 0) dx[T->from] = dx[T->from] - v;
        if (T->to >= 0) dx[T->to] = dx[T->to] + v;
    }
}

/* the observation mean g(x) */
static double obs_mean(const orc_ode_problem *P, const double *th, const double *x)
{
    if (P->obs_kind == OBS_SPECIES) return x[P->obs_species];
    double lam = th[P->fret_param[0]], bg = th[P->fret_param[1]], E = th[P->fret_param[2]];
    double fAA = th[P->fret_param[3]], fDD = th[P->fret_param[4]];
    double xa = x[P->obs_species], xb = x[P->obs_species2];
    double num = (E * fAA) * xa;
    double den = (xb + (1.0 - E) * xa) * fDD;
    return lam * (num / den + bg);
}

/* The step-size factor min(5, max(0.2, 0.9 err^(-1/5))), with err^(-1/5)
 * taken as 1 / exp(log(err) / 5) below 1 and exp(-log(err) / 5) from 1 on, so
 * that exp only sees non-positive arguments. */
static double step_factor(double err)
{
    double fac;
    if (err == 0.0) return 5.0;
    if (err < 1.0) fac = 0.9 / orc_exp(0.2 * orc_log(err));
    else fac = 0.9 * orc_exp(-0.2 * orc_log(err));
    if (fac > 5.0) fac = 5.0;
    if (fac < 0.2) fac = 0.2;
    return fac;
}

/* One trajectory: log-likelihood (and optionally the states at the
 * observation times and the number of step attempts). */
static int solve(const orc_ode_problem *P, int i, int m, double *ll_out, double *states_out,
                 int32_t *steps_out)
{
    const int U = P->U;
    const double *th = P->theta + (size_t)i * P->V;
    /* Dormand-Prince 5(4) tableau */
    const double c2 = 1.0 / 5.0, c3 = 3.0 / 10.0, c4 = 4.0 / 5.0, c5 = 8.0 / 9.0;
    const double a21 = 1.0 / 5.0;
    const double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
    const double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
    const double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0,
                 a54 = -212.0 / 729.0;
    const double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0,
                 a64 = 49.0 / 176.0, a65 = -5103.0 / 18656.0;
    const double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0,
                 b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
    const double e1 = 71.0 / 57600.0, e3 = -71.0 / 16695.0, e4 = 71.0 / 1920.0,
                 e5 = -17253.0 / 339200.0, e6 = 22.0 / 525.0, e7 = -1.0 / 40.0;
    (void)c2; (void)c3; (void)c4; (void)c5;   /* autonomous between stops: the input is constant */

    double x[ODE_MAXU], xn[ODE_MAXU], z[ODE_MAXU];
    double k1[ODE_MAXU], k2[ODE_MAXU], k3[ODE_MAXU], k4[ODE_MAXU], k5[ODE_MAXU], k6[ODE_MAXU],
        k7[ODE_MAXU];
    /* parameters are rates, constants, noise scales, initial values: all >= 0 */
    for (int v = 0; v < P->V; ++v)
        if (!(th[v] >= 0.0) || isinf(th[v])) {
            *ll_out = NAN;
            if (steps_out) *steps_out = 0;
            return ODE_BAD_THETA;
        }
    double sd = P->sd_param >= 0 ? th[P->sd_param] : P->sd_const;
    if (!(sd > 0.0)) {
        *ll_out = NAN;
        if (steps_out) *steps_out = 0;
        return ODE_BAD_THETA;
    }
    for (int s = 0; s < U; ++s)
        x[s] = P->x0_param[s] >= 0 ? th[P->x0_param[s]] : P->x0[(size_t)m * U + s];

    const int o0 = P->obs_offsets[m], T = P->obs_offsets[m + 1] - o0;
    const int q0 = P->in_offsets ? P->in_offsets[m] : 0;
    const int nq = P->in_offsets ? P->in_offsets[m + 1] - q0 : 0;
    double t = P->t0[m];
    const double span = P->t_obs[o0 + T - 1] - t;
    /* input in force at t0: the last breakpoint at or before it */
    double u = 0.0;
    int q = 0;
    while (q < nq && P->t_in[q0 + q] <= t) { u = P->u_in[q0 + q]; ++q; }
    double h = 0.01 * (P->t_obs[o0] - t);
    rhs(P, th, u, x, k1);
    int steps = 0, status = ODE_OK;
    double ll = 0.0;
    const double per = orc_log(sd) + 0.5 * orc_log(2.0 * 3.141592653589793);
    for (int k = 0; k < T && status == ODE_OK; ++k) {
        const double t_obs = P->t_obs[o0 + k];
        /* advance to each breakpoint before this observation, then to it */
        for (;;) {
            const int brk = q < nq && P->t_in[q0 + q] < t_obs;
            const double stop = brk ? P->t_in[q0 + q] : t_obs;
            while (t < stop) {
                if (steps >= P->max_steps || h < 1e-12 * span) { status = ODE_STEP_LIMIT; break; }
                const int last = t + h >= stop;
                const double hs = last ? stop - t : h;
                for (int s = 0; s < U; ++s) z[s] = x[s] + hs * (a21 * k1[s]);
                rhs(P, th, u, z, k2);
                for (int s = 0; s < U; ++s) z[s] = x[s] + hs * (a31 * k1[s] + a32 * k2[s]);
                rhs(P, th, u, z, k3);
                for (int s = 0; s < U; ++s)
                    z[s] = x[s] + hs * (a41 * k1[s] + a42 * k2[s] + a43 * k3[s]);
                rhs(P, th, u, z, k4);
                for (int s = 0; s < U; ++s)
                    z[s] = x[s] + hs * (a51 * k1[s] + a52 * k2[s] + a53 * k3[s] + a54 * k4[s]);
                rhs(P, th, u, z, k5);
                for (int s = 0; s < U; ++s)
                    z[s] = x[s] + hs * (a61 * k1[s] + a62 * k2[s] + a63 * k3[s] + a64 * k4[s] +
                                        a65 * k5[s]);
                rhs(P, th, u, z, k6);
                for (int s = 0; s < U; ++s)
                    xn[s] = x[s] + hs * (b1 * k1[s] + b3 * k3[s] + b4 * k4[s] + b5 * k5[s] +
                                         b6 * k6[s]);
                rhs(P, th, u, xn, k7);
                double err = 0.0;
                int bad = 0;
                for (int s = 0; s < U; ++s) {
                    double es = hs * (e1 * k1[s] + e3 * k3[s] + e4 * k4[s] + e5 * k5[s] +
                                      e6 * k6[s] + e7 * k7[s]);
                    double ax = fabs(x[s]), an = fabs(xn[s]);
                    double sc = P->atol + P->rtol * (ax > an ? ax : an);
                    double r = fabs(es) / sc;
                    if (isnan(r)) bad = 1;
                    else if (r > err) err = r;
                }
                steps = steps + 1;
                if (bad || isinf(err)) { status = ODE_NONFINITE; break; }
                const double fac = step_factor(err);
                if (err <= 1.0) {
                    t = last ? stop : t + hs;
                    for (int s = 0; s < U; ++s) { x[s] = xn[s]; k1[s] = k7[s]; }
                }
                h = hs * fac;
            }
            if (status != ODE_OK) break;
            if (!brk) break;
            /* the input switches at the breakpoint: f changes, so k1 is recomputed */
            u = P->u_in[q0 + q];
            ++q;
            rhs(P, th, u, x, k1);
        }
        if (status != ODE_OK) break;
        for (int s = 0; s < U; ++s)
            if (!isfinite(x[s])) status = ODE_NONFINITE;
        double g = obs_mean(P, th, x);
        if (!isfinite(g)) status = ODE_NONFINITE;
        if (status != ODE_OK) break;
        if (states_out) memcpy(states_out + (size_t)k * U, x, sizeof(double) * (size_t)U);
        double zz = (P->y[o0 + k] - g) / sd;
        double lp = -0.5 * (zz * zz);
        lp = lp - per;
        ll = ll + lp;
    }
    if (steps_out) *steps_out = steps;
    *ll_out = status == ODE_OK ? ll : NAN;
    return status;
}

typedef struct {
    const orc_ode_problem *P;
    int next, F;
    pthread_mutex_t lock;
    double *tll;
    int32_t *tst, *tsteps;
} ode_batch;

static void *ode_worker(void *arg)
{
    ode_batch *b = (ode_batch *)arg;
    for (;;) {
        pthread_mutex_lock(&b->lock);
        int f = b->next++;
        pthread_mutex_unlock(&b->lock);
        if (f >= b->F) return NULL;
        int i = f / b->P->n_traj, m = f % b->P->n_traj;
        b->tst[f] = solve(b->P, i, m, &b->tll[f], NULL, &b->tsteps[f]);
    }
}

/* Per theta: the sum over trajectories in order; status the first non-OK. */
int orc_ode_eval(const orc_ode_problem *P, int nthreads, double *loglik, int32_t *status,
                 double *traj_ll, int32_t *traj_status, int32_t *traj_steps)
{
    if (P->U < 1 || P->U > ODE_MAXU) return -1;
    const int F = P->n_theta * P->n_traj;
    ode_batch b;
    b.P = P;
    b.next = 0;
    b.F = F;
    pthread_mutex_init(&b.lock, NULL);
    b.tll = (double *)malloc(sizeof(double) * (size_t)(F > 0 ? F : 1));
    b.tst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F > 0 ? F : 1));
    b.tsteps = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F > 0 ? F : 1));
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    for (int k = 1; k < nthreads; ++k) pthread_create(&th[k], NULL, ode_worker, &b);
    ode_worker(&b);
    for (int k = 1; k < nthreads; ++k) pthread_join(th[k], NULL);
    for (int i = 0; i < P->n_theta; ++i) {
        double s = 0.0;
        int st = ODE_OK;
        for (int m = 0; m < P->n_traj; ++m) {
            int f = i * P->n_traj + m;
            if (st == ODE_OK && b.tst[f] != ODE_OK) st = b.tst[f];
            s = s + b.tll[f];
        }
        loglik[i] = st == ODE_OK ? s : NAN;
        if (status) status[i] = st;
    }
    if (traj_ll) memcpy(traj_ll, b.tll, sizeof(double) * (size_t)F);
    if (traj_status) memcpy(traj_status, b.tst, sizeof(int32_t) * (size_t)F);
    if (traj_steps) memcpy(traj_steps, b.tsteps, sizeof(int32_t) * (size_t)F);
    free(b.tll);
    free(b.tst);
    free(b.tsteps);
    pthread_mutex_destroy(&b.lock);
    return 0;
}

/* One trajectory's states at its observation times [T][U] and step count. */
int orc_ode_solve(const orc_ode_problem *P, int i, int m, double *states_out, int32_t *steps_out,
                  double *ll_out)
{
    return solve(P, i, m, ll_out, states_out, steps_out);
}
