/*
 * pf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential-per-filter CPU implementation of the bootstrap
 * particle-filter log-likelihood of Mikelson & Khammash, "A parallelizable
 * sampling method for parameter inference of large biochemical reaction
 * models" (arXiv 1606.08281):
 *
 *   - the network model of Sec. "Chemical Reaction Networks" (species X_u,
 *     reactions with consumed counts p_ru and produced counts q_ru, propensities
 *     depending on theta; mass-action kinetics as stated for the Lac-Gfp example
 *     in the Supplementary "Examples used"),
 *   - the observation model Y ~ p(. | X, theta) of Sec. "General Task", with
 *     the Gaussian and log-normal noise used by the workloads and the
 *     fluorescence model of the Supplementary "LacGfp example" (each molecule
 *     contributes an independent normal signal, plus a background),
 *   - a random initial state: the filter starts from H draws of the initial
 *     distribution (Supplementary I), here independent uniform integers per
 *     species as in the Lac-Gfp initial-distribution table,
 *   - the likelihood factorisation over trajectories and time points and the
 *     recursive estimate of Supplementary I ("Computing the Likelihood"),
 *   - the particle filter of Supplementary I, Algorithm "Likelihood
 *     Approximation using particle filter": resample, simulate, weight,
 *     accumulate the running mean of the weights,
 *   - forward simulation by Gillespie's stochastic simulation algorithm (the
 *     paper cites Gillespie 1977 for the SSA; the direct method is used).
 *
 * The paper leaves the random-number streams, the resampling scheme and the
 * floating-point details open.  This file follows the numerical contract
 * written out in the repository's design notes (Philox4x32-10 streams keyed by
 * (event, particle slot, interval, trajectory, theta id), the log/exp
 * evaluation schemes below, fixed-point systematic resampling).  It shares no
 * code with the GPU library; only tests, the smoke check and the CPU baseline
 * of the benchmark may load it.
 *
 * Build: gcc -O2 -mfma -ffp-contract=off -fPIC -shared -pthread (no fast-math:
 * every floating-point operation below is one IEEE-754 binary64/binary32
 * operation, rounded to nearest; fma() is the correctly rounded fused
 * multiply-add).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EVENT_CAP 1
#define ORC_COUNT_OVERFLOW 2
#define ORC_BAD_THETA 3

#define ORC_FP64 0
#define ORC_FP32_MIXED 1

#define ORC_OBS_GAUSSIAN 0
#define ORC_OBS_LOGNORMAL 1
#define ORC_OBS_FLUORESCENCE 2

/* Counts above this at the end of an interval flag COUNT_OVERFLOW. */
#define ORC_COUNT_LIMIT (1 << 30)

typedef struct orc_problem {
    int32_t n_species;            /* U */
    int32_t n_reactions;          /* R */
    const int32_t *reactant_orders; /* [R*U] p_ru */
    const int32_t *stoich;        /* [R*U] net change q_ru - p_ru */
    int32_t obs_kind;             /* ORC_OBS_* */
    int32_t n_observed;           /* P */
    const int32_t *observed;      /* [P] species observed, in order */
    double sigma;
    int32_t n_theta;
    const double *theta;          /* [n_theta*R] rate constants c_r */
    const uint32_t *theta_ids;    /* [n_theta] stream ids, or NULL for 0..n-1 */
    int32_t n_traj;               /* M */
    const int32_t *obs_offsets;   /* [M+1] */
    const double *t_obs;          /* [total] strictly increasing per trajectory */
    const double *y;              /* [total*P] */
    const double *t0;             /* [M] */
    const int32_t *x0;            /* [M*U] */
    int32_t n_particles;          /* H */
    uint64_t seed;
    int32_t precision;            /* ORC_FP64 | ORC_FP32_MIXED */
    uint64_t event_cap;           /* max events per particle per interval */
    /* fluorescence model: y ~ N(gain x + bg_mean, sigma^2 x + bg_sd^2) */
    double gain, bg_mean, bg_sd;
    /* [M*U] or NULL: initial counts uniform on the integers x0 .. x0_hi */
    const int32_t *x0_hi;
} orc_problem;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies, the     */
/* Weyl key schedule between rounds.                                          */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                         uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Logarithm and exponential.  Both sides of the comparison evaluate these   */
/* with the same sequence of correctly rounded operations, so the decisions  */
/* they feed (event times, resampling weights) are reproducible bit for bit. */
/*                                                                            */
/* log: reduce x = 2^e m with m in [sqrt(1/2), sqrt(2)], put s = f/(2+f) for  */
/* f = m-1, so that log m = 2 atanh s = 2s (1 + s^2/3 + s^4/5 + ...); the     */
/* series is truncated after s^20/21 (|s| <= 0.1716).  Then                   */
/* log x = e ln2_hi + (e ln2_lo + log m) with ln2_hi = ln 2 cut to 32         */
/* significant bits, ln2_lo the double nearest ln 2 - ln2_hi.                 */
/* exp (arguments d <= 0 only): k = floor(d/ln2 + 1/2), r = d - k ln2 (two    */
/* pieces), exp r by its Taylor series to r^13/13!, times 2^k; d < -708 -> 0. */
/* ------------------------------------------------------------------------ */
static const double LN2_HI = 0x1.62e42feep-1;          /* 32 significant bits */
static const double LN2_LO = 0x1.a39ef35793c76p-33;    /* ln 2 - LN2_HI */
static const double INV_LN2 = 0x1.71547652b82fep+0;    /* nearest to 1/ln 2 */
static const double SQRT2 = 0x1.6a09e667f3bcdp+0;      /* nearest to sqrt 2 */

static double bits_to_double(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }
static uint64_t double_to_bits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }
static float bits_to_float(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static uint32_t float_to_bits(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

double orc_log(double x)
{
    if (x == 0.0) return -INFINITY;
    if (!(x > 0.0)) return NAN;
    if (isinf(x)) return x;
    int e = 0;
    uint64_t b = double_to_bits(x);
    if ((b >> 52) == 0) {              /* subnormal: scale into the normal range */
        x = x * 0x1p54;
        e = -54;
        b = double_to_bits(x);
    }
    e += (int)(b >> 52) - 1023;
    double m = bits_to_double((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > SQRT2) {
        m = m * 0.5;
        e = e + 1;
    }
    double f = m - 1.0;
    double s = f / (2.0 + f);
    double z = s * s;
    /* Q(z) = 1/3 + z/5 + ... + z^9/21, Horner from the highest power. */
    double q = 1.0 / 21.0;
    q = fma(q, z, 1.0 / 19.0);
    q = fma(q, z, 1.0 / 17.0);
    q = fma(q, z, 1.0 / 15.0);
    q = fma(q, z, 1.0 / 13.0);
    q = fma(q, z, 1.0 / 11.0);
    q = fma(q, z, 1.0 / 9.0);
    q = fma(q, z, 1.0 / 7.0);
    q = fma(q, z, 1.0 / 5.0);
    q = fma(q, z, 1.0 / 3.0);
    double t = 2.0 * s;
    double w = t * z;
    double lm = fma(w, q, t);
    double ed = (double)e;
    return ed * LN2_HI + (ed * LN2_LO + lm);
}

double orc_exp(double d)
{
    if (!(d >= -708.0)) return 0.0;
    double kd = floor(d * INV_LN2 + 0.5);
    double r = (d - kd * LN2_HI) - kd * LN2_LO;
    /* 1/i! for i = 13 .. 0; every i! here is exact in binary64. */
    double p = 1.0 / 6227020800.0;
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 1.0 / 2.0);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    int k = (int)kd;
    return p * bits_to_double((uint64_t)(k + 1023) << 52);
}

/* binary32 logarithm for the FP32-mixed event times: same reduction, series
 * truncated after s^10/11; ln2 split as 16 significant bits + remainder. */
static const float LN2F_HI = 0x1.62e4p-1f;
static const float LN2F_LO = 0x1.7f7d1cp-20f;
static const float SQRT2F = 0x1.6a09e6p+0f;

float orc_logf(float x)
{
    if (x == 0.0f) return -INFINITY;
    if (!(x > 0.0f)) return NAN;
    if (isinf(x)) return x;
    int e = 0;
    uint32_t b = float_to_bits(x);
    if ((b >> 23) == 0) {
        x = x * 0x1p24f;
        e = -24;
        b = float_to_bits(x);
    }
    e += (int)(b >> 23) - 127;
    float m = bits_to_float((b & 0x007FFFFFu) | 0x3F800000u);
    if (m > SQRT2F) {
        m = m * 0.5f;
        e = e + 1;
    }
    float f = m - 1.0f;
    float s = f / (2.0f + f);
    float z = s * s;
    float q = 1.0f / 11.0f;
    q = fmaf(q, z, 1.0f / 9.0f);
    q = fmaf(q, z, 1.0f / 7.0f);
    q = fmaf(q, z, 1.0f / 5.0f);
    q = fmaf(q, z, 1.0f / 3.0f);
    float t = 2.0f * s;
    float w = t * z;
    float lm = fmaf(w, q, t);
    float ef = (float)e;
    return ef * LN2F_HI + (ef * LN2F_LO + lm);
}

/* ------------------------------------------------------------------------ */
/* Network model.                                                             */
/* ------------------------------------------------------------------------ */

/* Gillespie's combinatorial mass-action factor h_r(x) = prod_u C(x_u, p_ru),
 * returned as a binary64 value (exact for the count ranges allowed). */
static double mass_action_factor(const orc_problem *P, int r, const int32_t *x)
{
    int U = P->n_species;
    const int32_t *p = P->reactant_orders + (size_t)r * U;
    int first = -1, second = -1;
    for (int u = 0; u < U; ++u) {
        if (p[u] == 2) return 0.5 * ((double)x[u] * (double)(x[u] - 1));
        if (p[u] == 1) {
            if (first < 0) first = u;
            else second = u;
        }
    }
    if (first < 0) return 1.0;
    if (second < 0) return (double)x[first];
    return (double)x[first] * (double)x[second];
}

/* a_r = c_r h_r(x) for every r (binary64), as the propensity of reaction r. */
void orc_propensities(const orc_problem *P, const double *c, const int32_t *x,
                      int precision, double *a_out)
{
    for (int r = 0; r < P->n_reactions; ++r) {
        double h = mass_action_factor(P, r, x);
        if (precision == ORC_FP32_MIXED)
            a_out[r] = (double)((float)c[r] * (float)h);
        else
            a_out[r] = c[r] * h;
    }
}

/* ------------------------------------------------------------------------ */
/* Gillespie direct method for one particle over one observation interval.   */
/* Runs from time t_start to t_end; returns the number of events applied and */
/* writes the particle status (OK or EVENT_CAP).                              */
/* ------------------------------------------------------------------------ */
static uint64_t ssa_interval(const orc_problem *P, const double *c, int32_t *x,
                             double t_start, double t_end, uint32_t slot,
                             uint32_t c2, uint32_t theta_id, int *status, double *clock_out)
{
    int U = P->n_species, R = P->n_reactions;
    double a[256], S[256];
    double clock = t_start;
    uint64_t n = 0;
    *status = ORC_OK;
    for (;;) {
        /* propensities and their running sums S_r = a_0 + ... + a_r */
        orc_propensities(P, c, x, P->precision, a);
        double total;
        int r_sel = -1;
        uint32_t w[4];
        if (P->precision == ORC_FP32_MIXED) {
            float sf = 0.0f;
            for (int r = 0; r < R; ++r) {
                sf = sf + (float)a[r];
                S[r] = (double)sf;
            }
            total = (double)sf;
            if (!(sf > 0.0f)) break;
            if (n >= P->event_cap) { *status = ORC_EVENT_CAP; break; }
            /* half a block per event: events 2p and 2p + 1 share block p,
             * the first taking words 0 and 1, the second words 2 and 3,
             * each word's leading 24 bits */
            philox_block(P->seed, (uint32_t)(n >> 1), slot, c2, theta_id << 2, w);
            const int h = (int)(n & 1u) * 2;
            float u1 = (float)((w[h] >> 8) + 1u) * 0x1p-24f;     /* (0, 1] */
            float u2 = (float)(w[h + 1] >> 8) * 0x1p-24f;        /* [0, 1) */
            float tau = -orc_logf(u1) / sf;
            if (clock + (double)tau > t_end) break;
            float target = u2 * sf;
            for (int r = 0; r < R; ++r)
                if ((float)S[r] > target) { r_sel = r; break; }
            if (r_sel < 0)
                for (int r = R - 1; r >= 0; --r)
                    if ((float)a[r] > 0.0f) { r_sel = r; break; }
            for (int u = 0; u < U; ++u) x[u] += P->stoich[(size_t)r_sel * U + u];
            clock = clock + (double)tau;
        } else {
            double s = 0.0;
            for (int r = 0; r < R; ++r) {
                s = s + a[r];
                S[r] = s;
            }
            total = s;
            if (!(total > 0.0)) break;
            if (n >= P->event_cap) { *status = ORC_EVENT_CAP; break; }
            philox_block(P->seed, (uint32_t)n, slot, c2, theta_id << 2, w);
            uint64_t z1 = ((((uint64_t)w[1]) << 32) | w[0]) >> 11;
            uint64_t z2 = ((((uint64_t)w[3]) << 32) | w[2]) >> 11;
            double u1 = (double)(z1 + 1) * 0x1p-53;   /* (0, 1] */
            double u2 = (double)z2 * 0x1p-53;         /* [0, 1) */
            double tau = -orc_log(u1) / total;
            if (clock + tau > t_end) break;           /* pending event discarded */
            double target = u2 * total;
            for (int r = 0; r < R; ++r)
                if (S[r] > target) { r_sel = r; break; }
            if (r_sel < 0)
                for (int r = R - 1; r >= 0; --r)
                    if (a[r] > 0.0) { r_sel = r; break; }
            for (int u = 0; u < U; ++u) x[u] += P->stoich[(size_t)r_sel * U + u];
            clock = clock + tau;
        }
        n = n + 1;
    }
    if (clock_out) *clock_out = clock;   /* time of the last event, t_start if none */
    return n;
}

/* Particle-dependent part of log p(y_t | x): for each observed species in
 * order, -0.5 z^2 with z the standardised residual (Gaussian) or the
 * standardised log residual (log-normal; a zero count has density 0). */
static double obs_logweight(const orc_problem *P, const int32_t *x, const double *yt)
{
    double lw = 0.0;
    for (int k = 0; k < P->n_observed; ++k) {
        int32_t cnt = x[P->observed[k]];
        double z;
        if (P->obs_kind == ORC_OBS_FLUORESCENCE) {
            /* the sum of cnt independent N(gain, sigma^2) signals plus a
             * N(bg_mean, bg_sd^2) background: normal, with mean and variance
             * linear in the count; its variance term depends on the
             * particle, so log v stays in the weight */
            double xc = (double)cnt;
            double mean = P->gain * xc + P->bg_mean;
            double var = (P->sigma * P->sigma) * xc + P->bg_sd * P->bg_sd;
            double r = yt[k] - mean;
            lw = lw - 0.5 * ((r * r) / var);
            lw = lw - 0.5 * orc_log(var);
            continue;
        }
        if (P->obs_kind == ORC_OBS_LOGNORMAL) {
            if (cnt <= 0) return -INFINITY;
            z = (orc_log(yt[k]) - orc_log((double)cnt)) / P->sigma;
        } else {
            z = (yt[k] - (double)cnt) / P->sigma;
        }
        lw = lw - 0.5 * (z * z);
    }
    return lw;
}

/* The particle-independent part of log p(y_t | x): the normalising constant
 * of the noise density (and the Jacobian -log y of the log-normal). */
static double obs_logconst(const orc_problem *P, const double *yt)
{
    double half_log_2pi = 0.5 * orc_log(2.0 * 3.141592653589793);
    double per = P->obs_kind == ORC_OBS_FLUORESCENCE ? half_log_2pi
                                                     : orc_log(P->sigma) + half_log_2pi;
    double c = -((double)P->n_observed * per);
    if (P->obs_kind == ORC_OBS_LOGNORMAL)
        for (int k = 0; k < P->n_observed; ++k) c = c - orc_log(yt[k]);
    return c;
}

/* ------------------------------------------------------------------------ */
/* Systematic resampling with integer weights.  q_j = floor(e_j 2^32),        */
/* cumulative sums C_0 = 0, C_{j+1} = C_j + q_j, total Q; one offset rho in   */
/* [0, Q); slot j takes ancestor a_j = min{ i : H C_{i+1} > j Q + rho }.      */
/* ------------------------------------------------------------------------ */
void orc_resample(int32_t H, const double *e, uint64_t w64, int32_t *anc)
{
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)H + 1));
    C[0] = 0;
    for (int j = 0; j < H; ++j) C[j + 1] = C[j] + (uint64_t)(e[j] * 4294967296.0);
    uint64_t Q = C[H];
    uint64_t rho = (uint64_t)(((unsigned __int128)w64 * Q) >> 64);
    int i = 0;
    for (int j = 0; j < H; ++j) {
        uint64_t point = (uint64_t)j * Q + rho;
        while (!((uint64_t)H * C[i + 1] > point)) i = i + 1;
        anc[j] = i;
    }
    free(C);
}

uint64_t orc_resample_word(uint64_t seed, uint32_t theta_id, uint32_t traj, uint32_t t)
{
    uint32_t w[4];
    philox_block(seed, 0, 0, (traj << 16) | t, (theta_id << 2) | 1u, w);
    return ((uint64_t)w[1] << 32) | w[0];
}

/* ------------------------------------------------------------------------ */
/* One particle filter: theta index i against trajectory m.                  */
/* Optional trace (H small): per interval the propagated states [T][H][U],    */
/* log-weights [T][H] and the ancestors used before the interval [T][H].     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t *states;
    double *logw;
    int32_t *ancestors;
    double *ll_inc;
} orc_trace;

/* A rate vector the filter cannot run: a negative, infinite or NaN rate; in
 * FP32-mixed mode also a rate beyond the binary32 range (it would round to
 * infinity, and infinity times a zero mass-action factor is NaN). */
static int bad_theta(const orc_problem *P, const double *c)
{
    for (int r = 0; r < P->n_reactions; ++r) {
        if (!(c[r] >= 0.0) || isinf(c[r])) return 1;
        if (P->precision == ORC_FP32_MIXED && isinf((float)c[r])) return 1;
    }
    return 0;
}

/* Simulation of particles j0 .. j1-1 over one interval (the "Simulate" step):
 * each particle runs on its own state and stream, so the particles of an
 * interval may be split between threads; the interval's events are their
 * sum and its status their largest. */
typedef struct {
    const orc_problem *P;
    const double *c;
    int32_t *x;
    double t_start, t_end;
    uint32_t c2, theta_id;
    int j0, j1;
    uint64_t events;
    int worst;
} orc_span;

static void *simulate_span(void *arg)
{
    orc_span *s = (orc_span *)arg;
    int U = s->P->n_species;
    s->events = 0;
    s->worst = ORC_OK;
    for (int j = s->j0; j < s->j1; ++j) {
        int st;
        int32_t *xj = s->x + (size_t)j * U;
        s->events += ssa_interval(s->P, s->c, xj, s->t_start, s->t_end, (uint32_t)j, s->c2,
                                  s->theta_id, &st, NULL);
        for (int u = 0; u < U; ++u)
            if (xj[u] > ORC_COUNT_LIMIT) st = st > ORC_COUNT_OVERFLOW ? st : ORC_COUNT_OVERFLOW;
        if (st > s->worst) s->worst = st;
    }
    return NULL;
}

static int run_filter(const orc_problem *P, int i, int m, double *ll_out,
                      uint64_t *events_out, int32_t *final_state, orc_trace *tr,
                      int threads)
{
    int U = P->n_species, H = P->n_particles;
    const double *c = P->theta + (size_t)i * P->n_reactions;
    uint32_t theta_id = P->theta_ids ? P->theta_ids[i] : (uint32_t)i;
    if (bad_theta(P, c)) {
        *ll_out = NAN;
        *events_out = 0;
        return ORC_BAD_THETA;
    }
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * U);
    int32_t *xn = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * U);
    double *lw = (double *)malloc(sizeof(double) * (size_t)H);
    double *e = (double *)malloc(sizeof(double) * (size_t)H);
    int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * (size_t)H);
    const int32_t *lo = P->x0 + (size_t)m * U;
    for (int j = 0; j < H; ++j) {
        for (int u = 0; u < U; ++u) {
            int32_t v = lo[u];
            if (P->x0_hi) {
                /* draw X_0 of particle j: species u from word u % 4 of the
                 * Philox block (u / 4, j, m << 16, theta id << 2 | 2), mapped
                 * to lo + floor(word * (hi - lo + 1) / 2^32) */
                uint32_t w[4];
                philox_block(P->seed, (uint32_t)(u / 4), (uint32_t)j, (uint32_t)m << 16,
                             (theta_id << 2) | 2u, w);
                uint64_t span = (uint64_t)(P->x0_hi[(size_t)m * U + u] - lo[u]) + 1u;
                v = lo[u] + (int32_t)(((uint64_t)w[u % 4] * span) >> 32);
            }
            x[(size_t)j * U + u] = v;
        }
    }

    int first = P->obs_offsets[m], T = P->obs_offsets[m + 1] - first;
    double ll = 0.0;
    uint64_t events = 0;
    int status = ORC_OK;
    double t_prev = P->t0[m];
    for (int t = 0; t < T; ++t) {
        /* 1. resample with the weights of observation t-1 (identity at t = 0,
         *    where all particles start from x0 with equal weights) */
        if (t > 0) {
            orc_resample(H, e, orc_resample_word(P->seed, theta_id, (uint32_t)m, (uint32_t)t), anc);
            for (int j = 0; j < H; ++j)
                for (int u = 0; u < U; ++u)
                    xn[(size_t)j * U + u] = x[(size_t)anc[j] * U + u];
            int32_t *tmp = x; x = xn; xn = tmp;
        } else {
            for (int j = 0; j < H; ++j) anc[j] = j;
        }
        /* 2. simulate every particle forward to the observation time
         *    (in `threads` spans of consecutive particles) */
        double t_end = P->t_obs[first + t];
        int worst = ORC_OK;
        int nspan = threads < H ? threads : H;
        orc_span span[64];
        pthread_t th[64];
        for (int k = 0; k < nspan; ++k) {
            span[k].P = P;
            span[k].c = c;
            span[k].x = x;
            span[k].t_start = t_prev;
            span[k].t_end = t_end;
            span[k].c2 = ((uint32_t)m << 16) | (uint32_t)t;
            span[k].theta_id = theta_id;
            span[k].j0 = (int)(((int64_t)H * k) / nspan);
            span[k].j1 = (int)(((int64_t)H * (k + 1)) / nspan);
        }
        for (int k = 1; k < nspan; ++k) pthread_create(&th[k], NULL, simulate_span, &span[k]);
        simulate_span(&span[0]);
        for (int k = 1; k < nspan; ++k) pthread_join(th[k], NULL);
        for (int k = 0; k < nspan; ++k) {
            events += span[k].events;
            if (span[k].worst > worst) worst = span[k].worst;
        }
        if (worst != ORC_OK) { status = worst; break; }
        /* 3. weight */
        const double *yt = P->y + (size_t)(first + t) * P->n_observed;
        for (int j = 0; j < H; ++j) lw[j] = obs_logweight(P, x + (size_t)j * U, yt);
        if (tr) {
            memcpy(tr->states + (size_t)t * H * U, x, sizeof(int32_t) * (size_t)H * U);
            memcpy(tr->logw + (size_t)t * H, lw, sizeof(double) * (size_t)H);
            memcpy(tr->ancestors + (size_t)t * H, anc, sizeof(int32_t) * (size_t)H);
        }
        /* 4. log of the mean weight, added to the running log-likelihood */
        double mx = -INFINITY;
        for (int j = 0; j < H; ++j) if (lw[j] > mx) mx = lw[j];
        if (mx == -INFINITY) {
            ll = -INFINITY;
            if (tr) tr->ll_inc[t] = -INFINITY;
            break;
        }
        double S = 0.0;
        for (int j = 0; j < H; ++j) {
            e[j] = orc_exp(lw[j] - mx);
            S = S + e[j];
        }
        double inc = ((mx + orc_log(S)) - orc_log((double)H)) + obs_logconst(P, yt);
        if (tr) tr->ll_inc[t] = inc;
        ll = ll + inc;
        t_prev = t_end;
    }
    if (status != ORC_OK) ll = NAN;
    if (final_state) {
        for (int u = 0; u < U; ++u)
            for (int j = 0; j < H; ++j)
                final_state[(size_t)u * H + j] = x[(size_t)j * U + u];
    }
    *ll_out = ll;
    *events_out = events;
    free(x); free(xn); free(lw); free(e); free(anc);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Batch: every theta against every trajectory, filters spread over threads. */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_problem *P;
    int next;
    int inner;       /* threads per filter for its particles */
    pthread_mutex_t lock;
    double *fll;
    uint64_t *fev;
    int32_t *fst;
    int32_t *final_state;
} batch_ctx;

static void *worker(void *arg)
{
    batch_ctx *b = (batch_ctx *)arg;
    const orc_problem *P = b->P;
    int F = P->n_theta * P->n_traj;
    size_t per = (size_t)P->n_species * P->n_particles;
    for (;;) {
        pthread_mutex_lock(&b->lock);
        int f = b->next++;
        pthread_mutex_unlock(&b->lock);
        if (f >= F) break;
        int i = f / P->n_traj, m = f % P->n_traj;
        b->fst[f] = run_filter(P, i, m, &b->fll[f], &b->fev[f],
                               b->final_state ? b->final_state + per * f : NULL, NULL, b->inner);
    }
    return NULL;
}

/* Returns 0, or -1 on invalid arguments. loglik[i] = sum over m (in order) of
 * the filter log-likelihoods; status[i] = first failing filter's status. */
int orc_eval(const orc_problem *P, int nthreads, double *loglik, int32_t *status,
             double *filter_ll, uint64_t *filter_events, int32_t *final_state)
{
    if (P->n_species < 1 || P->n_reactions < 1 || P->n_reactions > 256 ||
        P->n_particles < 1 || P->n_theta < 0 || P->n_traj < 1)
        return -1;
    int F = P->n_theta * P->n_traj;
    batch_ctx b;
    b.P = P;
    b.next = 0;
    pthread_mutex_init(&b.lock, NULL);
    b.fll = (double *)malloc(sizeof(double) * (size_t)(F > 0 ? F : 1));
    b.fev = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(F > 0 ? F : 1));
    b.fst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F > 0 ? F : 1));
    b.final_state = final_state;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    /* fewer filters than threads: the spare threads share each filter's
     * particles (at most 64 per filter) */
    int outer = nthreads;
    b.inner = 1;
    if (F > 0 && F < nthreads) {
        outer = F;
        b.inner = nthreads / F;
        if (b.inner > 64) b.inner = 64;
    }
    pthread_t th[256];
    for (int k = 0; k < outer; ++k) pthread_create(&th[k], NULL, worker, &b);
    for (int k = 0; k < outer; ++k) pthread_join(th[k], NULL);
    for (int i = 0; i < P->n_theta; ++i) {
        double s = 0.0;
        int32_t st = ORC_OK;
        for (int m = 0; m < P->n_traj; ++m) {
            int f = i * P->n_traj + m;
            if (st == ORC_OK && b.fst[f] != ORC_OK) st = b.fst[f];
            s = s + b.fll[f];
        }
        loglik[i] = st == ORC_OK ? s : NAN;
        if (status) status[i] = st;
    }
    if (filter_ll) memcpy(filter_ll, b.fll, sizeof(double) * (size_t)F);
    if (filter_events) memcpy(filter_events, b.fev, sizeof(uint64_t) * (size_t)F);
    free(b.fll); free(b.fev); free(b.fst);
    pthread_mutex_destroy(&b.lock);
    return 0;
}

/* One filter with a full trace (for brute-force checks at small H). */
int orc_trace_filter(const orc_problem *P, int i, int m, int32_t *states, double *logw,
                     int32_t *ancestors, double *ll_inc, double *ll_out, uint64_t *events_out)
{
    orc_trace tr = {states, logw, ancestors, ll_inc};
    return run_filter(P, i, m, ll_out, events_out, NULL, &tr, 1);
}

/* Plain SSA paths (no observations): n_paths particles from x0 over
 * [t_start, t_end], particle slot j, interval index 0 of trajectory 0.
 * Output states [n_paths][U], per-path event counts and (clock_out not
 * NULL) each path's clock: the time of its last event, the sum of its
 * waiting times from t_start. */
int orc_ssa_paths(const orc_problem *P, const double *c, uint32_t theta_id,
                  const int32_t *x0, double t_start, double t_end, int32_t n_paths,
                  int32_t *states_out, uint64_t *events_out, double *clock_out)
{
    int U = P->n_species;
    for (int j = 0; j < n_paths; ++j) {
        int32_t *xj = states_out + (size_t)j * U;
        for (int u = 0; u < U; ++u) xj[u] = x0[u];
        int st;
        events_out[j] = ssa_interval(P, c, xj, t_start, t_end, (uint32_t)j, 0u, theta_id, &st,
                                     clock_out ? clock_out + j : NULL);
        if (st != ORC_OK) return st;
    }
    return 0;
}
