// ode.hip -- likelihood of deterministic models (Sec. "Chemical Reaction
// Networks": dX/dt = f(X, t, theta); Results: a deterministic model needs no
// particle filter, only its ODE solution and the noise density around it;
// Supplementary "Egf-Ras-Raf-Mek-Erk model": saturating and Hill rate laws,
// a time-dependent input, a FRET read-out).
//
// One lane integrates one (theta, trajectory) pair with the Dormand-Prince
// 5(4) pair under the step rule of include/lik.h, stopping exactly at every
// observation time and input breakpoint, and accumulates the normal
// log-density of each observation; a second kernel sums each theta's
// trajectories in order.  The model (its flux terms) is the same for every
// lane, so the term loop and its indices are wave-uniform.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <stdio.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "host.hpp"
#include "ode.hpp"

struct lik_ode_t_ {
    lik_ode_model m;
    std::vector<lik_ode_term> terms;
    std::vector<int32_t> x0_param;
    // the model-specialised kernel, per device
    std::mutex mu;
    std::map<int, std::pair<hipModule_t, hipFunction_t>> spec;
    // the terms and x0_param in device memory, per device (made on first use)
    std::map<int, char *> dev;
};

namespace {

using namespace lik;

template <int UMAX>
__global__ void __launch_bounds__(64) k_ode(OdeArgs a) {
    ode_run<OdeGeneric<UMAX>>(a);
}

// The order in which the lanes take trajectories: by stops (observations plus
// input breakpoints) from most to fewest, ties in index order; thread m
// places trajectory m at its rank.  Thread 0 also zeroes the pair counter.
__global__ void k_ode_order(const int32_t *obs_off, const int32_t *in_off, int32_t M,
                            int32_t *order, unsigned int *next) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m == 0) *next = 0u;
    if (m >= M) return;
    const int sm = (obs_off[m + 1] - obs_off[m]) + (in_off ? in_off[m + 1] - in_off[m] : 0);
    int rank = 0;
    for (int j = 0; j < M; ++j) {
        const int sj = (obs_off[j + 1] - obs_off[j]) + (in_off ? in_off[j + 1] - in_off[j] : 0);
        rank += (sj > sm || (sj == sm && j < m)) ? 1 : 0;
    }
    order[rank] = m;
}

// per theta: the sum over its trajectories in order; the first non-OK status
__global__ void k_ode_finish(const double *tll, const int32_t *tst, int32_t n_theta, int32_t M,
                             double *loglik, int32_t *status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_theta) return;
    double s = 0.0;
    int32_t st = LIK_STATUS_OK;
    for (int m = 0; m < M; ++m) {
        const int f = i * M + m;
        if (st == LIK_STATUS_OK && tst[f] != LIK_STATUS_OK) st = tst[f];
        s = s + tll[f];
    }
    loglik[i] = st == LIK_STATUS_OK ? s : __builtin_nan("");
    if (status) status[i] = st;
}

std::string hexd(double v) {
    char b[64];
    snprintf(b, sizeof(b), "%a", v);
    return b;
}

// Stride (in doubles) of the lanes' parameter slots in LDS: odd, so that the
// slots a wavefront reads at once fall in different banks, except at the
// largest V, where 64 slots of 128 fill the 64 KiB a workgroup may take.
int ode_par_stride(int V) { return V % 2 == 1 || V == LIK_ODE_MAX_PARAMS ? V : V + 1; }

// LDS bytes of the specialised kernel's launch: one parameter slot per lane.
size_t ode_par_lds(int V) { return (size_t)64 * ode_par_stride(V) * sizeof(double); }

// The model as code: its flux terms with constant indices (the same
// operations, in the same order, as OdeGeneric::rhs), the parameters of the
// lane's current theta read from its slot in LDS (copied there when the lane
// takes a pair), the observation mean with constant indices.
std::string ode_spec_source(const lik_ode_model &m) {
    const int U = m.n_species, V = m.n_params;
    std::ostringstream o;
    o << "typedef __hip_internal::uint32_t uint32_t;\n"
         "typedef __hip_internal::uint64_t uint64_t;\n"
         "typedef __hip_internal::int32_t int32_t;\n"
         "typedef __hip_internal::int64_t int64_t;\n"
         "#include \"ode.hpp\"\n"
         "extern __shared__ double lik_ode_par[];\n"
         "namespace lik {\n"
         "static_assert(sizeof(OdeArgs) == "
      << sizeof(OdeArgs) << ", \"OdeArgs layout\");\n"
      << "struct OdeSpec {\n  static constexpr int U = " << U << ";\n"
      << "  struct Params { int off; };\n"
      << "  __device__ static Params load(const OdeArgs &a, int i) {\n"
      << "    const int o = (int)threadIdx.x * " << ode_par_stride(V) << ";\n"
      << "    for (int k = 0; k < " << V << "; ++k) lik_ode_par[o + k] = a.theta[(size_t)i * "
      << V << " + k];\n    return Params{o};\n  }\n"
      // the offset passes through an empty asm so that every evaluation
      // reads its parameters from LDS anew instead of the compiler keeping
      // all of them in registers across the step loop
      << "  __device__ static const double *row(const Params &p) {\n"
      << "    int o = p.off;\n    asm volatile(\"\" : \"+v\"(o));\n"
      << "    return lik_ode_par + o;\n  }\n"
      << "  __device__ static void rhs(const OdeArgs &, const Params &p, double u, const double *x,"
         " double *dx) {\n    const double *pv = row(p);\n";
    for (int s = 0; s < U; ++s) o << "    dx[" << s << "] = 0.0;\n";
    for (int k = 0; k < m.n_terms; ++k) {
        const lik_ode_term &T = m.terms[k];
        o << "    { double v = " << hexd(T.rate_scale);
        if (T.rate_param >= 0) o << " * pv[" << T.rate_param << "]";
        o << ";\n";
        for (int f = 0; f < T.n_factors; ++f) {
            const std::string xs = "x[" + std::to_string(T.species[f]) + "]";
            const std::string K = "pv[" + std::to_string(T.param[f]) + "]";
            std::string phi;
            switch (T.kind[f]) {
                case LIK_ODE_INPUT: phi = "u"; break;
                case LIK_ODE_SPECIES: phi = xs; break;
                case LIK_ODE_SATURATING: phi = xs + " / (" + K + " + " + xs + ")"; break;
                case LIK_ODE_HILL2:
                    phi = "(" + xs + " * " + xs + ") / (" + K + " + " + xs + " * " + xs + ")";
                    break;
                default: phi = K + " / (" + K + " + " + xs + " * " + xs + ")"; break;
            }
            o << "      v = v * (" << phi << ");\n";
        }
        if (T.from >= 0) o << "      dx[" << T.from << "] = dx[" << T.from << "] - v;\n";
        if (T.to >= 0) o << "      dx[" << T.to << "] = dx[" << T.to << "] + v;\n";
        o << "    }\n";
    }
    o << "  }\n  __device__ static double obs(const OdeArgs &, const Params &p, const double *x) {\n"
         "    const double *pv = row(p);\n    (void)pv;\n";
    if (m.obs_kind == LIK_ODE_OBS_SPECIES) {
        o << "    return x[" << m.obs_species << "];\n";
    } else {
        auto P = [&](int k) { return "pv[" + std::to_string(m.fret_param[k]) + "]"; };
        o << "    const double xa = x[" << m.obs_species << "], xb = x[" << m.obs_species2 << "];\n"
          << "    const double num = (" << P(2) << " * " << P(3) << ") * xa;\n"
          << "    const double den = (xb + (1.0 - " << P(2) << ") * xa) * " << P(4) << ";\n"
          << "    return " << P(0) << " * (num / den + " << P(1) << ");\n";
    }
    o << "  }\n};\n}  // namespace lik\n"
         "extern \"C\" __global__ void __launch_bounds__(64) lik_ode_spec(lik::OdeArgs a) {\n"
         "  lik::ode_run<lik::OdeSpec>(a);\n}\n";
    return o.str();
}

// The specialised kernel on the current device (compiled or read from the
// disk cache on first use); nullptr with *err on failure.
hipFunction_t ode_spec_kernel(lik_ode_t_ &md, std::string *err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return nullptr;
    }
    std::lock_guard<std::mutex> g(md.mu);
    auto it = md.spec.find(dev);
    if (it != md.spec.end()) return it->second.second;
    std::vector<char> code;
    if (!rtc_code(ode_spec_source(md.m), &code, err)) return nullptr;
    hipModule_t mod = nullptr;
    hipError_t e = hipModuleLoadData(&mod, code.data());
    if (e != hipSuccess) {
        *err = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
        return nullptr;
    }
    hipFunction_t fn = nullptr;
    e = hipModuleGetFunction(&fn, mod, "lik_ode_spec");
    if (e != hipSuccess) {
        *err = std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
        (void)hipModuleUnload(mod);
        return nullptr;
    }
    md.spec[dev] = {mod, fn};
    return fn;
}

bool valid_param(int p, int V) { return p >= 0 && p < V; }

int check_model(const lik_ode_model *md) {
    if (!md) return fail(LIK_EINVAL, "model is NULL");
    const int U = md->n_species, V = md->n_params;
    if (U < 1 || U > LIK_ODE_MAX_SPECIES) return fail(LIK_EINVAL, "n_species out of [1, 32]");
    if (V < 1 || V > LIK_ODE_MAX_PARAMS) return fail(LIK_EINVAL, "n_params out of [1, 128]");
    if (md->n_terms < 1 || md->n_terms > LIK_ODE_MAX_TERMS || !md->terms)
        return fail(LIK_EINVAL, "n_terms out of [1, 128] or terms NULL");
    if (!md->x0_param) return fail(LIK_EINVAL, "x0_param is NULL");
    for (int k = 0; k < md->n_terms; ++k) {
        const lik_ode_term &T = md->terms[k];
        if (T.from < -1 || T.from >= U || T.to < -1 || T.to >= U)
            return fail(LIK_EINVAL, "term species out of range");
        if (T.rate_param < -1 || T.rate_param >= V) return fail(LIK_EINVAL, "rate_param out of range");
        if (!(T.rate_scale >= 0.0) || isinf(T.rate_scale))
            return fail(LIK_EINVAL, "rate_scale must be finite and >= 0");
        if (T.n_factors < 0 || T.n_factors > LIK_ODE_MAX_FACTORS)
            return fail(LIK_EINVAL, "n_factors out of [0, 3]");
        for (int f = 0; f < T.n_factors; ++f) {
            const int kind = T.kind[f];
            if (kind < LIK_ODE_SPECIES || kind > LIK_ODE_INPUT)
                return fail(LIK_EINVAL, "unknown factor kind");
            if (kind != LIK_ODE_INPUT && (T.species[f] < 0 || T.species[f] >= U))
                return fail(LIK_EINVAL, "factor species out of range");
            if ((kind == LIK_ODE_SATURATING || kind == LIK_ODE_HILL2 ||
                 kind == LIK_ODE_REPRESS2) && !valid_param(T.param[f], V))
                return fail(LIK_EINVAL, "factor param out of range");
        }
    }
    for (int s = 0; s < U; ++s)
        if (md->x0_param[s] < -1 || md->x0_param[s] >= V)
            return fail(LIK_EINVAL, "x0_param out of range");
    if (md->obs_kind != LIK_ODE_OBS_SPECIES && md->obs_kind != LIK_ODE_OBS_FRET)
        return fail(LIK_EINVAL, "unknown observation kind");
    if (md->obs_species < 0 || md->obs_species >= U) return fail(LIK_EINVAL, "obs_species out of range");
    if (md->obs_kind == LIK_ODE_OBS_FRET) {
        if (md->obs_species2 < 0 || md->obs_species2 >= U)
            return fail(LIK_EINVAL, "obs_species2 out of range");
        for (int k = 0; k < 5; ++k)
            if (!valid_param(md->fret_param[k], V)) return fail(LIK_EINVAL, "fret_param out of range");
    }
    if (md->sd_param < -1 || md->sd_param >= V) return fail(LIK_EINVAL, "sd_param out of range");
    if (md->sd_param < 0 && (!(md->sd_const > 0.0) || isinf(md->sd_const)))
        return fail(LIK_EINVAL, "sd_const must be finite and > 0");
    return LIK_OK;
}

// The model's terms and x0_param in device memory on the current device
// (copied on the first call there, kept until lik_ode_destroy).
int model_on_device(lik_ode_t_ &md, const lik_ode_term **terms, const int32_t **x0p) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(md.mu);
    const size_t tb = align256(md.terms.size() * sizeof(lik_ode_term));
    auto it = md.dev.find(dev);
    char *p = it != md.dev.end() ? it->second : nullptr;
    if (!p) {
        const size_t xb = md.x0_param.size() * sizeof(int32_t);
        if ((e = hipMalloc((void **)&p, tb + xb)) != hipSuccess)
            return fail(LIK_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        if ((e = hipMemcpy(p, md.terms.data(), md.terms.size() * sizeof(lik_ode_term),
                           hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p + tb, md.x0_param.data(), xb, hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(p);
            return hip_fail(e, "copy of the model to the device");
        }
        md.dev[dev] = p;
    }
    *terms = (const lik_ode_term *)p;
    *x0p = (const int32_t *)(p + tb);
    return LIK_OK;
}

// Arguments common to both entry points.
int check_call(lik_ode_t model, int32_t n_theta, const lik_ode_data *data, double rtol,
               double atol, int32_t max_steps, int32_t kernel) {
    if (!model) return fail(LIK_EINVAL, "model is NULL");
    if (kernel < LIK_KERNEL_AUTO || kernel > LIK_KERNEL_SPECIALIZED)
        return fail(LIK_EINVAL, "unknown kernel variant");
    if (!data) return fail(LIK_EINVAL, "data is NULL");
    if (n_theta < 0 || n_theta >= (1 << 26)) return fail(LIK_EINVAL, "n_theta out of range");
    if (!(rtol > 0.0) || !(atol > 0.0) || isinf(rtol) || isinf(atol))
        return fail(LIK_EINVAL, "rtol and atol must be finite and > 0");
    if (max_steps < 1 || max_steps > (1 << 30)) return fail(LIK_EINVAL, "max_steps out of [1, 2^30]");
    const int M = data->n_traj;
    if (M < 1 || M > LIK_MAX_TRAJ) return fail(LIK_EINVAL, "n_traj out of range");
    if ((int64_t)n_theta * M >= ((int64_t)1 << 30)) return fail(LIK_EINVAL, "too many trajectories");
    return LIK_OK;
}

// Input offsets (host copy): in_offsets[0] = 0, never decreasing; their total.
int check_in_offsets(const int32_t *in_offsets, int M, int64_t *n_in) {
    *n_in = 0;
    if (!in_offsets) return LIK_OK;
    if (in_offsets[0] != 0) return fail(LIK_EINVAL, "in_offsets[0] must be 0");
    for (int m = 0; m < M; ++m)
        if (in_offsets[m + 1] < in_offsets[m]) return fail(LIK_EINVAL, "in_offsets must not decrease");
    *n_in = in_offsets[M];
    return LIK_OK;
}

// The model's fields of the kernel arguments.
void model_args(const lik_ode_t_ &md, OdeArgs *a) {
    a->U = md.m.n_species;
    a->V = md.m.n_params;
    a->n_terms = md.m.n_terms;
    a->obs_kind = md.m.obs_kind;
    a->obs_species = md.m.obs_species;
    a->obs_species2 = md.m.obs_kind == LIK_ODE_OBS_FRET ? md.m.obs_species2 : -1;
    a->sd_param = md.m.sd_param;
    a->sd_const = md.m.sd_const;
    for (int k = 0; k < 5; ++k) a->fret[k] = md.m.fret_param[k];
}

// The specialised kernel when asked for (or by default, where it compiles).
int pick_kernel(lik_ode_t_ &md, int32_t kernel, hipFunction_t *spec) {
    *spec = nullptr;
    if (kernel == LIK_KERNEL_GENERIC) return LIK_OK;
    std::string msg;
    *spec = ode_spec_kernel(md, &msg);
    if (!*spec && kernel == LIK_KERNEL_SPECIALIZED)
        return fail(LIK_EDEVICE, "specialised ODE kernel unavailable: " + msg);
    return LIK_OK;
}

// Enqueues on s: the trajectory order (and the zeroed pair counter), the
// solver over every pair, and the per-theta sums.  Every pointer in a is a
// device pointer.
int ode_enqueue(const OdeArgs &a, hipFunction_t spec, double *loglik, int32_t *status,
                hipStream_t s) {
    const int U = a.U, V = a.V, M = a.M, n_theta = a.n_theta;
    const size_t F = (size_t)n_theta * M;
    hipLaunchKernelGGL(k_ode_order, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s,
                       a.obs_offsets, a.in_offsets, M, const_cast<int32_t *>(a.m_order), a.next);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ode order launch");
    // every lane takes pairs until none is left: as many workgroups as can
    // be resident at once (more would only find the counter spent)
    const unsigned lds = spec ? (unsigned)ode_par_lds(V) : 0u;
    const void *gen = U <= 4 ? (const void *)k_ode<4> : U <= 8 ? (const void *)k_ode<8>
                    : U <= 16 ? (const void *)k_ode<16> : (const void *)k_ode<32>;
    unsigned blocks = (unsigned)((F + 63) / 64);
    int per_cu = 0, cus = 0, dev_id = 0;
    const hipError_t eo = spec ? hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, spec,
                                                                                    64, lds)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gen, 64, 0);
    if (eo == hipSuccess && per_cu > 0 && hipGetDevice(&dev_id) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) == hipSuccess &&
        cus > 0)
        blocks = std::min(blocks, (unsigned)(per_cu * cus));
    hipEvent_t t0 = timing_begin(s);  // timed as a propagation launch
    if (spec) {
        OdeArgs ac = a;
        void *params[] = {(void *)&ac};
        e = hipModuleLaunchKernel(spec, blocks, 1, 1, 64, 1, 1, lds, s, params, nullptr);
        if (e != hipSuccess) return hip_fail(e, "ode launch");
    } else if (U <= 4) hipLaunchKernelGGL(k_ode<4>, dim3(blocks), dim3(64), 0, s, a);
    else if (U <= 8) hipLaunchKernelGGL(k_ode<8>, dim3(blocks), dim3(64), 0, s, a);
    else if (U <= 16) hipLaunchKernelGGL(k_ode<16>, dim3(blocks), dim3(64), 0, s, a);
    else hipLaunchKernelGGL(k_ode<32>, dim3(blocks), dim3(64), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "ode launch");
    timing_end_propagate(t0, s);
    hipLaunchKernelGGL(k_ode_finish, dim3((unsigned)((n_theta + 255) / 256)), dim3(256), 0, s,
                       a.tll, a.tst, n_theta, M, loglik, status);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "ode finish launch");
    return LIK_OK;
}

// Per-call device scratch after the inputs: trajectory log-likelihoods and
// statuses, step counts, the pair counter, the trajectory order.
size_t scratch_bytes(size_t F, int M) {
    return align256(F * 8) + align256(F * 4) + align256(F * 4) + align256(4) +
           align256((size_t)M * 4);
}

void carve_scratch(char *p, size_t F, int M, OdeArgs *a, int32_t *steps) {
    a->tll = (double *)p;
    p += align256(F * 8);
    a->tst = (int32_t *)p;
    p += align256(F * 4);
    a->tsteps = steps ? steps : (int32_t *)p;
    p += align256(F * 4);
    a->next = (unsigned int *)p;
    p += align256(4);
    a->m_order = (const int32_t *)p;
}

}  // namespace

extern "C" {

int lik_ode_create(const lik_ode_model *model, lik_ode_t *out) {
    if (!out) return fail(LIK_EINVAL, "out is NULL");
    int rc = check_model(model);
    if (rc) return rc;
    lik_ode_t_ *o = new (std::nothrow) lik_ode_t_;
    if (!o) return fail(LIK_ENOMEM, "allocation failed");
    o->m = *model;
    o->terms.assign(model->terms, model->terms + model->n_terms);
    o->x0_param.assign(model->x0_param, model->x0_param + model->n_species);
    o->m.terms = o->terms.data();
    o->m.x0_param = o->x0_param.data();
    *out = o;
    return LIK_OK;
}

int lik_ode_precompile(lik_ode_t model) {
    if (!model) return fail(LIK_EINVAL, "model is NULL");
    std::vector<char> code;
    std::string err;
    if (!rtc_code(ode_spec_source(model->m), &code, &err)) return fail(LIK_EDEVICE, err);
    return LIK_OK;
}

int lik_ode_destroy(lik_ode_t model) {
    if (model) {
        for (auto &kv : model->spec) (void)hipModuleUnload(kv.second.first);
        for (auto &kv : model->dev) (void)hipFree(kv.second);
    }
    delete model;
    return LIK_OK;
}

int lik_ode_eval(lik_ode_t model, int32_t n_theta, const double *theta, const lik_ode_data *data,
                 double rtol, double atol, int32_t max_steps, int32_t kernel,
                 double *loglik_out, int32_t *status_out, int32_t *steps_out) {
    int rc = check_call(model, n_theta, data, rtol, atol, max_steps, kernel);
    if (rc) return rc;
    const int M = data->n_traj, U = model->m.n_species, V = model->m.n_params;
    if (n_theta == 0) return LIK_OK;
    if (!theta || !loglik_out || !data->obs_offsets || !data->t_obs || !data->y || !data->t0 ||
        !data->x0)
        return fail(LIK_EINVAL, "NULL input or output pointer");
    int t_max = 0;
    int64_t total = 0, n_in = 0;
    if ((rc = check_offsets(data->obs_offsets, M, &t_max, &total))) return rc;
    if ((rc = check_in_offsets(data->in_offsets, M, &n_in))) return rc;
    if (n_in > 0 && (!data->t_in || !data->u_in)) return fail(LIK_EINVAL, "input arrays NULL");
    for (int m = 0; m < M; ++m) {
        double prev = data->t0[m];
        if (!isfinite(prev)) return fail(LIK_EINVAL, "t0 must be finite");
        for (int k = data->obs_offsets[m]; k < data->obs_offsets[m + 1]; ++k) {
            if (!(data->t_obs[k] > prev) || !isfinite(data->t_obs[k]))
                return fail(LIK_EINVAL, "observation times must increase strictly from t0");
            if (!isfinite(data->y[k])) return fail(LIK_EINVAL, "observations must be finite");
            prev = data->t_obs[k];
        }
        for (int s = 0; s < U; ++s)
            if (!isfinite(data->x0[(size_t)m * U + s])) return fail(LIK_EINVAL, "x0 must be finite");
        if (data->in_offsets)
            for (int k = data->in_offsets[m]; k < data->in_offsets[m + 1]; ++k) {
                if (!isfinite(data->t_in[k]) || !isfinite(data->u_in[k]) ||
                    (k > data->in_offsets[m] && !(data->t_in[k] > data->t_in[k - 1])))
                    return fail(LIK_EINVAL, "input breakpoints must be finite and increase strictly");
            }
    }
    hipFunction_t spec = nullptr;
    if ((rc = pick_kernel(*model, kernel, &spec))) return rc;
    OdeArgs a;
    memset(&a, 0, sizeof(a));
    if ((rc = model_on_device(*model, &a.terms, &a.x0_param))) return rc;
    model_args(*model, &a);

    const size_t F = (size_t)n_theta * M;
    // inputs, the per-theta results, then the solver's scratch
    const size_t sz[] = {(size_t)n_theta * V * 8, (size_t)(M + 1) * 4, (size_t)total * 8,
                         (size_t)total * 8, (size_t)M * 8, (size_t)M * U * 8,
                         data->in_offsets ? (size_t)(M + 1) * 4 : 0, (size_t)n_in * 8,
                         (size_t)n_in * 8, (size_t)n_theta * 8, (size_t)n_theta * 4};
    const void *src[] = {theta, data->obs_offsets, data->t_obs, data->y, data->t0, data->x0,
                         data->in_offsets, data->t_in, data->u_in, nullptr, nullptr};
    constexpr int kN = (int)(sizeof(sz) / sizeof(sz[0]));
    size_t bytes = scratch_bytes(F, M);
    for (size_t v : sz) bytes += align256(v);
    char *dev = nullptr;
    hipError_t e = hipMalloc((void **)&dev, bytes + 256);
    if (e != hipSuccess) return fail(LIK_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    void *ptr[kN];
    size_t off = 0;
    for (int k = 0; k < kN; ++k) {
        ptr[k] = sz[k] ? dev + off : nullptr;
        off += align256(sz[k]);
    }
    carve_scratch(dev + off, F, M, &a, nullptr);
    a.theta = (const double *)ptr[0];
    a.n_theta = n_theta;
    a.M = M;
    a.obs_offsets = (const int32_t *)ptr[1];
    a.t_obs = (const double *)ptr[2];
    a.y = (const double *)ptr[3];
    a.t0 = (const double *)ptr[4];
    a.x0 = (const double *)ptr[5];
    a.in_offsets = (const int32_t *)ptr[6];
    a.t_in = (const double *)ptr[7];
    a.u_in = (const double *)ptr[8];
    a.rtol = rtol;
    a.atol = atol;
    a.max_steps = max_steps;
    double *d_ll = (double *)ptr[9];
    int32_t *d_st = (int32_t *)ptr[10];
    hipStream_t s = nullptr;
    rc = LIK_OK;
    do {
        if ((e = hipStreamCreate(&s)) != hipSuccess) { rc = hip_fail(e, "hipStreamCreate"); break; }
        for (int k = 0; k < kN && e == hipSuccess; ++k)
            if (sz[k] && src[k]) e = hipMemcpyAsync(ptr[k], src[k], sz[k], hipMemcpyHostToDevice, s);
        if (e != hipSuccess) { rc = hip_fail(e, "copy to device"); break; }
        if ((rc = ode_enqueue(a, spec, d_ll, d_st, s))) break;
        if ((e = hipMemcpyAsync(loglik_out, d_ll, (size_t)n_theta * 8, hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (status_out && (e = hipMemcpyAsync(status_out, d_st, (size_t)n_theta * 4,
                                               hipMemcpyDeviceToHost, s)) != hipSuccess) ||
            (steps_out && (e = hipMemcpyAsync(steps_out, a.tsteps, F * 4, hipMemcpyDeviceToHost,
                                              s)) != hipSuccess)) {
            rc = hip_fail(e, "copy to host");
            break;
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = hip_fail(e, "synchronize"); break; }
    } while (0);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(dev);
    return rc;
}

size_t lik_ode_workspace_size(lik_ode_t model, int32_t n_theta, int32_t n_traj) {
    if (!model || n_theta < 0 || n_traj < 1) return 0;
    return scratch_bytes((size_t)n_theta * n_traj, n_traj) + 256;
}

int lik_ode_eval_device(lik_ode_t model, int32_t n_theta, const double *theta,
                        const lik_ode_data *data, const int32_t *obs_offsets_host,
                        const int32_t *in_offsets_host, double rtol, double atol,
                        int32_t max_steps, int32_t kernel, double *loglik, int32_t *status,
                        int32_t *steps, void *workspace, size_t workspace_bytes, void *stream) {
    int rc = check_call(model, n_theta, data, rtol, atol, max_steps, kernel);
    if (rc) return rc;
    const int M = data->n_traj;
    if (n_theta == 0) return LIK_OK;
    if (!theta || !loglik || !data->obs_offsets || !data->t_obs || !data->y || !data->t0 ||
        !data->x0 || !obs_offsets_host)
        return fail(LIK_EINVAL, "NULL input or output pointer");
    if ((data->in_offsets == nullptr) != (in_offsets_host == nullptr))
        return fail(LIK_EINVAL, "in_offsets and in_offsets_host must both be given or both NULL");
    int t_max = 0;
    int64_t total = 0, n_in = 0;
    if ((rc = check_offsets(obs_offsets_host, M, &t_max, &total))) return rc;
    if ((rc = check_in_offsets(in_offsets_host, M, &n_in))) return rc;
    if (n_in > 0 && (!data->t_in || !data->u_in)) return fail(LIK_EINVAL, "input arrays NULL");
    const size_t F = (size_t)n_theta * M;
    if (!workspace || workspace_bytes < lik_ode_workspace_size(model, n_theta, M))
        return fail(LIK_EINVAL, "workspace too small (see lik_ode_workspace_size)");
    hipFunction_t spec = nullptr;
    if ((rc = pick_kernel(*model, kernel, &spec))) return rc;
    OdeArgs a;
    memset(&a, 0, sizeof(a));
    if ((rc = model_on_device(*model, &a.terms, &a.x0_param))) return rc;
    model_args(*model, &a);
    carve_scratch((char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255), F, M, &a, steps);
    a.theta = theta;
    a.n_theta = n_theta;
    a.M = M;
    a.obs_offsets = data->obs_offsets;
    a.t_obs = data->t_obs;
    a.y = data->y;
    a.t0 = data->t0;
    a.x0 = data->x0;
    a.in_offsets = data->in_offsets;
    a.t_in = data->t_in;
    a.u_in = data->u_in;
    a.rtol = rtol;
    a.atol = atol;
    a.max_steps = max_steps;
    return ode_enqueue(a, spec, loglik, status, (hipStream_t)stream);
}

}  // extern "C"
