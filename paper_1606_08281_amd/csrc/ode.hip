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
};

namespace {

using namespace lik;

template <int UMAX>
__global__ void __launch_bounds__(64) k_ode(OdeArgs a) {
    ode_run<OdeGeneric<UMAX>>(a);
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
    if (model)
        for (auto &kv : model->spec) (void)hipModuleUnload(kv.second.first);
    delete model;
    return LIK_OK;
}

int lik_ode_eval(lik_ode_t model, int32_t n_theta, const double *theta, const lik_ode_data *data,
                 double rtol, double atol, int32_t max_steps, int32_t kernel,
                 double *loglik_out, int32_t *status_out, int32_t *steps_out) {
    if (!model) return fail(LIK_EINVAL, "model is NULL");
    if (kernel < LIK_KERNEL_AUTO || kernel > LIK_KERNEL_SPECIALIZED)
        return fail(LIK_EINVAL, "unknown kernel variant");
    if (!data) return fail(LIK_EINVAL, "data is NULL");
    if (n_theta < 0 || n_theta >= (1 << 26)) return fail(LIK_EINVAL, "n_theta out of range");
    if (!(rtol > 0.0) || !(atol > 0.0) || isinf(rtol) || isinf(atol))
        return fail(LIK_EINVAL, "rtol and atol must be finite and > 0");
    if (max_steps < 1 || max_steps > (1 << 30)) return fail(LIK_EINVAL, "max_steps out of [1, 2^30]");
    const int M = data->n_traj, U = model->m.n_species, V = model->m.n_params;
    if (M < 1 || M > LIK_MAX_TRAJ) return fail(LIK_EINVAL, "n_traj out of range");
    if ((int64_t)n_theta * M >= ((int64_t)1 << 30)) return fail(LIK_EINVAL, "too many trajectories");
    if (n_theta == 0) return LIK_OK;
    if (!theta || !loglik_out || !data->obs_offsets || !data->t_obs || !data->y || !data->t0 ||
        !data->x0)
        return fail(LIK_EINVAL, "NULL input or output pointer");
    int t_max = 0;
    int64_t total = 0;
    int rc = check_offsets(data->obs_offsets, M, &t_max, &total);
    if (rc) return rc;
    int64_t n_in = 0;
    if (data->in_offsets) {
        if (data->in_offsets[0] != 0) return fail(LIK_EINVAL, "in_offsets[0] must be 0");
        for (int m = 0; m < M; ++m)
            if (data->in_offsets[m + 1] < data->in_offsets[m])
                return fail(LIK_EINVAL, "in_offsets must not decrease");
        n_in = data->in_offsets[M];
        if (n_in > 0 && (!data->t_in || !data->u_in)) return fail(LIK_EINVAL, "input arrays NULL");
    }
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
    const size_t F = (size_t)n_theta * M;
    // Pairs are taken trajectory by trajectory, the trajectories with the
    // most stops (observations and input breakpoints, each a restart of the
    // step size) first: their pairs tend to take the most steps, and a lane
    // that ends the launch on a short pair leaves less of a tail.
    std::vector<int32_t> m_order(M);
    for (int m = 0; m < M; ++m) m_order[m] = m;
    auto stops = [&](int m) {
        return (data->obs_offsets[m + 1] - data->obs_offsets[m]) +
               (data->in_offsets ? data->in_offsets[m + 1] - data->in_offsets[m] : 0);
    };
    std::stable_sort(m_order.begin(), m_order.end(),
                     [&](int32_t x, int32_t y) { return stops(x) > stops(y); });
    const size_t sz[] = {(size_t)model->m.n_terms * sizeof(lik_ode_term), (size_t)U * 4,
                         (size_t)n_theta * V * 8, (size_t)(M + 1) * 4, (size_t)total * 8,
                         (size_t)total * 8, (size_t)M * 8, (size_t)M * U * 8,
                         data->in_offsets ? (size_t)(M + 1) * 4 : 0, (size_t)n_in * 8,
                         (size_t)n_in * 8, F * 8, F * 4, (size_t)n_theta * 8, (size_t)n_theta * 4,
                         F * 4, 4, (size_t)M * 4};
    const void *src[] = {model->m.terms, model->m.x0_param, theta, data->obs_offsets, data->t_obs,
                         data->y, data->t0, data->x0, data->in_offsets, data->t_in, data->u_in,
                         nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, m_order.data()};
    size_t bytes = 0;
    for (size_t v : sz) bytes += align256(v);
    char *dev = nullptr;
    hipError_t e = hipMalloc((void **)&dev, bytes + 256);
    if (e != hipSuccess) return fail(LIK_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    void *ptr[18];
    size_t off = 0;
    for (int k = 0; k < 18; ++k) {
        ptr[k] = sz[k] ? dev + off : nullptr;
        off += align256(sz[k]);
    }
    OdeArgs a;
    memset(&a, 0, sizeof(a));
    a.terms = (const lik_ode_term *)ptr[0];
    a.x0_param = (const int32_t *)ptr[1];
    a.U = U;
    a.V = V;
    a.n_terms = model->m.n_terms;
    a.obs_kind = model->m.obs_kind;
    a.obs_species = model->m.obs_species;
    a.obs_species2 = model->m.obs_kind == LIK_ODE_OBS_FRET ? model->m.obs_species2 : -1;
    a.sd_param = model->m.sd_param;
    a.sd_const = model->m.sd_const;
    for (int k = 0; k < 5; ++k) a.fret[k] = model->m.fret_param[k];
    a.theta = (const double *)ptr[2];
    a.n_theta = n_theta;
    a.M = M;
    a.obs_offsets = (const int32_t *)ptr[3];
    a.t_obs = (const double *)ptr[4];
    a.y = (const double *)ptr[5];
    a.t0 = (const double *)ptr[6];
    a.x0 = (const double *)ptr[7];
    a.in_offsets = (const int32_t *)ptr[8];
    a.t_in = (const double *)ptr[9];
    a.u_in = (const double *)ptr[10];
    a.rtol = rtol;
    a.atol = atol;
    a.max_steps = max_steps;
    a.tll = (double *)ptr[11];
    a.tst = (int32_t *)ptr[12];
    a.tsteps = (int32_t *)ptr[15];
    a.next = (unsigned int *)ptr[16];
    a.m_order = (const int32_t *)ptr[17];
    double *d_ll = (double *)ptr[13];
    int32_t *d_st = (int32_t *)ptr[14];
    hipFunction_t spec = nullptr;
    if (kernel != LIK_KERNEL_GENERIC) {
        std::string msg;
        spec = ode_spec_kernel(*model, &msg);
        if (!spec && kernel == LIK_KERNEL_SPECIALIZED) {
            (void)hipFree(dev);
            return fail(LIK_EDEVICE, "specialised ODE kernel unavailable: " + msg);
        }
    }
    hipStream_t s = nullptr;
    rc = LIK_OK;
    do {
        if ((e = hipStreamCreate(&s)) != hipSuccess) { rc = hip_fail(e, "hipStreamCreate"); break; }
        for (int k = 0; k < 18 && e == hipSuccess; ++k)
            if (sz[k] && src[k]) e = hipMemcpyAsync(ptr[k], src[k], sz[k], hipMemcpyHostToDevice, s);
        if (e != hipSuccess) { rc = hip_fail(e, "copy to device"); break; }
        if ((e = hipMemsetAsync(a.next, 0, 4, s)) != hipSuccess) { rc = hip_fail(e, "memset"); break; }
        // every lane takes pairs until none is left: as many workgroups as
        // can be resident at once (more would only find the counter spent)
        const unsigned lds = spec ? (unsigned)ode_par_lds(V) : 0u;
        const void *gen = U <= 4 ? (const void *)k_ode<4> : U <= 8 ? (const void *)k_ode<8>
                        : U <= 16 ? (const void *)k_ode<16> : (const void *)k_ode<32>;
        unsigned blocks = (unsigned)((F + 63) / 64);
        int per_cu = 0, cus = 0, dev_id = 0;
        const hipError_t eo = spec ? hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(
                                         &per_cu, spec, 64, lds)
                                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gen, 64, 0);
        if (eo == hipSuccess && per_cu > 0 && hipGetDevice(&dev_id) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) == hipSuccess &&
            cus > 0)
            blocks = std::min(blocks, (unsigned)(per_cu * cus));
        hipEvent_t t0 = timing_begin(s);  // timed as a propagation launch
        if (spec) {
            void *params[] = {(void *)&a};
            e = hipModuleLaunchKernel(spec, blocks, 1, 1, 64, 1, 1, lds, s, params, nullptr);
            if (e != hipSuccess) { rc = hip_fail(e, "ode launch"); break; }
        } else if (U <= 4) hipLaunchKernelGGL(k_ode<4>, dim3(blocks), dim3(64), 0, s, a);
        else if (U <= 8) hipLaunchKernelGGL(k_ode<8>, dim3(blocks), dim3(64), 0, s, a);
        else if (U <= 16) hipLaunchKernelGGL(k_ode<16>, dim3(blocks), dim3(64), 0, s, a);
        else hipLaunchKernelGGL(k_ode<32>, dim3(blocks), dim3(64), 0, s, a);
        if ((e = hipGetLastError()) != hipSuccess) { rc = hip_fail(e, "ode launch"); break; }
        timing_end_propagate(t0, s);
        hipLaunchKernelGGL(k_ode_finish, dim3((unsigned)((n_theta + 255) / 256)), dim3(256), 0, s,
                           a.tll, a.tst, n_theta, M, d_ll, d_st);
        if ((e = hipGetLastError()) != hipSuccess) { rc = hip_fail(e, "ode finish launch"); break; }
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

}  // extern "C"
