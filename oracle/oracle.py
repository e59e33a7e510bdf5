"""TEST INFRASTRUCTURE ONLY: ctypes binding of the CPU oracle (pf_oracle.c,
and ode_oracle.c for deterministic models).

The oracle is the plain CPU particle filter of Supplementary I (Algorithm
"Likelihood Approximation using particle filter") with Gillespie direct-method
propagation.  Only tests, the smoke check and the benchmark's CPU-baseline leg
may import this module; the GPU library never does.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "pf_oracle.c")
_SRC_ODE = os.path.join(_HERE, "ode_oracle.c")

OK, EVENT_CAP, COUNT_OVERFLOW, BAD_THETA = 0, 1, 2, 3
FP64, FP32_MIXED = 0, 1
OBS_GAUSSIAN, OBS_LOGNORMAL, OBS_FLUORESCENCE = 0, 1, 2


def build():
    """Compile the oracle: no fast-math, no FMA contraction (fma() explicit)."""
    cmd = ["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-pthread", "-o", _LIB_PATH, _SRC, _SRC_ODE, "-lm"]
    subprocess.run(cmd, check=True)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_species", ctypes.c_int32),
        ("n_reactions", ctypes.c_int32),
        ("reactant_orders", ctypes.c_void_p),
        ("stoich", ctypes.c_void_p),
        ("obs_kind", ctypes.c_int32),
        ("n_observed", ctypes.c_int32),
        ("observed", ctypes.c_void_p),
        ("sigma", ctypes.c_double),
        ("n_theta", ctypes.c_int32),
        ("theta", ctypes.c_void_p),
        ("theta_ids", ctypes.c_void_p),
        ("n_traj", ctypes.c_int32),
        ("obs_offsets", ctypes.c_void_p),
        ("t_obs", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("t0", ctypes.c_void_p),
        ("x0", ctypes.c_void_p),
        ("n_particles", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("precision", ctypes.c_int32),
        ("event_cap", ctypes.c_uint64),
        ("gain", ctypes.c_double),
        ("bg_mean", ctypes.c_double),
        ("bg_sd", ctypes.c_double),
        ("x0_hi", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
                os.path.getmtime(_SRC), os.path.getmtime(_SRC_ODE)):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, u32, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                                  ctypes.c_uint64, ctypes.c_double)
        L.orc_philox.argtypes = [vp, vp, vp]
        L.orc_log.argtypes = [dbl]
        L.orc_log.restype = dbl
        L.orc_exp.argtypes = [dbl]
        L.orc_exp.restype = dbl
        L.orc_logf.argtypes = [ctypes.c_float]
        L.orc_logf.restype = ctypes.c_float
        L.orc_propensities.argtypes = [vp, vp, vp, ctypes.c_int, vp]
        L.orc_resample.argtypes = [i32, vp, u64, vp]
        L.orc_resample_word.argtypes = [u64, u32, u32, u32]
        L.orc_resample_word.restype = u64
        L.orc_eval.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp]
        L.orc_eval.restype = ctypes.c_int
        L.orc_trace_filter.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_trace_filter.restype = ctypes.c_int
        L.orc_ssa_paths.argtypes = [vp, vp, u32, vp, dbl, dbl, i32, vp, vp, vp]
        L.orc_ssa_paths.restype = ctypes.c_int
        L.orc_ode_eval.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp]
        L.orc_ode_eval.restype = ctypes.c_int
        L.orc_ode_solve.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.orc_ode_solve.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class Problem:
    """Holds contiguous numpy copies of one batch and the C struct over them."""

    def __init__(self, reactant_orders, stoich, obs_kind, observed, sigma, theta,
                 trajectories, n_particles, seed, precision=FP64, event_cap=100_000_000,
                 theta_ids=None):
        self.orders = np.ascontiguousarray(reactant_orders, dtype=np.int32)
        self.stoich = np.ascontiguousarray(stoich, dtype=np.int32)
        R, U = self.orders.shape
        self.U, self.R = U, R
        self.observed = np.ascontiguousarray(observed, dtype=np.int32)
        self.theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, R))
        self.theta_ids = (None if theta_ids is None
                          else np.ascontiguousarray(theta_ids, dtype=np.uint32))
        P = len(self.observed)
        offs = [0]
        t_obs, ys, t0, x0, x0_hi = [], [], [], [], []
        for tr in trajectories:
            t_obs.append(np.asarray(tr["t_obs"], dtype=np.float64))
            ys.append(np.asarray(tr["y"], dtype=np.float64).reshape(-1, P))
            t0.append(float(tr.get("t0", 0.0)))
            x0.append(np.asarray(tr["x0"], dtype=np.int32))
            x0_hi.append(np.asarray(tr.get("x0_hi", tr["x0"]), dtype=np.int32))
            offs.append(offs[-1] + len(t_obs[-1]))
        random_start = any("x0_hi" in tr for tr in trajectories)
        self.offsets = np.array(offs, dtype=np.int32)
        self.t_obs = np.ascontiguousarray(np.concatenate(t_obs))
        self.y = np.ascontiguousarray(np.concatenate(ys))
        self.t0 = np.array(t0, dtype=np.float64)
        self.x0 = np.ascontiguousarray(np.stack(x0))
        self.x0_hi = np.ascontiguousarray(np.stack(x0_hi)) if random_start else None
        # sigma: the noise scale, or (sigma, gain, bg_mean, bg_sd) for the
        # fluorescence model
        sig = tuple(sigma) if isinstance(sigma, (tuple, list)) else (sigma, 0.0, 0.0, 0.0)
        self.H = int(n_particles)
        self.M = len(trajectories)
        self.n_theta = self.theta.shape[0]
        self.c = _Problem(
            U, R, _ptr(self.orders), _ptr(self.stoich), int(obs_kind), P,
            _ptr(self.observed), float(sig[0]), self.n_theta, _ptr(self.theta),
            _ptr(self.theta_ids), self.M, _ptr(self.offsets), _ptr(self.t_obs),
            _ptr(self.y), _ptr(self.t0), _ptr(self.x0), self.H, int(seed) & (2**64 - 1),
            int(precision), int(event_cap), float(sig[1]), float(sig[2]), float(sig[3]),
            _ptr(self.x0_hi))


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def log(x):
    return lib().orc_log(float(x))


def exp(d):
    return lib().orc_exp(float(d))


def logf(x):
    return lib().orc_logf(float(np.float32(x)))


def propensities(prob, c, x, precision=FP64):
    c = np.ascontiguousarray(c, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.int32)
    out = np.zeros(prob.R, dtype=np.float64)
    lib().orc_propensities(ctypes.byref(prob.c), c.ctypes.data, x.ctypes.data,
                           int(precision), out.ctypes.data)
    return out


def resample(e, w64):
    e = np.ascontiguousarray(e, dtype=np.float64)
    anc = np.zeros(len(e), dtype=np.int32)
    lib().orc_resample(len(e), e.ctypes.data, int(w64), anc.ctypes.data)
    return anc


def resample_word(seed, theta_id, traj, t):
    return lib().orc_resample_word(int(seed), int(theta_id), int(traj), int(t))


def evaluate(prob, nthreads=None, want_final_state=False):
    """Returns dict: loglik[n_theta], status[n_theta], filter_ll[F], events[F]
    (and final_state[F, U, H] if requested)."""
    if nthreads is None:
        nthreads = min(os.cpu_count() or 1, 16)
    F = prob.n_theta * prob.M
    ll = np.zeros(prob.n_theta, dtype=np.float64)
    st = np.zeros(prob.n_theta, dtype=np.int32)
    fll = np.zeros(max(F, 1), dtype=np.float64)
    fev = np.zeros(max(F, 1), dtype=np.uint64)
    fs = np.zeros((max(F, 1), prob.U, prob.H), dtype=np.int32) if want_final_state else None
    rc = lib().orc_eval(ctypes.byref(prob.c), int(nthreads), ll.ctypes.data, st.ctypes.data,
                        fll.ctypes.data, fev.ctypes.data, _ptr(fs))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    out = {"loglik": ll, "status": st, "filter_ll": fll[:F], "events": fev[:F]}
    if want_final_state:
        out["final_state"] = fs[:F]
    return out


def trace_filter(prob, i, m):
    """Full trace of filter (theta i, trajectory m): states [T,H,U], logw [T,H],
    ancestors [T,H], ll_inc [T], loglik, events, status."""
    T = int(prob.offsets[m + 1] - prob.offsets[m])
    H, U = prob.H, prob.U
    states = np.zeros((T, H, U), dtype=np.int32)
    logw = np.full((T, H), np.nan)
    anc = np.zeros((T, H), dtype=np.int32)
    inc = np.full(T, np.nan)
    ll = ctypes.c_double()
    ev = ctypes.c_uint64()
    st = lib().orc_trace_filter(ctypes.byref(prob.c), int(i), int(m), states.ctypes.data,
                                logw.ctypes.data, anc.ctypes.data, inc.ctypes.data,
                                ctypes.byref(ll), ctypes.byref(ev))
    return {"states": states, "logw": logw, "ancestors": anc, "ll_inc": inc,
            "loglik": ll.value, "events": ev.value, "status": st}


def ssa_paths(prob, c, x0, t_start, t_end, n_paths, theta_id=0, clocks=False):
    """n_paths independent direct-method SSA paths from x0 (no filtering):
    (final states, event counts, status), and with clocks=True each path's
    clock (time of its last event) after them."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    states = np.zeros((n_paths, prob.U), dtype=np.int32)
    ev = np.zeros(n_paths, dtype=np.uint64)
    clk = np.zeros(n_paths, dtype=np.float64)
    st = lib().orc_ssa_paths(ctypes.byref(prob.c), c.ctypes.data, int(theta_id),
                             x0.ctypes.data, float(t_start), float(t_end), int(n_paths),
                             states.ctypes.data, ev.ctypes.data, clk.ctypes.data)
    return (states, ev, st, clk) if clocks else (states, ev, st)


# -- deterministic models (ode_oracle.c) -------------------------------------

STEP_LIMIT, NONFINITE = 7, 8
ODE_SPECIES, ODE_SATURATING, ODE_HILL2, ODE_REPRESS2, ODE_INPUT = 0, 1, 2, 3, 4
ODE_OBS_SPECIES, ODE_OBS_FRET = 0, 1


class _OdeTerm(ctypes.Structure):
    _fields_ = [("frm", ctypes.c_int32), ("to", ctypes.c_int32), ("rate_param", ctypes.c_int32),
                ("n_factors", ctypes.c_int32), ("rate_scale", ctypes.c_double),
                ("kind", ctypes.c_int32 * 3), ("species", ctypes.c_int32 * 3),
                ("param", ctypes.c_int32 * 3)]


class _OdeProblem(ctypes.Structure):
    _fields_ = [("U", ctypes.c_int32), ("V", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("terms", ctypes.c_void_p), ("x0_param", ctypes.c_void_p),
                ("obs_kind", ctypes.c_int32), ("obs_species", ctypes.c_int32),
                ("obs_species2", ctypes.c_int32), ("sd_param", ctypes.c_int32),
                ("sd_const", ctypes.c_double), ("fret_param", ctypes.c_int32 * 5),
                ("n_theta", ctypes.c_int32), ("theta", ctypes.c_void_p),
                ("n_traj", ctypes.c_int32), ("obs_offsets", ctypes.c_void_p),
                ("t_obs", ctypes.c_void_p), ("y", ctypes.c_void_p), ("t0", ctypes.c_void_p),
                ("x0", ctypes.c_void_p), ("in_offsets", ctypes.c_void_p),
                ("t_in", ctypes.c_void_p), ("u_in", ctypes.c_void_p),
                ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("max_steps", ctypes.c_int32)]


class OdeProblem:
    """A deterministic batch.  model: dict with U, V, terms (list of dicts
    frm, to, rate_param, rate_scale, factors [(kind, species, param)]),
    x0_param [U], obs_kind, obs_species, obs_species2, sd_param, sd_const,
    fret_param [5].  trajectories: dicts t_obs, y, t0, x0 and optionally
    t_in, u_in (piecewise-constant input)."""

    def __init__(self, model, theta, trajectories, rtol=1e-6, atol=1e-9, max_steps=100000):
        U, V = int(model["U"]), int(model["V"])
        terms = model["terms"]
        self.terms = (_OdeTerm * len(terms))()
        for k, t in enumerate(terms):
            T = self.terms[k]
            T.frm, T.to = int(t.get("frm", -1)), int(t.get("to", -1))
            T.rate_param = int(t.get("rate_param", -1))
            T.rate_scale = float(t.get("rate_scale", 1.0))
            fs = t.get("factors", [])
            T.n_factors = len(fs)
            for j, (kind, sp, par) in enumerate(fs):
                T.kind[j], T.species[j], T.param[j] = int(kind), int(sp), int(par)
        self.x0_param = np.ascontiguousarray(model.get("x0_param", [-1] * U), dtype=np.int32)
        self.theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, V))
        offs, t_obs, ys, t0, x0, ioff, tin, uin = [0], [], [], [], [], [0], [], []
        for tr in trajectories:
            t_obs.append(np.asarray(tr["t_obs"], np.float64))
            ys.append(np.asarray(tr["y"], np.float64).ravel())
            t0.append(float(tr.get("t0", 0.0)))
            x0.append(np.asarray(tr.get("x0", np.zeros(U)), np.float64))
            offs.append(offs[-1] + len(t_obs[-1]))
            tin.append(np.asarray(tr.get("t_in", []), np.float64))
            uin.append(np.asarray(tr.get("u_in", []), np.float64))
            ioff.append(ioff[-1] + len(tin[-1]))
        self.offsets = np.array(offs, np.int32)
        self.t_obs = np.ascontiguousarray(np.concatenate(t_obs))
        self.y = np.ascontiguousarray(np.concatenate(ys))
        self.t0 = np.array(t0, np.float64)
        self.x0 = np.ascontiguousarray(np.stack(x0))
        self.in_offsets = np.array(ioff, np.int32)
        self.t_in = np.ascontiguousarray(np.concatenate(tin)) if ioff[-1] else np.zeros(1)
        self.u_in = np.ascontiguousarray(np.concatenate(uin)) if ioff[-1] else np.zeros(1)
        self.n_theta, self.M, self.U = self.theta.shape[0], len(trajectories), U
        fret = (ctypes.c_int32 * 5)(*[int(v) for v in model.get("fret_param", [0] * 5)])
        self.c = _OdeProblem(
            U, V, len(terms), ctypes.addressof(self.terms), _ptr(self.x0_param),
            int(model.get("obs_kind", 0)), int(model.get("obs_species", 0)),
            int(model.get("obs_species2", 0)), int(model.get("sd_param", -1)),
            float(model.get("sd_const", 1.0)), fret, self.n_theta, _ptr(self.theta), self.M,
            _ptr(self.offsets), _ptr(self.t_obs), _ptr(self.y), _ptr(self.t0), _ptr(self.x0),
            _ptr(self.in_offsets) if ioff[-1] else None, _ptr(self.t_in), _ptr(self.u_in),
            float(rtol), float(atol), int(max_steps))


def ode_eval(prob, nthreads=None):
    """dict loglik [n_theta], status [n_theta], traj_ll [F], traj_status [F]."""
    if nthreads is None:
        nthreads = min(os.cpu_count() or 1, 16)
    F = prob.n_theta * prob.M
    ll = np.zeros(max(prob.n_theta, 1))
    st = np.zeros(max(prob.n_theta, 1), np.int32)
    tll = np.zeros(max(F, 1))
    tst = np.zeros(max(F, 1), np.int32)
    tsteps = np.zeros(max(F, 1), np.int32)
    if lib().orc_ode_eval(ctypes.byref(prob.c), int(nthreads), ll.ctypes.data, st.ctypes.data,
                          tll.ctypes.data, tst.ctypes.data, tsteps.ctypes.data) != 0:
        raise ValueError("oracle rejected the problem")
    return {"loglik": ll[:prob.n_theta], "status": st[:prob.n_theta], "traj_ll": tll[:F],
            "traj_status": tst[:F], "traj_steps": tsteps[:F]}


def ode_solve(prob, i, m):
    """(states [T, U] at the observation times, step attempts, loglik, status)."""
    T = int(prob.offsets[m + 1] - prob.offsets[m])
    states = np.zeros((T, prob.U))
    steps = ctypes.c_int32()
    ll = ctypes.c_double()
    st = lib().orc_ode_solve(ctypes.byref(prob.c), int(i), int(m), states.ctypes.data,
                             ctypes.byref(steps), ctypes.byref(ll))
    return states, steps.value, ll.value, st
