"""Pins of the oracle's deterministic-model likelihood (Sec. "Chemical
Reaction Networks", deterministic formulation; Results, deterministic models;
Supplementary "Egf-Ras-Raf-Mek-Erk model").

* closed forms: immigration-death rate equations (exponential relaxation),
  Michaelis-Menten degradation (implicit solution, root-found by scipy), an
  input-driven production with a piecewise-constant input (piecewise
  exponential relaxation through the breakpoints), and pure input-driven
  production, which a Runge-Kutta step integrates exactly between
  breakpoints (so its error stays at rounding level whatever the tolerance);
* a network with every rate-law factor against scipy's DOP853 at tight
  tolerances, integrated piece by piece between breakpoints;
* the log-likelihood is the normal log-density of the observations around
  the solution (scipy), for a species read-out and the FRET ratio;
* the solver's error falls with its tolerance; statuses (bad parameters, step
  limit, blow-up).
"""
import math

import numpy as np
import pytest
from scipy import optimize, stats
from scipy.integrate import solve_ivp

SP, SAT, HILL, REP, INP = 0, 1, 2, 3, 4


def imm_death_model(sd=0.5):
    # 0 -> X at theta0, X -> 0 at theta1 * X
    return {"U": 1, "V": 2, "terms": [{"to": 0, "rate_param": 0},
                                      {"frm": 0, "rate_param": 1, "factors": [(SP, 0, 0)]}],
            "x0_param": [-1], "obs_kind": 0, "obs_species": 0, "sd_param": -1, "sd_const": sd}


def test_immigration_death_closed_form(orc):
    k1, k2, x0 = 7.0, 0.4, 2.0
    t = np.linspace(0.5, 12.0, 24)
    exact = k1 / k2 + (x0 - k1 / k2) * np.exp(-k2 * t)
    y = exact + np.random.default_rng(0).normal(0, 0.5, len(t))
    P = orc.OdeProblem(imm_death_model(), [[k1, k2]], [{"t_obs": t, "y": y, "x0": [x0]}],
                       rtol=1e-11, atol=1e-12)
    states, steps, ll, st = orc.ode_solve(P, 0, 0)
    assert st == 0 and steps > 10
    assert np.allclose(states[:, 0], exact, rtol=1e-9, atol=0)
    want = stats.norm.logpdf(y, exact, 0.5).sum()
    assert ll == pytest.approx(want, rel=1e-9)
    assert orc.ode_eval(P)["loglik"][0] == ll


def test_michaelis_menten_degradation(orc):
    # x' = -V x / (K + x): K log(x / x0) + (x - x0) = -V t
    V, K, x0 = 3.0, 2.0, 10.0
    model = {"U": 1, "V": 2, "terms": [{"frm": 0, "rate_param": 0, "factors": [(SAT, 0, 1)]}],
             "x0_param": [-1], "sd_const": 1.0}
    t = np.array([0.3, 1.0, 2.0, 3.5, 5.0])
    P = orc.OdeProblem(model, [[V, K]], [{"t_obs": t, "y": np.zeros(5), "x0": [x0]}],
                       rtol=1e-11, atol=1e-13)
    states, _, _, st = orc.ode_solve(P, 0, 0)
    exact = [optimize.brentq(lambda x: K * math.log(x / x0) + (x - x0) + V * tt, 1e-12, x0,
                             xtol=1e-15) for tt in t]
    assert st == 0
    assert np.allclose(states[:, 0], exact, rtol=1e-8)


def test_piecewise_input_relaxation(orc):
    # x' = k u(t) - g x, u switching at breakpoints (and zero before the first)
    k, g, x0 = 2.0, 0.5, 1.0
    t_in, u_in = np.array([1.0, 2.5, 4.0]), np.array([3.0, 0.0, 1.5])
    model = {"U": 1, "V": 2, "terms": [{"to": 0, "rate_param": 0, "factors": [(INP, 0, 0)]},
                                       {"frm": 0, "rate_param": 1, "factors": [(SP, 0, 0)]}],
             "x0_param": [-1], "sd_const": 1.0}
    t = np.array([0.5, 1.0, 2.0, 3.0, 4.0, 6.0])

    def exact(tt):
        x, tc, u = x0, 0.0, 0.0
        for tb, ub in zip(np.r_[t_in, np.inf], np.r_[u_in, 0.0]):
            te = min(tb, tt)
            x = k * u / g + (x - k * u / g) * math.exp(-g * (te - tc))
            if tt <= tb:
                return x
            tc, u = tb, ub
        return x
    P = orc.OdeProblem(model, [[k, g]], [{"t_obs": t, "y": np.zeros(6), "x0": [x0],
                                          "t_in": t_in, "u_in": u_in}], rtol=1e-11, atol=1e-13)
    states, _, _, st = orc.ode_solve(P, 0, 0)
    assert st == 0
    assert np.allclose(states[:, 0], [exact(tt) for tt in t], rtol=1e-9)


def test_input_driven_production_is_exact_between_breakpoints(orc):
    # x' = k u(t) with u piecewise constant: between breakpoints the right-hand
    # side is constant, every stage of an explicit Runge-Kutta step equals it
    # and the step is exact, so x(t) = x0 + k * integral of u to rounding, at
    # any tolerance.  A step that carried the first stage over from before a
    # breakpoint (the old input's slope) would be accepted once its error
    # estimate fell under the loose tolerance, leaving an error of that size.
    k, x0 = 1.7, 3.0
    t_in, u_in = np.array([0.7, 1.9, 2.2, 4.1]), np.array([5.0, 0.25, 9.0, 2.0])
    model = {"U": 1, "V": 1, "terms": [{"to": 0, "rate_param": 0, "factors": [(INP, 0, 0)]}],
             "x0_param": [-1], "sd_const": 1.0}
    t = np.array([0.5, 1.0, 2.0, 2.3, 3.0, 4.1, 5.0, 7.5])

    def exact(tt):
        area, tc, u = 0.0, 0.0, 0.0
        for tb, ub in zip(np.r_[t_in, np.inf], np.r_[u_in, 0.0]):
            te = min(tb, tt)
            area += u * (te - tc)
            if tt <= tb:
                return x0 + k * area
            tc, u = tb, ub
        return x0 + k * area
    for rtol, atol in ((1e-4, 1e-4), (1e-6, 1e-6)):
        P = orc.OdeProblem(model, [[k]], [{"t_obs": t, "y": np.zeros(len(t)), "x0": [x0],
                                           "t_in": t_in, "u_in": u_in}], rtol=rtol, atol=atol)
        states, steps, _, st = orc.ode_solve(P, 0, 0)
        assert st == 0
        want = np.array([exact(tt) for tt in t])
        assert np.max(np.abs(states[:, 0] - want)) <= 1e-12 * np.max(np.abs(want)), \
            (rtol, states[:, 0] - want)


def every_factor_model():
    """Four species with every factor kind: A -> A* (k0 u A/(K1 + A)),
    A* -> A (k2 A*), B produced at k3 K4/(K4 + A*^2), B -> 0 (k5 B),
    C produced at k6 B^2/(K7 + B^2), C -> A (k8 C)."""
    terms = [{"frm": 0, "to": 1, "rate_param": 0, "factors": [(INP, 0, 0), (SAT, 0, 1)]},
             {"frm": 1, "to": 0, "rate_param": 2, "factors": [(SP, 1, 0)]},
             {"to": 2, "rate_param": 3, "factors": [(REP, 1, 4)]},
             {"frm": 2, "rate_param": 5, "factors": [(SP, 2, 0)]},
             {"to": 3, "rate_param": 6, "rate_scale": 0.5, "factors": [(HILL, 2, 7)]},
             {"frm": 3, "to": 0, "rate_param": 8, "factors": [(SP, 3, 0)]}]
    return {"U": 4, "V": 10, "terms": terms, "x0_param": [9, -1, -1, -1], "obs_kind": 1,
            "obs_species": 1, "obs_species2": 0, "sd_param": -1, "sd_const": 0.05,
            "fret_param": [4, 5, 6, 7, 8]}


def every_factor_rhs(th, u):
    def f(t, x):
        A, As, B, C = x
        v = [th[0] * u * A / (th[1] + A), th[2] * As, th[3] * th[4] / (th[4] + As * As),
             th[5] * B, 0.5 * th[6] * B * B / (th[7] + B * B), th[8] * C]
        return [-v[0] + v[1] + v[5], v[0] - v[1], v[2] - v[3], v[4] - v[5]]
    return f


def test_every_factor_against_dop853_and_fret_density(orc):
    th = np.array([1.3, 0.8, 0.4, 2.0, 0.3, 0.7, 1.1, 0.5, 0.2, 2.5])
    x0 = [0.0, 0.0, 0.4, 0.1]          # species 0 from theta[9]
    t = np.linspace(0.4, 8.0, 20)
    t_in, u_in = np.array([0.0, 3.0, 5.0]), np.array([1.0, 0.2, 2.0])
    y = np.random.default_rng(1).normal(1.0, 0.05, len(t))
    P = orc.OdeProblem(every_factor_model(), [th], [{"t_obs": t, "y": y, "x0": x0,
                                                     "t_in": t_in, "u_in": u_in}],
                       rtol=1e-11, atol=1e-13)
    states, _, ll, st = orc.ode_solve(P, 0, 0)
    assert st == 0
    # reference: DOP853 piece by piece
    x, tc, ref = [th[9]] + x0[1:], 0.0, []
    edges = list(t_in[1:]) + [np.inf]
    us = list(u_in)
    for k, (te, uu) in enumerate(zip(edges, us)):
        ts = [tt for tt in t if tc < tt <= te]
        end = min(te, t[-1])
        if end <= tc:
            break
        sol = solve_ivp(every_factor_rhs(th, uu), (tc, end), x, method="DOP853", rtol=1e-13,
                        atol=1e-15, t_eval=ts, dense_output=True)
        ref += list(sol.y.T)
        x, tc = list(sol.sol(end)), end
    ref = np.array(ref)
    assert np.allclose(states, ref, rtol=1e-8, atol=1e-11)
    # FRET read-out: lambda (E fAA A* / ((A + (1 - E) A*) fDD) + bg)
    lam, bg, E, fAA, fDD = th[4], th[5], th[6], th[7], th[8]
    As, A = ref[:, 1], ref[:, 0]
    g = lam * (E * fAA * As / ((A + (1 - E) * As) * fDD) + bg)
    assert ll == pytest.approx(stats.norm.logpdf(y, g, 0.05).sum(), rel=1e-7)


def test_error_follows_the_tolerance(orc):
    k1, k2, x0 = 7.0, 0.4, 2.0
    t = np.array([10.0])
    exact = k1 / k2 + (x0 - k1 / k2) * math.exp(-k2 * 10.0)
    errs = []
    for rtol in (1e-4, 1e-6, 1e-8, 1e-10):
        P = orc.OdeProblem(imm_death_model(), [[k1, k2]], [{"t_obs": t, "y": [0.0], "x0": [x0]}],
                           rtol=rtol, atol=rtol * 1e-3)
        errs.append(abs(orc.ode_solve(P, 0, 0)[0][0, 0] - exact) / exact)
    assert all(e < 50 * r for e, r in zip(errs, (1e-4, 1e-6, 1e-8, 1e-10)))
    assert errs[0] > errs[1] > errs[2] > errs[3]


def test_statuses(orc):
    t = np.array([1.0, 2.0])
    tr = {"t_obs": t, "y": [0.0, 0.0], "x0": [1.0]}
    P = orc.OdeProblem(imm_death_model(), [[1.0, 0.5], [-1.0, 0.5], [np.nan, 0.5], [1.0, np.inf]],
                       [tr])
    assert list(orc.ode_eval(P)["status"]) == [0, 3, 3, 3]
    # sd taken from theta: zero is a bad parameter vector
    m = dict(imm_death_model(), V=3, sd_param=2)
    assert list(orc.ode_eval(orc.OdeProblem(m, [[1.0, 0.5, 0.0], [1.0, 0.5, 0.1]], [tr]))
                ["status"]) == [3, 0]
    # step limit
    P = orc.OdeProblem(imm_death_model(), [[1.0, 0.5]], [tr], max_steps=3)
    assert orc.ode_eval(P)["status"][0] == 7
    # blow-up: x' = x^2 from 1 reaches infinity at t = 1
    blow = {"U": 1, "V": 1, "terms": [{"to": 0, "rate_param": 0, "factors": [(SP, 0, 0), (SP, 0, 0)]}],
            "x0_param": [-1], "sd_const": 1.0}
    out = orc.ode_eval(orc.OdeProblem(blow, [[1.0]], [{"t_obs": [0.5, 2.0], "y": [0.0, 0.0],
                                                        "x0": [1.0]}]))
    assert out["status"][0] in (7, 8) and np.isnan(out["loglik"][0])


def test_sum_over_trajectories_in_order(orc):
    t = np.array([1.0, 3.0])
    trs = [{"t_obs": t, "y": [2.0, 3.0], "x0": [1.0]}, {"t_obs": t + 0.5, "y": [4.0, 1.0], "x0": [5.0]}]
    P = orc.OdeProblem(imm_death_model(), [[2.0, 0.3], [1.0, 0.9]], trs)
    out = orc.ode_eval(P)
    for i in range(2):
        assert out["loglik"][i] == out["traj_ll"][2 * i] + out["traj_ll"][2 * i + 1]
