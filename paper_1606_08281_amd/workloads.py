"""Seeded synthetic workloads: reaction networks, parameter draws, observed data.

This module is shared by the tests, the benchmark and the CPU oracle's callers.
It holds none of the likelihood arithmetic: it defines networks (reactant
orders p_ru and net changes q_ru - p_ru, Sec. "Chemical Reaction Networks"),
draws rate vectors from log-uniform priors with numpy's PCG64, and simulates
observation trajectories with Gillespie's *first-reaction* method under numpy's
generator, then adds measurement noise (Sec. "General Task": Y ~ p(.|X, theta)).
The likelihood path uses the direct method with Philox streams; the data
simulator shares neither algorithm nor random numbers with it.

Workloads:
  * immigration-death (the birth-death model of the Results section, with the
    degradation rate and prior box of the benchmark configuration): 0 -> X
    (k1 = 10), X -> 0 (k2 = 0.1), X(0) = 0, y = X + N(0, 2^2) at t = 5..100.
  * telegraph gene expression (the RNA model of Supplementary II extended by
    translation and protein decay): G_off <-> G_on, G_on -> G_on + M, M -> 0,
    M -> M + P, P -> 0; log y = log P + N(0, 0.1^2) at t = 2, 4, ..., 100.
  * a seeded random mass-action network with 20 species and 40 reactions.
  * Lac-Gfp (Supplementary "LacGfp example"): 9 species, 18 mass-action
    reactions, 18 parameters (the LACI degradation rate rises linearly with
    the inducer, theta_4 + theta_5 [IPTG]; GFP and mature GFP share the
    degradation rate theta_17), random initial counts, and fluorescence of
    mature GFP observed with per-molecule normal signal plus background.
"""
import functools
import math

import numpy as np

SEED_NET, SEED_DATA, SEED_NOISE, SEED_THETA, SEED_FILTER = 1, 2, 3, 4, 5

OBS_GAUSSIAN, OBS_LOGNORMAL, OBS_FLUORESCENCE = 0, 1, 2


class Network:
    """Reactant orders p[r, u] and net changes nu[r, u] = q[r, u] - p[r, u]."""

    def __init__(self, name, species, orders, stoich, reaction_names=None):
        self.name = name
        self.species = list(species)
        self.orders = np.asarray(orders, dtype=np.int32)
        self.stoich = np.asarray(stoich, dtype=np.int32)
        self.R, self.U = self.orders.shape
        self.reaction_names = reaction_names or [f"R{r}" for r in range(self.R)]

    def propensity_factors(self, X):
        """propensity_factor for every row of X [K, U]: [K, R]."""
        self.propensity_factor(X[0])   # builds the index tables
        X = np.asarray(X, dtype=np.float64)
        a = X[:, self._first]
        h = np.where(self._order == 0, 1.0, a)
        h = np.where(self._homo, a * (a - 1.0) / 2.0, h)
        return np.where(self._second >= 0, h * X[:, np.maximum(self._second, 0)], h)

    def propensity_factor(self, x):
        """Mass-action combinatorial factors prod_u C(x_u, p_ru) (float64):
        products of exact integers, so any evaluation order gives the same
        values."""
        if not hasattr(self, "_first"):
            first = np.zeros(self.R, dtype=np.int64)
            second = np.full(self.R, -1, dtype=np.int64)
            homo = np.zeros(self.R, dtype=bool)
            order = self.orders.sum(axis=1)
            for r in range(self.R):
                us = np.nonzero(self.orders[r])[0]
                if len(us):
                    first[r] = us[0]
                if len(us) == 2:
                    second[r] = us[1]
                homo[r] = len(us) == 1 and self.orders[r, us[0]] == 2
            self._first, self._second, self._homo, self._order = first, second, homo, order
        x = np.asarray(x, dtype=np.float64)
        a = x[self._first]
        h = np.where(self._order == 0, 1.0, a)
        h = np.where(self._homo, a * (a - 1.0) / 2.0, h)
        two = self._second >= 0
        return np.where(two, h * x[np.maximum(self._second, 0)], h)


def immigration_death():
    return Network("immigration-death", ["X"], [[0], [1]], [[1], [-1]],
                   ["0->X", "X->0"])


def telegraph():
    # species: G_off, G_on, M, P
    orders = [[1, 0, 0, 0],   # G_off -> G_on       k_on
              [0, 1, 0, 0],   # G_on -> G_off       k_off
              [0, 1, 0, 0],   # G_on -> G_on + M    k_m
              [0, 0, 1, 0],   # M -> 0              gamma_m
              [0, 0, 1, 0],   # M -> M + P          k_p
              [0, 0, 0, 1]]   # P -> 0              gamma_p
    stoich = [[-1, 1, 0, 0],
              [1, -1, 0, 0],
              [0, 0, 1, 0],
              [0, 0, -1, 0],
              [0, 0, 0, 1],
              [0, 0, 0, -1]]
    return Network("telegraph", ["G_off", "G_on", "M", "P"], orders, stoich,
                   ["k_on", "k_off", "k_m", "gamma_m", "k_p", "gamma_p"])


TELEGRAPH_TRUTH = np.array([0.05, 0.05, 10.0, 1.0, 2.0, 0.1])
TELEGRAPH_X0 = np.array([0, 1, 10, 100], dtype=np.int32)
IMMDEATH_TRUTH = np.array([10.0, 0.1])


def first_reaction_path(net, c, x0, t_points, rng, max_events=50_000_000):
    """States at t_points of one path simulated by the first-reaction method:
    every reaction draws its own exponential waiting time and the earliest
    fires.  Returns an int64 array [len(t_points), U]."""
    x = np.array(x0, dtype=np.int64)
    t = 0.0
    out = np.zeros((len(t_points), net.U), dtype=np.int64)
    k = 0
    events = 0
    while k < len(t_points):
        a = c * net.propensity_factor(x)
        pos = a > 0
        if not pos.any():
            while k < len(t_points):
                out[k] = x
                k += 1
            break
        waits = np.full(net.R, np.inf)
        waits[pos] = rng.exponential(1.0 / a[pos])
        r = int(np.argmin(waits))
        t_next = t + waits[r]
        while k < len(t_points) and t_points[k] < t_next:
            out[k] = x
            k += 1
        x = x + net.stoich[r]
        t = t_next
        events += 1
        if events > max_events:
            raise RuntimeError("data simulation exceeded its event budget")
    return out


def first_reaction_paths(net, c, x0s, t_points, rng, max_events=50_000_000):
    """first_reaction_path for several paths at once (rows of x0s), stepped
    together: every unfinished path fires its next reaction per step.
    Returns int64 [K, len(t_points), U]."""
    X = np.array(x0s, dtype=np.int64)
    K = X.shape[0]
    t = np.zeros(K)
    k = np.zeros(K, dtype=np.int64)
    T = len(t_points)
    tp = np.append(np.asarray(t_points, dtype=np.float64), np.inf)
    out = np.zeros((K, T, net.U), dtype=np.int64)
    nu = net.stoich.astype(np.int64)
    live = np.arange(K)
    steps = 0
    while len(live):
        a = c * net.propensity_factors(X[live])
        pos = a > 0
        with np.errstate(divide="ignore"):
            waits = np.where(pos, rng.exponential(1.0, a.shape) / np.where(pos, a, 1.0), np.inf)
        r = np.argmin(waits, axis=1)
        t_next = t[live] + waits[np.arange(len(live)), r]
        # observations passed before the next event keep the current counts
        for i in np.nonzero(tp[k[live]] < t_next)[0]:
            p = live[i]
            while tp[k[p]] < t_next[i]:
                out[p, k[p]] = X[p]
                k[p] += 1
        fire = np.isfinite(t_next)
        X[live[fire]] += nu[r[fire]]
        t[live] = t_next
        live = live[k[live] < T]
        steps += 1
        if steps > max_events:
            raise RuntimeError("data simulation exceeded its event budget")
    return out


def log_uniform(rng, lo, hi, n):
    lo = np.broadcast_to(np.asarray(lo, dtype=np.float64), (len(np.atleast_1d(lo)),))
    hi = np.broadcast_to(np.asarray(hi, dtype=np.float64), lo.shape)
    u = rng.random((n, lo.shape[0]))
    return np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))


class Workload:
    """One batch: network, observation model, theta[n_theta, R], trajectories."""

    def __init__(self, name, net, obs_kind, observed, sigma, theta, trajectories,
                 n_particles, seed=SEED_FILTER, truth=None):
        self.name = name
        self.net = net
        self.obs_kind = obs_kind
        self.observed = list(observed)
        # the noise scale, or (sigma, gain, bg_mean, bg_sd) for the fluorescence model
        self.sigma = tuple(float(v) for v in sigma) if isinstance(sigma, (tuple, list)) \
            else float(sigma)
        self.theta = np.ascontiguousarray(theta, dtype=np.float64)
        self.trajectories = trajectories
        self.n_particles = int(n_particles)
        self.seed = int(seed)
        self.truth = truth

    @property
    def n_theta(self):
        return self.theta.shape[0]

    @property
    def n_traj(self):
        return len(self.trajectories)

    def subset(self, theta_idx, traj_idx=None, n_particles=None):
        """A smaller batch; theta stream ids are kept via theta_ids."""
        trajs = (self.trajectories if traj_idx is None
                 else [self.trajectories[m] for m in traj_idx])
        w = Workload(self.name, self.net, self.obs_kind, self.observed, self.sigma,
                     self.theta[np.asarray(theta_idx)], trajs,
                     n_particles or self.n_particles, self.seed, self.truth)
        w.theta_ids = np.asarray(theta_idx, dtype=np.uint32)
        return w

    theta_ids = None


def immigration_death_workload(n_theta=64, n_particles=256, t_obs=None, seed_data=SEED_DATA):
    """64 rate vectors log-uniform on [1e-2, 1e2]^2, one trajectory observed at
    t = 5, 10, ..., 100 with Gaussian noise sd 2, X(0) = 0."""
    net = immigration_death()
    t_obs = np.arange(5.0, 100.0 + 1e-9, 5.0) if t_obs is None else np.asarray(t_obs, float)
    rng = np.random.Generator(np.random.PCG64(seed_data))
    states = first_reaction_path(net, IMMDEATH_TRUTH, [0], t_obs, rng)
    noise = np.random.Generator(np.random.PCG64(SEED_NOISE)).normal(0.0, 2.0, len(t_obs))
    y = states[:, 0] + noise
    theta = log_uniform(np.random.Generator(np.random.PCG64(SEED_THETA)),
                        [1e-2, 1e-2], [1e2, 1e2], n_theta)
    traj = {"t_obs": t_obs, "y": y.reshape(-1, 1), "t0": 0.0, "x0": np.array([0], np.int32),
            "x_true": states}
    return Workload("immigration-death", net, OBS_GAUSSIAN, [0], 2.0, theta, [traj],
                    n_particles, truth=IMMDEATH_TRUTH)


def telegraph_workload(n_theta=1024, n_traj=10, n_obs=50, n_particles=1000, dt=2.0):
    """Telegraph model: n_traj trajectories of P observed at dt, 2dt, ... with
    log-normal noise sigma 0.1; theta log-uniform on [truth/10, 10 truth]."""
    net = telegraph()
    t_obs = dt * np.arange(1, n_obs + 1, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(SEED_DATA))
    nrng = np.random.Generator(np.random.PCG64(SEED_NOISE))
    trajs = []
    while len(trajs) < n_traj:
        states = first_reaction_path(net, TELEGRAPH_TRUTH, TELEGRAPH_X0, t_obs, rng)
        if (states[:, 3] <= 0).any():
            continue  # a zero protein count has no log-normal observation
        y = states[:, 3] * np.exp(nrng.normal(0.0, 0.1, n_obs))
        trajs.append({"t_obs": t_obs, "y": y.reshape(-1, 1), "t0": 0.0,
                      "x0": TELEGRAPH_X0.copy(), "x_true": states})
    theta = log_uniform(np.random.Generator(np.random.PCG64(SEED_THETA)),
                        TELEGRAPH_TRUTH / 10.0, TELEGRAPH_TRUTH * 10.0, n_theta)
    return Workload("telegraph", net, OBS_LOGNORMAL, [3], 0.1, theta, trajs,
                    n_particles, truth=TELEGRAPH_TRUTH)


def random_network(n_species=20, n_reactions=40, seed=SEED_NET):
    """Seeded random mass-action network: orders 0-2, net changes in -2..2,
    net change >= -order for every reactant (nothing consumed that is not
    used), zeroth-order reactions only create, and every reaction of order
    >= 1 conserves or destroys molecules overall (no autocatalytic blow-up)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U, R = n_species, n_reactions
    orders = np.zeros((R, U), dtype=np.int32)
    stoich = np.zeros((R, U), dtype=np.int32)
    for r in range(R):
        order = int(rng.choice([0, 1, 1, 1, 2, 2])) if r >= 4 else (0 if r < 2 else 1)
        if order == 1:
            orders[r, rng.integers(U)] = 1
        elif order == 2:
            if rng.random() < 0.3:
                orders[r, rng.integers(U)] = 2
            else:
                a, b = rng.choice(U, size=2, replace=False)
                orders[r, a] = orders[r, b] = 1
        while True:
            nu = np.zeros(U, dtype=np.int32)
            for u in np.nonzero(orders[r])[0]:
                nu[u] = -rng.integers(0, orders[r, u] + 1)   # consume some of each reactant
            for _ in range(int(rng.integers(1, 3))):           # and produce one or two species
                nu[rng.integers(U)] += int(rng.integers(1, 3))
            nu = np.clip(nu, -2, 2)
            nu = np.maximum(nu, -orders[r])
            if order == 0 and (nu < 0).any():
                continue
            if order >= 1 and nu.sum() > 0:
                continue
            if not nu.any():
                continue
            break
        stoich[r] = nu
    # every species needs a way out, otherwise zeroth-order inflow accumulates
    for u in range(U):
        if not ((stoich[:, u] < 0)).any():
            r = 4 + u % (R - 4)
            orders[r] = 0
            orders[r, u] = 1
            stoich[r] = 0
            stoich[r, u] = -1
    return Network("random-20x40", [f"S{u}" for u in range(U)], orders, stoich)


def tau_leap_path(net, c, x0, t_points, rng, n_sub=200):
    """Approximate path for synthetic data only: Poisson tau-leaping with
    n_sub sub-steps per observation interval, counts clipped at zero."""
    x = np.array(x0, dtype=np.int64)
    out = np.zeros((len(t_points), net.U), dtype=np.int64)
    t_prev = 0.0
    for k, t in enumerate(t_points):
        tau = (t - t_prev) / n_sub
        for _ in range(n_sub):
            a = c * net.propensity_factor(x)
            fires = rng.poisson(np.maximum(a, 0.0) * tau)
            x = np.maximum(x + fires @ net.stoich, 0)
        out[k] = x
        t_prev = t
    return out


def mean_field_path(net, c, x0, t_points):
    """The network's rate equations dx/dt = sum_r nu_r c_r h_r(x) (mass-action
    factors of continuous counts) from x0, solved by scipy's stiff LSODA, at
    t_points: a deterministic synthetic data path where an exact stochastic
    one is too slow to simulate (float64 [len(t_points), U], clipped at 0)."""
    from scipy.integrate import solve_ivp
    nu = net.stoich.astype(np.float64)

    def rhs(_, x):
        return (c * net.propensity_factor(np.maximum(x, 0.0))) @ nu

    sol = solve_ivp(rhs, (0.0, float(t_points[-1])), np.asarray(x0, dtype=np.float64),
                    method="LSODA", t_eval=np.asarray(t_points, dtype=np.float64),
                    rtol=1e-7, atol=1e-6)
    if not sol.success:
        raise RuntimeError("mean-field data path: " + sol.message)
    return np.maximum(sol.y.T, 0.0)


def random_network_x0(net):
    return np.random.Generator(np.random.PCG64(SEED_NET + 100)).poisson(100, net.U).astype(np.int32)


def random_network_theta(net, n_theta):
    return log_uniform(np.random.Generator(np.random.PCG64(SEED_THETA)),
                       np.full(net.R, 1e-3), np.full(net.R, 1.0), n_theta)


# Observation interval at which the median rate vector of the 20 x 40
# network's prior realises 1e4 direct-method events per particle per interval
# (tests/helpers/calibrate_random_interval.py: exact SSA paths of 256 prior
# draws from x0 over 100 intervals; median 9,973, mean 11,673, p99 34,696
# events per interval).  The network relaxes fast from x0, so this interval
# is ~4,200 times the one at which the median rate vector's total propensity
# at x0 gives 1e4 events.
RANDOM_DT_1E4 = 2797.88


def random_network_workload(n_theta=4096, n_particles=512, n_obs=100, events_per_interval=1e4,
                            dt=None):
    """20 species / 40 reactions, x0 ~ Poisson(100) once, rates log-uniform on
    [1e-3, 1]; Gaussian noise sigma 10 on species 0 and 1.

    dt None: the observation interval is set so that the median over the
    drawn rate vectors of the total propensity *at x0* times the interval is
    `events_per_interval` (the network then relaxes and realises far fewer,
    ~36 events per particle per interval at 1e4); data from a tau-leaped path
    at rates 10^-1.5.  dt given (RANDOM_DT_1E4 for ~1e4 realised events per
    particle per interval): that interval, and data from the rate equations'
    mean-field path at rates 10^-1.5 (tau-leaping is unstable at that
    interval, and an exact path takes millions of events)."""
    net = random_network()
    x0 = random_network_x0(net)
    theta = random_network_theta(net, n_theta)
    truth = np.full(net.R, 10 ** -1.5)
    if dt is None:
        a0 = np.array([(th * net.propensity_factor(x0)).sum() for th in theta])
        dt = float(events_per_interval / np.median(a0))
        t_obs = dt * np.arange(1, n_obs + 1, dtype=np.float64)
        rng = np.random.Generator(np.random.PCG64(SEED_DATA))
        states = tau_leap_path(net, truth, x0, t_obs, rng, n_sub=20)
        name = "random-20x40"
    else:
        t_obs = float(dt) * np.arange(1, n_obs + 1, dtype=np.float64)
        states = mean_field_path(net, truth, x0, t_obs)
        name = "random-20x40-1e4"
    y = states[:, :2] + np.random.Generator(np.random.PCG64(SEED_NOISE)).normal(0, 10.0, (n_obs, 2))
    traj = {"t_obs": t_obs, "y": y, "t0": 0.0, "x0": x0, "x_true": states}
    return Workload(name, net, OBS_GAUSSIAN, [0, 1], 10.0, theta, [traj],
                    n_particles, truth=truth)


# ---------------------------------------------------------------------------
# Lac-Gfp (Supplementary "LacGfp example": species and initial-distribution
# table, reaction list, prior table, observation model)
# ---------------------------------------------------------------------------
LACGFP_SPECIES = ["lacI", "LACI", "LACI2", "PLac", "O2Lac", "O4Lac", "gfp", "GFP", "mGFP"]
# theta* of the prior table
LACGFP_TRUTH = np.array([1.215, 7.430, 1.439, 3.971, 1.173, 1716.683, 6.282, 0.433, 0.679,
                         173.576, 0.623, 119.232, 0.120, 0.006, 1.673, 32.318, 1.196, 2.102])
# prior intervals (log-uniform); theta_10's upper bound is read as 1600 (the
# table prints 1.600 with theta* = 173.576 inside the interval)
LACGFP_PRIOR_LO = np.array([1, 0.1, 1, 0.1, 1, 0.16, 0.1, 0.0016, 0.1, 0.16, 0.1, 1, 0.1, 1e-5,
                            0.1, 1, 0.1, 0.1])
LACGFP_PRIOR_HI = np.array([50, 30, 50, 20, 100, 3000, 20, 1.6, 20, 1600, 20, 150, 15, 1, 20, 50,
                            20, 20], dtype=np.float64)
LACGFP_IPTG = 10.0
# initial counts uniform on the integers lo..hi (lacI, LACI, O4Lac random)
LACGFP_X0_LO = np.array([0, 0, 0, 0, 0, 50, 0, 0, 0], dtype=np.int32)
LACGFP_X0_HI = np.array([5, 10, 0, 0, 0, 70, 0, 0, 0], dtype=np.int32)
# fluorescence: 22.85 per molecule, sd 5.72 per molecule; the background is
# read as normal (the paper's is an empirical flow-cytometry distribution)
LACGFP_GAIN, LACGFP_SD = 22.85, 5.72
LACGFP_BG_MEAN, LACGFP_BG_SD = 400.0, 120.0


def lacgfp():
    """The 9-species, 18-reaction Lac-Gfp network, reactions in the paper's
    order."""
    lacI, LACI, LACI2, PLac, O2Lac, O4Lac, gfp, GFP, mGFP = range(9)
    reac = [({}, {lacI: 1}), ({lacI: 1}, {}), ({lacI: 1}, {lacI: 1, LACI: 1}), ({LACI: 1}, {}),
            ({LACI: 2}, {LACI2: 1}), ({LACI2: 1}, {LACI: 2}),
            ({LACI2: 1, PLac: 1}, {O2Lac: 1}), ({O2Lac: 1}, {LACI2: 1, PLac: 1}),
            ({O2Lac: 2}, {O4Lac: 1}), ({O4Lac: 1}, {O2Lac: 2}),
            ({PLac: 1}, {PLac: 1, gfp: 1}), ({O2Lac: 1}, {O2Lac: 1, gfp: 1}),
            ({O4Lac: 1}, {O4Lac: 1, gfp: 1}), ({gfp: 1}, {}), ({gfp: 1}, {gfp: 1, GFP: 1}),
            ({GFP: 1}, {}), ({GFP: 1}, {mGFP: 1}), ({mGFP: 1}, {})]
    U, R = 9, len(reac)
    orders = np.zeros((R, U), dtype=np.int32)
    stoich = np.zeros((R, U), dtype=np.int32)
    for r, (cons, prod) in enumerate(reac):
        for u, v in cons.items():
            orders[r, u] = v
            stoich[r, u] -= v
        for u, v in prod.items():
            stoich[r, u] += v
    return Network("lac-gfp", LACGFP_SPECIES, orders, stoich, [f"R{r + 1}" for r in range(R)])


def lacgfp_rates(theta, iptg=LACGFP_IPTG):
    """Rate constants c [n, 18] of parameter vectors theta [n, 18]: reaction 4
    degrades LACI at theta_4 + theta_5 [IPTG], reactions 5-17 take theta_6 ..
    theta_18, and reaction 18 (mature GFP degradation) shares theta_17."""
    th = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    return np.concatenate([th[:, 0:3], (th[:, 3] + iptg * th[:, 4])[:, None], th[:, 5:18],
                           th[:, 16:17]], axis=1)


@functools.lru_cache(maxsize=4)
def _lacgfp_data(n_traj, n_obs, dt):
    """The Lac-Gfp data paths (exact, ~1.5e5 events each: simulated once per
    process and argument set)."""
    net = lacgfp()
    t_obs = dt * np.arange(1, n_obs + 1, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(SEED_DATA))
    nrng = np.random.Generator(np.random.PCG64(SEED_NOISE))
    c_true = lacgfp_rates(LACGFP_TRUTH)[0]
    x0s = np.stack([rng.integers(LACGFP_X0_LO, LACGFP_X0_HI + 1) for _ in range(n_traj)])
    paths = first_reaction_paths(net, c_true, x0s, t_obs, rng)
    trajs = []
    for x0, states in zip(x0s.astype(np.int32), paths):
        x = states[:, 8].astype(np.float64)
        y = (nrng.normal(LACGFP_GAIN * x, LACGFP_SD * np.sqrt(x))
             + nrng.normal(LACGFP_BG_MEAN, LACGFP_BG_SD, n_obs))
        trajs.append({"t_obs": t_obs, "y": y.reshape(-1, 1), "t0": 0.0,
                      "x0": LACGFP_X0_LO.copy(), "x0_hi": LACGFP_X0_HI.copy(),
                      "x_true": states, "x0_drawn": x0})
    return trajs


def lacgfp_population(n_theta, spread=0.3):
    """Parameter vectors log-normal around theta* (sd `spread` per log
    parameter): the shape of a late level of the sampler's population."""
    rng = np.random.Generator(np.random.PCG64(SEED_THETA))
    return LACGFP_TRUTH * np.exp(rng.normal(0.0, spread, (n_theta, len(LACGFP_TRUTH))))


def lacgfp_workload(n_theta=256, n_traj=5, n_obs=29, dt=1.0, n_particles=200, theta=None):
    """Lac-Gfp batch: rate vectors from parameters log-uniform on the prior
    box (or the given parameters), n_traj paths simulated exactly (first-
    reaction method) at theta* from random initial counts, mature GFP observed
    at dt, 2dt, ..., n_obs dt through the fluorescence model.  w.params holds
    the parameter vectors, w.theta their rate constants."""
    net = lacgfp()
    c_true = lacgfp_rates(LACGFP_TRUTH)[0]
    trajs = [{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in tr.items()}
             for tr in _lacgfp_data(int(n_traj), int(n_obs), float(dt))]
    if theta is None:
        theta = log_uniform(np.random.Generator(np.random.PCG64(SEED_THETA)),
                            LACGFP_PRIOR_LO, LACGFP_PRIOR_HI, n_theta)
    params = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    w = Workload("lac-gfp", net, OBS_FLUORESCENCE, [8],
                 (LACGFP_SD, LACGFP_GAIN, LACGFP_BG_MEAN, LACGFP_BG_SD), lacgfp_rates(params),
                 trajs, n_particles, truth=c_true)
    w.params = params
    return w


# ---------------------------------------------------------------------------
# Egf-Ras-Raf-Mek-Erk (Supplementary "Egf-Ras-Raf-Mek-Erk model": species and
# initial-value table, reaction equations, parameter and FRET prior tables)
# as a deterministic model: a term list for the ODE likelihood (the spec
# format of lik.OdeModel and of the oracle's OdeProblem)
# ---------------------------------------------------------------------------
ERK_SPECIES = ["EGFR", "EGFR*", "Ras", "Ras*", "Raf", "Raf*", "MEK", "MEK*", "ERK", "ERK*",
               "NFB", "NFB*", "dusp", "DUSP"]
ERK_PARAMS = ["k1", "gamma1", "k2", "K2", "gamma2", "D2", "k3", "K3", "K_NFB", "gamma3", "D3",
              "k4", "K4", "gamma4", "D4", "k5", "K5", "gamma5", "D5", "k6", "K6", "K6R", "gamma6",
              "D6", "dusp_basal", "dusp_ind", "K_dusp", "EGFR0", "NFB0", "dusp0",
              "bg", "lambda", "sigma", "E", "fAA", "fDD"]
ERK_PRIOR_LO = np.exp(np.r_[np.full(27, -10.0), np.full(3, -8.0), -7.0, -7.0, -8.0, -4.0, -8.0,
                            -8.0])
ERK_PRIOR_HI = np.exp(np.r_[np.full(27, 5.0), np.full(3, 1.0), 6.0, 6.0, -3.0, -0.5, 5.0, 5.0])
# a reference point inside the prior box (the paper's table leaves its theta
# column empty): rates per minute, concentrations in the table's units
ERK_REF = np.array([1.0, 0.5, 2.0, 0.1, 0.5, 0.1, 2.0, 0.5, 0.1, 0.5, 0.5, 2.0, 0.5, 0.5, 0.5,
                    2.0, 0.3, 2.0, 0.3, 0.5, 0.1, 0.3, 0.05, 0.1, 0.01, 10.0, 0.01, 0.1, 0.05,
                    0.001, 0.5, 1.0, 0.01, 0.3, 1.0, 1.0])
ERK_T_HALF = 90.0   # minutes, dusp and DUSP (fixed in the table)


def erk_model():
    """The 14 reaction equations as 17 flux terms over the engine's 36
    parameters (erk_engine_params): conversions between inactive and active
    forms, dusp production (basal and ERK-induced) and decay, DUSP
    translation and decay; observed through the FRET ratio of ERK* / ERK."""
    SP, SAT, HILL, REP, INP = 0, 1, 2, 3, 4
    (EGFR, EGFRa, Ras, Rasa, Raf, Rafa, MEK, MEKa, ERK, ERKa, NFB, NFBa, dusp, DUSP) = range(14)
    P = {n: k for k, n in enumerate(ERK_PARAMS)}
    dec = math.log10(2.0) / ERK_T_HALF   # the printed factor log10(2) / T
    terms = [
        dict(frm=EGFR, to=EGFRa, rate_param=P["k1"], factors=[(INP, 0, 0), (SP, EGFR, 0)]),
        dict(frm=EGFRa, to=EGFR, rate_param=P["gamma1"], factors=[(SP, EGFRa, 0)]),
        dict(frm=Ras, to=Rasa, rate_param=P["k2"], factors=[(SP, EGFRa, 0), (SAT, Ras, P["K2"])]),
        dict(frm=Rasa, to=Ras, rate_param=P["gamma2"], factors=[(SAT, Rasa, P["D2"])]),
        dict(frm=Raf, to=Rafa, rate_param=P["k3"],
             factors=[(SP, Rasa, 0), (SAT, Raf, P["K3"]), (REP, NFBa, P["K_NFB"])]),
        dict(frm=Rafa, to=Raf, rate_param=P["gamma3"], factors=[(SAT, Rafa, P["D3"])]),
        dict(frm=MEK, to=MEKa, rate_param=P["k4"], factors=[(SP, Rafa, 0), (SAT, MEK, P["K4"])]),
        dict(frm=MEKa, to=MEK, rate_param=P["gamma4"], factors=[(SAT, MEKa, P["D4"])]),
        dict(frm=ERK, to=ERKa, rate_param=P["k5"], factors=[(SP, MEKa, 0), (SAT, ERK, P["K5"])]),
        dict(frm=ERKa, to=ERK, rate_param=P["gamma5"], factors=[(SP, DUSP, 0), (SAT, ERKa, P["D5"])]),
        dict(frm=NFB, to=NFBa, rate_param=P["k6"],
             factors=[(SP, ERKa, 0), (SAT, NFB, P["K6"]), (HILL, EGFRa, P["K6R"])]),
        dict(frm=NFBa, to=NFB, rate_param=P["gamma6"], factors=[(SAT, NFBa, P["D6"])]),
        dict(to=dusp, rate_param=P["dusp_basal"], rate_scale=dec),
        dict(to=dusp, rate_param=P["dusp_ind"], rate_scale=dec, factors=[(HILL, ERKa, P["K_dusp"])]),
        dict(frm=dusp, rate_scale=dec, factors=[(SP, dusp, 0)]),
        dict(to=DUSP, rate_scale=dec, factors=[(SP, dusp, 0)]),
        dict(frm=DUSP, rate_scale=dec, factors=[(SP, DUSP, 0)]),
    ]
    x0_param = [-1] * 14
    x0_param[EGFR], x0_param[NFB] = P["EGFR0"], P["NFB0"]
    x0_param[dusp] = x0_param[DUSP] = P["dusp0"]
    return {"U": 14, "V": len(ERK_PARAMS), "terms": terms, "x0_param": x0_param,
            "obs_kind": 1, "obs_species": ERKa, "obs_species2": ERK, "sd_param": P["sigma"],
            "sd_const": 1.0, "fret_param": [P["lambda"], P["bg"], P["E"], P["fAA"], P["fDD"]]}


def erk_engine_params(theta):
    """The model's parameters as the engine reads them: the two repression and
    activation constants that enter squared (K_NFB, K6R) are squared, and the
    induced dusp rate is dusp_basal * dusp_ind."""
    th = np.array(np.atleast_2d(theta), dtype=np.float64)
    P = {n: k for k, n in enumerate(ERK_PARAMS)}
    th[:, P["K_NFB"]] = th[:, P["K_NFB"]] ** 2
    th[:, P["K6R"]] = th[:, P["K6R"]] ** 2
    th[:, P["dusp_ind"]] = th[:, P["dusp_basal"]] * th[:, P["dusp_ind"]]
    return th


ERK_X0 = np.array([0, 0, 0.1, 0, 0.7, 0, 0.68, 0, 0.26, 0, 0, 0, 0, 0], dtype=np.float64)


def erk_inputs():
    """Six EGF input patterns over 0-120 min (reading: a sustained step, a
    single 10-min pulse, 3-min pulses every 10, 20 and 30 min, and a staircase),
    as breakpoints and values of a piecewise-constant input."""
    pats = [([0.0], [1.0]), ([0.0, 10.0], [1.0, 0.0])]
    for period in (10.0, 20.0, 30.0):
        t, u = [], []
        for s in np.arange(0.0, 120.0, period):
            t += [s, s + 3.0]
            u += [1.0, 0.0]
        pats.append((t, u))
    pats.append(([0.0, 30.0, 60.0, 90.0], [0.25, 0.5, 0.75, 1.0]))
    return pats


def ode_spec_rhs(spec, th, u):
    """numpy right-hand side of a term list (data generation only)."""
    U = spec["U"]

    def f(t, x):
        dx = np.zeros(U)
        for T in spec["terms"]:
            v = T.get("rate_scale", 1.0) * (th[T["rate_param"]] if T.get("rate_param", -1) >= 0 else 1.0)
            for kind, sp, par in T.get("factors", []):
                xs = x[sp]
                v *= (u if kind == 4 else xs if kind == 0 else xs / (th[par] + xs) if kind == 1
                      else xs * xs / (th[par] + xs * xs) if kind == 2 else th[par] / (th[par] + xs * xs))
            if T.get("frm", -1) >= 0:
                dx[T["frm"]] -= v
            if T.get("to", -1) >= 0:
                dx[T["to"]] += v
        return dx
    return f


def erk_workload(n_theta=256, spread=0.3, n_obs=60, dt=2.0, theta=None):
    """ERK batch: engine parameter vectors log-normal (sd `spread`) around the
    reference point, six input patterns, FRET observations every dt minutes
    simulated from the reference point (scipy DOP853, piece by piece between
    input breakpoints) plus normal noise of the reference sigma."""
    from scipy.integrate import solve_ivp
    spec = erk_model()
    ref = erk_engine_params(ERK_REF)[0]
    t_obs = dt * np.arange(1, n_obs + 1, dtype=np.float64)
    nrng = np.random.Generator(np.random.PCG64(SEED_NOISE))
    P = {n: k for k, n in enumerate(ERK_PARAMS)}
    trajs = []
    for t_in, u_in in erk_inputs():
        x = ERK_X0.copy()
        for s, p in enumerate(spec["x0_param"]):
            if p >= 0:
                x[s] = ref[p]
        edges = list(t_in[1:]) + [t_obs[-1]]
        states = []
        tc = 0.0
        for te, uu in zip(edges, u_in):
            te = min(te, t_obs[-1])
            if te <= tc:
                continue
            ts = [tt for tt in t_obs if tc < tt <= te]
            sol = solve_ivp(ode_spec_rhs(spec, ref, uu), (tc, te), x, method="DOP853", rtol=1e-10,
                            atol=1e-12, t_eval=ts, dense_output=True)
            states += list(sol.y.T)
            x, tc = sol.sol(te), te
        states = np.array(states)
        lam, bg, E, fAA, fDD = (ref[P[k]] for k in ("lambda", "bg", "E", "fAA", "fDD"))
        a, b = states[:, 9], states[:, 8]
        g = lam * (E * fAA * a / ((b + (1 - E) * a) * fDD) + bg)
        y = g + nrng.normal(0.0, ref[P["sigma"]], len(g))
        trajs.append({"t_obs": t_obs, "y": y, "t0": 0.0, "x0": ERK_X0.copy(),
                      "t_in": np.asarray(t_in, np.float64), "u_in": np.asarray(u_in, np.float64),
                      "x_true": states})
    if theta is None:
        rng = np.random.Generator(np.random.PCG64(SEED_THETA))
        theta = ERK_REF * np.exp(rng.normal(0.0, spread, (n_theta, len(ERK_REF))))
    params = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    return {"spec": spec, "params": params, "theta": erk_engine_params(params), "trajectories": trajs}
