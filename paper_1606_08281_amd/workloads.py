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
"""
import numpy as np

SEED_NET, SEED_DATA, SEED_NOISE, SEED_THETA, SEED_FILTER = 1, 2, 3, 4, 5

OBS_GAUSSIAN, OBS_LOGNORMAL = 0, 1


class Network:
    """Reactant orders p[r, u] and net changes nu[r, u] = q[r, u] - p[r, u]."""

    def __init__(self, name, species, orders, stoich, reaction_names=None):
        self.name = name
        self.species = list(species)
        self.orders = np.asarray(orders, dtype=np.int32)
        self.stoich = np.asarray(stoich, dtype=np.int32)
        self.R, self.U = self.orders.shape
        self.reaction_names = reaction_names or [f"R{r}" for r in range(self.R)]

    def propensity_factor(self, x):
        """Mass-action combinatorial factors prod_u C(x_u, p_ru) (float64)."""
        h = np.ones(self.R)
        for r in range(self.R):
            for u in range(self.U):
                p = self.orders[r, u]
                if p == 1:
                    h[r] *= x[u]
                elif p == 2:
                    h[r] *= x[u] * (x[u] - 1) / 2.0
        return h


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
        self.sigma = float(sigma)
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
