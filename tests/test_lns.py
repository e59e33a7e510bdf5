"""Host level-set sampler: threshold, rejection and DP-GMM rules, termination
and posterior recovery, each pinned to a closed form, a library routine or a
law that a plausible mistake breaks (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_1606_08281_amd import lns


# -- alpha-quantile thresholds (Remark "Use quantiles for the computation of
#    epsilon_{k+1}"; the first level keeps floor((1 - alpha) N) particles)

@pytest.mark.parametrize("N,alpha", [(10, 0.3), (7, 0.3), (200, 0.3), (200, 0.5), (33, 0.1)])
def test_threshold_keeps_floor_of_one_minus_alpha_N(N, alpha):
    ll = np.random.default_rng(N).normal(size=N)
    eps = lns.threshold(ll, alpha)
    assert np.sum(ll >= eps) == math.floor((1 - alpha) * N + 1e-9)
    assert np.sum(ll < eps) == math.ceil(alpha * N - 1e-9)


def test_threshold_puts_failed_evaluations_lowest():
    ll = np.array([-3.0, -np.inf, np.nan, -1.0, -2.0, 0.5, -0.5, -4.0, -np.inf, 1.0])
    # four values below the 0.4-quantile: the two -inf, the nan and -4
    assert lns.threshold(ll, 0.4) == -3.0
    assert lns.threshold(ll, 0.1) == -np.inf


# -- rejection step (Supplementary "Rejection Sampling", "Choice of M_k")

def test_accept_probability_is_min_one_m_over_q():
    q = np.array([0.01, 0.2, 0.5, 2.0, 8.0])
    m = 0.5
    p = lns.accept_probability(np.log(q), math.log(m))
    assert np.allclose(p, np.minimum(1.0, m / q))


def test_m_is_the_five_percent_quantile():
    v = np.random.default_rng(1).normal(size=401)
    s = np.sort(v)
    # 5 % of 400 gaps: exactly the 21st smallest value
    assert lns.log_m_quantile(v) == pytest.approx(s[20], abs=0)


def test_rejection_turns_the_proposal_into_the_level_set():
    """theta* ~ q' = q_prev restricted to the level set, thinned with
    min(1, M / q_prev) and M = min of q_prev on the set: the survivors are
    uniform on the set (the ratio q' M / q_prev is constant there).  q_prev
    is a standard normal and the level set |theta| <= 1.2."""
    rng = np.random.default_rng(2)
    a = 1.2
    th = stats.truncnorm.rvs(-a, a, size=200_000, random_state=rng)
    log_q = stats.norm.logpdf(th)
    keep = rng.random(len(th)) < lns.accept_probability(log_q, stats.norm.logpdf(a))
    out = th[keep]
    assert stats.kstest(out, stats.uniform(-a, 2 * a).cdf).pvalue > 1e-3
    # thinning the other way round (q_prev / M) keeps the normal shape
    wrong = th[rng.random(len(th)) < np.minimum(1.0, np.exp(log_q - stats.norm.logpdf(0.0)))]
    assert stats.kstest(wrong, stats.uniform(-a, 2 * a).cdf).pvalue < 1e-6


# -- DP-GMM (Remark "DP-GMM for density estimation")

def test_student_t_density_matches_scipy():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(3, 3))
    shape = A @ A.T + np.eye(3)
    mu = rng.normal(size=3)
    x = rng.normal(size=(50, 3)) * 2
    ref = stats.multivariate_t(loc=mu, shape=shape, df=4.5).logpdf(x)
    got = lns.student_t_logpdf(x, mu, np.linalg.cholesky(shape), 4.5)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_predictive_tends_to_the_sample_moments():
    """With many points the posterior predictive of one cluster has the
    sample mean as its location and the sample covariance as its scale."""
    rng = np.random.default_rng(4)
    X = rng.multivariate_normal([1.0, -2.0], [[1.0, 0.6], [0.6, 2.0]], size=200_000)
    g = lns.DPGMM()
    g._base(X)
    mu, L, dof = g.predictive(len(X), X.sum(0), X.T @ X)
    assert np.allclose(mu, X.mean(0), atol=1e-3)
    assert np.allclose(L @ L.T * dof / (dof - 2), np.cov(X.T), rtol=2e-3)


def test_dpgmm_separates_two_clusters_and_is_a_density():
    rng = np.random.default_rng(5)
    X = np.vstack([rng.normal([-3, 0], 0.4, size=(120, 2)), rng.normal([3, 1], 0.6, size=(80, 2))])
    g = lns.DPGMM(sweeps=15, rng=np.random.default_rng(6)).fit(X)
    truth = np.r_[np.zeros(120, int), np.ones(80, int)]
    # the two groups end up in different clusters, each group in one cluster
    # apart from at most a few points
    big = [np.bincount(g.z[truth == t]).argmax() for t in (0, 1)]
    assert big[0] != big[1]
    assert np.mean(g.z[truth == 0] == big[0]) > 0.95 and np.mean(g.z[truth == 1] == big[1]) > 0.95
    # integrates to one over a box that holds the mass
    h = 0.05
    xs, ys = np.meshgrid(np.arange(-9, 9, h), np.arange(-8, 9, h))
    dens = np.exp(g.logpdf(np.c_[xs.ravel(), ys.ravel()]))
    assert dens.sum() * h * h == pytest.approx(1.0, abs=0.02)
    # its draws follow it: mean and left-cluster share
    s = g.sample(40_000, np.random.default_rng(7))
    assert np.allclose(s.mean(0), X.mean(0), atol=0.15)
    assert np.mean(s[:, 0] < 0) == pytest.approx(0.6, abs=0.03)


def test_dpgmm_warm_start_keeps_a_converged_assignment():
    rng = np.random.default_rng(8)
    X = np.vstack([rng.normal([-3, 0], 0.4, size=(100, 2)), rng.normal([3, 1], 0.4, size=(100, 2))])
    g = lns.DPGMM(sweeps=15, rng=np.random.default_rng(9)).fit(X)
    # drop thirty points, add thirty unlabelled ones: one warm sweep
    keep = np.arange(30, 200)
    Y = np.vstack([X[keep], rng.normal([3, 1], 0.4, size=(30, 2))])
    h = lns.DPGMM(sweeps=1, rng=np.random.default_rng(10)).fit(
        Y, z_init=np.r_[g.z[keep], np.full(30, -1)])
    same = np.mean([h.z[i] == h.z[j] for i in range(0, 170, 7) for j in range(0, 170, 11)
                    if g.z[keep[i]] == g.z[keep[j]]])
    assert same > 0.95
    # the new points join clusters of the right-hand group only
    right = set(h.z[170:])
    assert all(np.all(Y[h.z == c, 0] > 0) for c in right)


# -- the sampler on a likelihood with a closed form

D = 2
MU = np.array([-1.0, 1.0])
SD = 0.5
C = -D * math.log(SD * math.sqrt(2 * math.pi))


def gauss_ll(rates):
    x = np.log(rates)
    return -0.5 * np.sum(((x - MU) / SD) ** 2, axis=1) + C, np.zeros(len(x), np.int32)


def prior2():
    return lns.LogUniformPrior(np.full(D, math.exp(-5)), np.full(D, math.exp(5)))


@pytest.fixture(scope="module")
def gauss_run():
    s = lns.LNS(prior2(), gauss_ll, N=100, alpha=0.3, batch=16, seed=11)
    s.run(max_levels=12)
    return s


def test_levels_hold_N_particles_above_their_threshold(gauss_run):
    s = gauss_run
    eps = [r["eps"] for r in s.levels]
    assert len(s.levels) == 12
    assert np.all(np.diff(eps) > 0)
    for r in s.levels:
        assert r["kept"] == 70 and r["accepted"] == r["needed"] == 30
        assert r["passed"] <= r["evaluated"] and r["passed"] >= r["accepted"]
        new_ll = gauss_ll(np.exp(r["new"]))[0]
        assert np.all(new_ll >= r["eps"])
    assert len(s.X) == 100 and np.all(s.ll >= eps[-1])
    assert np.allclose(gauss_ll(np.exp(s.X))[0], s.ll)
    # the level sets close in on the maximum C
    assert C - eps[-1] < 1.0 and s.levels[-1]["max_loglik"] <= C


def test_first_level_thins_nothing_later_levels_do(gauss_run):
    """q_0 is the (constant) prior: M_1 = q_0, so every in-support proposal of
    the first level is evaluated; later levels thin with M_k / q_{k-1}."""
    r = gauss_run.levels
    assert r[0]["thinned"] == 0 and r[0]["in_support"] == r[0]["evaluated"]
    assert sum(x["thinned"] for x in r[1:]) > 0


def test_synchronous_and_in_flight_paths_agree():
    """With one batch in flight, submit/collect draws and evaluates in the
    same order as the synchronous path."""
    a = lns.LNS(prior2(), gauss_ll, N=60, alpha=0.3, batch=8, seed=12)
    a.run(max_levels=4)
    b = lns.LNS(prior2(), N=60, alpha=0.3, batch=8, seed=12, submit=lambda r: r,
                collect=gauss_ll, inflight=1)
    b.run(max_levels=4)
    assert [x["eps"] for x in a.levels] == [x["eps"] for x in b.levels]
    assert np.array_equal(a.X, b.X)


def test_in_flight_batches_keep_the_level_rules():
    s = lns.LNS(prior2(), N=60, alpha=0.3, batch=8, seed=13, submit=lambda r: r,
                collect=gauss_ll, inflight=4)
    s.run(max_levels=5)
    for r in s.levels:
        assert r["accepted"] == r["needed"] == 18
        assert np.all(gauss_ll(np.exp(r["new"]))[0] >= r["eps"])


# -- termination ("Termination Criterion")

def test_spread_and_acceptance_criteria_stop_the_run():
    s = lns.LNS(prior2(), gauss_ll, N=60, alpha=0.3, batch=8, seed=14, spread_stop=2.0)
    s.run(max_levels=40)
    assert s.levels[-1]["spread"] < 2.0 and all(r["spread"] >= 2.0 for r in s.levels[:-1])
    s = lns.LNS(prior2(), gauss_ll, N=60, alpha=0.3, batch=8, seed=14, acceptance_stop=1.01)
    s.run(max_levels=40)
    assert len(s.levels) == 1


def test_a_level_that_cannot_refill_ends_the_run():
    """Every evaluation after S_0 fails (status != 0, l = -inf): the first
    level spends its proposal budget and the run stops there."""
    calls = []

    def ll(rates):
        calls.append(len(rates))
        v, st = gauss_ll(rates)
        return v, (st if len(calls) == 1 else np.full(len(rates), 3, np.int32))
    s = lns.LNS(prior2(), ll, N=40, alpha=0.5, batch=8, seed=15, max_proposals_per_level=400)
    s.run(max_levels=10)
    assert len(s.levels) == 1
    r = s.levels[0]
    assert r["accepted"] == 0 and r["needed"] == 20 and r["passed"] == 0
    assert r["proposals"] > 400 and len(s.X) == 20 and np.all(np.isfinite(s.ll))


def test_a_prior_without_finite_likelihoods_is_an_error():
    def ll(rates):
        return np.zeros(len(rates)), np.full(len(rates), 3, np.int32)
    s = lns.LNS(prior2(), ll, N=20, alpha=0.3, seed=16)
    with pytest.raises(ValueError, match="finite"):
        s.run(max_levels=3)


# -- posterior from level sets (Supplementary "Approximating the full posterior")

def test_level_set_weights_closed_form():
    covs = [np.diag([4.0, 1.0]), np.diag([1.0, 0.25])]
    eps = [-3.0, -1.0]
    w = lns.level_set_weights(eps, covs)
    assert w[0] == pytest.approx(0.5 * math.log(4.0) - 3.0)
    assert w[1] == pytest.approx(0.5 * math.log(0.25) + math.log(math.exp(-1.0) - math.exp(-3.0)))


def test_exact_level_sets_recover_a_gaussian_posterior():
    """Level sets of l(theta) = exp(-theta^2 / 2) sampled exactly (uniform on
    |theta| <= r_k) at fine thresholds: the g_k delta_k mixture is the
    normalised likelihood, mean 0 and standard deviation 1 (a dropped g_k
    or a delta in log-likelihood units gives a visibly wrong width)."""
    rng = np.random.default_rng(16)
    prior = lns.LogUniformPrior([math.exp(-6.0)], [math.exp(6.0)])
    eps = np.log(np.linspace(0.002, 0.998, 400))
    levels = []
    for e in eps:
        r = math.sqrt(-2.0 * e)
        levels.append({"eps": float(e), "new": rng.uniform(-r, r, size=(400, 1))})
    X, w = lns.posterior_sample(levels, prior, 200_000, rng)
    m = float(np.sum(w * X[:, 0]))
    sd = math.sqrt(float(np.sum(w * (X[:, 0] - m) ** 2)))
    assert abs(m) < 0.02 and sd == pytest.approx(1.0, abs=0.02)
    # the two plausible slips: g_k dropped (too narrow) and delta_k taken in
    # log-likelihood units (too wide)
    g = np.log([np.std(r["new"]) for r in levels])

    def width(lw):
        p = np.exp(lw - lw.max())
        k = rng.choice(len(levels), size=50_000, p=p / p.sum())
        return np.std([levels[i]["new"][rng.integers(400), 0] for i in k])
    assert width(np.log(np.diff(np.r_[0.0, np.exp(eps)]))) < 0.9
    assert width(g + np.log(np.diff(np.r_[eps[0] - 1.0, eps]))) > 1.3


def test_sampler_posterior_is_centred_on_the_mode(gauss_run):
    X, w = lns.posterior_sample(gauss_run.levels, prior2(), 20_000, np.random.default_rng(17))
    m = np.sum(w[:, None] * X, axis=0)
    sd = np.sqrt(np.sum(w[:, None] * (X - m) ** 2, axis=0))
    assert np.allclose(m, MU, atol=0.12)
    assert np.all((sd > 0.3) & (sd < 0.6))


# -- the served stream's plumbing, against a stand-in server (CPU)

class _FakeServer:
    """submit -> ticket; a ticket is done on the second zero-timeout poll."""

    def __init__(self):
        self.polls, self.subs = {}, []

    def submit(self, net, obs_kind, observed, sigma, theta, trajs, H, seed, theta_ids=None):
        t = len(self.subs) + 1
        self.subs.append((net, np.array(theta), H, seed))
        self.polls[t] = 0
        return t

    def wait(self, t, timeout_s=None):
        self.polls[t] += 1
        if self.polls[t] < 2:
            return None
        theta = self.subs[t - 1][1]
        return gauss_ll(theta[:, :D])


def test_sampler_stream_plumbing_with_side_requests():
    from paper_1606_08281_amd import serve_lns

    class WL:
        def __init__(self, name, n):
            self.name, self.obs_kind, self.observed, self.sigma = name, 0, [0], 1.0
            self.theta = np.exp(np.random.default_rng(0).normal(size=(n, D)))
            self.trajectories = []

        @property
        def n_theta(self):
            return len(self.theta)
    tel, side = WL("tel", 1), WL("side", 64)
    srv = _FakeServer()
    stream = serve_lns.Stream(srv, {"tel": "net-tel", "side": "net-side"}, side=side, side_every=3)
    t = serve_lns.Tenant(stream, tel, [], 256, seed_base=1000)
    s = lns.LNS(prior2(), N=40, alpha=0.3, batch=8, seed=18, submit=t.submit, collect=t.collect,
                inflight=3)
    s.run(max_levels=3)
    for r in stream.log:
        r["event"].wait()
    stream.close()
    tags = [r["tag"] for r in stream.log]
    n_tel = tags.count("telegraph-H256")
    # one side request after every two sampler requests: a third of the stream
    assert tags.count("random-20x40") == n_tel // 2
    assert all(1 <= len(r["theta"]) <= 8 for r in stream.log)
    assert all(r["t_done"] >= r["t_submit"] for r in stream.log)
    seeds = [r["seed"] for r in stream.log if r["tag"] == "telegraph-H256"]
    assert seeds == list(range(1001, 1001 + n_tel))
    assert [x[0] for x in srv.subs].count("net-side") == tags.count("random-20x40")
    assert all(x["accepted"] == x["needed"] for x in s.levels)
