"""Likelihood nested sampling on the host: the level-set sampler that sits
upstream of the likelihood engine and emits its requests.

What it computes follows the paper's Likelihood Nested Sampling algorithm,
its Remarks ("Use quantiles for the computation of epsilon_{k+1}", "DP-GMM
for density estimation"), Supplementary "Rejection Sampling" (with "Choice of
M_k"), "Termination Criterion" and "Approximating the full posterior":

  S_0   N rate vectors from the prior p_0, each with an estimated
        log-likelihood l(theta) (a particle filter, evaluated by the engine);
  level k = 1, 2, ...
    eps_k    the alpha-quantile of the log-likelihoods of S_{k-1}: the value
             with ceil(alpha N) values below it, so floor((1 - alpha) N)
             particles are kept when there are no ties;
    S'_k     the particles of S_{k-1} with l >= eps_k;
    q'_k     a DP-GMM density fitted to S'_k, warm-started from the labels of
             the previous fit;
    q_{k-1}  the DP-GMM density of S_{k-1} (q_0 = p_0);
    M_k      the 5 % quantile of q_{k-1} over the particles of S'_k;
    refill   draw theta* ~ q'_k; keep it with probability
             min(1, M_k / q_{k-1}(theta*)) if it lies in the prior's support;
             estimate l(theta*) and add it to S'_k if l(theta*) >= eps_k,
             until S'_k holds N particles; S_k = S'_k.
  stop      when the spread max l - min l of a level, or its acceptance rate
            (evaluated proposals with l >= eps_k over all evaluated), falls
            below a set value, when a level cannot be refilled within its
            proposal budget, or after a set number of levels.

Readings where the paper leaves a choice: the level-set inequality is >= for
keeping and for accepting; M_k is taken over S'_k (the retained particles,
which are the proposal's own samples), so that about 95 % of proposals in the
bulk of q'_k are thinned; everything works in log-parameter space, where the
log-uniform priors used here are uniform, so q_0 is constant and the first
level accepts every in-support proposal.

Proposal survivors go to the engine in batches (one request per batch); with
`submit`/`collect` callables several batches are in flight while the next is
drawn, and a level's surplus results are discarded once it is full.

The DP-GMM is the collapsed Gibbs sampler of a Dirichlet-process mixture of
Gaussians with a conjugate normal-inverse-Wishart base measure: each sweep
reassigns every point to an existing cluster with probability proportional to
the cluster's size times its posterior predictive density (a multivariate
Student t), or to a new cluster with probability proportional to the
concentration times the prior predictive.  The fitted density is the
posterior-predictive mixture of the final assignment, new-cluster term
included.  Warm-started labels make later levels converge in a few sweeps.

Posterior recovery uses the newly sampled particles of each level as samples
of the level set L_k, g_k = sqrt(det Cov L_k) (in log-parameter space) and
delta_k = eps_k - eps_{k-1} in likelihood units (eps_0 = 0), formed in log
space so that log-likelihoods of any size stay finite.
"""
import math

import numpy as np
from scipy.special import gammaln, logsumexp


class LogUniformPrior:
    """Independent log-uniform rates on [lo_r, hi_r]: uniform in log space."""

    def __init__(self, lo, hi):
        self.lo = np.log(np.asarray(lo, dtype=np.float64))
        self.hi = np.log(np.asarray(hi, dtype=np.float64))
        self.d = len(self.lo)
        self.log_density = -float(np.sum(self.hi - self.lo))

    def sample(self, n, rng):
        return self.lo + rng.random((n, self.d)) * (self.hi - self.lo)

    def inside(self, x):
        return np.all((x >= self.lo) & (x <= self.hi), axis=-1)

    def logpdf(self, x):
        x = np.atleast_2d(x)
        return np.where(self.inside(x), self.log_density, -np.inf)


def student_t_logpdf(x, mu, chol, dof):
    """log density of the multivariate Student t with location mu, scale
    matrix chol chol^T and dof degrees of freedom, at the rows of x."""
    x = np.atleast_2d(x)
    d = mu.shape[-1]
    z = np.linalg.solve(chol, (x - mu).T)
    maha = np.sum(z * z, axis=0)
    logdet = 2.0 * np.sum(np.log(np.diag(chol)))
    return (gammaln((dof + d) / 2.0) - gammaln(dof / 2.0) - 0.5 * d * math.log(dof * math.pi)
            - 0.5 * logdet - 0.5 * (dof + d) * np.log1p(maha / dof))


class DPGMM:
    """Dirichlet-process Gaussian mixture fitted by collapsed Gibbs sampling.

    Base measure: normal-inverse-Wishart with mean mu0 = the data mean,
    kappa0, nu0 = d + 2 and scale psi0 chosen so that a new cluster's prior
    mean covariance is `scale` times the data covariance."""

    def __init__(self, alpha=1.0, kappa0=0.05, scale=0.2, sweeps=20, rng=None):
        self.alpha = float(alpha)
        self.kappa0 = float(kappa0)
        self.scale = float(scale)
        self.sweeps = int(sweeps)
        self.rng = rng if rng is not None else np.random.default_rng(0)
        self.z = None

    def _base(self, X):
        n, d = X.shape
        self.d = d
        self.mu0 = X.mean(axis=0)
        cov = np.atleast_2d(np.cov(X.T)) if n > 1 else np.eye(d)
        jitter = 1e-6 * max(float(np.trace(cov)) / d, 1e-12)
        self.nu0 = d + 2.0
        self.psi0 = (cov + jitter * np.eye(d)) * self.scale * (self.nu0 - d - 1.0)

    def predictive(self, n, s, ss):
        """Posterior predictive (mu, chol of the scale, dof) of a cluster with
        count n, coordinate sum s and sum of outer products ss."""
        d = self.d
        k = self.kappa0 + n
        mu = (self.kappa0 * self.mu0 + s) / k
        psi = self.psi0 + ss + self.kappa0 * np.outer(self.mu0, self.mu0) - k * np.outer(mu, mu)
        dof = self.nu0 + n - d + 1.0
        scale = psi * (k + 1.0) / (k * dof)
        return mu, np.linalg.cholesky(0.5 * (scale + scale.T)), dof

    def fit(self, X, z_init=None, sweeps=None):
        """Fits the rows of X.  z_init: labels from a previous fit (-1 for
        rows that had none): the warm start across levels."""
        X = np.asarray(X, dtype=np.float64)
        n, d = X.shape
        self._base(X)
        rng = self.rng
        z = np.full(n, -1, dtype=np.int64)
        if z_init is not None:
            relabel = {}
            for i, c in enumerate(np.asarray(z_init, dtype=np.int64)):
                if c >= 0:
                    z[i] = relabel.setdefault(int(c), len(relabel))
        cap = n + 1
        cnt = np.zeros(cap)
        S = np.zeros((cap, d))
        SS = np.zeros((cap, d, d))
        outer = np.einsum("ni,nj->nij", X, X)
        for i in np.nonzero(z >= 0)[0]:
            cnt[z[i]] += 1
            S[z[i]] += X[i]
            SS[z[i]] += outer[i]
        # per cluster slot: predictive location, inverse Cholesky factor of
        # the scale, degrees of freedom and the density's constant term
        loc = np.zeros((cap, d))
        winv = np.zeros((cap, d, d))
        dof = np.ones(cap)
        const = np.zeros(cap)

        def t_const(L, nu):
            return (gammaln((nu + d) / 2.0) - gammaln(nu / 2.0) - 0.5 * d * math.log(nu * math.pi)
                    - np.sum(np.log(np.diag(L))))

        def refresh(c):
            mu, L, nu = self.predictive(cnt[c], S[c], SS[c])
            loc[c], winv[c], dof[c], const[c] = mu, np.linalg.inv(L), nu, t_const(L, nu)

        for c in np.nonzero(cnt > 0)[0]:
            refresh(c)
        prior = self.predictive(0, np.zeros(d), np.zeros((d, d)))
        p_loc, p_winv, p_dof = prior[0], np.linalg.inv(prior[1]), prior[2]
        p_const = t_const(prior[1], p_dof) + math.log(self.alpha)
        for _ in range(max(self.sweeps if sweeps is None else int(sweeps), 1)):
            for i in rng.permutation(n):
                x = X[i]
                if z[i] >= 0:
                    c = z[i]
                    cnt[c] -= 1
                    S[c] -= x
                    SS[c] -= outer[i]
                    if cnt[c] <= 0:          # an emptied cluster restarts from exact zeros
                        S[c] = 0.0
                        SS[c] = 0.0
                    else:
                        refresh(c)
                live = np.nonzero(cnt > 0)[0]
                r = np.einsum("kij,kj->ki", winv[live], x - loc[live])
                nu = dof[live]
                logp = np.empty(len(live) + 1)
                logp[:-1] = (np.log(cnt[live]) + const[live]
                             - 0.5 * (nu + d) * np.log1p(np.sum(r * r, axis=1) / nu))
                r0 = p_winv @ (x - p_loc)
                logp[-1] = p_const - 0.5 * (p_dof + d) * math.log1p(float(r0 @ r0) / p_dof)
                cum = np.cumsum(np.exp(logp - logp.max()))
                j = min(int(np.searchsorted(cum, rng.random() * cum[-1], side="right")),
                        len(logp) - 1)
                c = int(live[j]) if j < len(live) else int(np.nonzero(cnt <= 0)[0][0])
                z[i] = c
                cnt[c] += 1
                S[c] += x
                SS[c] += outer[i]
                refresh(c)
        live = np.nonzero(cnt > 0)[0]
        remap = np.full(cap, -1, dtype=np.int64)
        remap[live] = np.arange(len(live))
        self.z = remap[z]
        self.n = n
        self.weights = np.append(cnt[live], self.alpha) / (n + self.alpha)
        self.comps = [self.predictive(cnt[c], S[c], SS[c]) for c in live] + [prior]
        return self

    @property
    def n_clusters(self):
        return len(self.weights) - 1

    def logpdf(self, x):
        x = np.atleast_2d(np.asarray(x, dtype=np.float64))
        parts = [math.log(w) + student_t_logpdf(x, *comp)
                 for w, comp in zip(self.weights, self.comps)]
        return logsumexp(np.vstack(parts), axis=0)

    def sample(self, m, rng):
        """m draws of the mixture (Student t: Gaussian over sqrt(chi2/dof))."""
        k = rng.choice(len(self.weights), size=m, p=self.weights)
        out = np.empty((m, self.d))
        for c in np.unique(k):
            sel = np.nonzero(k == c)[0]
            mu, L, dof = self.comps[c]
            g = rng.standard_normal((len(sel), self.d)) @ L.T
            w = rng.chisquare(dof, size=len(sel)) / dof
            out[sel] = mu + g / np.sqrt(w)[:, None]
        return out


def threshold(loglik, alpha):
    """eps: the alpha-quantile of a level's log-likelihoods, the value with
    ceil(alpha N) values below it (non-finite values count as lowest)."""
    v = np.asarray(loglik, dtype=np.float64)
    v = np.sort(np.where(np.isnan(v), -np.inf, v))
    k = min(max(int(math.ceil(alpha * len(v) - 1e-12)), 0), len(v) - 1)
    return float(v[k])


def log_m_quantile(logq_prev, q=0.05):
    """log M_k: the q-quantile of log q_{k-1} over the retained particles."""
    return float(np.quantile(np.asarray(logq_prev, dtype=np.float64), q))


def accept_probability(logq_prev_at, log_m):
    """Rejection step: keep theta* with probability min(1, M_k / q_{k-1}(theta*))."""
    return np.exp(np.minimum(0.0, log_m - np.asarray(logq_prev_at, dtype=np.float64)))


class LNS:
    """The level-set sampler.

    loglik(rates [n, R]) -> (loglik [n], status [n]) evaluates synchronously;
    or submit(rates) -> handle and collect(handle) -> (loglik, status) keep up
    to `inflight` proposal batches at the engine together.  Rates are passed
    as rates (exp of the sampler's log coordinates); a nonzero status counts
    as l = -inf."""

    def __init__(self, prior, loglik=None, N=200, alpha=0.3, batch=32, seed=0, submit=None,
                 collect=None, inflight=4, sweeps_first=20, sweeps_warm=5,
                 max_proposals_per_level=None, spread_stop=None, acceptance_stop=None):
        if loglik is None and (submit is None or collect is None):
            raise ValueError("need loglik, or submit and collect")
        self.prior = prior
        self.loglik_fn = loglik
        self.submit_fn, self.collect_fn = submit, collect
        self.N = int(N)
        self.alpha = float(alpha)
        self.batch = int(batch)
        self.rng = np.random.default_rng(seed)
        self.inflight = max(int(inflight), 1)
        self.sweeps_first, self.sweeps_warm = int(sweeps_first), int(sweeps_warm)
        self.max_props = int(max_proposals_per_level or 500 * self.N)
        self.spread_stop = spread_stop
        self.acceptance_stop = acceptance_stop
        self.levels = []
        self.evals = 0
        self.X = None

    @staticmethod
    def _ll(ll, st):
        return np.where(np.asarray(st) == 0, np.asarray(ll, dtype=np.float64), -np.inf)

    def initial(self):
        """S_0 from the prior."""
        X = self.prior.sample(self.N, self.rng)
        if self.loglik_fn is not None:
            ll = self._ll(*self.loglik_fn(np.exp(X)))
        else:   # batches of at most `batch`, all at the engine together
            hs = [self.submit_fn(np.exp(X[i:i + self.batch])) for i in range(0, self.N, self.batch)]
            ll = np.concatenate([self._ll(*self.collect_fn(h)) for h in hs])
        self.evals += len(X)
        self.X, self.ll, self.z, self.q_prev = X, ll, None, None
        return self

    def _logq_prev(self, X):
        return self.prior.logpdf(X) if self.q_prev is None else self.q_prev.logpdf(X)

    def _proposals(self, qk, log_m, count):
        """Up to `batch` rejection-step survivors (theta* ~ q'_k, in the
        prior's support, kept with probability min(1, M_k / q_{k-1})); an
        empty array once the level's proposal budget is spent.  count:
        [drawn, in support, thinned by the M_k rule], updated."""
        while count[0] <= self.max_props:
            cand = qk.sample(self.batch, self.rng)
            count[0] += len(cand)
            cand = cand[self.prior.inside(cand)]
            count[1] += len(cand)
            if len(cand):
                u = self.rng.random(len(cand))
                ok = u < accept_probability(self._logq_prev(cand), log_m)
                count[2] += int(np.sum(~ok))
                cand = cand[ok]
            if len(cand):
                return cand
        return np.empty((0, self.prior.d))

    def level(self):
        """One level; returns its record and replaces the particle set."""
        if self.X is None:
            self.initial()
        eps = threshold(self.ll, self.alpha)
        keep = np.isfinite(self.ll) & (self.ll >= eps)
        Xk, llk = self.X[keep], self.ll[keep]
        if len(Xk) < 2:
            raise ValueError("fewer than two particles with a finite log-likelihood above the "
                             "threshold: no level-set density to fit")
        zk = None if self.z is None else self.z[keep]
        qk = DPGMM(sweeps=self.sweeps_first if self.z is None else self.sweeps_warm,
                   rng=self.rng).fit(Xk, z_init=zk)
        log_m = log_m_quantile(self._logq_prev(Xk))
        need = self.N - len(Xk)
        newX, newll = [], []
        count = [0, 0, 0]
        evaluated = passed = 0
        pending = []
        while len(newX) < need:
            if self.loglik_fn is not None:
                cand = self._proposals(qk, log_m, count)
                if not len(cand):
                    break
                ll = self._ll(*self.loglik_fn(np.exp(cand)))
            else:
                while len(pending) < self.inflight:
                    cand = self._proposals(qk, log_m, count)
                    if not len(cand):
                        break
                    pending.append((cand, self.submit_fn(np.exp(cand))))
                if not pending:
                    break
                cand, h = pending.pop(0)
                ll = self._ll(*self.collect_fn(h))
            self.evals += len(cand)
            evaluated += len(cand)
            ok = ll >= eps
            passed += int(np.sum(ok))
            newX.extend(cand[ok])
            newll.extend(ll[ok])
        for cand, h in pending:      # batches still at the engine when the level filled
            self.collect_fn(h)
            self.evals += len(cand)
            evaluated += len(cand)
        newX = np.asarray(newX[:need], dtype=np.float64).reshape(-1, self.prior.d)
        newll = np.asarray(newll[:need], dtype=np.float64)
        self.X = np.vstack([Xk, newX])
        self.ll = np.concatenate([llk, newll])
        self.q_prev = DPGMM(sweeps=self.sweeps_warm, rng=self.rng).fit(
            self.X, z_init=np.concatenate([qk.z, np.full(len(newX), -1)]))
        self.z = self.q_prev.z
        fin = self.ll[np.isfinite(self.ll)]
        rec = {"eps": eps, "kept": int(len(Xk)), "needed": int(need), "accepted": int(len(newX)),
               "evaluated": int(evaluated), "passed": passed, "proposals": int(count[0]),
               "in_support": int(count[1]), "thinned": int(count[2]),
               "acceptance": passed / max(evaluated, 1),
               "spread": float(fin.max() - fin.min()) if len(fin) else float("inf"),
               "max_loglik": float(fin.max()) if len(fin) else -float("inf"),
               "min_loglik": float(fin.min()) if len(fin) else -float("inf"),
               "clusters": int(qk.n_clusters), "log_m": log_m, "new": newX.copy()}
        self.levels.append(rec)
        return rec

    def done(self):
        """A termination criterion holds for the last level."""
        if not self.levels:
            return False
        r = self.levels[-1]
        if r["accepted"] < r["needed"]:
            return True
        if self.spread_stop is not None and r["spread"] < self.spread_stop:
            return True
        return self.acceptance_stop is not None and r["acceptance"] < self.acceptance_stop

    def run(self, max_levels=20):
        if self.X is None:
            self.initial()
        for _ in range(int(max_levels)):
            self.level()
            if self.done():
                break
        return self.levels


def level_set_weights(eps, covs):
    """Log weights log(g_k delta_k) of the level-set mixture for thresholds
    eps_1 < eps_2 < ... (log-likelihoods) and the covariance matrices of the
    level sets: g_k = sqrt(det Cov L_k), delta_1 = exp(eps_1), delta_k =
    exp(eps_k) - exp(eps_{k-1})."""
    out = []
    prev = -np.inf
    for e, cov in zip(eps, covs):
        sign, logdet = np.linalg.slogdet(np.atleast_2d(cov))
        if sign <= 0 or not np.isfinite(e) or e <= prev:
            out.append(-np.inf)
        else:
            log_delta = e if not np.isfinite(prev) else e + math.log1p(-math.exp(prev - e))
            out.append(0.5 * logdet + log_delta)
        if np.isfinite(e):
            prev = max(prev, e)
    return np.array(out)


def posterior_sample(levels, prior, m, rng):
    """Weighted posterior samples from a run's levels: a level drawn with
    probability proportional to g_k delta_k, one of its newly sampled
    particles uniformly, weighted by the prior density.  Returns (log
    parameters [m, d], normalised weights [m])."""
    use = [r for r in levels if len(r["new"]) > 1]
    lw = level_set_weights([r["eps"] for r in use], [np.cov(r["new"].T) for r in use])
    w = np.exp(lw - logsumexp(lw))
    ks = rng.choice(len(use), size=m, p=w)
    out = np.empty((m, prior.d))
    for k in np.unique(ks):
        sel = np.nonzero(ks == k)[0]
        X = use[k]["new"]
        out[sel] = X[rng.integers(0, len(X), len(sel))]
    pw = np.exp(prior.logpdf(out) - prior.log_density)
    return out, pw / pw.sum()
