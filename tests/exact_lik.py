"""Exact likelihoods of small networks, independent of both implementations.

* immigration-death (0 -> X at rate k1, X -> 0 at rate k2 per molecule): the
  transition law over a step dt is Binomial(x, exp(-k2 dt)) survivors plus
  Poisson(k1/k2 (1 - exp(-k2 dt))) arrivals (an M/M/infinity queue).
* any small network: the chemical master equation on a truncated state box
  (finite state projection, Munsky & Khammash 2006, which the paper uses as
  its "almost exact" reference in Supplementary II), propagated with
  scipy.sparse.linalg.expm_multiply.

Both feed a forward algorithm: alpha_t(x) = sum_x' alpha_{t-1}(x') P(x' -> x)
times the observation density p(y_t | x); log p(y) = sum_t log sum_x alpha_t.
"""
import itertools

import numpy as np
import scipy.sparse as sp
from scipy import stats
from scipy.special import comb
from scipy.sparse.linalg import expm_multiply


def obs_density(kind, sigma, y, x):
    """Observation density of scalar y given counts x (array)."""
    x = np.asarray(x, dtype=np.float64)
    if kind == 0:
        return stats.norm.pdf(y, loc=x, scale=sigma)
    out = np.zeros_like(x)
    pos = x > 0
    out[pos] = stats.lognorm.pdf(y, s=sigma, scale=x[pos])
    return out


def immigration_death_loglik(k1, k2, x0, t0, t_obs, y, sigma, n_max=300):
    """Exact log p(y) for y_t = X(t_t) + N(0, sigma^2)."""
    states = np.arange(n_max + 1)
    alpha = np.zeros(n_max + 1)
    alpha[x0] = 1.0
    ll = 0.0
    t_prev = t0
    for t, yt in zip(t_obs, y):
        dt = t - t_prev
        p = np.exp(-k2 * dt)
        lam = k1 / k2 * (1.0 - p)
        surv = stats.binom.pmf(states[None, :], states[:, None], p)   # [x, s]
        arr = stats.poisson.pmf(states, lam)
        # P[x, x'] = sum_s surv[x, s] arr[x' - s]
        P = np.zeros((n_max + 1, n_max + 1))
        for s in range(n_max + 1):
            P[:, s:] += surv[:, s:s + 1] * arr[None, :n_max + 1 - s]
        alpha = alpha @ P
        alpha = alpha * obs_density(0, sigma, yt, states)
        z = alpha.sum()
        ll += np.log(z)
        alpha /= z
        t_prev = t
    return ll


class FSP:
    """Truncated CME generator of a mass-action network on a box of counts."""

    def __init__(self, orders, stoich, rates, bounds):
        orders = np.asarray(orders)
        stoich = np.asarray(stoich)
        self.bounds = list(bounds)
        self.U = len(bounds)
        self.states = np.array(list(itertools.product(*[range(b + 1) for b in bounds])),
                               dtype=np.int64)
        index = {tuple(s): k for k, s in enumerate(self.states)}
        n = len(self.states)
        rows, cols, vals = [], [], []
        out_rate = np.zeros(n)
        for k, s in enumerate(self.states):
            for r in range(len(rates)):
                a = rates[r]
                for u in range(self.U):
                    # Gillespie's combinatorial factor C(x_u, p_ru)
                    a *= float(comb(int(s[u]), int(orders[r, u]), exact=True))
                if a <= 0:
                    continue
                out_rate[k] += a
                tgt = tuple(s + stoich[r])
                if tgt in index:
                    rows.append(index[tgt])
                    cols.append(k)
                    vals.append(a)
                # transitions leaving the box are lost (sink)
        rows += list(range(n))
        cols += list(range(n))
        vals += list(-out_rate)
        self.A = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))  # d p / dt = A p

    def index_of(self, x):
        strides = np.cumprod([1] + [b + 1 for b in self.bounds[::-1]])[::-1][1:]
        return int(np.dot(np.asarray(x), strides))

    def propagate(self, p, dt):
        return expm_multiply(self.A * dt, p)

    def loglik(self, x0, t0, t_obs, y, obs_kind, observed, sigma):
        p = np.zeros(len(self.states))
        p[self.index_of(x0)] = 1.0
        ll, t_prev, lost = 0.0, t0, 0.0
        y = np.asarray(y).reshape(len(t_obs), -1)
        for t, yt in zip(t_obs, y):
            p = self.propagate(p, t - t_prev)
            lost = max(lost, 1.0 - p.sum())
            w = np.ones(len(p))
            for k, s in enumerate(observed):
                w *= obs_density(obs_kind, sigma, yt[k], self.states[:, s])
            p = p * w
            z = p.sum()
            ll += np.log(z)
            p /= z
            t_prev = t
        return ll, lost

    def marginal(self, x0, dt, species):
        p = np.zeros(len(self.states))
        p[self.index_of(x0)] = 1.0
        p = self.propagate(p, dt)
        out = np.zeros(self.bounds[species] + 1)
        np.add.at(out, self.states[:, species], p)
        return out
