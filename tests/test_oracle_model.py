"""Pins of the oracle's model pieces against exact or closed-form results.

* propensities: Gillespie's combinatorial mass action (0th, 1st, 2nd order,
  homo- and hetero-dimeric) against exact integer combinatorics, one rounding.
* systematic resampling: the defining properties (offspring counts within
  floor/ceil of H w_i, total H, ancestors non-decreasing, expectation H w_i
  over the offset), the degenerate cases (equal weights -> identity, one
  non-zero weight -> all copies).
* direct-method SSA: marginals against closed forms (immigration-death from 0
  is Poisson, pure death is Binomial, a two-state switch has an explicit
  occupation probability, pure immigration counts events as a Poisson
  process) and against the truncated CME for second-order reactions;
  conservation laws along paths; the random-number stream of each mode
  (which Philox words an event's uniforms come from, and how they are
  rounded), recomputed path by path, clocks included; reaction choices put
  on the boundary of the second uniform.  Every one of these runs in both
  arithmetic modes: the binary64 step and the FP32-mixed step (binary32
  propensities, uniforms and waiting times, binary64 clock), whose event
  loop is a separate branch of the oracle.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from tests.exact_lik import FSP


def _problem(orc, orders, stoich, **kw):
    U = np.asarray(orders).shape[1]
    traj = {"t_obs": [1.0], "y": [[1.0]], "t0": 0.0, "x0": np.zeros(U, np.int32)}
    args = dict(obs_kind=0, observed=[0], sigma=1.0, theta=np.ones((1, len(orders))),
                trajectories=[traj], n_particles=1, seed=kw.pop("seed", 5))
    args.update(kw)
    return orc.Problem(orders, stoich, **args)


def test_propensity_mass_action_exact(orc):
    # species A, B; reactions: 0 -> A, A -> 0, 2A -> B, A + B -> 0, B -> A
    orders = [[0, 0], [1, 0], [2, 0], [1, 1], [0, 1]]
    stoich = [[1, 0], [-1, 0], [-2, 1], [-1, -1], [1, -1]]
    P = _problem(orc, orders, stoich)
    rng = np.random.default_rng(7)
    for _ in range(300):
        x = [int(v) for v in rng.integers(0, 2**30, size=2)]
        if rng.random() < 0.3:
            x = [int(v) for v in rng.integers(0, 4, size=2)]
        c = rng.uniform(0, 100, size=5) * 10.0 ** rng.integers(-6, 3, size=5)
        got = orc.propensities(P, c, x)
        h = [1, x[0], x[0] * (x[0] - 1) // 2, x[0] * x[1], x[1]]
        for r in range(5):
            # one rounding of the exact integer factor, one of the product
            want = float(c[r]) * float(Fraction(h[r]))
            assert got[r] == want, (r, x, got[r], want)
        got32 = orc.propensities(P, c, x, precision=orc.FP32_MIXED)
        for r in range(5):
            want = float(np.float32(c[r]) * np.float32(float(h[r])))
            assert got32[r] == want


def _offspring(anc, H):
    return np.bincount(anc, minlength=H)


def test_resampling_invariants(orc):
    rng = np.random.default_rng(8)
    for trial in range(400):
        H = int(rng.integers(1, 70))
        lw = rng.normal(0, rng.choice([0.1, 3.0, 30.0]), size=H)
        if trial % 5 == 0:
            lw[rng.random(H) < 0.5] = -np.inf
            lw[0] = 0.0
        e = np.array([orc.exp(v - lw.max()) for v in lw])
        w64 = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        anc = orc.resample(e, w64)
        assert np.all(np.diff(anc) >= 0)
        assert anc.min() >= 0 and anc.max() < H
        q = np.floor(e * 2.0**32)
        Q = q.sum()
        off = _offspring(anc, H)
        assert off.sum() == H
        lo = np.floor(H * q / Q)
        hi = np.ceil(H * q / Q)
        assert np.all(off >= lo) and np.all(off <= hi), (off, H * q / Q)
        assert np.all(off[q == 0] == 0)


def test_resampling_expectation_over_offset(orc):
    # systematic resampling is unbiased: averaged over the uniform offset,
    # particle i receives H w_i copies
    H = 7
    e = np.array([1.0, 0.3, 0.0, 0.05, 0.9, 0.5, 1e-3])
    q = np.floor(e * 2.0**32)
    want = H * q / q.sum()
    n = 4000
    acc = np.zeros(H)
    for k in range(n):
        w64 = (k * 2**64) // n + 12345
        acc += _offspring(orc.resample(e, w64), H)
    assert np.allclose(acc / n, want, atol=2e-3)


def test_resampling_degenerate_cases(orc):
    for H in [1, 2, 5, 64, 1000]:
        e = np.ones(H)
        for w64 in [0, 2**63, 2**64 - 1]:
            assert np.array_equal(orc.resample(e, w64), np.arange(H))
        one = np.zeros(H)
        one[H // 2] = 1.0
        assert np.all(orc.resample(one, 2**62) == H // 2)


IMM_DEATH = ([[0], [1]], [[1], [-1]])


PRECISIONS = [0, 1]   # binary64 step, FP32-mixed step


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("k1,k2,t", [(10.0, 0.1, 5.0), (3.0, 1.0, 2.5), (50.0, 2.0, 10.0)])
def test_ssa_immigration_death_poisson(orc, k1, k2, t, precision):
    P = _problem(orc, *IMM_DEATH, precision=precision)
    n = 20000
    states, ev, st = orc.ssa_paths(P, [k1, k2], [0], 0.0, t, n, theta_id=int(k1))
    assert st == 0
    lam = k1 / k2 * (1 - math.exp(-k2 * t))
    x = states[:, 0]
    # chi-square against the Poisson law on bins with expected count >= 20
    kmax = int(lam + 8 * math.sqrt(lam) + 10)
    obs = np.bincount(np.minimum(x, kmax), minlength=kmax + 1).astype(float)
    exp_ = stats.poisson.pmf(np.arange(kmax + 1), lam) * n
    exp_[-1] += stats.poisson.sf(kmax, lam) * n
    keep = exp_ >= 20
    o = np.append(obs[keep], obs[~keep].sum())
    ex = np.append(exp_[keep], exp_[~keep].sum())
    chi2 = ((o - ex) ** 2 / np.maximum(ex, 1e-12)).sum()
    p = stats.chi2.sf(chi2, len(o) - 1)
    assert p > 1e-4, (chi2, p)


def test_fp32_mixed_takes_half_a_block_per_event(orc):
    # The FP32-mixed stream layout, recomputed here from Philox blocks (pinned
    # to rocRAND) and the binary32 log (pinned to mpmath): events 2p and
    # 2p + 1 of a path share block p = (p, path, 0, theta_id << 2) under key
    # (seed), the first taking u1, u2 from words 0, 1 and the second from
    # words 2, 3, the leading 24 bits of each.  Two birth reactions, so that
    # both the waiting times (u1) and the choice of reaction (u2) are checked;
    # each path's clock, the binary64 sum of its binary32 waiting times, is
    # compared bit for bit, so that a uniform off by half an ulp shows.
    rates, t_end, n_paths, theta_id, seed = (2.0, 1.0), 3.0, 150, 7, 5
    P = _problem(orc, [[0, 0], [0, 0]], [[1, 0], [0, 1]], precision=1, seed=seed)
    states, ev, st, clk = orc.ssa_paths(P, list(rates), [0, 0], 0.0, t_end, n_paths,
                                        theta_id=theta_id, clocks=True)
    assert st == 0
    key = [seed & 0xFFFFFFFF, seed >> 32]
    a = [np.float32(r) for r in rates]          # float(c) * float(1) for order 0
    sf = np.float32(a[0] + a[1])
    for j in range(n_paths):
        clock, n, x = 0.0, 0, [0, 0]
        while True:
            w = orc.philox([n >> 1, j, 0, theta_id << 2], key)
            h = 2 * (n & 1)
            u1 = np.float32(((int(w[h]) >> 8) + 1) * 2.0**-24)
            u2 = np.float32((int(w[h + 1]) >> 8) * 2.0**-24)
            tau = np.float32(-np.float32(orc.logf(u1))) / sf
            if clock + float(tau) > t_end:
                break
            r = 0 if a[0] > np.float32(u2 * sf) else 1
            x[r] += 1
            clock += float(tau)
            n += 1
        assert int(ev[j]) == n and list(states[j]) == x, (j, n, x)
        assert clk[j] == clock, (j, clk[j], clock)
    assert ev.mean() > 5


def test_fp64_takes_a_block_per_event(orc):
    # The binary64 stream layout, recomputed from Philox blocks (pinned to
    # rocRAND) and the binary64 log (pinned to mpmath): event n of a path
    # takes block (n, path, 0, theta_id << 2) under key (seed), u1 from the
    # leading 53 bits of words 1:0 plus one ulp (so in (0, 1]) and u2 from the
    # leading 53 bits of words 3:2; the waiting time is -log(u1) / a0 and the
    # reaction the first whose running sum exceeds u2 a0.  Events, states and
    # each path's clock are compared exactly.
    rates, t_end, n_paths, theta_id, seed = (2.0, 1.0), 3.0, 150, 11, 9
    P = _problem(orc, [[0, 0], [0, 0]], [[1, 0], [0, 1]], precision=0, seed=seed)
    states, ev, st, clk = orc.ssa_paths(P, list(rates), [0, 0], 0.0, t_end, n_paths,
                                        theta_id=theta_id, clocks=True)
    assert st == 0
    key = [seed & 0xFFFFFFFF, seed >> 32]
    a0 = rates[0] + rates[1]
    for j in range(n_paths):
        clock, n, x = 0.0, 0, [0, 0]
        while True:
            w = [int(v) for v in orc.philox([n, j, 0, theta_id << 2], key)]
            z1 = ((w[1] << 32) | w[0]) >> 11
            z2 = ((w[3] << 32) | w[2]) >> 11
            u1 = (z1 + 1) * 2.0**-53
            u2 = z2 * 2.0**-53
            tau = -orc.log(u1) / a0
            if clock + tau > t_end:
                break
            r = 0 if rates[0] > u2 * a0 else 1
            x[r] += 1
            clock += tau
            n += 1
        assert int(ev[j]) == n and list(states[j]) == x and clk[j] == clock, (j, n, x)
    assert ev.mean() > 5


def _event_uniforms(orc, precision, seed, theta_id, j, n):
    """(u1, u2) of event n of path j under the stream layout of each mode:
    binary64 takes block n, 53 leading bits of words 1:0 and 3:2; FP32-mixed
    takes half of block n >> 1, 24 leading bits of each word."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    if precision == 1:
        w = [int(v) for v in orc.philox([n >> 1, j, 0, theta_id << 2], key)]
        h = 2 * (n & 1)
        return (np.float32(((w[h] >> 8) + 1) * 2.0**-24),
                np.float32((w[h + 1] >> 8) * 2.0**-24))
    w = [int(v) for v in orc.philox([n, j, 0, theta_id << 2], key)]
    return (((((w[1] << 32) | w[0]) >> 11) + 1) * 2.0**-53,
            (((w[3] << 32) | w[2]) >> 11) * 2.0**-53)


def _two_births_path(orc, precision, k1, t_end, seed, theta_id, j, u2_at=None):
    """Path j of the two-birth network with rates (k1, 1 - k1), whose total
    propensity is exactly 1 in both modes, recomputed event by event; u2_at =
    (n, value) replaces event n's second uniform (a planted deviation)."""
    f = np.float32 if precision == 1 else float
    a1 = f(k1)
    a0 = f(a1 + f(1.0 - k1))
    assert a0 == 1.0
    clock, n, x = 0.0, 0, [0, 0]
    while True:
        u1, u2 = _event_uniforms(orc, precision, seed, theta_id, j, n)
        if u2_at is not None and u2_at[0] == n:
            u2 = f(u2_at[1])
        if precision == 1:
            tau = float(np.float32(-np.float32(orc.logf(u1))) / a0)
        else:
            tau = -orc.log(u1) / a0
        if clock + tau > t_end:
            break
        x[0 if a1 > f(u2 * a0) else 1] += 1
        clock += tau
        n += 1
    return n, x


@pytest.mark.parametrize("precision", PRECISIONS)
def test_reaction_choice_on_the_boundary(orc, precision):
    # The second uniform only picks the reaction: the first whose running sum
    # exceeds u2 a0.  With random rates a wrong rounding of u2 moves a choice
    # with probability of about one grid step per event, which no path count
    # resolves.  Here the boundary is put on the uniform itself: two birth
    # reactions with rates (b, 1 - b), exact in both modes, so a0 = 1 and the
    # first reaction fires iff u2 < b.  With b = u2 of a chosen event, the
    # correct u2 takes the second reaction and any smaller one the first;
    # with b one grid step above u2 (u2 >= 1/2, where that step is the ulp),
    # the correct u2 takes the first reaction and any larger one the second.
    # Each case is checked to tell the planted neighbour from the correct
    # value; the oracle's path must agree with the correct one.
    f32 = precision == 1
    grid = 2.0**-24 if f32 else 2.0**-53
    seed, theta_id, t_end = 13, 3, 6.0
    cases = {"below": 0, "above": 0}
    for j in range(48):
        for n in range(4):                 # both halves of an FP32-mixed block
            _, u2 = _event_uniforms(orc, precision, seed, theta_id, j, n)
            u2 = float(u2)
            for side, b, planted in (("below", u2, np.nextafter(u2, 0.0)),
                                     ("above", u2 + grid, u2 + grid)):
                if cases[side] >= 8 or u2 == 0.0 or (side == "above" and u2 < 0.5):
                    continue
                if f32:
                    planted = float(np.nextafter(np.float32(u2), np.float32(0.0))) \
                        if side == "below" else planted
                want = _two_births_path(orc, precision, b, t_end, seed, theta_id, j)
                if want[0] <= n:
                    continue                # the event falls after t_end
                bad = _two_births_path(orc, precision, b, t_end, seed, theta_id, j,
                                       u2_at=(n, planted))
                assert bad != want, (side, j, n)
                P = _problem(orc, [[0, 0], [0, 0]], [[1, 0], [0, 1]],
                             precision=precision, seed=seed)
                states, ev, st = orc.ssa_paths(P, [b, 1.0 - b], [0, 0], 0.0, t_end, j + 1,
                                               theta_id=theta_id)
                assert st == 0
                assert (int(ev[j]), list(states[j])) == want, (side, j, n, b)
                cases[side] += 1
    assert cases == {"below": 8, "above": 8}


@pytest.mark.parametrize("precision", PRECISIONS)
def test_ssa_pure_death_binomial(orc, precision):
    P = _problem(orc, *IMM_DEATH, precision=precision)
    n, x0, k2, t = 20000, 40, 0.3, 2.0
    states, ev, st = orc.ssa_paths(P, [0.0, k2], [x0], 0.0, t, n)
    x = states[:, 0]
    p = math.exp(-k2 * t)
    obs = np.bincount(x, minlength=x0 + 1).astype(float)
    exp_ = stats.binom.pmf(np.arange(x0 + 1), x0, p) * n
    keep = exp_ >= 20
    o = np.append(obs[keep], obs[~keep].sum())
    ex = np.append(exp_[keep], exp_[~keep].sum())
    chi2 = ((o - ex) ** 2 / ex).sum()
    assert stats.chi2.sf(chi2, len(o) - 1) > 1e-4
    # every event is a death: events = x0 - x
    assert np.array_equal(ev.astype(np.int64), x0 - x.astype(np.int64))


@pytest.mark.parametrize("precision", PRECISIONS)
def test_ssa_pure_immigration_event_count(orc, precision):
    P = _problem(orc, *IMM_DEATH, precision=precision)
    n, k1, t = 20000, 7.0, 3.0
    states, ev, st = orc.ssa_paths(P, [k1, 0.0], [0], 0.0, t, n)
    assert np.array_equal(states[:, 0].astype(np.uint64), ev)
    m, v = ev.mean(), ev.var()
    se = math.sqrt(k1 * t / n)
    assert abs(m - k1 * t) < 5 * se
    assert abs(v / (k1 * t) - 1) < 0.05


@pytest.mark.parametrize("precision", PRECISIONS)
def test_ssa_telegraph_switch_and_conservation(orc, precision):
    from paper_1606_08281_amd.workloads import telegraph
    net = telegraph()
    P = _problem(orc, net.orders, net.stoich, precision=precision)
    kon, koff, t = 0.7, 0.3, 1.5
    c = [kon, koff, 5.0, 1.0, 2.0, 0.5]
    n = 20000
    states, ev, st = orc.ssa_paths(P, c, [1, 0, 0, 0], 0.0, t, n)
    assert np.all(states.sum(axis=0) >= 0) and np.all(states >= 0)
    assert np.all(states[:, 0] + states[:, 1] == 1)
    p_on = kon / (kon + koff) * (1 - math.exp(-(kon + koff) * t))
    frac = states[:, 1].mean()
    assert abs(frac - p_on) < 5 * math.sqrt(p_on * (1 - p_on) / n)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("case", ["dimer", "hetero"])
def test_ssa_second_order_against_cme(orc, case, precision):
    if case == "dimer":   # 2A -> B, B -> 2A
        orders, stoich, c, x0, bounds = [[2, 0], [0, 1]], [[-2, 1], [2, -1]], [0.05, 0.4], [20, 0], [20, 10]
    else:                 # A + B -> C, C -> A + B
        orders = [[1, 1, 0], [0, 0, 1]]
        stoich = [[-1, -1, 1], [1, 1, -1]]
        c, x0, bounds = [0.08, 0.5], [12, 9, 0], [12, 9, 9]
    P = _problem(orc, orders, stoich, precision=precision)
    t, n = 1.3, 20000
    states, ev, st = orc.ssa_paths(P, c, x0, 0.0, t, n)
    fsp = FSP(orders, stoich, c, bounds)
    want = fsp.marginal(x0, t, 0) * n
    obs = np.bincount(states[:, 0], minlength=len(want)).astype(float)[:len(want)]
    keep = want >= 20
    o = np.append(obs[keep], obs[~keep].sum())
    ex = np.append(want[keep], want[~keep].sum())
    chi2 = ((o - ex) ** 2 / ex).sum()
    assert stats.chi2.sf(chi2, len(o) - 1) > 1e-4, chi2
