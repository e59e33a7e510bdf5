"""GPU path (liblik.so, HIP kernels) against the CPU oracle, element by element.

The bar: bit-exact integer results (per-filter event counts, final particle
counts, statuses) and log-likelihoods within 1e-9 relative (binary64 and
FP32-mixed alike: both modes share the binary64 weight/log-sum-exp path,
whose only freedom is the summation order of the particle weights); the
FP32-mixed results are also held to 1e-4 absolute against the oracle's
FP32-mixed mode.
"""
import numpy as np
import pytest

from paper_1606_08281_amd import workloads as W

pytestmark = pytest.mark.gpu

REL = 1e-9
FP32_ABS = 1e-4


def _oracle(orc, wl, theta=None, theta_ids=None, H=None, precision=0, event_cap=100_000_000,
            trajectories=None, seed=None):
    P = orc.Problem(wl.net.orders, wl.net.stoich, wl.obs_kind, wl.observed, wl.sigma,
                    wl.theta if theta is None else theta,
                    wl.trajectories if trajectories is None else trajectories,
                    H or wl.n_particles, wl.seed if seed is None else seed,
                    precision=precision, event_cap=event_cap, theta_ids=theta_ids)
    return orc.evaluate(P, want_final_state=True)


def _gpu(wl, theta=None, theta_ids=None, H=None, precision=0, event_cap=0, trajectories=None,
         seed=None, kernel=1, tuning=None):
    from paper_1606_08281_amd import lik
    net = lik.Network(wl.net.orders, wl.net.stoich)
    if tuning:
        net.set_tuning(**tuning)
    return lik.eval_batch(net, wl.obs_kind, wl.observed, wl.sigma,
                          wl.theta if theta is None else theta,
                          wl.trajectories if trajectories is None else trajectories,
                          H or wl.n_particles, wl.seed if seed is None else seed,
                          precision=precision, event_cap=event_cap, theta_ids=theta_ids,
                          aux=True, kernel=kernel)


def assert_parity(got, ref, check_state=True, abs_tol=None):
    assert np.array_equal(got["status"], ref["status"]), (got["status"], ref["status"])
    ok_theta = ref["status"] == 0
    M = len(ref["events"]) // max(len(ref["status"]), 1)
    ok_f = np.repeat(ok_theta, M)
    assert np.array_equal(got["filter_events"][ok_f], ref["events"][ok_f])
    if check_state:
        assert np.array_equal(got["final_state"][ok_f], ref["final_state"][ok_f])
    a, b = got["loglik"], ref["loglik"]
    assert np.array_equal(np.isnan(a), np.isnan(b))
    assert np.array_equal(np.isneginf(a), np.isneginf(b))
    fin = np.isfinite(b)
    err = np.abs(a[fin] - b[fin])
    assert np.all(err <= REL * np.abs(b[fin])), (err.max(), a[fin][np.argmax(err)], b[fin][np.argmax(err)])
    if abs_tol is not None:
        assert np.all(err <= abs_tol), err.max()
    fa, fb = got["filter_loglik"][ok_f], ref["filter_ll"][ok_f]
    fin = np.isfinite(fb)
    assert np.all(np.abs(fa[fin] - fb[fin]) <= REL * np.abs(fb[fin]))


def _say(*a):
    print("[gpu case]", *a, flush=True)


KERNELS = [1, 2]   # generic, network-specialised


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [0, 1])
def test_immigration_death_full_batch(orc, precision, kernel):
    wl = W.immigration_death_workload()
    _say("immigration-death 64x256x20", "precision", precision, "kernel", kernel)
    assert_parity(_gpu(wl, precision=precision, kernel=kernel),
                  _oracle(orc, wl, precision=precision), abs_tol=FP32_ABS if precision else None)


def _telegraph_subset(n_obs=50):
    wl = W.telegraph_workload(n_theta=1024, n_obs=n_obs)
    # a cost-stratified sample of the prior draws the oracle finishes quickly:
    # rates that matter most for the event count are k_m k_p / gamma_m
    th = wl.theta
    cost = th[:, 2] / th[:, 3] * th[:, 4] + th[:, 2]
    order = np.argsort(cost)
    idx = np.concatenate([order[:6], order[300:303], order[600:602]])
    return wl, np.sort(idx)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [0, 1])
def test_telegraph_subset_full_shape(orc, precision, kernel):
    wl, idx = _telegraph_subset()
    trajs = wl.trajectories[:3]
    _say("telegraph subset", idx.tolist(), "M=3 H=1000 T=50 precision", precision, "kernel", kernel)
    got = _gpu(wl, theta=wl.theta[idx], theta_ids=idx, trajectories=trajs, precision=precision,
               kernel=kernel)
    ref = _oracle(orc, wl, theta=wl.theta[idx], theta_ids=idx, trajectories=trajs,
                  precision=precision)
    assert_parity(got, ref, abs_tol=FP32_ABS if precision else None)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("H", [1, 63, 64, 65, 200, 4096])
def test_particle_counts_ragged(orc, H, kernel):
    wl = W.immigration_death_workload(n_theta=5, n_particles=H)
    _say("ragged H", H, "kernel", kernel)
    assert_parity(_gpu(wl, kernel=kernel), _oracle(orc, wl))


def test_uneven_trajectory_lengths(orc):
    wl = W.telegraph_workload(n_theta=4, n_traj=3, n_obs=20, n_particles=130)
    trajs = []
    for m, T in enumerate([1, 20, 7]):
        tr = dict(wl.trajectories[m])
        tr["t_obs"] = tr["t_obs"][:T]
        tr["y"] = tr["y"][:T]
        trajs.append(tr)
    theta = np.vstack([W.TELEGRAPH_TRUTH * s for s in [1.0, 0.5, 2.0, 1.3]])
    _say("uneven T", [1, 20, 7])
    assert_parity(_gpu(wl, theta=theta, trajectories=trajs),
                  _oracle(orc, wl, theta=theta, trajectories=trajs))


@pytest.mark.parametrize("kernel", KERNELS)
def test_statuses_and_degenerate_inputs(orc, kernel):
    wl = W.immigration_death_workload(n_theta=6, n_particles=70)
    theta = np.array([[10, 0.1], [-1, 0.1], [np.nan, 1], [np.inf, 1], [0, 0], [1e-300, 1e-300]])
    _say("statuses kernel", kernel)
    assert_parity(_gpu(wl, theta=theta, kernel=kernel), _oracle(orc, wl, theta=theta))
    _say("event cap 3")
    assert_parity(_gpu(wl, theta=wl.theta[:3], event_cap=3, kernel=kernel),
                  _oracle(orc, wl, theta=wl.theta[:3], event_cap=3), check_state=False)
    tw = W.telegraph_workload(n_theta=2, n_traj=1, n_obs=4, n_particles=16)
    tr = dict(tw.trajectories[0])
    tr["x0"] = np.array([1, 0, 0, 0], np.int32)
    th = np.vstack([np.zeros(6), [0.1, 0.1, 0.0, 1.0, 0.0, 1.0]])
    _say("log-normal, zero protein -> -inf")
    got = _gpu(tw, theta=th, trajectories=[tr], kernel=kernel)
    assert np.all(got["loglik"] == -np.inf)
    assert_parity(got, _oracle(orc, tw, theta=th, trajectories=[tr]))


def test_batch_composition_does_not_change_results(orc):
    wl = W.immigration_death_workload(n_theta=16, n_particles=96)
    _say("composition")
    full = _gpu(wl)
    idx = np.array([9, 3, 15])
    sub = _gpu(wl, theta=wl.theta[idx], theta_ids=idx)
    assert np.array_equal(sub["loglik"], full["loglik"][idx])
    assert np.array_equal(sub["final_state"], full["final_state"][idx])
    again = _gpu(wl)
    assert np.array_equal(again["loglik"], full["loglik"])


def test_device_entry_point_matches_host_entry_point(orc):
    import torch
    from paper_1606_08281_amd import lik
    wl = W.telegraph_workload(n_theta=8, n_traj=2, n_obs=10, n_particles=256)
    net = lik.Network(wl.net.orders, wl.net.stoich)
    _say("device entry point")
    host = lik.eval_batch(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta, wl.trajectories,
                          wl.n_particles, wl.seed)
    db = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories,
                         wl.n_theta, wl.n_particles)
    theta = torch.from_numpy(wl.theta).cuda()
    for _ in range(2):
        ll, st = db.run(theta, wl.seed)
        torch.cuda.synchronize()
        assert np.array_equal(ll.cpu().numpy(), host["loglik"])
        assert np.array_equal(st.cpu().numpy(), host["status"])


@pytest.mark.parametrize("precision", [0, 1])
def test_random_network_20x40_small(orc, precision):
    # 20 species, 40 reactions of orders 0-2: both kernel variants, short run
    wl = W.random_network_workload(n_theta=64, n_particles=96, n_obs=3, events_per_interval=300)
    idx = np.arange(0, 64, 8)
    for kernel in KERNELS:
        _say("random 20x40 theta", idx.tolist(), "H=96 T=3 precision", precision, "kernel", kernel)
        got = _gpu(wl, theta=wl.theta[idx], theta_ids=idx, precision=precision, kernel=kernel)
        ref = _oracle(orc, wl, theta=wl.theta[idx], theta_ids=idx, precision=precision)
        assert_parity(got, ref, abs_tol=FP32_ABS if precision else None)


def _small_random_workload(U, R, n_theta=6, n_particles=128, n_obs=4, events=200.0):
    # seeded random network of U species and R reactions, x0 ~ Poisson(50),
    # rates log-uniform on [1e-2, 1], observation interval set for about
    # `events` events per particle, synthetic Gaussian data on species 0, 1
    net = W.random_network(n_species=U, n_reactions=R, seed=W.SEED_NET + 1000 * U + R)
    rng = np.random.Generator(np.random.PCG64(W.SEED_DATA + 1000 * U + R))
    x0 = rng.poisson(50, U).astype(np.int32)
    theta = W.log_uniform(rng, np.full(R, 1e-2), np.full(R, 1.0), n_theta)
    a0 = np.median([(th * net.propensity_factor(x0)).sum() for th in theta])
    t_obs = (events / a0) * np.arange(1, n_obs + 1, dtype=np.float64)
    y = rng.normal(50.0, 10.0, (n_obs, 2))
    traj = {"t_obs": t_obs, "y": y, "t0": 0.0, "x0": x0}
    return W.Workload(f"random-{U}x{R}", net, W.OBS_GAUSSIAN, [0, 1], 10.0, theta, [traj],
                      n_particles)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("shape", [(3, 12), (4, 9), (6, 10), (8, 16)])
def test_net_change_packing(orc, shape, precision):
    # net changes are packed as bytes for at most four species and as 4-bit
    # fields beyond; the generic kernel runs a network of at most four
    # species but more than eight reactions in a wider instance, which must
    # still read bytes.  Both kernel variants against the oracle.
    U, R = shape
    wl = _small_random_workload(U, R)
    ref = _oracle(orc, wl, precision=precision)
    assert np.all(ref["status"] == 0), ref["status"]
    for kernel in KERNELS:
        _say("net-change packing U", U, "R", R, "precision", precision, "kernel", kernel)
        got = _gpu(wl, precision=precision, kernel=kernel)
        assert_parity(got, ref, abs_tol=FP32_ABS if precision else None)


def test_graph_replays_match_eager():
    # the captured launch sequence, replayed with a new seed each time and
    # with eager work in between, equals eager launches every time
    import torch
    from paper_1606_08281_amd import lik
    wl = W.telegraph_workload(n_theta=24, n_traj=2, n_obs=12, n_particles=200)
    for kernel in KERNELS:
        net = lik.Network(wl.net.orders, wl.net.stoich)
        eager = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories,
                                wl.n_theta, wl.n_particles, kernel=kernel)
        graph = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories,
                                wl.n_theta, wl.n_particles, kernel=kernel, graph=True)
        theta = torch.from_numpy(wl.theta).cuda()
        for k in range(4):
            _say("graph replay", k, "kernel", kernel)
            ll_e = eager.run(theta, wl.seed + k)[0].clone()
            ev_e = eager.events.clone()
            junk = torch.randn(4096, device="cuda").sum()   # eager work between replays
            ll_g = graph.run(theta, wl.seed + k)[0].clone()
            ev_g = graph.events.clone()
            torch.cuda.synchronize()
            assert float(junk) == float(junk)
            assert torch.equal(ll_e, ll_g), k
            assert torch.equal(ev_e, ev_g), k
        host = lik.eval_batch(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta, wl.trajectories,
                              wl.n_particles, wl.seed + 3, kernel=kernel)
        assert np.array_equal(ll_g.cpu().numpy(), host["loglik"])


_COST_ORDER = []


def telegraph_cost_order(orc):
    """The benchmark telegraph batch's rate vectors, most SSA events first,
    ranked by an oracle run of every theta at 16 particles against two
    trajectories (a cheap, deterministic ranking; a few seconds)."""
    if not _COST_ORDER:
        wl = W.telegraph_workload()
        P = orc.Problem(wl.net.orders, wl.net.stoich, wl.obs_kind, wl.observed, wl.sigma,
                        wl.theta, wl.trajectories[:2], 16, wl.seed)
        ev = orc.evaluate(P)["events"].reshape(wl.n_theta, 2).sum(axis=1)
        _COST_ORDER.append(np.argsort(ev, kind="stable")[::-1].copy())
    return _COST_ORDER[0]


def heaviest_telegraph_theta(orc, k):
    return telegraph_cost_order(orc)[:k]


@pytest.mark.parametrize("precision", [0, 1])
def test_telegraph_full_batch_sampled(orc, precision):
    # the benchmark's batch and launch configuration (device entry point,
    # automatic kernel choice, default schedule): 1024 theta x 10 trajectories
    # x 1000 particles x 50 observations.  The oracle recomputes a sample that
    # spans the cost range -- by an oracle ranking of the batch, the six
    # heaviest rate vectors (up to 1.2e5 events per particle: long pools,
    # drain draws at thousands of events, protein counts in the thousands),
    # then ranks 10, 30, 100, 300, 600 and 900 and the three lightest -- with
    # all ten trajectories each: per-filter event counts, final particle
    # counts and log-likelihoods.
    import torch
    from paper_1606_08281_amd import lik
    wl = W.telegraph_workload()
    net = lik.Network(wl.net.orders, wl.net.stoich)
    db = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories, wl.n_theta,
                         wl.n_particles, precision=precision)
    final = torch.empty((wl.n_theta * wl.n_traj, wl.net.U, wl.n_particles), dtype=torch.int32,
                        device="cuda")
    _say("telegraph full batch 1024x10x1000x50 precision", precision)
    ll, st = db.run(torch.from_numpy(wl.theta).cuda(), wl.seed, final_state=final)
    torch.cuda.synchronize()
    ll, st = ll.cpu().numpy(), st.cpu().numpy()
    M = wl.n_traj
    events = db.events.cpu().numpy().astype(np.uint64).reshape(wl.n_theta, M)
    fll = db.filter_loglik.cpu().numpy().reshape(wl.n_theta, M)
    th = wl.theta
    order = telegraph_cost_order(orc)
    heavy = order[:6]
    idx = np.unique(order[[0, 1, 2, 3, 4, 5, 10, 30, 100, 300, 600, 900, 1021, 1022, 1023]])
    _say("oracle sample", idx.tolist(), "heaviest", heavy.tolist())
    ref = _oracle(orc, wl, theta=th[idx], theta_ids=idx, precision=precision)
    fs = final.view(wl.n_theta, M, wl.net.U, wl.n_particles)[torch.from_numpy(idx).cuda()]
    fs = fs.cpu().numpy().reshape(len(idx) * M, wl.net.U, wl.n_particles)
    assert np.array_equal(st[idx], ref["status"])
    assert np.array_equal(events[idx].ravel(), ref["events"])
    assert np.array_equal(fs, ref["final_state"])
    assert np.all(np.abs(fll[idx].ravel() - ref["filter_ll"]) <= REL * np.abs(ref["filter_ll"]))
    assert np.all(np.abs(ll[idx] - ref["loglik"]) <= REL * np.abs(ref["loglik"]))
    if precision:
        assert np.all(np.abs(ll[idx] - ref["loglik"]) <= FP32_ABS)
    # the sample reaches the top of the batch (a check of coverage, by the
    # events the GPU ran): a rate vector among the heaviest five, and most of
    # the heavy six among the heaviest 3 %
    rank = np.argsort(np.argsort(-events.sum(axis=1).astype(np.int64)))
    _say("batch ranks of the sample", dict(zip(idx.tolist(), rank[idx].tolist())))
    assert rank[idx].min() < 5, rank[idx]
    assert np.sum(rank[heavy] < 31) >= 4, rank[heavy]
    assert np.all(st == 0) and np.all(np.isfinite(ll))


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [0, 1])
def test_heaviest_theta_at_4096_particles(orc, precision, kernel):
    # the four heaviest telegraph rate vectors at the largest particle count
    # (pools of several groups of 64, drain draws at thousands of events per
    # particle), one trajectory, five observations: bit-exact
    wl = W.telegraph_workload()
    heavy = np.sort(heaviest_telegraph_theta(orc, 4))
    trajs = [dict(wl.trajectories[3], t_obs=wl.trajectories[3]["t_obs"][:5],
                  y=wl.trajectories[3]["y"][:5])]
    _say("heaviest theta", heavy.tolist(), "H=4096 T=5 precision", precision, "kernel", kernel)
    got = _gpu(wl, theta=wl.theta[heavy], theta_ids=heavy, H=4096, trajectories=trajs,
               precision=precision, kernel=kernel)
    ref = _oracle(orc, wl, theta=wl.theta[heavy], theta_ids=heavy, H=4096, trajectories=trajs,
                  precision=precision)
    assert_parity(got, ref, abs_tol=FP32_ABS if precision else None)
    assert ref["events"].min() > 4096 * 5 * 100


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [0, 1])
def test_count_overflow(orc, precision, kernel):
    # counts started just below 2^30 under immigration: a filter stops with
    # COUNT_OVERFLOW at the first interval whose end count exceeds 2^30, on
    # both sides, after the same events; the others run to the end
    wl = W.immigration_death_workload(n_theta=4, n_particles=130)
    limit = 1 << 30
    tr = dict(wl.trajectories[0])
    tr["x0"] = np.array([limit - 300], np.int32)
    tr["y"] = tr["y"] + float(limit - 300)
    theta = np.array([[10.0, 0.0], [10.0, 1e-9], [0.5, 0.0], [1e-3, 1e-9]])
    _say("count overflow precision", precision, "kernel", kernel)
    got = _gpu(wl, theta=theta, trajectories=[tr], precision=precision, kernel=kernel)
    ref = _oracle(orc, wl, theta=theta, trajectories=[tr], precision=precision)
    assert list(ref["status"]) == [2, 2, 0, 0], ref["status"]
    assert_parity(got, ref)
    assert np.array_equal(got["filter_events"], ref["events"])   # the stopped ones too


def _boundary_batch(orc, precision, n_theta, H, seed, t1):
    """Rate vectors (b, 1 - b) of two birth reactions (total propensity exactly
    1), each putting one event of one particle of the first interval on the
    second uniform's boundary: b at that event's u2 (any smaller u2 flips the
    choice) or, for u2 >= 1/2, one grid step above it (any larger u2 does).
    Row i is stream theta_id i; the first interval of trajectory 0 uses the
    same counters as a plain path (c2 = 0), so the uniforms are those of the
    oracle's pinned stream layout."""
    from tests.test_oracle_model import _event_uniforms, _two_births_path
    grid = 2.0**-24 if precision == 1 else 2.0**-53
    theta = []
    for i in range(n_theta):
        side = "below" if i % 2 == 0 else "above"
        for k in range(4 * H):
            j, n = (i * 7 + k) % H, k % 4
            u2 = float(_event_uniforms(orc, precision, seed, i, j, n)[1])
            if u2 == 0.0 or (side == "above" and u2 < 0.5):
                continue
            b = u2 if side == "below" else u2 + grid
            if _two_births_path(orc, precision, b, t1, seed, i, j)[0] > n:
                theta.append([b, 1.0 - b])
                break
        else:
            raise AssertionError(("no boundary event", i))
    return np.array(theta)


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [0, 1])
def test_reaction_choice_on_the_boundary(orc, precision, kernel, schedule):
    # every rate vector puts one event of the first interval exactly on the
    # second uniform's boundary (the oracle is pinned there); the GPU path,
    # its drain draws included (40 particles), must take the same choices:
    # same final counts, same log-likelihoods
    H, t1 = 40, 4.0
    net = W.Network("two births", ["A", "B"], [[0, 0], [0, 0]], [[1, 0], [0, 1]])
    tr = {"t_obs": np.array([t1, 2 * t1]), "y": np.array([[2.0], [4.5]]), "t0": 0.0,
          "x0": np.zeros(2, np.int32)}
    wl = W.Workload("two births", net, W.OBS_GAUSSIAN, [0], 1.0, np.ones((1, 2)), [tr], H)
    theta = _boundary_batch(orc, precision, 24, H, wl.seed, t1)
    ids = np.arange(len(theta), dtype=np.uint32)
    _say("boundary choices precision", precision, "kernel", kernel, "schedule", schedule)
    got = _gpu(wl, theta=theta, theta_ids=ids, precision=precision, kernel=kernel,
               tuning=dict(schedule=schedule))
    ref = _oracle(orc, wl, theta=theta, theta_ids=ids, precision=precision)
    assert np.all(ref["status"] == 0)
    assert_parity(got, ref, abs_tol=FP32_ABS if precision else None)


@pytest.mark.parametrize("kernel", KERNELS)
def test_fp32_rates_beyond_binary32(orc, kernel):
    # a rate beyond the binary32 range is a bad rate vector for the
    # FP32-mixed step only; both sides agree in both modes
    wl = W.immigration_death_workload(n_theta=3, n_particles=64)
    theta = np.array([[10, 0.1], [1e39, 0.1], [0.1, 5e38]])
    for precision in (0, 1):
        _say("rates beyond binary32, precision", precision, "kernel", kernel)
        got = _gpu(wl, theta=theta, precision=precision, event_cap=10_000, kernel=kernel)
        ref = _oracle(orc, wl, theta=theta, precision=precision, event_cap=10_000)
        want = [0, 1, 0] if precision == 0 else [0, 3, 3]
        assert list(ref["status"]) == want, ref["status"]
        assert_parity(got, ref, abs_tol=FP32_ABS if precision else None)


TUNINGS = [dict(pool_min=1, pool_max=1, pool_events=0, pool_first=1, refill_min=1, priority=0,
                items_per_cu=0, persistent=0, schedule=0),
           dict(pool_min=2, pool_max=4, pool_events=1024, pool_first=2, refill_min=1, priority=1,
                items_per_cu=0, persistent=0, schedule=0),
           dict(pool_min=2, pool_max=8, pool_events=8192, pool_first=2, refill_min=7, priority=1,
                items_per_cu=1, persistent=0, schedule=0),
           dict(pool_min=3, pool_max=5, pool_events=1, pool_first=7, refill_min=64, priority=0,
                items_per_cu=0, persistent=0, schedule=0),
           dict(pool_min=64, pool_max=64, pool_events=0, pool_first=64, refill_min=33,
                priority=1, items_per_cu=0, persistent=0, schedule=0),
           dict(pool_min=1, pool_max=4, pool_events=1024, pool_first=1, refill_min=1, priority=0,
                items_per_cu=160, persistent=1, schedule=0),
           dict(pool_min=1, pool_max=1, pool_events=0, pool_first=1, refill_min=9, priority=0,
                items_per_cu=0, persistent=1, schedule=0),
           dict(pool_min=4, pool_max=4, pool_events=0, pool_first=4, refill_min=64, priority=0,
                items_per_cu=0, persistent=1, schedule=0),
           dict(pool_min=1, pool_max=6, pool_events=1536, pool_first=1, refill_min=1, priority=0,
                items_per_cu=160, persistent=0, schedule=1),
           dict(pool_min=1, pool_max=1, pool_events=0, pool_first=1, refill_min=1, priority=0,
                items_per_cu=0, persistent=1, schedule=1, urgent_events=0),
           dict(pool_min=64, pool_max=64, pool_events=0, pool_first=64, refill_min=5,
                priority=0, items_per_cu=0, persistent=0, schedule=1, urgent_events=1),
           dict(pool_min=1, pool_max=4, pool_events=1024, pool_first=2, refill_min=1, priority=0,
                items_per_cu=0, persistent=0, schedule=1, urgent_events=3000, backlog_per_cu=1)]

FLOW = dict(schedule=1)
PER_INTERVAL = dict(schedule=0)


@pytest.mark.parametrize("kernel", KERNELS)
def test_work_partitioning_never_changes_results(orc, kernel):
    # pools of 1..64 groups of 64 particles per wavefront, lane refill in
    # any order: every output is bit-identical, and the oracle agrees
    from paper_1606_08281_amd import lik
    wl, idx = _telegraph_subset(n_obs=20)
    trajs = wl.trajectories[:2]
    net = lik.Network(wl.net.orders, wl.net.stoich)
    first = {}
    for t in TUNINGS:
        net.set_tuning(**t)
        for H in (1000, 4096, 65):
            _say("partitioning", t, "H", H, "kernel", kernel)
            got = lik.eval_batch(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta[idx], trajs,
                                 H, wl.seed, theta_ids=idx, aux=True, kernel=kernel)
            if H not in first:
                first[H] = got
                continue
            for k in ("loglik", "status", "filter_events", "filter_loglik", "final_state"):
                assert np.array_equal(got[k], first[H][k], equal_nan=True), (t, H, k)
    sub = idx[:4]
    ref = _oracle(orc, wl, theta=wl.theta[sub], theta_ids=sub, trajectories=trajs)
    net.set_tuning(**TUNINGS[-1])
    assert_parity(lik.eval_batch(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta[sub], trajs,
                                 wl.n_particles, wl.seed, theta_ids=sub, aux=True, kernel=kernel),
                  ref)


@pytest.mark.parametrize("kernel", KERNELS)
def test_flow_schedule_equals_per_interval_schedule(orc, kernel):
    # one persistent launch, filters advancing independently: bit-identical
    # to one launch sequence per interval, over statuses, stopped filters,
    # uneven trajectory lengths, ragged particle counts and both precisions
    wl = W.immigration_death_workload(n_theta=6, n_particles=70)
    theta = np.array([[10, 0.1], [-1, 0.1], [np.nan, 1], [np.inf, 1], [0, 0], [1e-300, 1e-300]])
    cases = [("statuses", dict(wl=wl, theta=theta), True),
             ("event cap 3", dict(wl=wl, theta=wl.theta[:3], event_cap=3), False)]
    tw = W.telegraph_workload(n_theta=4, n_traj=3, n_obs=20, n_particles=130)
    trajs = []
    for m, T in enumerate([1, 20, 7]):
        tr = dict(tw.trajectories[m])
        tr["t_obs"] = tr["t_obs"][:T]
        tr["y"] = tr["y"][:T]
        trajs.append(tr)
    th = np.vstack([W.TELEGRAPH_TRUTH * s for s in [1.0, 0.5, 2.0, 1.3]])
    cases.append(("uneven T", dict(wl=tw, theta=th, trajectories=trajs), True))
    z = W.telegraph_workload(n_theta=2, n_traj=1, n_obs=4, n_particles=16)
    zt = dict(z.trajectories[0])
    zt["x0"] = np.array([1, 0, 0, 0], np.int32)
    zth = np.vstack([np.zeros(6), [0.1, 0.1, 0.0, 1.0, 0.0, 1.0]])
    cases.append(("-inf", dict(wl=z, theta=zth, trajectories=[zt]), True))
    for H in (1, 65, 4096):
        iw = W.immigration_death_workload(n_theta=5, n_particles=H)
        cases.append((f"H={H}", dict(wl=iw), True))
    for prec in (0, 1):
        sw = W.telegraph_workload(n_theta=8, n_traj=2, n_obs=12, n_particles=1000)
        cases.append((f"telegraph precision {prec}", dict(wl=sw, precision=prec), True))
    for name, kw, state in cases:
        _say("flow vs per-interval:", name, "kernel", kernel)
        a = _gpu(kernel=kernel, tuning=PER_INTERVAL, **kw)
        b = _gpu(kernel=kernel, tuning=FLOW, **kw)
        for k in ("loglik", "status", "filter_events", "filter_loglik", "final_state"):
            assert np.array_equal(a[k], b[k], equal_nan=True), (name, k)
        ref = _oracle(orc, kw["wl"], theta=kw.get("theta"), trajectories=kw.get("trajectories"),
                      event_cap=kw.get("event_cap") or 100_000_000,
                      precision=kw.get("precision", 0))
        assert_parity(b, ref, check_state=state,
                      abs_tol=FP32_ABS if kw.get("precision") else None)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [0, 1])
def test_pool_drain_draws(orc, precision, kernel):
    # Once a pool's particles are all taken and at most 32 lanes still run,
    # the idle lanes compute the running lanes' coming draws.  Particle
    # counts around 32 and 64 start an item at or just above that point,
    # staged pools of up to five groups reach it mid-item, and an event cap
    # that stops the heaviest filters lands among the last particles (two
    # of the four theta finish, two stop).  Bit-exact against the oracle.
    tw = W.telegraph_workload(n_theta=4, n_traj=1, n_obs=10, n_particles=97)
    th = np.vstack([W.TELEGRAPH_TRUTH * s for s in [1.0, 0.7, 1.5, 2.0]])
    trajs = tw.trajectories[:1]
    big_pools = dict(pool_min=2, pool_max=5, pool_events=1 << 20, pool_first=5, refill_min=1,
                     priority=0, items_per_cu=0, persistent=0, schedule=1)
    for H in (31, 32, 33, 63, 97, 129, 320):
        for cap in (0, 240):
            ref = _oracle(orc, tw, theta=th, H=H, trajectories=trajs, precision=precision,
                          event_cap=cap or 100_000_000)
            for t in (FLOW, PER_INTERVAL, big_pools):
                _say("drain draws H", H, "cap", cap, "tuning", t, "precision", precision,
                     "kernel", kernel)
                got = _gpu(tw, theta=th, H=H, trajectories=trajs, precision=precision,
                           event_cap=cap, kernel=kernel, tuning=t)
                assert_parity(got, ref, abs_tol=FP32_ABS if precision else None)
            if cap:
                assert set(ref["status"]) == {0, 1}, ref["status"]


def test_flow_schedule_graph_replays_and_random_network(orc):
    import torch
    from paper_1606_08281_amd import lik
    wl = W.telegraph_workload(n_theta=24, n_traj=2, n_obs=12, n_particles=200)
    net = lik.Network(wl.net.orders, wl.net.stoich)
    net.set_tuning(**FLOW)
    eager = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories,
                            wl.n_theta, wl.n_particles)
    graph = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories,
                            wl.n_theta, wl.n_particles, graph=True)
    theta = torch.from_numpy(wl.theta).cuda()
    for k in range(3):
        _say("flow graph replay", k)
        ll_e = eager.run(theta, wl.seed + k)[0].clone()
        junk = torch.randn(4096, device="cuda").sum()
        ll_g = graph.run(theta, wl.seed + k)[0].clone()
        ev_g = graph.events.clone()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert torch.equal(ll_e, ll_g), k
    # the last replay against the oracle directly (same seed)
    ref = _oracle(orc, wl, seed=wl.seed + 2)
    assert np.array_equal(ev_g.cpu().numpy().astype(np.uint64), ref["events"])
    got = ll_g.cpu().numpy()
    assert np.all(np.abs(got - ref["loglik"]) <= REL * np.abs(ref["loglik"]))
    rw = W.random_network_workload(n_theta=64, n_particles=96, n_obs=3, events_per_interval=300)
    idx = np.arange(0, 64, 8)
    for kernel in KERNELS:
        _say("flow random 20x40 kernel", kernel)
        a = _gpu(rw, theta=rw.theta[idx], theta_ids=idx, kernel=kernel, tuning=PER_INTERVAL)
        b = _gpu(rw, theta=rw.theta[idx], theta_ids=idx, kernel=kernel, tuning=FLOW)
        for k in ("loglik", "status", "filter_events", "final_state"):
            assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_flow_scheduler_gives_up_cleanly(monkeypatch):
    # the flow schedule's bounded waits, forced to their limit from the host
    # (1 us without a finished work item): the launch ends, unfinished
    # filters report LIK_STATUS_SCHEDULER with NaN, finished ones are exact
    wl = W.telegraph_workload(n_theta=8, n_traj=2, n_obs=20, n_particles=256)
    ref = _gpu(wl, tuning=PER_INTERVAL)
    monkeypatch.setenv("LIK_FLOW_STALL_US", "1")
    _say("flow give-up path, stall limit 1 us")
    got = _gpu(wl, tuning=FLOW)
    st = got["status"]
    assert set(np.unique(st).tolist()) <= {0, 4}, st
    assert (st == 4).any()
    assert np.all(np.isnan(got["loglik"][st == 4]))
    assert np.array_equal(got["loglik"][st == 0], ref["loglik"][st == 0])
    monkeypatch.delenv("LIK_FLOW_STALL_US")
    again = _gpu(wl, tuning=FLOW)
    assert np.array_equal(again["loglik"], ref["loglik"])


def test_autotune_picks_a_candidate_and_keeps_results():
    import torch
    from paper_1606_08281_amd import lik
    wl = W.telegraph_workload(n_theta=64, n_traj=2, n_obs=10, n_particles=1000)
    net = lik.Network(wl.net.orders, wl.net.stoich)
    db = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories, wl.n_theta,
                         wl.n_particles)
    theta = torch.from_numpy(wl.theta).cuda()
    ll0 = db.run(theta, wl.seed)[0].cpu().numpy()
    _say("autotune 64x2x1000x10")
    chosen = db.autotune(theta, wl.seed + 1)
    torch.cuda.synchronize()
    assert chosen == net.tuning()
    assert 1 <= chosen["pool_min"] <= chosen["pool_max"] <= 64
    assert np.array_equal(db.run(theta, wl.seed)[0].cpu().numpy(), ll0)


@pytest.mark.parametrize("precision", [0, 1])
def test_gpu_estimator_unbiased_vs_exact(precision):
    # The GPU estimate itself against the exact immigration-death likelihood
    # (closed-form transition kernel): 2000 independent streams per theta
    # (one theta id each); the mean of exp(l_hat - l*) is 1 within 4
    # standard errors.  The estimator is unbiased up to the fixed-point
    # resampling weights (relative bias at most H 2^-32 per observation).
    import math
    from paper_1606_08281_amd import lik
    from tests.exact_lik import immigration_death_loglik
    wl = W.immigration_death_workload(n_theta=1, n_particles=256)
    tr = wl.trajectories[0]
    net = lik.Network(wl.net.orders, wl.net.stoich)
    R = 2000
    for theta in [(10.0, 0.1), (12.0, 0.13), (9.0, 0.085)]:
        lstar = immigration_death_loglik(theta[0], theta[1], 0, 0.0, tr["t_obs"], tr["y"][:, 0],
                                         2.0)
        _say("unbiasedness theta", theta, "precision", precision, "R", R)
        got = lik.eval_batch(net, wl.obs_kind, wl.observed, wl.sigma, np.tile(theta, (R, 1)),
                             [tr], 256, 77, theta_ids=np.arange(R, dtype=np.uint32),
                             precision=precision)
        assert np.all(got["status"] == 0)
        z = np.exp(got["loglik"] - lstar)
        se = z.std(ddof=1) / math.sqrt(R)
        assert abs(z.mean() - 1.0) <= 4 * se + 1e-3, (theta, z.mean(), se)


@pytest.mark.parametrize("precision", [0, 1])
def test_random_network_full_batch_sampled(orc, precision):
    # the 20-species, 40-reaction network at full size (4096 theta x 512
    # particles x 100 observations) through the device entry point; a seeded
    # sample of theta is recomputed by the oracle
    import torch
    from paper_1606_08281_amd import lik
    wl = W.random_network_workload()
    net = lik.Network(wl.net.orders, wl.net.stoich)
    db = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories, wl.n_theta,
                         wl.n_particles, precision=precision)
    _say("random 20x40 full batch 4096x512x100 precision", precision)
    ll, st = db.run(torch.from_numpy(wl.theta).cuda(), wl.seed)
    torch.cuda.synchronize()
    ll, st = ll.cpu().numpy(), st.cpu().numpy()
    events = db.events.cpu().numpy().astype(np.uint64)
    idx = np.sort(np.random.default_rng(11).choice(wl.n_theta, 4, replace=False))
    _say("oracle sample", idx.tolist())
    ref = _oracle(orc, wl, theta=wl.theta[idx], theta_ids=idx, precision=precision)
    assert np.array_equal(st[idx], ref["status"])
    assert np.array_equal(events[idx], ref["events"])
    fin = np.isfinite(ref["loglik"])
    err = np.abs(ll[idx][fin] - ref["loglik"][fin])
    assert np.all(err <= REL * np.abs(ref["loglik"][fin]))
    if precision:
        assert np.all(err <= FP32_ABS)
    assert np.all(st == 0) and np.all(np.isfinite(ll))


@pytest.mark.parametrize("precision", [0, 1])
def test_random_network_1e4_events_full_batch_sampled(orc, precision):
    # the 20-species, 40-reaction network at the interval where the median
    # rate vector realises 1e4 SSA events per particle per interval
    # (4096 theta x 512 particles x 100 observations, ~2.4e12 events), in the
    # benchmark's launch configuration; two seeded rate vectors recomputed by
    # the oracle at full size: statuses, event counts, final particle counts,
    # log-likelihoods
    import torch
    from paper_1606_08281_amd import lik
    wl = W.random_network_workload(dt=W.RANDOM_DT_1E4)
    net = lik.Network(wl.net.orders, wl.net.stoich)
    db = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories, wl.n_theta,
                         wl.n_particles, precision=precision)
    final = torch.empty((wl.n_theta, wl.net.U, wl.n_particles), dtype=torch.int32,
                        device="cuda")
    _say("random 20x40 at 1e4 events/interval, full batch 4096x512x100 precision", precision)
    ll, st = db.run(torch.from_numpy(wl.theta).cuda(), wl.seed, final_state=final)
    torch.cuda.synchronize()
    ll, st = ll.cpu().numpy(), st.cpu().numpy()
    events = db.events.cpu().numpy().astype(np.uint64)
    idx = np.sort(np.random.default_rng(23).choice(wl.n_theta, 2, replace=False))
    _say("oracle sample", idx.tolist(), "events", events[idx].tolist())
    ref = _oracle(orc, wl, theta=wl.theta[idx], theta_ids=idx, precision=precision)
    assert np.array_equal(st[idx], ref["status"])
    assert np.array_equal(events[idx], ref["events"])
    assert np.array_equal(final[torch.from_numpy(idx).cuda()].cpu().numpy(), ref["final_state"])
    fin = np.isfinite(ref["loglik"])
    err = np.abs(ll[idx][fin] - ref["loglik"][fin])
    assert np.all(err <= REL * np.abs(ref["loglik"][fin]))
    if precision:
        assert np.all(err <= FP32_ABS)
    # the batch realises ~1e4 events per particle per interval at its median
    per = events.astype(np.float64) / (wl.n_particles * len(wl.trajectories[0]["t_obs"]))
    assert 5e3 < np.median(per[st == 0]) < 2e4, np.median(per[st == 0])
    assert np.mean(st == 0) > 0.99
