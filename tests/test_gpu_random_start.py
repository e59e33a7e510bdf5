"""Random initial counts and the fluorescence observation model on the GPU,
against the oracle (Supplementary I: the filter starts from H draws of the
initial distribution; Supplementary "LacGfp example": uniform initial counts,
per-molecule normal signal plus background, the 9-species, 18-reaction
Lac-Gfp network).  Same bar as the other parity tests: integer results bit
for bit, log-likelihoods within 1e-9 relative."""
import numpy as np
import pytest

from paper_1606_08281_amd import workloads as W
from tests.test_gpu_parity import _gpu, _oracle, _say, assert_parity

pytestmark = pytest.mark.gpu

FLUO = (1.5, 3.0, 2.0, 1.2)


def fluo_immigration_death(n_theta=48, M=2, lo=0, hi=20):
    """Immigration-death paths observed through the fluorescence model,
    started from a uniform count."""
    wl = W.immigration_death_workload(n_theta=n_theta, n_particles=64)
    rng = np.random.default_rng(21)
    trajs = []
    for m in range(M):
        tr = dict(wl.trajectories[0])
        x = tr["x_true"][:, 0].astype(np.float64) + 3 * m
        y = rng.normal(FLUO[1] * x + FLUO[2], np.sqrt(FLUO[0] ** 2 * x + FLUO[3] ** 2))
        tr.update(y=y.reshape(-1, 1), x0=np.array([lo], np.int32), x0_hi=np.array([hi], np.int32))
        trajs.append(tr)
    return W.Workload("immigration-death", wl.net, W.OBS_FLUORESCENCE, [0], FLUO, wl.theta, trajs,
                      64)


TUNINGS = [{"schedule": 0}, {"schedule": 1}, {"schedule": 0, "persistent": 1}]


@pytest.mark.parametrize("tuning", TUNINGS)
@pytest.mark.parametrize("kernel", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_random_start_fluorescence_parity(orc, precision, kernel, tuning):
    wl = fluo_immigration_death()
    for H in (1, 37, 64, 300, 1000):
        _say("random start + fluorescence, immigration-death", precision, kernel, tuning, H)
        got = _gpu(wl, H=H, precision=precision, kernel=kernel, tuning=tuning)
        ref = _oracle(orc, wl, H=H, precision=precision)
        assert_parity(got, ref)


@pytest.fixture(scope="module")
def lacgfp_near_truth():
    """theta* and seven parameter vectors around it (log-normal, sd 0.3):
    rates the oracle evaluates in seconds at 64 particles."""
    rng = np.random.default_rng(23)
    params = np.vstack([W.LACGFP_TRUTH,
                        W.LACGFP_TRUTH * np.exp(rng.normal(0.0, 0.3, (7, 18)))])
    return W.lacgfp_workload(n_traj=2, theta=params, n_particles=64)


@pytest.mark.parametrize("kernel", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_lacgfp_parity(orc, lacgfp_near_truth, precision, kernel):
    wl = lacgfp_near_truth
    _say("lac-gfp 8 theta x 2 traj x 64 particles x 29 obs", precision, kernel)
    got = _gpu(wl, precision=precision, kernel=kernel)
    ref = _oracle(orc, wl, precision=precision)
    assert np.all(ref["status"] == 0) and np.all(np.isfinite(ref["loglik"]))
    assert ref["events"].min() > 0
    assert_parity(got, ref)


def test_lacgfp_served_and_batched_equal_alone(lacgfp_near_truth):
    from paper_1606_08281_amd import lik
    lw = lacgfp_near_truth
    tw = W.telegraph_workload(n_theta=4, n_traj=2, n_obs=20, n_particles=128)
    nl = lik.Network(lw.net.orders, lw.net.stoich)
    nt = lik.Network(tw.net.orders, tw.net.stoich)
    reqs = [dict(net=nl, obs_kind=lw.obs_kind, observed=lw.observed, sigma=lw.sigma,
                 theta=lw.theta[:4], trajectories=lw.trajectories, n_particles=64, seed=7),
            dict(net=nt, obs_kind=tw.obs_kind, observed=tw.observed, sigma=tw.sigma,
                 theta=tw.theta, trajectories=tw.trajectories, n_particles=128, seed=8),
            dict(net=nl, obs_kind=lw.obs_kind, observed=lw.observed, sigma=lw.sigma,
                 theta=lw.theta[4:], trajectories=lw.trajectories[:1], n_particles=100, seed=9)]
    alone = [lik.eval_batch(r["net"], r["obs_kind"], r["observed"], r["sigma"], r["theta"],
                            r["trajectories"], r["n_particles"], r["seed"]) for r in reqs]
    _say("lac-gfp requests through lik_eval_requests")
    ll, st, _ = lik.eval_requests(reqs)
    for a, b, s in zip(alone, ll, st):
        assert np.array_equal(a["loglik"], b, equal_nan=True) and np.array_equal(a["status"], s)
    _say("lac-gfp requests through the server")
    with lik.Server(arena_bytes=1 << 30) as srv:
        tickets = [srv.submit(r["net"], r["obs_kind"], r["observed"], r["sigma"], r["theta"],
                              r["trajectories"], r["n_particles"], r["seed"]) for r in reqs]
        for a, t in zip(alone, tickets):
            ll, st = srv.wait(t)
            assert np.array_equal(a["loglik"], ll, equal_nan=True)
            assert np.array_equal(a["status"], st)


def test_random_start_graph_replays_equal_eager():
    import torch
    from paper_1606_08281_amd import lik
    wl = fluo_immigration_death(n_theta=32)
    net = lik.Network(wl.net.orders, wl.net.stoich)
    theta = torch.from_numpy(wl.theta.ravel().copy()).cuda()
    eager = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories, 32, 200)
    graph = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories, 32, 200,
                            graph=True)
    for seed in (3, 4, 3, 5):
        _say("random start graph replay, seed", seed)
        a = eager.run(theta, seed)[0].cpu().numpy().copy()
        torch.cuda.synchronize()
        b = graph.run(theta, seed)[0].cpu().numpy().copy()
        torch.cuda.synchronize()
        assert np.array_equal(a, b, equal_nan=True)
    # the seed reaches the initial draws too
    assert not np.array_equal(eager.run(theta, 3)[0].cpu().numpy(),
                              eager.run(theta, 4)[0].cpu().numpy())


def test_lacgfp_bench_batch_sampled(orc):
    """The bench's Lac-Gfp batch at full size (1024 theta x 5 trajectories x
    200 particles x 29 observations) on the GPU, a sample recomputed by the
    oracle: the cheapest, a middle and the two heaviest theta of an oracle
    cost ranking (events of every theta at 8 particles on one trajectory)."""
    import time
    from paper_1606_08281_amd import lik
    wl = W.lacgfp_workload(theta=W.lacgfp_population(1024), n_traj=5, n_particles=200)
    P = orc.Problem(wl.net.orders, wl.net.stoich, wl.obs_kind, wl.observed, wl.sigma, wl.theta,
                    wl.trajectories[:1], 8, wl.seed)
    rank = np.argsort(-orc.evaluate(P)["events"])
    pick = np.array([rank[-1], rank[512], rank[1], rank[0]])
    _say("lac-gfp bench batch 1024 x 5 x 200 x 29 on the GPU")
    net = lik.Network(wl.net.orders, wl.net.stoich)
    got = lik.eval_batch(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta, wl.trajectories,
                         200, wl.seed, aux=True)
    t0 = time.time()
    ref = _oracle(orc, wl, theta=wl.theta[pick], theta_ids=pick.astype(np.uint32))
    _say("oracle sample", pick, f"{time.time() - t0:.1f} s")
    F = np.concatenate([np.arange(5 * i, 5 * i + 5) for i in pick])
    sub = {"status": got["status"][pick], "loglik": got["loglik"][pick],
           "filter_events": got["filter_events"][F], "filter_loglik": got["filter_loglik"][F],
           "final_state": got["final_state"][F]}
    assert np.all(ref["status"] == 0)
    assert_parity(sub, ref)
