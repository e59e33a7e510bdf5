"""lik_eval_requests: many requests of several networks, particle counts and
trajectory lengths in one flow launch (or shared per-interval iterations).
Every request's result equals the same request evaluated alone
(lik_eval_batch) bit for bit, under every kernel variant and schedule, and a
sample matches the CPU oracle to the parity bar."""
import numpy as np
import pytest

from paper_1606_08281_amd import workloads as W

pytestmark = pytest.mark.gpu

REL = 1e-9


def _say(*a):
    print("[gpu case]", *a, flush=True)


def mixed_requests(lik, n=24, precision=0, with_random=False, seed=3):
    """Requests of immigration-death and telegraph (and optionally the
    20 x 40 network): H in {64, 128, 200, 512, 1024}, lengths 3-40, 1-4 theta,
    their own seeds; a few carry a bad rate, an event cap or zero rates."""
    rng = np.random.default_rng(seed)
    imm = W.immigration_death_workload(n_theta=64, n_particles=128,
                                       t_obs=np.arange(5.0, 200.0 + 1e-9, 5.0))
    tel = W.telegraph_workload(n_theta=64, n_traj=3, n_obs=40, n_particles=128)
    rnd = W.random_network_workload(n_theta=64, n_particles=96, n_obs=4,
                                    events_per_interval=200) if with_random else None
    nets = {"imm": lik.Network(imm.net.orders, imm.net.stoich),
            "tel": lik.Network(tel.net.orders, tel.net.stoich)}
    if rnd is not None:
        nets["rnd"] = lik.Network(rnd.net.orders, rnd.net.stoich)
    reqs, src = [], []
    for k in range(n):
        kind = ("rnd" if with_random and k % 5 == 4 else "imm" if k % 2 == 0 else "tel")
        wl = {"imm": imm, "tel": tel, "rnd": rnd}[kind]
        nt = int(rng.integers(1, 5))
        i0 = int(rng.integers(0, wl.n_theta - nt))
        theta = wl.theta[i0:i0 + nt].copy()
        T = int(rng.integers(3, 41)) if kind != "rnd" else 4
        M = int(rng.integers(1, 4)) if kind == "tel" else 1
        trajs = [dict(tr, t_obs=tr["t_obs"][:T], y=tr["y"][:T]) for tr in wl.trajectories[:M]]
        cap = 0
        if k == 3:
            theta[0, 0] = -1.0            # bad rate: BAD_THETA
        if k == 5:
            cap = 30                      # event cap: EVENT_CAP
        if k == 7:
            theta[:] = 0.0                # nothing happens
        reqs.append(dict(net=nets[kind], obs_kind=wl.obs_kind, observed=wl.observed,
                         sigma=wl.sigma, theta=theta, trajectories=trajs,
                         n_particles=int(rng.choice([64, 128, 200, 512, 1024])),
                         seed=100 + k, precision=precision, event_cap=cap,
                         theta_ids=np.arange(i0, i0 + nt)))
        src.append(wl)
    return reqs, src, nets


def _alone(lik, r):
    return lik.eval_batch(r["net"], r["obs_kind"], r["observed"], r["sigma"], r["theta"],
                          r["trajectories"], r["n_particles"], r["seed"],
                          precision=r["precision"], event_cap=r["event_cap"],
                          theta_ids=r["theta_ids"])


@pytest.mark.parametrize("schedule", [1, 0])
@pytest.mark.parametrize("kernel", [0, 1, 2])
def test_requests_equal_alone(kernel, schedule):
    from paper_1606_08281_amd import lik
    reqs, _, _ = mixed_requests(lik)
    _say("eval_requests kernel", kernel, "schedule", schedule)
    ll, st, done = lik.eval_requests(reqs, tuning=dict(schedule=schedule), kernel=kernel)
    statuses = set()
    for k, r in enumerate(reqs):
        a = _alone(lik, r)
        assert np.array_equal(st[k], a["status"]), (k, st[k], a["status"])
        assert np.array_equal(ll[k], a["loglik"], equal_nan=True), (k, ll[k], a["loglik"])
        statuses |= set(st[k].tolist())
    assert {0, 1, 3} <= statuses
    ran = np.array([np.any(s == 0) or np.any(s == 1) for s in st])
    assert np.all(done[ran] > 0.0) and np.all(done >= 0.0)


def test_requests_against_oracle(orc):
    from paper_1606_08281_amd import lik
    reqs, src, _ = mixed_requests(lik, n=12, seed=5)
    _say("eval_requests vs oracle")
    ll, st, _ = lik.eval_requests(reqs)
    for k, (r, wl) in enumerate(zip(reqs, src)):
        P = orc.Problem(wl.net.orders, wl.net.stoich, r["obs_kind"], r["observed"], r["sigma"],
                        r["theta"], r["trajectories"], r["n_particles"], r["seed"],
                        precision=r["precision"], event_cap=r["event_cap"] or 100_000_000,
                        theta_ids=r["theta_ids"])
        ref = orc.evaluate(P)
        assert np.array_equal(st[k], ref["status"]), k
        fin = np.isfinite(ref["loglik"])
        assert np.array_equal(np.isfinite(ll[k]), fin)
        assert np.all(np.abs(ll[k][fin] - ref["loglik"][fin]) <= REL * np.abs(ref["loglik"][fin]))


def test_requests_fp32_and_large_network():
    # FP32-mixed requests; and a set that includes the 20 x 40 network, whose
    # flow kernel keeps too few wavefronts resident: per-interval iterations
    from paper_1606_08281_amd import lik
    for precision, with_random in ((1, False), (0, True)):
        reqs, _, _ = mixed_requests(lik, n=15, precision=precision, with_random=with_random,
                                    seed=7)
        _say("eval_requests precision", precision, "random network", with_random)
        ll, st, _ = lik.eval_requests(reqs)
        for k, r in enumerate(reqs):
            a = _alone(lik, r)
            assert np.array_equal(st[k], a["status"]), k
            assert np.array_equal(ll[k], a["loglik"], equal_nan=True), k


def test_autotune_requests_keeps_results():
    from paper_1606_08281_amd import lik
    reqs, _, _ = mixed_requests(lik, n=10, seed=9)
    _say("autotune_requests")
    t = lik.autotune_requests(reqs)
    assert 1 <= t["pool_min"] <= t["pool_max"] <= 64
    ll1, _, _ = lik.eval_requests(reqs, tuning=t)
    ll0, _, _ = lik.eval_requests(reqs)
    for a, b in zip(ll0, ll1):
        assert np.array_equal(a, b, equal_nan=True)


def test_uneven_batch_one_launch_sampled(orc):
    # the 8192-request uneven batch (immigration-death and telegraph halves,
    # T 10-200, H 128-4096) in one call; a seeded sample of requests against
    # lik_eval_batch (bit-identical) and against the oracle
    from paper_1606_08281_amd import lik
    from paper_1606_08281_amd import serve_bench as SB
    reqs = SB.uneven_batch()
    nets = SB.make_networks(reqs, precompile=False)
    rq = SB.as_requests(reqs, nets)
    _say("uneven batch 8192 requests, one launch")
    ll, st, done = lik.eval_requests(rq)
    assert np.all(np.concatenate(st) == 0)
    assert np.all(done > 0)
    idx = np.random.default_rng(31).choice(len(rq), 12, replace=False)
    for k in idx:
        r = dict(rq[k], precision=0, event_cap=0)
        a = _alone(lik, r)
        assert np.array_equal(ll[k], a["loglik"]), k
    for k in idx[:4]:
        r, wl = rq[k], reqs[k]["wl"]
        _say("oracle request", int(k), "H", r["n_particles"], "T", len(r["trajectories"][0]["t_obs"]))
        P = orc.Problem(wl.net.orders, wl.net.stoich, r["obs_kind"], r["observed"], r["sigma"],
                        r["theta"], r["trajectories"], r["n_particles"], r["seed"],
                        theta_ids=r["theta_ids"])
        ref = orc.evaluate(P)
        assert np.array_equal(st[k], ref["status"])
        assert np.all(np.abs(ll[k] - ref["loglik"]) <= REL * np.abs(ref["loglik"]))


def test_requests_on_the_reaction_boundary(orc):
    # every request is one rate vector that puts one event of its first
    # interval exactly on the second uniform's boundary (the construction of
    # the batch-path test); one launch per precision (a call takes one), each
    # request against the oracle, with a margin that a flipped choice would
    # break
    from paper_1606_08281_amd import lik
    from tests.test_gpu_parity import _boundary_batch
    H, t1 = 40, 4.0
    wl_net = W.Network("two births", ["A", "B"], [[0, 0], [0, 0]], [[1, 0], [0, 1]])
    tr = {"t_obs": np.array([t1, 2 * t1]), "y": np.array([[2.0], [4.5]]), "t0": 0.0,
          "x0": np.zeros(2, np.int32)}
    net = lik.Network(wl_net.orders, wl_net.stoich)
    for precision in (0, 1):
        reqs, refs = [], []
        theta = _boundary_batch(orc, precision, 16, H, W.SEED_FILTER, t1)
        f = np.float32 if precision else float
        flipped = theta.copy()
        for i in range(len(theta)):
            b = f(theta[i, 0])
            b2 = float(np.nextafter(b, f(1.0) if i % 2 == 0 else f(0.0)))
            flipped[i] = [b2, 1.0 - b2]

        def oracle(th):
            P = orc.Problem(wl_net.orders, wl_net.stoich, W.OBS_GAUSSIAN, [0], 1.0, th, [tr],
                            H, W.SEED_FILTER, precision=precision,
                            theta_ids=np.arange(len(th), dtype=np.uint32))
            return orc.evaluate(P)["loglik"]

        ref, ref_flip = oracle(theta), oracle(flipped)
        assert np.all(np.abs(ref_flip - ref) > 10 * REL * np.abs(ref)), precision
        for i in range(len(theta)):
            reqs.append(dict(net=net, obs_kind=W.OBS_GAUSSIAN, observed=[0], sigma=1.0,
                             theta=theta[i:i + 1], trajectories=[tr], n_particles=H,
                             seed=W.SEED_FILTER, precision=precision, event_cap=0,
                             theta_ids=np.array([i])))
            refs.append(ref[i])
        _say("eval_requests on the reaction boundary, precision", precision)
        ll, st, _ = lik.eval_requests(reqs)
        for k, want in enumerate(refs):
            assert st[k][0] == 0, k
            assert abs(ll[k][0] - want) <= REL * abs(want), (k, ll[k][0], want)
