"""Continuous-batching server: every request's result is bit-identical to the
same request evaluated alone (lik_eval_batch), whatever else shares the GPU,
and matches the CPU oracle to the parity bar; admission by memory;
cancellation while queued and while resident, per-request time limits;
statistics; shutdown drains."""
import threading
import time

import numpy as np
import pytest

from paper_1606_08281_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _mixed_requests():
    """Requests of two networks, several particle counts, lengths and
    precisions, each with its own seed."""
    imm = W.immigration_death_workload(n_theta=24, n_particles=128)
    tel = W.telegraph_workload(n_theta=16, n_traj=3, n_obs=20, n_particles=128)
    reqs = []
    for k in range(10):
        if k % 2 == 0:
            wl = imm
            th = imm.theta[2 * k:2 * k + 3]
            trajs = imm.trajectories
            T = 5 + 3 * k
            trajs = [dict(trajs[0], t_obs=trajs[0]["t_obs"][:T], y=trajs[0]["y"][:T])]
        else:
            wl = tel
            th = np.vstack([W.TELEGRAPH_TRUTH * (1 + 0.1 * k), W.TELEGRAPH_TRUTH / (1 + 0.05 * k)])
            trajs = [dict(tr, t_obs=tr["t_obs"][:4 + k], y=tr["y"][:4 + k])
                     for tr in tel.trajectories]
        reqs.append(dict(wl=wl, theta=th, trajs=trajs, H=[64, 128, 200, 1000, 65][k % 5],
                         seed=100 + k, precision=k % 3 == 2))
    return reqs


def _alone(lik, req, nets):
    wl = req["wl"]
    return lik.eval_batch(nets[wl.name], wl.obs_kind, wl.observed, wl.sigma, req["theta"],
                          req["trajs"], req["H"], req["seed"], precision=int(req["precision"]))


def _oracle_check(orc, req, got):
    # the served result against the CPU oracle on the same inputs: statuses
    # equal, log-likelihoods within 1e-9 relative (and 1e-4 absolute for
    # FP32-mixed, against the oracle's FP32-mixed mode)
    wl = req["wl"]
    P = orc.Problem(wl.net.orders, wl.net.stoich, wl.obs_kind, wl.observed, wl.sigma,
                    req["theta"], req["trajs"], req["H"], req["seed"],
                    precision=int(req["precision"]))
    ref = orc.evaluate(P)
    assert np.array_equal(got[1], ref["status"])
    a, b = got[0], ref["loglik"]
    assert np.array_equal(np.isfinite(a), np.isfinite(b))
    fin = np.isfinite(b)
    err = np.abs(a[fin] - b[fin])
    assert np.all(err <= 1e-9 * np.abs(b[fin])), err.max()
    if req["precision"]:
        assert np.all(err <= 1e-4)


def _device_bytes(n_theta, M, total_obs, U, R, P, H, with_ids):
    # a request's arena footprint as the server computes it: each input array
    # rounded up to 256 bytes, then the particle state of its n_theta * M
    # filters -- counts twice (U x Hp each), log-weights (2 Hp words),
    # ancestors, event counts and final propensities (Hp words each)
    a = lambda n: (n + 255) // 256 * 256
    Hp = (H + 63) // 64 * 64
    inputs = (a(n_theta * R * 8) + a(n_theta * 4 if with_ids else 0) + a((M + 1) * 4) +
              a(total_obs * 8) + a(total_obs * P * 8) + a(M * 8) + a(M * U * 4))
    return inputs + a(n_theta * M * (2 * U * Hp + 5 * Hp) * 4)


@pytest.mark.parametrize("kernel,tuning", [
    (1, None), (2, None),
    (2, dict(pool_min=4, pool_max=4, pool_first=4, items_per_cu=0, refill_min=5, priority=1))])
def test_served_results_equal_alone(orc, kernel, tuning):
    from paper_1606_08281_amd import lik
    reqs = _mixed_requests()
    nets = {r["wl"].name: lik.Network(r["wl"].net.orders, r["wl"].net.stoich) for r in reqs}
    _say("server mixed requests, kernel", kernel, "tuning", tuning)
    with lik.Server(arena_bytes=256 << 20, kernel=kernel, tuning=tuning) as srv:
        tickets = []
        for k, r in enumerate(reqs):
            wl = r["wl"]
            tickets.append(srv.submit(nets[wl.name], wl.obs_kind, wl.observed, wl.sigma,
                                      r["theta"], r["trajs"], r["H"], r["seed"],
                                      precision=int(r["precision"])))
            if k % 3 == 0:
                time.sleep(0.002)  # arrivals while others are resident
        got = [srv.wait(t, timeout_s=120) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["p99_latency_us"] >= st["p50_latency_us"] > 0
    for r, g in zip(reqs, got):
        assert g is not None
        ref = _alone(lik, r, nets)
        assert np.array_equal(g[1], ref["status"])
        assert np.array_equal(g[0], ref["loglik"]), (g[0], ref["loglik"])
        _oracle_check(orc, r, g)


def test_small_arena_admits_by_memory():
    # an arena that holds one request at a time: the three requests run one
    # after another (8 iterations each, none overlapping), with the results
    # of the whole batch
    from paper_1606_08281_amd import lik
    wl = W.telegraph_workload(n_theta=6, n_traj=2, n_obs=8, n_particles=512)
    net = lik.Network(wl.net.orders, wl.net.stoich)
    one = _device_bytes(2, 2, 16, 4, 6, 1, 512, True)
    _say("server small arena", one)
    with lik.Server(arena_bytes=one + one // 2, kernel=1) as srv:
        tickets = [srv.submit(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta[2 * k:2 * k + 2],
                              wl.trajectories, 512, 7, theta_ids=[2 * k, 2 * k + 1])
                   for k in range(3)]
        out = [srv.wait(t, timeout_s=120) for t in tickets]
        st = srv.stats()
    assert st["iterations"] >= 3 * 8, st
    whole = lik.eval_batch(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta, wl.trajectories,
                           512, 7)
    got = np.concatenate([o[0] for o in out])
    assert np.array_equal(got, whole["loglik"])
    # an arena one byte short of a request rejects it at submission
    with lik.Server(arena_bytes=one - 256, kernel=1) as srv:
        with pytest.raises(lik.LikError):
            srv.submit(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta[:2], wl.trajectories,
                       512, 7, theta_ids=[0, 1])


def _long_request(orc):
    # the heaviest telegraph rate vectors against all ten trajectories:
    # hundreds of milliseconds of GPU work over fifty iterations
    from tests.test_gpu_parity import heaviest_telegraph_theta
    wl = W.telegraph_workload()
    idx = np.sort(heaviest_telegraph_theta(orc, 4))
    return wl, idx


def test_cancel_queued_and_resident(orc):
    from paper_1606_08281_amd import lik
    long_wl, long_idx = _long_request(orc)
    imm = W.immigration_death_workload(n_theta=8, n_particles=128)
    nets = {"telegraph": lik.Network(long_wl.net.orders, long_wl.net.stoich),
            "immigration-death": lik.Network(imm.net.orders, imm.net.stoich)}
    short = dict(wl=imm, theta=imm.theta[:3], trajs=imm.trajectories, H=128, seed=31,
                 precision=0)

    def sub(srv, req, **kw):
        wl = req["wl"]
        return srv.submit(nets[wl.name], wl.obs_kind, wl.observed, wl.sigma, req["theta"],
                          req["trajs"], req["H"], req["seed"], **kw)

    long_req = dict(wl=long_wl, theta=long_wl.theta[long_idx], trajs=long_wl.trajectories,
                    H=1000, seed=32, precision=0)
    # (1) queued: an arena for one long request; a second one waits in the
    # queue behind it and is cancelled there; the first is unaffected
    one = _device_bytes(4, 10, 500, 4, 6, 1, 1000, False)
    _say("cancel while queued")
    with lik.Server(arena_bytes=one + one // 2, kernel=2) as srv:
        ta = sub(srv, long_req)
        tb = sub(srv, dict(long_req, seed=33))
        srv.cancel(tb)
        ll_b, st_b = srv.wait(tb, timeout_s=120)
        assert np.all(st_b == lik.STATUS_CANCELLED) and np.all(np.isnan(ll_b))
        ll_a, st_a = srv.wait(ta, timeout_s=120)
        stats = srv.stats()
        with pytest.raises(lik.LikError):
            srv.cancel(123456)
    assert stats["cancelled"] == 1 and stats["completed"] == 1
    alone = _alone(lik, long_req, nets)
    assert np.array_equal(ll_a, alone["loglik"]) and np.array_equal(st_a, alone["status"])
    # (2) resident: the long request runs beside a short one; once the short
    # one has finished the long one is certainly resident, and is cancelled
    # mid-run; requests before and after it are unaffected
    _say("cancel while resident")
    with lik.Server(arena_bytes=1 << 30, kernel=2) as srv:
        ta = sub(srv, long_req)
        tb = sub(srv, short)
        got_b = srv.wait(tb, timeout_s=120)
        srv.cancel(ta)
        ll_a, st_a = srv.wait(ta, timeout_s=120)
        tc = sub(srv, dict(short, seed=34))
        got_c = srv.wait(tc, timeout_s=120)
        stats = srv.stats()
    assert np.all(st_a == lik.STATUS_CANCELLED) and np.all(np.isnan(ll_a))
    assert stats["cancelled"] == 1 and stats["completed"] == 2
    for req, g in ((short, got_b), (dict(short, seed=34), got_c)):
        ref = _alone(lik, req, nets)
        assert np.array_equal(g[0], ref["loglik"]) and np.array_equal(g[1], ref["status"])
        _oracle_check(orc, req, g)


def test_request_time_limit(orc):
    from paper_1606_08281_amd import lik
    long_wl, long_idx = _long_request(orc)
    imm = W.immigration_death_workload(n_theta=8, n_particles=128)
    tnet = lik.Network(long_wl.net.orders, long_wl.net.stoich)
    inet = lik.Network(imm.net.orders, imm.net.stoich)
    _say("per-request time limit")
    with lik.Server(arena_bytes=1 << 30, kernel=2) as srv:
        ta = srv.submit(tnet, long_wl.obs_kind, long_wl.observed, long_wl.sigma,
                        long_wl.theta[long_idx], long_wl.trajectories, 1000, 41, timeout_s=0.002)
        tb = srv.submit(inet, imm.obs_kind, imm.observed, imm.sigma, imm.theta[:4],
                        imm.trajectories, 128, 42, timeout_s=60)
        ll_a, st_a = srv.wait(ta, timeout_s=120)
        ll_b, st_b = srv.wait(tb, timeout_s=120)
        stats = srv.stats()
    assert np.all(st_a == lik.STATUS_TIMED_OUT) and np.all(np.isnan(ll_a))
    ref = lik.eval_batch(inet, imm.obs_kind, imm.observed, imm.sigma, imm.theta[:4],
                         imm.trajectories, 128, 42)
    assert np.array_equal(ll_b, ref["loglik"]) and np.array_equal(st_b, ref["status"])
    assert stats["cancelled"] == 1


def test_concurrent_clients_and_shutdown():
    from paper_1606_08281_amd import lik
    wl = W.immigration_death_workload(n_theta=32, n_particles=64)
    net = lik.Network(wl.net.orders, wl.net.stoich)
    results = {}
    _say("server concurrent clients")
    srv = lik.Server(kernel=1)

    def client(c):
        t = srv.submit(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta[4 * c:4 * c + 4],
                       wl.trajectories, 64, 11, theta_ids=np.arange(4 * c, 4 * c + 4))
        results[c] = srv.wait(t, timeout_s=120)

    threads = [threading.Thread(target=client, args=(c,)) for c in range(8)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    # requests still queued or running when the server is closed are finished first
    pending = [srv.submit(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta[:2], wl.trajectories,
                          64, 11) for _ in range(3)]
    assert pending
    srv.close()
    whole = lik.eval_batch(net, wl.obs_kind, wl.observed, wl.sigma, wl.theta, wl.trajectories,
                           64, 11)
    got = np.concatenate([results[c][0] for c in range(8)])
    assert np.array_equal(got, whole["loglik"])


def test_server_rejects_invalid_tuning():
    from paper_1606_08281_amd import lik
    with pytest.raises(lik.LikError):
        lik.Server(arena_bytes=64 << 20, tuning=dict(pool_min=0))
