"""Served likelihood requests: continuous batching against plain per-request
launches on one MI355X.

The request stream mixes three networks: telegraph (60 %: 1-32 rate vectors
drawn from the prior, as a level-set sampler emits them in a proposal round,
against 1-3 trajectories of 10-50 observations, 128-1000 filter particles),
immigration-death (20 %: 1-32 rate vectors, one trajectory of 10-20
observations) and the 20-species, 40-reaction random network (20 %: 1-8 rate
vectors, its trajectory of 100 observations, 512 particles); each request has
its own seed.

  1. saturation: all requests submitted at once, to the server and, one after
     another, to lik_eval_batch (plain launches per request);
  2. Poisson arrivals at a fixed rate (a fraction of the plain path's
     saturated rate): latency submit -> result, p50/p99, and evals/s.

Prints one JSON line.  python -m paper_1606_08281_amd.serve_bench [--requests N]
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1606_08281_amd import lik  # noqa: E402
from paper_1606_08281_amd import workloads as W  # noqa: E402


def request_stream(n, seed=13):
    rng = np.random.default_rng(seed)
    tel = W.telegraph_workload(n_theta=2048, n_traj=3, n_obs=50, n_particles=1000)
    imm = W.immigration_death_workload(n_theta=2048, n_particles=256)
    rnd = W.random_network_workload(n_theta=2048)
    reqs = []
    for k in range(n):
        u = rng.random()
        wl = tel if u < 0.6 else imm if u < 0.8 else rnd
        n_theta = int(rng.integers(1, 9 if wl is rnd else 33))
        start = int(rng.integers(0, wl.n_theta - n_theta))
        M = int(rng.integers(1, 4)) if wl is tel else 1
        T = (int(rng.integers(10, 51)) if wl is tel else int(rng.integers(10, 21)) if wl is imm
             else 100)
        H = 512 if wl is rnd else int(rng.choice([128, 512, 1000]))
        trajs = [dict(tr, t_obs=tr["t_obs"][:T], y=tr["y"][:T]) for tr in wl.trajectories[:M]]
        reqs.append(dict(wl=wl, theta=wl.theta[start:start + n_theta],
                         ids=np.arange(start, start + n_theta, dtype=np.uint32), trajs=trajs,
                         H=H, seed=int(1000 + k)))
    return reqs


def uneven_batch(n=8192, seed=17):
    """One rate vector per request from the immigration-death or telegraph
    prior (half each), one trajectory of 10-200 observations, 128-4096 filter
    particles: the uneven batch the engine runs in shared iterations."""
    rng = np.random.default_rng(seed)
    tel = W.telegraph_workload(n_theta=n, n_traj=1, n_obs=200, n_particles=1000)
    imm = W.immigration_death_workload(n_theta=n, n_particles=256,
                                       t_obs=np.arange(5.0, 1000.0 + 1e-9, 5.0))
    reqs = []
    for k in range(n):
        wl = tel if k % 2 else imm
        T = int(rng.integers(10, 201))
        tr = wl.trajectories[0]
        reqs.append(dict(wl=wl, theta=wl.theta[k:k + 1], ids=np.array([k], np.uint32),
                         trajs=[dict(tr, t_obs=tr["t_obs"][:T], y=tr["y"][:T])],
                         H=int(rng.choice([128, 512, 1024, 4096])), seed=int(5000 + k)))
    return reqs


def run_plain(reqs, nets, arrivals=None):
    """Requests one at a time through lik_eval_batch, in arrival order."""
    lat = []
    t0 = time.perf_counter()
    for k, r in enumerate(reqs):
        if arrivals is not None:
            wait = t0 + arrivals[k] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
        wl = r["wl"]
        lik.eval_batch(nets[wl.name], wl.obs_kind, wl.observed, wl.sigma, r["theta"], r["trajs"],
                       r["H"], r["seed"], theta_ids=r["ids"])
        done = time.perf_counter()
        lat.append(done - (t0 + (arrivals[k] if arrivals is not None else 0.0)))
    return time.perf_counter() - t0, np.array(lat)


def run_server(reqs, nets, arrivals=None, tuning=None):
    lat = np.zeros(len(reqs))
    with lik.Server(arena_bytes=8 << 30, kernel=lik.KERNEL_SPECIALIZED, tuning=tuning) as srv:
        t0 = time.perf_counter()
        tickets = [None] * len(reqs)
        sub_t = np.zeros(len(reqs))

        def waiter():
            for k in range(len(reqs)):
                while tickets[k] is None:
                    time.sleep(1e-4)
                srv.wait(tickets[k])
                lat[k] = time.perf_counter() - sub_t[k]

        th = threading.Thread(target=waiter)
        th.start()
        for k, r in enumerate(reqs):
            if arrivals is not None:
                wait = t0 + arrivals[k] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
            wl = r["wl"]
            sub_t[k] = time.perf_counter()
            tickets[k] = srv.submit(nets[wl.name], wl.obs_kind, wl.observed, wl.sigma, r["theta"],
                                    r["trajs"], r["H"], r["seed"], theta_ids=r["ids"])
        th.join()
        total = time.perf_counter() - t0
        stats = srv.stats()
    return total, lat, stats


def check_equal(reqs, nets, n=8):
    """Served results equal alone results, bit for bit (a sample)."""
    with lik.Server(arena_bytes=2 << 30, kernel=lik.KERNEL_SPECIALIZED) as srv:
        ts = []
        for r in reqs[:n]:
            wl = r["wl"]
            ts.append(srv.submit(nets[wl.name], wl.obs_kind, wl.observed, wl.sigma, r["theta"],
                                 r["trajs"], r["H"], r["seed"], theta_ids=r["ids"]))
        served = [srv.wait(t)[0] for t in ts]
    for r, s in zip(reqs[:n], served):
        wl = r["wl"]
        alone = lik.eval_batch(nets[wl.name], wl.obs_kind, wl.observed, wl.sigma, r["theta"],
                               r["trajs"], r["H"], r["seed"], theta_ids=r["ids"])["loglik"]
        if not np.array_equal(alone, s, equal_nan=True):
            return False
    return True


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--uneven", action="store_true",
                    help="the 8192-request uneven batch (all submitted at once) instead")
    ap.add_argument("--plain-sample", type=int, default=512)
    ap.add_argument("--load", type=float, default=0.8,
                    help="arrival rate as a fraction of the plain path's saturated rate")
    ap.add_argument("--tuning", default=None,
                    help="server work partitioning pool_min,pool_max,pool_events,pool_first,"
                         "refill_min,priority,items_per_cu,persistent,schedule,urgent_events,backlog_per_cu "
                         "(default: the library's)")
    args = ap.parse_args()
    tuning = None
    if args.tuning:
        keys = ("pool_min", "pool_max", "pool_events", "pool_first", "refill_min", "priority",
                "items_per_cu", "persistent", "schedule", "urgent_events", "backlog_per_cu")
        tuning = dict(zip(keys, (int(v) for v in args.tuning.split(","))))
    import torch
    torch.cuda.set_device(0)
    reqs = uneven_batch() if args.uneven else request_stream(args.requests)
    nets = {}
    for r in reqs:
        wl = r["wl"]
        if wl.name not in nets:
            nets[wl.name] = lik.Network(wl.net.orders, wl.net.stoich)
            nets[wl.name].precompile(lik.FP64)
    n_evals = sum(len(r["theta"]) for r in reqs)
    if args.uneven:
        run_server(reqs[:8], nets, tuning=tuning)
        print("[serve] warm", flush=True, file=sys.stderr)
        t_srv, lat, st = run_server(reqs, nets, tuning=tuning)
        print(f"[serve] uneven batch served in {t_srv:.2f} s", flush=True, file=sys.stderr)
        sample = reqs[:args.plain_sample]
        if args.plain_sample == 0:
            out = {"requests": len(reqs), "makespan_s": t_srv, "server_evals_per_s": n_evals / t_srv,
                   "tuning": tuning}
            print(json.dumps(out), flush=True)
            return
        t_plain, _ = run_plain(sample, nets)
        out = {"metric": "uneven batch: likelihood evals/s, makespan, p50/p99 completion",
               "requests": len(reqs), "makespan_s": t_srv, "server_evals_per_s": n_evals / t_srv,
               "p50_completion_ms": float(np.percentile(lat, 50) * 1e3),
               "p99_completion_ms": float(np.percentile(lat, 99) * 1e3),
               "plain_evals_per_s": len(sample) / t_plain,
               "plain_sample": f"first {len(sample)} requests one at a time via lik_eval_batch",
               "server_stats": st,
               "workload": "8192 single-theta requests, immigration-death and telegraph halves, "
                           "T uniform 10-200, H in {128, 512, 1024, 4096}; FP64"}
        print(json.dumps(out), flush=True)
        return
    # warm both paths (kernel loads, allocator)
    run_plain(reqs[:4], nets)
    run_server(reqs[:4], nets, tuning=tuning)
    print("[serve] warm", flush=True, file=sys.stderr)
    t_plain, _ = run_plain(reqs, nets)
    print(f"[serve] plain saturated {n_evals / t_plain:.1f} evals/s", flush=True, file=sys.stderr)
    t_srv, _, st_sat = run_server(reqs, nets, tuning=tuning)
    print(f"[serve] server saturated {n_evals / t_srv:.1f} evals/s", flush=True, file=sys.stderr)
    rate = args.load * len(reqs) / t_plain   # requests per second
    arrivals = np.cumsum(np.random.default_rng(6).exponential(1.0 / rate, len(reqs)))
    tp, lat_p = run_plain(reqs, nets, arrivals)
    print("[serve] plain at load done", flush=True, file=sys.stderr)
    ts, lat_s, st = run_server(reqs, nets, arrivals, tuning=tuning)
    print("[serve] server at load done", flush=True, file=sys.stderr)
    equal = check_equal(reqs, nets)
    out = {
        "metric": "served likelihood evals/s; p50/p99 latency",
        "requests": len(reqs), "evals": n_evals,
        "saturated": {"server_evals_per_s": n_evals / t_srv, "plain_evals_per_s": n_evals / t_plain,
                      "speedup": t_plain / t_srv},
        "at_load": {"arrival_rate_req_per_s": rate, "load_vs_plain_saturation": args.load,
                    "server": {"evals_per_s": n_evals / ts,
                               "p50_ms": float(np.percentile(lat_s, 50) * 1e3),
                               "p99_ms": float(np.percentile(lat_s, 99) * 1e3)},
                    "plain": {"evals_per_s": n_evals / tp,
                              "p50_ms": float(np.percentile(lat_p, 50) * 1e3),
                              "p99_ms": float(np.percentile(lat_p, 99) * 1e3)}},
        "server_stats": st,
        "served_equals_alone": equal,
        "workload": "telegraph (60%: 1-32 theta, 1-3 trajectories, 10-50 observations, H in "
                    "{128, 512, 1000}), immigration-death (20%: 1-32 theta, 10-20 observations) "
                    "and random 20x40 network (20%: 1-8 theta, 100 observations, H 512) "
                    "requests; FP64",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
