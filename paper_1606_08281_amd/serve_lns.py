"""A served stream that the level-set sampler emits: several likelihood nested
sampling runs on the telegraph model share one lik_server, with requests of
the 20-species, 40-reaction random network mixed in.

  1. closed loop: each sampler run (its own particle count H) draws proposal
     batches (the rejection step's survivors, 1-64 rate vectors), submits
     each batch as one request and keeps up to `inflight` of them at the
     server while it draws the next; every ninth request overall is a
     random-network request (1-8 rate vectors, 100 observations, H 512).
     Reported: per-request latency (submit -> result, one poller thread, no
     head-of-line effect), evals/s, the samplers' level records, and a sample
     of requests re-evaluated alone (lik_eval_batch) that must equal the
     served results bit for bit.
  2. open loop: the emitted requests (repeated with fresh seeds up to
     `replay` requests) submitted all at once (saturated evals/s), then with
     Poisson arrivals at fractions of that rate; p50/p99 latency from the
     server's own per-request record.

python -m paper_1606_08281_amd.serve_lns [--levels L] [--replay N]
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
from paper_1606_08281_amd import lns  # noqa: E402
from paper_1606_08281_amd import workloads as W  # noqa: E402


class Poller:
    """Completion times of server tickets, taken by one thread that polls
    every outstanding ticket (a zero-timeout wait) about every 0.1 ms."""

    def __init__(self, srv):
        self.srv = srv
        self.pending = {}
        self.lock = threading.Lock()
        self.stop = False
        self.thread = threading.Thread(target=self._run, daemon=True)
        self.thread.start()

    def add(self, ticket, on_done):
        with self.lock:
            self.pending[ticket] = on_done

    def _run(self):
        while True:
            with self.lock:
                items = list(self.pending.items())
            if not items and self.stop:
                return
            for t, cb in items:
                r = self.srv.wait(t, timeout_s=0)
                if r is not None:
                    now = time.perf_counter()
                    with self.lock:
                        del self.pending[t]
                    cb(r, now)
            time.sleep(1e-4)

    def close(self):
        self.stop = True
        self.thread.join()


class Stream:
    """Shared submission path: records every request and its completion."""

    def __init__(self, srv, nets, side=None, side_every=9, seed=0):
        self.srv = srv
        self.nets = nets
        self.poller = Poller(srv)
        self.log = []
        self.lock = threading.Lock()
        self.side = side
        self.side_every = int(side_every)
        self.side_rng = np.random.default_rng(seed + 99)
        self.count = 0

    def submit(self, wl, theta, trajs, H, seed, tag, done_cb=None, primary=True):
        ids = np.arange(len(theta), dtype=np.uint32)
        rec = {"wl": wl, "theta": np.array(theta, dtype=np.float64), "ids": ids, "trajs": trajs,
               "H": int(H), "seed": int(seed), "tag": tag, "t_submit": time.perf_counter(),
               "t_done": None, "result": None}
        ev = threading.Event()

        def on_done(r, now):
            rec["t_done"] = now
            rec["result"] = r
            ev.set()
            if done_cb is not None:
                done_cb(rec)
        rec["event"] = ev
        ticket = self.srv.submit(self.nets[wl.name], wl.obs_kind, wl.observed, wl.sigma,
                                 rec["theta"], trajs, H, seed, theta_ids=ids)
        self.poller.add(ticket, on_done)
        with self.lock:
            self.log.append(rec)
            self.count += int(primary)
            # one side request after every side_every - 1 primary ones
            side = (primary and self.side is not None
                    and self.count % (self.side_every - 1) == 0)
            n_side = int(self.side_rng.integers(1, 9)) if side else 0
            k_side = self.count
        if side:
            wl2 = self.side
            start = int(self.side_rng.integers(0, wl2.n_theta - n_side))
            self.submit(wl2, wl2.theta[start:start + n_side], wl2.trajectories, 512,
                        700_000 + k_side, "random-20x40", primary=False)
        return rec

    def close(self):
        self.poller.close()


class Tenant:
    """One sampler run's submit/collect callables on the shared stream."""

    def __init__(self, stream, wl, trajs, H, seed_base):
        self.stream, self.wl, self.trajs, self.H = stream, wl, trajs, H
        self.seed_base = int(seed_base)
        self.k = 0

    def submit(self, rates):
        self.k += 1
        return self.stream.submit(self.wl, rates, self.trajs, self.H, self.seed_base + self.k,
                                  f"telegraph-H{self.H}")

    def collect(self, rec):
        rec["event"].wait()
        return rec["result"]


def telegraph_data(n_traj=3, n_obs=50):
    return W.telegraph_workload(n_theta=1, n_traj=n_traj, n_obs=n_obs, n_particles=1000)


def _pct(v):
    v = np.asarray(v, dtype=np.float64) * 1e3
    if not len(v):
        return {"n": 0}
    return {"n": int(len(v)), "p50_ms": float(np.percentile(v, 50)),
            "p99_ms": float(np.percentile(v, 99)), "max_ms": float(v.max())}


def closed_loop(H_list=(128, 512, 1024, 4096), N=200, alpha=0.3, batch=64, inflight=4,
                levels=8, check=32, log=None, arena_bytes=8 << 30):
    """Sampler runs (one per H) sharing one server, plus random-network side
    requests.  Returns (report, stream log, networks)."""
    say = log or (lambda *a: None)
    tel = telegraph_data()
    rnd = W.random_network_workload(n_theta=4096)
    nets = {}
    for wl in (tel, rnd):
        nets[wl.name] = lik.Network(wl.net.orders, wl.net.stoich)
        nets[wl.name].precompile(lik.FP64)
    prior = lns.LogUniformPrior(W.TELEGRAPH_TRUTH / 10.0, W.TELEGRAPH_TRUTH * 10.0)
    runs = []
    with lik.Server(arena_bytes=arena_bytes, kernel=lik.KERNEL_SPECIALIZED) as srv:
        stream = Stream(srv, nets, side=rnd)
        samplers = []
        for i, H in enumerate(H_list):
            t = Tenant(stream, tel, tel.trajectories, H, seed_base=100_000 * (i + 1))
            samplers.append(lns.LNS(prior, N=N, alpha=alpha, batch=batch, seed=31 + i,
                                    submit=t.submit, collect=t.collect, inflight=inflight))
        errors = []

        def drive(s):
            try:
                s.run(max_levels=levels)
            except Exception as e:     # reported, not swallowed
                errors.append(repr(e))
        t0 = time.perf_counter()
        threads = [threading.Thread(target=drive, args=(s,)) for s in samplers]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        # side requests submitted last may still be running
        for rec in list(stream.log):
            rec["event"].wait()
        wall = time.perf_counter() - t0
        stream.close()
        stats = srv.stats()
    if errors:
        raise RuntimeError("sampler run failed: " + "; ".join(errors))
    recs = stream.log
    say(f"closed loop: {len(recs)} requests in {wall:.2f} s")
    lat = {}
    for r in recs:
        lat.setdefault(r["tag"], []).append(r["t_done"] - r["t_submit"])
    all_lat = [r["t_done"] - r["t_submit"] for r in recs]
    n_evals = sum(len(r["theta"]) for r in recs)
    sizes = np.array([len(r["theta"]) for r in recs if r["tag"].startswith("telegraph")])
    # a sample re-evaluated alone, synchronously
    rng = np.random.default_rng(5)
    pick = rng.choice(len(recs), size=min(check, len(recs)), replace=False)
    equal = True
    for k in pick:
        r = recs[int(k)]
        wl = r["wl"]
        alone = lik.eval_batch(nets[wl.name], wl.obs_kind, wl.observed, wl.sigma, r["theta"],
                               r["trajs"], r["H"], r["seed"], theta_ids=r["ids"])
        ll, st = alone["loglik"], alone["status"]
        equal &= bool(np.array_equal(ll, r["result"][0], equal_nan=True) and
                      np.array_equal(st, r["result"][1]))
    for i, s in enumerate(samplers):
        runs.append({"H": H_list[i], "levels": len(s.levels), "evals": s.evals,
                     "eps": [round(x["eps"], 3) for x in s.levels],
                     "max_loglik": [round(x["max_loglik"], 3) for x in s.levels],
                     "acceptance": [round(x["acceptance"], 3) for x in s.levels],
                     "clusters": [x["clusters"] for x in s.levels]})
    report = {"requests": len(recs), "evals": n_evals, "wall_s": wall,
              "evals_per_s": n_evals / wall,
              "latency": dict(all=_pct(all_lat), **{k: _pct(v) for k, v in sorted(lat.items())}),
              "server_stats": stats,
              "telegraph_batch_size": {"min": int(sizes.min()), "mean": float(sizes.mean()),
                                       "max": int(sizes.max())},
              "served_equals_alone": bool(equal), "checked_alone": int(len(pick)),
              "samplers": runs}
    return report, recs, nets


def replay(recs, nets, n_total, loads=(0.5, 0.8), log=None, arena_bytes=8 << 30):
    """The emitted requests repeated with fresh seeds up to n_total, submitted
    at once and then with Poisson arrivals at fractions of the saturated
    rate.  Latency percentiles are the server's own (submit -> result)."""
    say = log or (lambda *a: None)
    base = sorted(recs, key=lambda r: r["t_submit"])
    reqs = []
    k = 0
    while len(reqs) < n_total:
        r = base[k % len(base)]
        rep = k // len(base)
        reqs.append(dict(r, seed=r["seed"] + 10_000_000 * rep))
        k += 1
    n_evals = sum(len(r["theta"]) for r in reqs)

    def serve(reqs, arrivals):
        with lik.Server(arena_bytes=arena_bytes, kernel=lik.KERNEL_SPECIALIZED) as srv:
            t0 = time.perf_counter()
            tickets = []
            for i, r in enumerate(reqs):
                if arrivals is not None:
                    wait = t0 + arrivals[i] - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                wl = r["wl"]
                tickets.append(srv.submit(nets[wl.name], wl.obs_kind, wl.observed, wl.sigma,
                                          r["theta"], r["trajs"], r["H"], r["seed"],
                                          theta_ids=r["ids"]))
            for t in tickets:
                srv.wait(t)
            wall = time.perf_counter() - t0
            st = srv.stats()
        return wall, st

    serve(reqs[:64], None)      # kernel loads, allocator
    wall, st = serve(reqs, None)
    sat = n_evals / wall
    say(f"replay saturated {sat:.0f} evals/s over {len(reqs)} requests")
    out = {"requests": len(reqs), "evals": n_evals,
           "saturated": {"evals_per_s": sat, "wall_s": wall,
                         "p50_ms": st["p50_latency_us"] / 1e3, "p99_ms": st["p99_latency_us"] / 1e3},
           "at_load": []}
    # the same requests in one lik_eval_requests call: one persistent flow
    # launch over every interval of every filter, the upper bound for a
    # server that fed the flow kernel
    rq = [dict(net=nets[r["wl"].name], obs_kind=r["wl"].obs_kind, observed=r["wl"].observed,
               sigma=r["wl"].sigma, theta=r["theta"], trajectories=r["trajs"], n_particles=r["H"],
               seed=r["seed"], theta_ids=r["ids"]) for r in reqs]
    lik.eval_requests(rq[:64])
    t0 = time.perf_counter()
    lik.eval_requests(rq)
    flow_wall = time.perf_counter() - t0
    out["one_flow_launch"] = {"evals_per_s": n_evals / flow_wall, "wall_s": flow_wall,
                              "path": "every request at once through lik_eval_requests "
                                      "(synchronous; copies and allocation included)"}
    say(f"one flow launch {n_evals / flow_wall:.0f} evals/s")
    mean_evals = n_evals / len(reqs)
    for load in loads:
        rate = load * sat / mean_evals
        arrivals = np.cumsum(np.random.default_rng(7).exponential(1.0 / rate, len(reqs)))
        wall, st = serve(reqs, arrivals)
        say(f"replay at {load:.1f}x: p50 {st['p50_latency_us'] / 1e3:.1f} ms")
        out["at_load"].append({"load": load, "arrival_rate_req_per_s": rate,
                               "evals_per_s": n_evals / wall, "wall_s": wall,
                               "p50_ms": st["p50_latency_us"] / 1e3,
                               "p99_ms": st["p99_latency_us"] / 1e3})
    return out


WORKLOAD = ("level-set sampler runs on the telegraph model (N 200, alpha 0.3, DP-GMM proposals "
            "with M_k rejection; 3 trajectories x 50 log-normal observations; one run per H in "
            "{128, 512, 1024, 4096}; proposal batches of 1-64 rate vectors, 4 in flight per "
            "run) and every ninth request a random 20x40 network request (1-8 rate vectors, "
            "100 observations, H 512); FP64")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--N", type=int, default=200)
    ap.add_argument("--replay", type=int, default=10_000)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)

    def say(m):
        print("[lns-serve]", m, flush=True, file=sys.stderr)
    report, recs, nets = closed_loop(N=args.N, levels=args.levels, log=say)
    out = {"metric": "served likelihood evals/s and p50/p99 latency under the level-set "
                     "sampler's own request stream",
           "closed_loop": report, "workload": WORKLOAD}
    if args.replay:
        out["replay"] = replay(recs, nets, args.replay, log=say)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
