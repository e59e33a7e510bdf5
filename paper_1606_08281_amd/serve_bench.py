"""Served likelihood requests: continuous batching against plain per-request
launches of the same kernels on one MI355X.

The request stream mixes three networks: telegraph (60 %: 1-32 rate vectors
drawn from the prior, as a level-set sampler emits them in a proposal round,
against 1-3 trajectories of 10-50 observations, 128-1000 filter particles),
immigration-death (20 %: 1-32 rate vectors, one trajectory of 10-20
observations) and the 20-species, 40-reaction random network (20 %: 1-8 rate
vectors, its trajectory of 100 observations, 512 particles); each request has
its own seed.

The plain path is the same network-specialised kernels launched once per
request through lik_eval_batch_device: device buffers and the workspace are
allocated once, for the largest request, and reused; every request copies
its inputs in, runs on one long-lived stream and copies its results back
before the next starts.  The served path submits the same requests to a
lik_server.

  1. saturation: every request submitted at once to the server, and one
     after another through the plain path;
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

STREAM_WORKLOAD = ("telegraph (60%: 1-32 theta, 1-3 trajectories, 10-50 observations, H in "
                   "{128, 512, 1000}), immigration-death (20%: 1-32 theta, 10-20 observations) "
                   "and random 20x40 network (20%: 1-8 theta, 100 observations, H 512) "
                   "requests; FP64")


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


def as_requests(reqs, nets):
    """The request dicts of lik.eval_requests for a request list."""
    out = []
    for r in reqs:
        wl = r["wl"]
        out.append(dict(net=nets[wl.name], obs_kind=wl.obs_kind, observed=wl.observed,
                        sigma=wl.sigma, theta=r["theta"], trajectories=r["trajs"],
                        n_particles=r["H"], seed=r["seed"], theta_ids=r["ids"]))
    return out


def uneven_block(reqs=None, nets=None, autotune=True, log=None):
    """The uneven batch in one persistent launch (lik_eval_requests): wall
    makespan of the call, evals/s, p50/p99 request completion on the device
    clock, with the autotuner's partitioning (timed on the same batch)."""
    say = log or (lambda *a: None)
    reqs = uneven_batch() if reqs is None else reqs
    nets = make_networks(reqs) if nets is None else nets
    rq = as_requests(reqs, nets)
    n_evals = sum(len(r["theta"]) for r in reqs)
    lik.eval_requests(rq[:64])   # kernel loads
    tuning = lik.autotune_requests(rq) if autotune else None
    say(f"tuning {tuning}")
    lik.timing_read()
    lik.timing_enable(True)
    t0 = time.perf_counter()
    ll, st, done = lik.eval_requests(rq, tuning=tuning)
    wall = time.perf_counter() - t0
    lik.timing_enable(False)
    tm = lik.timing_read()
    return {"requests": len(reqs), "evals": n_evals, "makespan_s": wall,
            "evals_per_s": n_evals / wall,
            "kernel_ms": tm["propagate_ms"], "kernel_launches": tm["propagate_launches"],
            "p50_completion_ms": float(np.percentile(done, 50)),
            "p99_completion_ms": float(np.percentile(done, 99)),
            "max_completion_ms": float(done.max()),
            "status_counts": {str(k): int(v) for k, v in
                              zip(*np.unique(np.concatenate(st), return_counts=True))},
            "tuning": tuning,
            "path": "lik_eval_requests: one admission launch, one persistent flow launch over "
                    "every interval of every filter (each work item with its own network's "
                    "specialised body), one finishing launch; makespan is the whole "
                    "synchronous call (input copies and allocation included); completion on "
                    "the device clock from the admission launch",
            "workload": "8192 single-theta requests, immigration-death and telegraph halves, "
                        "T uniform 10-200, H in {128, 512, 1024, 4096}; FP64"}


def make_networks(reqs, precompile=True):
    nets = {}
    for r in reqs:
        wl = r["wl"]
        if wl.name not in nets:
            nets[wl.name] = lik.Network(wl.net.orders, wl.net.stoich)
            if precompile:
                nets[wl.name].precompile(lik.FP64)
    return nets


class PlainRunner:
    """The same kernels once per request through lik_eval_batch_device, with
    device buffers and the workspace allocated once (for the largest request
    of the set) and one long-lived stream."""

    def __init__(self, reqs, nets, kernel=lik.KERNEL_SPECIALIZED):
        import torch
        self.torch = torch
        self.nets = nets
        self.kernel = kernel
        self.packed = []
        mx = dict(theta=1, ids=1, obs_offsets=2, t_obs=1, y=1, t0=1, x0=1, ws=256, out=1)
        for r in reqs:
            wl = r["wl"]
            d = lik.pack_trajectories(r["trajs"], len(wl.observed))
            self.packed.append(d)
            net = nets[wl.name]
            mx["theta"] = max(mx["theta"], r["theta"].size)
            mx["ids"] = max(mx["ids"], len(r["ids"]))
            for k in ("obs_offsets", "t_obs", "y", "t0", "x0"):
                mx[k] = max(mx[k], d[k].size)
            mx["ws"] = max(mx["ws"], lik.workspace_size(net, len(r["theta"]), len(r["trajs"]),
                                                        r["H"]))
            mx["out"] = max(mx["out"], len(r["theta"]))
        dev = "cuda"
        self.theta = torch.empty(mx["theta"], dtype=torch.float64, device=dev)
        self.ids = torch.empty(mx["ids"], dtype=torch.int32, device=dev)
        self.data = {"obs_offsets": torch.empty(mx["obs_offsets"], dtype=torch.int32, device=dev),
                     "t_obs": torch.empty(mx["t_obs"], dtype=torch.float64, device=dev),
                     "y": torch.empty(mx["y"], dtype=torch.float64, device=dev),
                     "t0": torch.empty(mx["t0"], dtype=torch.float64, device=dev),
                     "x0": torch.empty(mx["x0"], dtype=torch.int32, device=dev)}
        self.ws_bytes = mx["ws"]
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        self.ll = torch.empty(mx["out"], dtype=torch.float64, device=dev)
        self.st = torch.empty(mx["out"], dtype=torch.int32, device=dev)
        self.ll_host = torch.empty(mx["out"], dtype=torch.float64).pin_memory()
        self.stream = torch.cuda.Stream()   # default priority

    def run_one(self, k, r):
        """Inputs in, one evaluation, results out; returns the log-likelihoods."""
        torch = self.torch
        wl = r["wl"]
        d = self.packed[k]
        n = len(r["theta"])
        with torch.cuda.stream(self.stream):
            self.theta[:r["theta"].size].copy_(torch.from_numpy(r["theta"].ravel()),
                                               non_blocking=True)
            self.ids[:n].copy_(torch.from_numpy(r["ids"].astype(np.int32)), non_blocking=True)
            view = {}
            for key, t in self.data.items():
                t[:d[key].size].copy_(torch.from_numpy(d[key].ravel()), non_blocking=True)
                view[key] = t
            lik.eval_batch_device(self.nets[wl.name], wl.obs_kind, wl.observed, wl.sigma,
                                  self.theta[:r["theta"].size], view, d["obs_offsets"], r["H"],
                                  r["seed"], self.ll, self.st, self.ws, self.ws_bytes + 256,
                                  self.stream, kernel=self.kernel, theta_ids_dev=self.ids)
            self.ll_host[:n].copy_(self.ll[:n], non_blocking=True)
        self.stream.synchronize()
        return self.ll_host[:n].numpy().copy()

    def run(self, reqs, arrivals=None):
        """Requests one at a time, in arrival order.  Returns (wall seconds,
        latencies, results)."""
        lat, out = [], []
        t0 = time.perf_counter()
        for k, r in enumerate(reqs):
            if arrivals is not None:
                wait = t0 + arrivals[k] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
            out.append(self.run_one(k, r))
            lat.append(time.perf_counter() - (t0 + (arrivals[k] if arrivals is not None else 0.0)))
        return time.perf_counter() - t0, np.array(lat), out


def run_server(reqs, nets, arrivals=None, tuning=None, arena_bytes=8 << 30):
    """Every request through one server.  Returns (wall seconds, latencies,
    statistics, results)."""
    lat = np.zeros(len(reqs))
    results = [None] * len(reqs)
    with lik.Server(arena_bytes=arena_bytes, kernel=lik.KERNEL_SPECIALIZED, tuning=tuning) as srv:
        t0 = time.perf_counter()
        tickets = [None] * len(reqs)
        sub_t = np.zeros(len(reqs))

        def waiter():
            for k in range(len(reqs)):
                while tickets[k] is None:
                    time.sleep(1e-4)
                results[k] = srv.wait(tickets[k])[0]
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
    return total, lat, stats, results


def _ms(lat):
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3)}


def compare(reqs, nets, load=0.8, tuning=None, log=None):
    """Saturated and at-load comparison of the served and plain paths on one
    request set; the served results must equal the plain ones bit for bit."""
    say = log or (lambda *a: None)
    n_evals = sum(len(r["theta"]) for r in reqs)
    plain = PlainRunner(reqs, nets)
    plain.run(reqs[:4])          # kernel loads, allocator, stream
    run_server(reqs[:4], nets, tuning=tuning)
    say("warm")
    t_plain, _, res_plain = plain.run(reqs)
    say(f"plain saturated {n_evals / t_plain:.1f} evals/s")
    t_srv, _, st_sat, res_srv = run_server(reqs, nets, tuning=tuning)
    say(f"server saturated {n_evals / t_srv:.1f} evals/s")
    equal = all(np.array_equal(a, b, equal_nan=True) for a, b in zip(res_plain, res_srv))
    rate = load * len(reqs) / t_plain   # requests per second
    arrivals = np.cumsum(np.random.default_rng(6).exponential(1.0 / rate, len(reqs)))
    tp, lat_p, _ = plain.run(reqs, arrivals)
    say("plain at load done")
    ts, lat_s, st, res_load = run_server(reqs, nets, arrivals, tuning=tuning)
    say("server at load done")
    equal = equal and all(np.array_equal(a, b, equal_nan=True) for a, b in zip(res_plain, res_load))
    return {
        "requests": len(reqs), "evals": n_evals,
        "saturated": {"served_evals_per_s": n_evals / t_srv, "plain_evals_per_s": n_evals / t_plain,
                      "speedup": t_plain / t_srv},
        "at_load": {"arrival_rate_req_per_s": rate, "load_vs_plain_saturation": load,
                    "served": dict(evals_per_s=n_evals / ts, **_ms(lat_s)),
                    "plain": dict(evals_per_s=n_evals / tp, **_ms(lat_p))},
        "server_stats": st,
        "served_equals_alone": bool(equal),
        "plain_path": "same specialised kernels once per request via lik_eval_batch_device; "
                      "buffers and workspace allocated once, one long-lived stream, inputs "
                      "copied in and results out per request",
        "workload": STREAM_WORKLOAD,
    }


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
    nets = make_networks(reqs)
    n_evals = sum(len(r["theta"]) for r in reqs)

    def say(m):
        print("[serve]", m, flush=True, file=sys.stderr)

    if args.uneven:
        out = uneven_block(reqs, nets, log=say)
        out["metric"] = "uneven batch in one persistent launch: evals/s, makespan, p50/p99 completion"
        run_server(reqs[:8], nets, tuning=tuning)
        t_srv, lat, st, _ = run_server(reqs, nets, tuning=tuning)
        say(f"uneven batch through the server in {t_srv:.2f} s")
        out["server"] = {"makespan_s": t_srv, "evals_per_s": n_evals / t_srv,
                         "p50_completion_ms": float(np.percentile(lat, 50) * 1e3),
                         "p99_completion_ms": float(np.percentile(lat, 99) * 1e3),
                         "path": "the same requests submitted at once to a lik_server "
                                 "(per-interval iterations)"}
        if args.plain_sample:
            sample = reqs[:args.plain_sample]
            plain = PlainRunner(sample, nets)
            plain.run(sample[:4])
            t_plain, _, _ = plain.run(sample)
            out["plain_evals_per_s"] = len(sample) / t_plain
            out["plain_sample"] = f"first {len(sample)} requests one at a time (plain path)"
        print(json.dumps(out), flush=True)
        return
    out = compare(reqs, nets, load=args.load, tuning=tuning, log=say)
    out["metric"] = "served likelihood evals/s; p50/p99 latency"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
