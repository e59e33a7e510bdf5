"""Throughput of the particle-filter likelihood on one MI355X.

A step is one lik_eval_batch_device call: the whole hot path (direct-method
SSA propagation, observation weighting, log-sum-exp, systematic resampling,
per-theta reduction) over one batch.  Default workload: the telegraph
gene-expression batch, 1,024 rate vectors x 10 observed trajectories x 1,000
filter particles x 50 log-normal observations, binary64.  --workload random:
the seeded 20-species, 40-reaction mass-action network, 4,096 rate vectors x
1 trajectory x 512 particles x 100 Gaussian observations, at the observation
interval where the median rate vector realises 1e4 SSA events per particle
per interval (~2.4e12 events per batch).  --workload lacgfp: the Lac-Gfp
model, 1,024 parameter vectors around theta* x 5 trajectories x 200
particles x 29 fluorescence observations, random initial counts.  Inputs are
resident in device
memory before the timed region.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload telegraph|random|lacgfp|erk]
                  [--precision 0|1] [--no-cpu-baseline] [--no-serving]

The VALU roofline is priced with the lane-op issue slots per SSA event that
rocprofv3 measured on the same kernel sources (SQ_THREAD_CYCLES_VALU divided
by the launch's events, from the committed profile record); where no such
record matches the sources, with the model count of the event's operations
at their measured gfx950 issue costs.  Beside the whole-run rate the line
carries each timed step's device time (median, min, max, spread: HIP events
on the launch stream between steps) and the clocks and power rocm-smi reports
right after the timed steps.
"""
import argparse
import json
import os
import shutil
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one wave64 instruction per SIMD per 4 cycles), in lane-operations/s.
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


# Issue cost in full-rate VALU slots on gfx950, measured by
# microbench/isa_cost.hip (four wavefronts per SIMD, 4.3-4.5 cycles for a
# full-rate instruction; the table is in the profile summaries): a
# 32 x 32 -> 64 multiply-add takes one slot, the IEEE-correct binary64 divide
# sequence fifteen (58 cycles), the binary32 one ten (42 cycles); the log's
# in-range division (the same sequence less its two scalings and its fix-up)
# three slots less.
SLOTS_MAD_U64 = 1
SLOTS_DIV_F64 = 15
SLOTS_DIV_F32 = 10
SLOTS_DIV_INRANGE_F64 = SLOTS_DIV_F64 - 3
SLOTS_DIV_INRANGE_F32 = SLOTS_DIV_F32 - 3


def ops_per_event(R, U, precision):
    """Model count of the VALU issue slots one direct-method SSA event needs
    (lane operations, each instruction weighted by its measured issue cost).
    It counts the method's arithmetic, independent of how the kernel
    realises it; the design notes itemise it."""
    if precision == 0:
        philox = 10 * (2 * SLOTS_MAD_U64 + 2)   # 10 rounds: two 32x32->64 products, two 3-way xors
        uniforms = 2 * 6                # 53-bit assembly, int->binary64, scale (two uniforms)
        log = 7 + SLOTS_DIV_INRANGE_F64 + 3 + 10 + 5   # reduction, divide, squares, series, sum
        tau = SLOTS_DIV_F64             # IEEE binary64 divide
    else:
        philox = 10 * (2 * SLOTS_MAD_U64 + 2) // 2   # half a block per event
        uniforms = 2 * 3                # 24-bit shift, int->binary32, scale (two uniforms)
        log = 7 + SLOTS_DIV_INRANGE_F32 + 3 + 6 + 5
        tau = SLOTS_DIV_F32
    propensity = 3 * R                  # count -> float, times rate, running sum
    select = 1 + 2 * (R - 1)            # target, compare + select per reaction
    update = 2                          # species changed by one reaction (at most two here)
    clock = 3                           # a0 > 0, clock + tau, compare
    count = 2                           # event counter, cap test
    return philox + uniforms + log + tau + propensity + select + update + clock + count


def host_cores():
    """Cores this process may run on, the machine's count and CPU model."""
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return usable, os.cpu_count(), model


def cpu_baseline(wl, budget_s=15.0, share=16, per_call=2, t_sub=None):
    """Time the CPU oracle on a seeded random sample of theta (all
    trajectories, full particle count), per_call theta per call, on every
    core this process may use up to the GPU's host share.  t_sub: time only
    the first t_sub observations of each trajectory and scale the rate by
    t_sub / T (equal observation intervals: a bounded sample where one whole
    theta is minutes of CPU work)."""
    from oracle import oracle
    rng = np.random.default_rng(7)
    order = rng.permutation(wl.n_theta)
    usable, machine, model = host_cores()
    nthreads = max(1, min(share, usable))
    T = len(wl.trajectories[0]["t_obs"])
    trajs = wl.trajectories
    if t_sub:
        trajs = [dict(tr, t_obs=tr["t_obs"][:t_sub], y=tr["y"][:t_sub]) for tr in trajs]
    scale = (t_sub / T) if t_sub else 1.0
    done, t_total, events = [], 0.0, 0
    k = 0
    while t_total < budget_s and k < len(order):
        idx = order[k:k + per_call]
        k += len(idx)
        P = oracle.Problem(wl.net.orders, wl.net.stoich, wl.obs_kind, wl.observed, wl.sigma,
                           wl.theta[idx], trajs, wl.n_particles, wl.seed, theta_ids=idx)
        t0 = time.perf_counter()
        out = oracle.evaluate(P, nthreads=nthreads)
        t_total += time.perf_counter() - t0
        events += int(out["events"].sum())
        done += idx.tolist()
    return {"value": len(done) * scale / t_total, "unit": "likelihood evals/s", "cores": nthreads,
            "kind": "oracle",
            "host": {"cores_usable": usable, "cores_machine": machine, "cpu_model": model,
                     "threads_used": nthreads, "rule": "one oracle thread per usable core, at "
                     "most the GPU's host share of 16"},
            "sample": f"{len(done)} theta of the same batch (seeded random pick: "
                      f"{done}), all {wl.n_traj} trajectories, H={wl.n_particles}, "
                      + (f"the first {t_sub} of T={T} observations (rate scaled by {t_sub}/{T})"
                         if t_sub else f"T={T}")
                      + f"; {t_total:.1f} s wall, {events / t_total:.3g} SSA events/s"}


def workload(name):
    """(workload, description, record tag) of a bench workload."""
    from paper_1606_08281_amd import workloads as W
    if name == "telegraph":
        return (W.telegraph_workload(),
                "telegraph gene expression, 6 mass-action rates log-uniform over two decades; "
                "1024 theta x 10 trajectories x 1000 filter particles x 50 log-normal "
                "observations (sigma 0.1)", "telegraph_1024x10x1000x50")
    if name == "random":
        return (W.random_network_workload(dt=W.RANDOM_DT_1E4),
                "seeded random mass-action network, 20 species x 40 reactions (orders 0-2, net "
                "changes -2..2), rates log-uniform on [1e-3, 1]; 4096 theta x 1 trajectory x 512 "
                "filter particles x 100 Gaussian observations (sigma 10, species 0 and 1) at the "
                "interval where the median theta realises 1e4 SSA events per particle per "
                "interval", "random20x40_4096x1x512x100")
    if name == "lacgfp":
        return (W.lacgfp_workload(theta=W.lacgfp_population(1024), n_traj=5, n_particles=200),
                "Lac-Gfp, 9 species x 18 mass-action reactions, 18 parameters log-normal (sd 0.3) "
                "around theta* (a late level of the sampler's population); 1024 theta x 5 "
                "trajectories x 200 filter particles x 29 fluorescence observations of mature "
                "GFP; initial counts uniform per particle", "lacgfp_1024x5x200x29")
    raise SystemExit(f"unknown workload {name!r}")


def ode_step_work(spec):
    """(binary64 operations, lane-op issue slots) of one Dormand-Prince step
    attempt of a term-list model, a model count: six right-hand sides (the
    seventh stage is the next step's first) and, per species, the stage
    combinations (2i - 1 operations for stage i = 2..6), the fifth-order
    update (11), the error estimate (12) and its scaled norm (4, one of them a
    divide).  Slots: one per operation, the IEEE divide sequence SLOTS_DIV_F64,
    and the step-size factor's log and exp (~65)."""
    ops = divs = 0
    for T in spec["terms"]:
        ops += 1 if T.get("rate_param", -1) >= 0 else 0
        for kind, _, _ in T.get("factors", []):
            ops += {0: 1, 1: 3, 2: 4, 3: 4, 4: 1}[kind]
            divs += kind in (1, 2, 3)
        ops += (T.get("frm", -1) >= 0) + (T.get("to", -1) >= 0)
    ops, divs = 6 * ops, 6 * divs
    ops += spec["U"] * ((3 + 5 + 7 + 9 + 11) + 11 + 12 + 4)
    divs += spec["U"]
    return ops, ops - divs + SLOTS_DIV_F64 * divs + 65


def bench_erk(args):
    """The deterministic (ODE) likelihood of the Egf-Ras-Raf-Mek-Erk model:
    lik_ode_eval_device over a population of parameter vectors, six input
    patterns each, with the trajectories, parameter vectors and workspace
    resident on the device; the host entry point (copies and allocation in
    every call) is timed beside it.  The roofline uses the solver kernel's
    own HIP-event time."""
    import torch
    from paper_1606_08281_amd import lik
    from paper_1606_08281_amd import workloads as W
    torch.cuda.set_device(0)
    n = 65536
    wl = W.erk_workload(n_theta=n, spread=0.3)
    model = lik.OdeModel(wl["spec"])
    trajs = wl["trajectories"]
    kw = dict(rtol=1e-6, atol=1e-9, max_steps=100000)
    say = lambda m: print("[bench]", m, flush=True, file=sys.stderr)  # noqa: E731
    db = lik.OdeDeviceBatch(model, trajs, n, steps=True)
    theta = torch.from_numpy(np.ascontiguousarray(wl["theta"])).cuda()
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    say(f"erk workload ready: {n} theta x {len(trajs)} input patterns x 60 FRET observations")
    steps_sum = torch.zeros((), dtype=torch.float64, device="cuda")
    for w in range(args.warmup):
        db.run(theta, **kw)
        steps_sum.add_(db.steps[:n * len(trajs)].to(torch.float64).sum())
        torch.cuda.synchronize()
        say(f"warmup {w + 1}/{args.warmup} done")
    steps_sum.zero_()
    lik.timing_read()
    lik.timing_enable(True)
    mark, step_summary = step_clock(torch, args.steps, torch.cuda.current_stream())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mark()
    for k in range(args.steps):
        db.run(theta, **kw)
        steps_sum.add_(db.steps[:n * len(trajs)].to(torch.float64).sum())
        mark()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dev_state = device_state()
    lik.timing_enable(False)
    tm = lik.timing_read()
    say(f"{args.steps} steps done")
    steps_total = int(steps_sum.item())
    st = db.status[:n].cpu().numpy()
    # the host entry point on the same batch (PCIe copies and allocation included)
    h0 = time.perf_counter()
    ll_h, st_h = lik.ode_eval(model, wl["theta"], trajs, **kw)
    host_s = time.perf_counter() - h0
    same = bool(np.array_equal(ll_h, db.loglik[:n].cpu().numpy(), equal_nan=True))
    flops, slots = ode_step_work(wl["spec"])
    kernel_s = tm["propagate_ms"] / 1e3
    achieved = steps_total * slots / kernel_s / 1e12
    from paper_1606_08281_amd import profsum_ode
    rec = profsum_ode.read_record(os.path.join(
        ROOT, "profiles", "lik_ode_spec_traffic_erk_65536x6x60_fp64.txt"))
    out = {
        "metric": "deterministic likelihood evals/s", "value": n * args.steps / elapsed,
        "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Egf-Ras-Raf-Mek-Erk ODE model (14 species, 17 flux terms, 36 "
                               "parameters log-normal sd 0.3 around a reference point), 6 "
                               "piecewise-constant EGF input patterns x 60 FRET observations; "
                               "Dormand-Prince 5(4), rtol 1e-6, atol 1e-9", "n_theta": n},
        "status_counts": {str(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
        "step_ms": step_summary(),
        "device": dev_state,
        "solver_steps_per_eval": steps_total / (n * args.steps),
        "host_entry_point": {"evals_per_s": n / host_s, "ms": host_s * 1e3,
                             "path": "lik_ode_eval: host buffers, input copies, allocation and "
                                     "synchronisation in the call",
                             "equals_device_entry_point": same},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved / (VALU_PEAK_LANE_OPS / 1e12),
                     "traffic": float(rec["hbm_bytes_per_launch"]) if rec else None,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated; null unless the committed counter "
                                     "record matches the solver sources)",
                     "measured_slots_per_attempt": (float(rec["lane_slots_per_attempt"])
                                                    if rec else None),
                     "lane_utilisation": float(rec["lane_utilisation"]) if rec else None,
                     "fp64_tflops": steps_total * flops / kernel_s / 1e12,
                     "kernel": "lik_ode_spec (the model compiled with hipRTC): lanes take "
                               "(theta, input pattern) pairs from a shared counter",
                     "basis": "lane-op slots of the step attempts (model count, "
                              f"{slots} per attempt; {flops} binary64 operations) over the "
                              "solver kernel's HIP-event time",
                     "avg_launch_ms": tm["propagate_ms"] / max(tm["propagate_launches"], 1)},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import oracle
        usable, machine, model_name = host_cores()
        nth = max(1, min(16, usable))
        P = oracle.OdeProblem(wl["spec"], wl["theta"], trajs, **kw)
        c0 = time.perf_counter()
        oracle.ode_eval(P, nthreads=nth)
        ct = time.perf_counter() - c0
        out["cpu_baseline"] = {"value": n / ct, "unit": "deterministic likelihood evals/s",
                               "cores": nth, "kind": "oracle",
                               "sample": f"the whole batch ({n} theta, all 6 patterns); "
                                         f"{ct:.1f} s wall on {nth} threads"}
    print(json.dumps(out), flush=True)


def step_clock(torch, n_steps, stream):
    """HIP events recorded on the launch stream before the first timed step
    and after each one: per-step device times with no host synchronisation
    inside the timed region.  mark() after each step; summary() once the
    stream has been synchronised."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_steps + 1)]
    state = {"k": 0}

    def mark():
        ev[state["k"]].record(stream)
        state["k"] += 1

    def summary():
        ms = [a.elapsed_time(b) for a, b in zip(ev[:-1], ev[1:])]
        med = float(np.median(ms))
        return {"median": med, "min": float(min(ms)), "max": float(max(ms)),
                "spread": float((max(ms) - min(ms)) / med) if med > 0 else None,
                "each": [round(float(v), 3) for v in ms],
                "basis": "HIP events between consecutive timed steps on the launch stream"}

    return mark, summary


def device_state():
    """Clocks and power as rocm-smi reports them, read once right after the
    timed steps (a child process; null fields if the tool is unavailable).
    The tool is a Python script: it runs under this interpreter, so no
    launcher process (its `env` line) stands between; and it is not started
    at all under a profiler, whose preloaded library the child would inherit."""
    preload = os.environ.get("LD_PRELOAD", "")
    if "rocprof" in preload or any(k.startswith("ROCPROF") for k in os.environ):
        return {"rocm_smi": None, "skipped": "running under a profiler"}
    try:
        tool = shutil.which("rocm-smi")
        if tool is None:
            raise FileNotFoundError("rocm-smi not on PATH")
        r = subprocess.run([sys.executable, os.path.realpath(tool), "--showclocks",
                            "--showpower", "--showmaxpower", "--json"],
                           capture_output=True, text=True, timeout=30)
        txt = r.stdout[r.stdout.find("{"):]
        d = json.loads(txt) if txt else {}
        card = next((v for k, v in d.items() if k.startswith("card")), {})
        keep = {k: v for k, v in card.items()
                if any(w in k.lower() for w in ("clk", "clock", "power"))}
        return {"rocm_smi": keep or None}
    except (OSError, ValueError, subprocess.SubprocessError) as e:
        return {"rocm_smi": None, "error": str(e)[:200]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the served-vs-plain block (continuous batching against the same "
                         "kernels launched once per request)")
    ap.add_argument("--serving-requests", type=int, default=160)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--workload", default="telegraph",
                    choices=["telegraph", "random", "lacgfp", "erk"])
    ap.add_argument("--graph", action="store_true",
                    help="replay the step's launch sequence as a captured HIP graph")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device (a known-size reference for "
                         "hardware byte counters)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate work partitionings on this batch first and keep "
                         "the fastest (default: the library's default partitioning)")
    ap.add_argument("--tuning", default=None,
                    help="work partitioning pool_min,pool_max,pool_events,pool_first,refill_min,"
                         "priority,items_per_cu,persistent,schedule,urgent_events,backlog_per_cu "
                         "(default: the library's)")
    ap.add_argument("--kernel", type=int, default=0,
                    help="0 auto, 1 generic, 2 network-specialised propagation kernel")
    ap.add_argument("--no-compare", action="store_true",
                    help="FP32-mixed: skip the binary64 runs of the same batch that the "
                         "per-result difference is taken against (profiling passes, whose "
                         "counters must see the timed kernel's launches only)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the likelihood path is built and timed on a "
              "single MI355X (see the design notes for how it shards); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "erk":
        bench_erk(args)
        return

    import torch
    from paper_1606_08281_amd import lik
    from paper_1606_08281_amd import workloads as W

    torch.cuda.set_device(0)
    wl, wl_desc, wl_tag = workload(args.workload)
    net = lik.Network(wl.net.orders, wl.net.stoich)
    db = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories, wl.n_theta,
                         wl.n_particles, precision=args.precision, kernel=args.kernel,
                         graph=args.graph)
    theta = torch.from_numpy(wl.theta).cuda()
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] workload ready: {wl.n_theta} theta x {wl.n_traj} traj x "
          f"{wl.n_particles} particles x {len(wl.trajectories[0]['t_obs'])} obs", flush=True,
          file=sys.stderr)

    if args.tuning:
        keys = ("pool_min", "pool_max", "pool_events", "pool_first", "refill_min", "priority",
                "items_per_cu", "persistent", "schedule", "urgent_events", "backlog_per_cu")
        net.set_tuning(**dict(zip(keys, (int(v) for v in args.tuning.split(",")))))
    tuning = net.tuning()
    if args.autotune:
        tuning = db.autotune(theta, wl.seed, stream=stream)
        print(f"[bench] autotuned: {tuning}", flush=True, file=sys.stderr)

    # per-step event totals and maxima accumulate on the device, in stream
    # order, so the timed steps run back to back with no host round trip
    ev_sum = torch.zeros((), dtype=torch.float64, device="cuda")
    ev_max = torch.zeros((), dtype=torch.float64, device="cuda")

    def count_events():
        ev = db.events.to(torch.float64)
        ev_sum.add_(ev.sum())
        torch.maximum(ev_max, ev.max(), out=ev_max)

    for w in range(args.warmup):
        db.run(theta, wl.seed, stream=stream)
        count_events()  # (the warmup also loads torch's reduction kernels)
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", flush=True, file=sys.stderr)
    ev_sum.zero_()
    ev_max.zero_()

    lik.timing_read()
    lik.timing_enable(True)
    mark, step_summary = step_clock(torch, args.steps, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mark()
    for k in range(args.steps):
        db.run(theta, wl.seed + k, stream=stream)
        count_events()
        mark()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] {args.steps} steps done", flush=True, file=sys.stderr)
    dev_state = device_state()
    events = int(ev_sum.item())
    max_per_particle = float(ev_max.item()) / wl.n_particles
    lik.timing_enable(False)
    tm = lik.timing_read()
    status = db.status.cpu().numpy()

    fp32_error = None
    if args.precision == 1 and not args.no_compare:
        # the same batch and seed in binary64, and again under another seed:
        # the two precisions draw different random numbers, so FP32-mixed
        # against FP64 is a Monte-Carlo difference, read beside FP64's own
        # seed-to-seed difference
        ll32 = db.loglik.cpu().numpy().copy()
        ev32 = db.events.cpu().numpy().copy()
        db64 = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories,
                               wl.n_theta, wl.n_particles, precision=lik.FP64,
                               kernel=args.kernel)
        db64.run(theta, wl.seed + args.steps - 1, stream=stream)
        ll64 = db64.loglik.cpu().numpy().copy()
        ev64 = db64.events.cpu().numpy().copy()
        # Monte Carlo scale: the binary64 estimate under another seed
        db64.run(theta, wl.seed + args.steps, stream=stream)
        ll64b = db64.loglik.cpu().numpy().copy()

        def diff(a, b):
            ok = np.isfinite(a) & np.isfinite(b)
            err = np.abs(a[ok] - b[ok])
            if not err.size:
                return {"n": 0}
            rel = err / np.abs(b[ok])
            q = (10, 25, 50, 75, 90, 99)
            return {"n": int(ok.sum()), "abs_max": float(err.max()),
                    "abs_p50": float(np.median(err)), "abs_p99": float(np.percentile(err, 99)),
                    "rel_max": float(rel.max()),
                    "identical": int((err == 0).sum()),
                    "abs_quantiles": {f"p{k}": float(np.percentile(err, k)) for k in q},
                    "rel_quantiles": {f"p{k}": float(np.percentile(rel, k)) for k in q}}
        # (the two precisions draw different random numbers, so this is a
        # Monte-Carlo difference; filters_diverged: event totals that differ)
        fp32_error = dict(diff(ll32, ll64), vs="f64 path, same seed",
                          filters_diverged=float(np.mean(ev32 != ev64)),
                          filters=int(ev32.size),
                          f64_seed_to_seed=diff(ll64b, ll64))
        out_dir = os.path.join(ROOT, "gpurun_out")
        if os.path.isdir(out_dir):   # every result: FP32-mixed, FP64, FP64 under another seed
            np.save(os.path.join(out_dir, f"fp32_vs_fp64_{args.workload}.npy"),
                    np.stack([ll32, ll64, ll64b]))
        del db64

    # HBM bytes per launch from the committed rocprofv3 counter summary of
    # this kernel and configuration; null once the kernel sources differ.
    # The schedule that ran: the flow schedule makes one propagation launch
    # per step (the library takes the per-interval one where the flow
    # kernel's occupancy is too low, whatever the tuning asks for).
    flow = tm["propagate_launches"] == args.steps and tuning.get("schedule", 0) == 1
    kname = "lik_flow_spec" if flow else "lik_propagate_spec"
    fp = "fp64" if args.precision == 0 else "fp32mixed"
    traffic = None
    if args.kernel in (0, 2) and not args.tuning and not args.autotune:
        from paper_1606_08281_amd import profsum
        rec = profsum.read_traffic(os.path.join(ROOT, "profiles",
                                                f"{kname}_traffic_{wl_tag}_{fp}.txt"))
        if rec is not None:
            traffic = float(rec["hbm_bytes_per_launch"])

    evals = wl.n_theta * args.steps
    model_ope = ops_per_event(wl.net.R, wl.net.U, args.precision)
    # measured lane-op issue time per event (the committed counter record of
    # this kernel, configuration and sources), else the model count
    ope, ope_basis = model_ope, "model count at measured instruction costs (no counter record " \
                                "matches the current kernel sources)"
    passes = None
    if args.kernel in (0, 2) and not args.tuning and not args.autotune:
        from paper_1606_08281_amd import profsum
        rec_name = f"{kname}_valu_{wl_tag}_{fp}.txt"
        rec = profsum.read_record(os.path.join(ROOT, "profiles", rec_name))
        if rec is not None:
            passes = float(rec["lane_slots_per_event"])
        if rec is not None and "lane_time_slots_per_event" in rec:
            ope = float(rec["lane_time_slots_per_event"])
            ope_basis = ("measured: SQ_THREAD_CYCLES_VALU / SSA events of this kernel on these "
                         "sources, issue passes priced at the issue time per pass of its "
                         "instruction classes (profiles/" + rec_name + ")")
        elif rec is not None:
            ope = float(rec["lane_slots_per_event"])
            ope_basis = ("measured: SQ_THREAD_CYCLES_VALU / SSA events of this kernel on these "
                         "sources, issue passes (profiles/" + rec_name + ")")
    prop_s = tm["propagate_ms"] / 1e3
    # A replayed graph records no per-kernel events: its roofline is taken
    # over the whole step instead (a lower bound for the kernel's).
    basis = "propagation kernel time (HIP events on its stream)"
    if prop_s <= 0:
        prop_s = elapsed
        basis = "whole step time (graph replay: no per-kernel events)"
    achieved = events * ope / prop_s / 1e12
    peak = VALU_PEAK_LANE_OPS / 1e12
    out = {
        "metric": "likelihood evals/s",
        "value": evals / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32-mixed (f64 clock/weights)",
        "data": "synthetic",
        "config": {
            "workload": wl_desc,
            "n_theta": wl.n_theta, "n_traj": wl.n_traj, "n_particles": wl.n_particles,
            "n_obs": len(wl.trajectories[0]["t_obs"]), "precision": args.precision,
            "kernel": ["auto", "generic", "specialised"][args.kernel],
            "graph": bool(args.graph),
        },
        "step_ms": step_summary(),
        "device": dev_state,
        "reaction_events_per_s": events / elapsed,
        "events_per_step": events // args.steps,
        "max_events_per_particle": max_per_particle,
        "status_counts": {str(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))},
        "kernel_ms_per_step": {"propagate": tm["propagate_ms"] / args.steps,
                               "weigh_resample": tm["weigh_ms"] / args.steps},
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tlane-op/s",
            "frac": achieved / peak, "traffic": traffic,
            "kernel": (kname + ": every interval in one launch (direct-method SSA work items "
                       "and each filter's weighing/resampling)") if flow else
                      (kname + ": direct-method SSA to the next observation, one launch per "
                       "interval"),
            "basis": basis,
            "ops_per_event": ope,
            "ops_per_event_basis": ope_basis,
            "issue_passes_per_event": passes,
            "model_ops_per_event": model_ope,
            "model_frac": events * model_ope / prop_s / 1e12 / peak,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "avg_launch_ms": tm["propagate_ms"] / max(tm["propagate_launches"], 1),
            "launches": tm["propagate_launches"],
        },
        "cpu_baseline": None,
        "tuning": tuning,
    }
    if fp32_error is not None:
        out["fp32_error_vs_fp64"] = fp32_error
    if not args.no_serving:
        print("[bench] serving block: served vs plain per-request launches", flush=True,
              file=sys.stderr)
        from paper_1606_08281_amd import serve_bench as SB
        reqs = SB.request_stream(args.serving_requests)
        t_s0 = time.perf_counter()
        nets = SB.make_networks(reqs)
        out["serving"] = SB.compare(reqs, nets, load=0.8,
                                    log=lambda m: print("[bench] serving:", m, flush=True,
                                                        file=sys.stderr))
        out["serving"]["wall_s"] = time.perf_counter() - t_s0
        print("[bench] uneven block: 8192 mixed requests in one persistent launch", flush=True,
              file=sys.stderr)
        t_u0 = time.perf_counter()
        out["uneven"] = SB.uneven_block(log=lambda m: print("[bench] uneven:", m, flush=True,
                                                            file=sys.stderr))
        out["uneven"]["wall_s"] = time.perf_counter() - t_u0
        print("[bench] sampler-stream block: level-set sampler runs against one server",
              flush=True, file=sys.stderr)
        from paper_1606_08281_amd import serve_lns as SL
        t_l0 = time.perf_counter()
        say_l = lambda m: print("[bench] sampler:", m, flush=True, file=sys.stderr)  # noqa: E731
        rep, recs, nets_l = SL.closed_loop(N=120, levels=4, check=16, log=say_l)
        rep.pop("samplers", None)
        rep["replay"] = SL.replay(recs, nets_l, 1500, log=say_l)
        rep["workload"] = SL.WORKLOAD.replace("N 200", "N 120") + "; 4 levels"
        rep["wall_s"] = time.perf_counter() - t_l0
        out["sampler_stream"] = rep
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", flush=True, file=sys.stderr)
        out["cpu_baseline"] = (cpu_baseline(wl, per_call=1, t_sub=10) if args.workload == "random"
                               else cpu_baseline(wl))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
