"""Summaries of rocprofv3 output for the profiles/ folder, and the source
fingerprint that ties a hardware-counter reading to the kernel it was taken on.

  python -m paper_1606_08281_amd.profsum --stats DIR --fetch DIR --write DIR \\
      [--util DIR] [--valu DIR --valu-bench JSON --valu-record profiles/NAME.txt] \\
      [--isa FILE] --bench BENCH_JSON --out profiles/NAME.md --traffic profiles/NAME.txt

DIR arguments are rocprofv3 output folders written with --output-format csv
(--kernel-trace --stats for --stats; --pmc FETCH_SIZE / WRITE_SIZE /
VALUBusy VALUUtilization for the others, each run with bench.py
--copy-calibration so that a device-to-device copy of 1 GiB is in the same
trace).  FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is scaled by
the ratio of the copy's known bytes to what the counter read for it.

--valu: a pass with SQ_THREAD_CYCLES_VALU, SQ_ACTIVE_INST_VALU, SQ_INSTS_VALU
and GRBM_GUI_ACTIVE over one bench step whose JSON line is --valu-bench.
SQ_THREAD_CYCLES_VALU counts VALU issue passes times the lanes active in
them: a wave64 instruction with every lane active is 64, whatever its issue
time, v_rcp_f32 128 and v_rcp_f64 256.  Divided by the SSA events of the
launch it is the measured lane-op issue passes per event, the
per-event count of issue passes.  --isa adds the table printed by
microbench/isa_cost.hip.

--types: two passes with the SQ_INSTS_VALU_<class> counters (INT32, INT64,
CVT, ADD/MUL/FMA/TRANS per precision; the rest is "other") over one bench
step, and --mix the isamix JSON of the kernel.  Every class is priced at the
issue time per pass of its instructions in the event loop: the passes per
event times that ratio are the lane-op issue time per event (in full-rate
slots), which bench.py prices the VALU roofline with.
"""
import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 1 << 30  # bench.py --copy-calibration: 2^28 float32 copied device to device

# Sources that decide what the propagation kernel executes and how work is cut
# into pools (and so its memory traffic).
KERNEL_SOURCES = ["paper_1606_08281_amd/csrc/propagate.hpp",
                  "paper_1606_08281_amd/csrc/devmath.hpp",
                  "paper_1606_08281_amd/csrc/lik_internal.hpp",
                  "paper_1606_08281_amd/csrc/weigh.hpp",
                  "paper_1606_08281_amd/csrc/flow.hpp",
                  "paper_1606_08281_amd/csrc/kernels.hip",
                  "paper_1606_08281_amd/csrc/specialize.cpp",
                  "paper_1606_08281_amd/csrc/host.hpp",
                  "paper_1606_08281_amd/csrc/api.cpp",
                  "include/lik.h"]


def _code_only(text):
    """C/C++ source without comments and blank space runs: the fingerprint
    follows the code the counters were taken on, not edits to its comments."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"' or c == "'":  # string or character literal, copied whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_sha256():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        h.update(rel.encode())
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def _kind(name):
    if "propagate" in name:
        return "lik_propagate_spec" if "spec" in name else "lik::k_propagate"
    if "lik_flow_spec" in name:
        return "lik_flow_spec"
    for k in ("k_flow_init", "k_flow_seed", "k_flow_check", "k_flow", "k_order_count",
              "k_order_scan", "k_order_place", "k_order_reset", "k_order", "k_weigh",
              "k_admit", "k_finish", "k_aux_filters", "k_aux_state"):
        if k in name:
            return "lik::" + k
    if "copyBuffer" in name:
        return "__amd_rocclr_copyBuffer"
    if "reduce_kernel" in name:
        return "torch reduce"
    if "elementwise" in name:
        return "torch elementwise"
    return name[:40]


def _one(pattern):
    hits = glob.glob(pattern, recursive=True)
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def kernel_stats(stats_dir):
    rows = list(csv.DictReader(open(_one(os.path.join(stats_dir, "**", "*kernel_stats.csv")))))
    out = []
    for r in rows:
        out.append({"kernel": _kind(r["Name"]), "calls": int(r["Calls"]),
                    "total_ms": float(r["TotalDurationNs"]) / 1e6,
                    "avg_us": float(r["AverageNs"]) / 1e3, "min_us": float(r["MinNs"]) / 1e3,
                    "max_us": float(r["MaxNs"]) / 1e3, "pct": float(r["Percentage"])})
    return out


def counter_means(pmc_dir):
    """{(kernel kind, counter): (mean per dispatch, dispatches)}"""
    rows = list(csv.DictReader(open(_one(os.path.join(pmc_dir, "**",
                                                      "*counter_collection.csv")))))
    acc = {}
    for r in rows:
        key = (_kind(r["Kernel_Name"]), r["Counter_Name"])
        acc.setdefault(key, []).append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def dispatches(pmc_dir, kind):
    """Number of dispatches of a kernel kind in a --pmc folder."""
    rows = list(csv.DictReader(open(_one(os.path.join(pmc_dir, "**",
                                                      "*counter_collection.csv")))))
    return len({r["Dispatch_Id"] for r in rows if _kind(r["Kernel_Name"]) == kind})


def check_dispatches(pmc_dir, kind, expect):
    """Counter means are taken per dispatch of a kernel kind: a folder that
    also holds other launches of the same kernel name (FP32-mixed runs that
    also ran binary64 batches, say) would mix their counts in."""
    n = dispatches(pmc_dir, kind)
    if n != expect:
        raise SystemExit(f"{pmc_dir}: {n} dispatches of {kind}, the profiled bench step "
                         f"launches {expect}")


def counter_sum(pmc_dir, kind, counter):
    rows = list(csv.DictReader(open(_one(os.path.join(pmc_dir, "**",
                                                      "*counter_collection.csv")))))
    return sum(float(r["Counter_Value"]) for r in rows
               if _kind(r["Kernel_Name"]) == kind and r["Counter_Name"] == counter)


def traffic(fetch_dir, write_dir, kernel="lik_flow_spec"):
    fetch_copy_kib = counter_sum(fetch_dir, "__amd_rocclr_copyBuffer", "FETCH_SIZE")
    write_copy_kib = counter_sum(write_dir, "__amd_rocclr_copyBuffer", "WRITE_SIZE")
    fs = COPY_BYTES / (fetch_copy_kib * 1024.0)
    ws = COPY_BYTES / (write_copy_kib * 1024.0)
    f_kib, n_f = counter_means(fetch_dir)[(kernel, "FETCH_SIZE")]
    w_kib, n_w = counter_means(write_dir)[(kernel, "WRITE_SIZE")]
    fb = f_kib * 1024.0 * fs
    wb = w_kib * 1024.0 * ws
    return {"fetch_copy_kib": fetch_copy_kib, "write_copy_kib": write_copy_kib,
            "fetch_scale": fs, "write_scale": ws, "fetch_kib_per_launch": f_kib,
            "write_kib_per_launch": w_kib, "launches": min(n_f, n_w),
            "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
            "hbm_bytes_per_launch": fb + wb}


def read_record(path):
    """A record written by this module (traffic or VALU work), or None if
    absent or taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("source_sha256") != source_sha256():
        return None
    return rec


read_traffic = read_record


VALU_COUNTERS = ("SQ_THREAD_CYCLES_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU",
                 "GRBM_GUI_ACTIVE")


def valu_work(valu_dir, bench_line, kernel):
    """Per-launch VALU counters of `kernel` and the per-event figures."""
    means = counter_means(valu_dir)
    c = {n: means[(kernel, n)][0] for n in VALU_COUNTERS if (kernel, n) in means}
    launches = bench_line["roofline"]["launches"]
    events = bench_line["events_per_step"] * bench_line["steps"] / max(launches, 1)
    out = {"events_per_launch": events, "launches_profiled": means[(kernel, VALU_COUNTERS[0])][1]}
    out.update({n.lower(): v for n, v in c.items()})
    out["lane_slots_per_event"] = c["SQ_THREAD_CYCLES_VALU"] / events
    out["wave_insts_per_event"] = c["SQ_INSTS_VALU"] / events
    out["lane_utilisation"] = c["SQ_THREAD_CYCLES_VALU"] / (c["SQ_ACTIVE_INST_VALU"] * 64.0)
    return out


TYPE_COUNTERS = ("INT32", "INT64", "CVT", "FMA_F32", "ADD_F32", "MUL_F32", "TRANS_F32",
                 "FMA_F64", "ADD_F64", "MUL_F64", "TRANS_F64")
DEFAULT_PASSES = {"TRANS_F64": 4, "TRANS_F32": 2}


def issue_time(type_dirs, kernel, mix, events):
    """Issue time per issue pass of `kernel`'s VALU work: the kernel's own
    SQ_INSTS_VALU_<class> totals (two --pmc passes), each class priced at the
    time and passes per instruction of the same class in the event loop's mix
    (isamix).  A class the loop lacks is priced at one slot per pass."""
    means = {}
    for d in type_dirs:
        for (k, c), (v, n) in counter_means(d).items():
            if k == kernel:
                means[c] = v
    total = means["SQ_INSTS_VALU"]
    counts = {t: means.get("SQ_INSTS_VALU_" + t, 0.0) for t in TYPE_COUNTERS}
    counts["other"] = total - sum(counts.values())
    rows, time, passes = [], 0.0, 0.0
    for t, n in counts.items():
        m = mix["per_class"].get(t)
        if m:
            p_i, w_i = m["passes"] / m["n"], m["time"] / m["n"]
        else:
            p_i = DEFAULT_PASSES.get(t, 1)
            w_i = float(p_i)
        time += n * w_i
        passes += n * p_i
        rows.append((t, n / events, m["n"] if m else 0, p_i, w_i))
    return {"rows": rows, "time_per_pass": time / passes, "passes_per_event": passes / events,
            "insts_per_event": total / events}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--util")
    ap.add_argument("--valu", help="rocprofv3 --pmc folder with the VALU work counters")
    ap.add_argument("--valu-bench", help="bench.py JSON line of the --valu run")
    ap.add_argument("--valu-record", help="record file of the measured VALU work per event")
    ap.add_argument("--isa", help="output of microbench/isa_cost.hip")
    ap.add_argument("--types", nargs=2, metavar="DIR",
                    help="two rocprofv3 --pmc folders with the SQ_INSTS_VALU_<class> counters")
    ap.add_argument("--types-bench", help="bench.py JSON line of the first --types run")
    ap.add_argument("--mix", help="isamix JSON of the same kernel")
    ap.add_argument("--bench", required=True, help="bench.py JSON line of the same configuration")
    ap.add_argument("--kernel", default="lik_flow_spec", help="kernel whose traffic is recorded")
    ap.add_argument("--title", default="lik_flow_spec — telegraph 1024 theta x 10 traj x "
                                       "1000 particles x 50 obs (FP64)")
    ap.add_argument("--commands", required=True, help="text file with the commands that ran")
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic", required=True)
    a = ap.parse_args()

    stats = kernel_stats(a.stats)
    bench = json.loads(open(a.bench).read().strip().splitlines()[-1])
    per_step = bench["roofline"]["launches"] // bench["steps"]
    calls = [s["calls"] for s in stats if s["kernel"] == a.kernel]
    if calls != [per_step * (bench["steps"] + bench["warmup"])]:
        raise SystemExit(f"{a.stats}: {a.kernel} calls {calls}, the bench line's steps launch "
                         f"{per_step * (bench['steps'] + bench['warmup'])}")
    # every --pmc pass profiles one bench step without warm-up
    for d in [a.fetch, a.write, a.util, a.valu] + list(a.types or []):
        if d:
            check_dispatches(d, a.kernel, per_step)
    tr = traffic(a.fetch, a.write, a.kernel)
    util = counter_means(a.util) if a.util else {}
    sha = source_sha256()
    lines = [f"# {a.title}", "",
             ("One bench step = k_admit, the flow set-up kernels, one lik_flow_spec launch (every "
              "interval: SSA work items and each filter's weighing) and k_finish."
              if a.kernel == "lik_flow_spec" else
              "Engine iteration = k_order_count + k_order_scan + k_order_place + "
              f"lik_propagate_spec + k_weigh; {per_step} iterations per "
              "bench step."), "", "Commands (repository root on one MI355X, `R` = its path):", "",
             "```"] + open(a.commands).read().strip().splitlines() + ["```", "",
             "Kernel statistics (rocprofv3 --kernel-trace --stats):", "",
             "| kernel | calls | total ms | average us | min us | max us | % |",
             "|---|---|---|---|---|---|---|"]
    for s in stats:
        lines.append(f"| {s['kernel']} | {s['calls']} | {s['total_ms']:.2f} | {s['avg_us']:.1f} | "
                     f"{s['min_us']:.1f} | {s['max_us']:.1f} | {s['pct']:.3f} |")
    rl = bench["roofline"]
    lines += ["", f"bench.py, same configuration: {bench['value']:.1f} evals/s, "
                  f"{bench['ms_per_step']:.1f} ms per step; {a.kernel} average per launch "
                  f"{rl['avg_launch_ms']:.3f} ms (HIP events on the launch stream).", "",
              f"HBM traffic of {a.kernel} (rocprofv3 --pmc, one pass per counter):", "",
              f"- copy calibration (1 GiB device-to-device): FETCH_SIZE read "
              f"{tr['fetch_copy_kib']:.0f} KiB -> scale {tr['fetch_scale']:.4f}; WRITE_SIZE read "
              f"{tr['write_copy_kib']:.0f} KiB -> scale {tr['write_scale']:.4f}",
              f"- per launch ({tr['launches']} launches): FETCH_SIZE {tr['fetch_kib_per_launch']:.0f}"
              f" KiB -> {tr['fetch_bytes_per_launch'] / 1e6:.1f} MB; WRITE_SIZE "
              f"{tr['write_kib_per_launch']:.0f} KiB -> {tr['write_bytes_per_launch'] / 1e6:.1f} MB;"
              f" total {tr['hbm_bytes_per_launch'] / 1e6:.1f} MB"]
    vw = None
    if a.valu:
        vb = json.loads(open(a.valu_bench).read().strip().splitlines()[-1])
        vw = valu_work(a.valu, vb, a.kernel)
        lines += ["", f"VALU work of {a.kernel} (rocprofv3 --pmc "
                      f"{' '.join(VALU_COUNTERS)}, one bench step):", "",
                  f"- SSA events in the launch: {vw['events_per_launch']:.6g}",
                  f"- SQ_THREAD_CYCLES_VALU {vw['sq_thread_cycles_valu']:.6g}, "
                  f"SQ_ACTIVE_INST_VALU {vw['sq_active_inst_valu']:.6g}, SQ_INSTS_VALU "
                  f"{vw['sq_insts_valu']:.6g}, GRBM_GUI_ACTIVE {vw.get('grbm_gui_active', 0):.6g}",
                  f"- lane-op issue slots per event (SQ_THREAD_CYCLES_VALU / events): "
                  f"{vw['lane_slots_per_event']:.2f}",
                  f"- wave64 VALU instructions per event (SQ_INSTS_VALU / events): "
                  f"{vw['wave_insts_per_event']:.3f}",
                  f"- active lanes per VALU issue slot: {vw['lane_utilisation']:.3f}"]
    if vw is not None and a.types:
        tb = json.loads(open(a.types_bench).read().strip().splitlines()[-1])
        ev = tb["events_per_step"] * tb["steps"] / max(tb["roofline"]["launches"], 1)
        mix = json.load(open(a.mix))
        it = issue_time(a.types, a.kernel, mix, ev)
        vw["time_per_pass"] = it["time_per_pass"]
        vw["lane_time_slots_per_event"] = vw["lane_slots_per_event"] * it["time_per_pass"]
        lines += ["", f"Issue time of the VALU work (rocprofv3 --pmc SQ_INSTS_VALU_<class>, two "
                      f"passes; event-loop mix from isamix, loop {mix['loop'][0]}..{mix['loop'][1]}"
                      f", {mix['valu_instructions']} VALU instructions, {mix['time_per_pass']:.3f} "
                      "slots per pass):", "",
                  "SQ_THREAD_CYCLES_VALU credits every wave64 VALU instruction with one issue "
                  "pass (the transcendental ones four or two); gfx950 issues the plain 32-bit "
                  "operations in about 0.6 of one.  Each class of the kernel's instructions is "
                  "priced at the issue time per pass of the same class in the event loop.", "",
                  "| class | wave64 instructions per event | in the loop | passes each | "
                  "slots each |", "|---|---|---|---|---|"]
        for t, n, nl, p_i, w_i in it["rows"]:
            lines.append(f"| {t} | {n:.4f} | {nl} | {p_i:.2f} | {w_i:.3f} |")
        lines += ["", f"- issue passes per event from the class counts: "
                      f"{it['passes_per_event']:.3f} wave64 (SQ_ACTIVE_INST_VALU / events: "
                      f"{vw['sq_active_inst_valu'] / vw['events_per_launch']:.3f})",
                  f"- issue time per issue pass: {it['time_per_pass']:.4f}",
                  f"- lane-op issue time per event: {vw['lane_slots_per_event']:.2f} passes x "
                  f"{it['time_per_pass']:.4f} = {vw['lane_time_slots_per_event']:.2f} slots"]
        # the bench line's launches: events per launch at its average launch time
        ev_b = bench["events_per_step"] * bench["steps"] / max(rl["launches"], 1)
        rate = ev_b / (rl["avg_launch_ms"] / 1e3)
        lines.append(f"- VALU fraction of the bench line's launches: {rate:.4g} events/s x "
                     f"{vw['lane_time_slots_per_event']:.2f} slots / {rl['peak']:.2f} T = "
                     f"{rate * vw['lane_time_slots_per_event'] / (rl['peak'] * 1e12):.3f} "
                     f"(issue passes alone: "
                     f"{rate * vw['lane_slots_per_event'] / (rl['peak'] * 1e12):.3f})")
        if mix.get("unpriced"):
            lines.append(f"- instructions of the loop priced at one slot (not timed by the "
                         f"microbenchmark): {mix['unpriced']}")
    if a.isa:
        lines += ["", "Issue cost of the event loop's instructions on gfx950 "
                      "(microbench/isa_cost.hip, one compute unit):", "", "```"]
        lines += open(a.isa).read().strip().splitlines() + ["```"]
    if util:
        lines += ["", "Utilisation counters (mean per dispatch):", ""]
        for (k, c), (v, n) in sorted(util.items()):
            if k in ("lik_propagate_spec", "lik_flow_spec", "lik::k_weigh", "lik::k_order_count",
                     "lik::k_order_scan", "lik::k_order_place"):
                lines.append(f"- {k} {c}: {v:.2f} ({n} dispatches)")
    lines += ["", f"Kernel sources fingerprint (sha256): {sha}", ""]
    open(a.out, "w").write("\n".join(lines))
    with open(a.traffic, "w") as f:
        f.write(f"# HBM traffic of {a.kernel} per launch, {a.title},\n"
                "# default work partitioning; read by bench.py while the kernel sources match.\n")
        f.write(f"source_sha256: {sha}\n")
        for k in ("fetch_scale", "write_scale", "fetch_bytes_per_launch",
                  "write_bytes_per_launch", "hbm_bytes_per_launch"):
            f.write(f"{k}: {tr[k]:.6g}\n")
    if vw is not None and a.valu_record:
        with open(a.valu_record, "w") as f:
            f.write(f"# VALU work of {a.kernel} per SSA event, {a.title};\n"
                    "# read by bench.py while the kernel sources match.\n")
            f.write(f"source_sha256: {sha}\n")
            for k in ("events_per_launch", "sq_thread_cycles_valu", "sq_active_inst_valu",
                      "sq_insts_valu", "lane_slots_per_event", "wave_insts_per_event",
                      "lane_utilisation", "time_per_pass", "lane_time_slots_per_event"):
                if k in vw:
                    f.write(f"{k}: {vw[k]:.6g}\n")
    print(a.out, a.traffic)


if __name__ == "__main__":
    main()
