"""Summary of rocprofv3 output for the deterministic-model (ODE) solver kernel,
for the profiles/ folder, and the source fingerprint of that kernel.

  python -m paper_1606_08281_amd.profsum_ode --stats DIR --fetch DIR --write DIR \\
      --util DIR --valu DIR --valu-bench JSON --bench JSON --commands FILE \\
      --out profiles/NAME.md --traffic profiles/NAME.txt

The folders are rocprofv3 outputs written with --output-format csv, as for
profsum (the FETCH_SIZE and WRITE_SIZE passes run with bench.py
--copy-calibration).  The unit of work is a step attempt of the
Dormand-Prince solver: SQ_THREAD_CYCLES_VALU divided by the launch's step
attempts is the measured lane-op issue slots per attempt.
"""
import argparse
import hashlib
import json
import os

from paper_1606_08281_amd import profsum as P

KERNEL = "lik_ode_spec"
# Sources that decide what the solver kernel executes.
ODE_SOURCES = ["paper_1606_08281_amd/csrc/ode.hpp",
               "paper_1606_08281_amd/csrc/ode.hip",
               "paper_1606_08281_amd/csrc/devmath.hpp",
               "paper_1606_08281_amd/csrc/specialize.cpp",
               "include/lik.h"]


def source_sha256():
    h = hashlib.sha256()
    for rel in ODE_SOURCES:
        h.update(rel.encode())
        with open(os.path.join(P.ROOT, rel), encoding="utf-8") as f:
            h.update(P._code_only(f.read()).encode())
    return h.hexdigest()


def read_record(path):
    """A record written by this module, or None if absent or taken on other
    solver sources."""
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    return rec if rec.get("source_sha256") == source_sha256() else None


def _kind(name):
    return KERNEL if KERNEL in name else P._kind(name)


def _means(pmc_dir):
    acc = {}
    for (k, c), (v, n) in P.counter_means(pmc_dir).items():
        acc[(_kind(k), c)] = (v, n)
    return acc


def main():
    ap = argparse.ArgumentParser()
    for k in ("--stats", "--fetch", "--write", "--util", "--valu", "--valu-bench", "--bench",
              "--commands", "--out", "--traffic"):
        ap.add_argument(k, required=True)
    ap.add_argument("--title", default="lik_ode_spec — Egf-Ras-Raf-Mek-Erk ODE model, "
                                       "65536 theta x 6 input patterns x 60 FRET obs (FP64)")
    a = ap.parse_args()

    stats = P.kernel_stats(a.stats)
    for s in stats:
        if KERNEL in s["kernel"]:
            s["kernel"] = KERNEL
    tr = P.traffic(a.fetch, a.write, KERNEL)
    bench = json.loads(open(a.bench).read().strip().splitlines()[-1])
    vb = json.loads(open(a.valu_bench).read().strip().splitlines()[-1])
    vm = _means(a.valu)
    attempts = vb["solver_steps_per_eval"] * vb["config"]["n_theta"]  # one step: one launch
    c = {n: vm[(KERNEL, n)][0] for n in P.VALU_COUNTERS if (KERNEL, n) in vm}
    slots = c["SQ_THREAD_CYCLES_VALU"] / attempts
    lane_util = c["SQ_THREAD_CYCLES_VALU"] / (c["SQ_ACTIVE_INST_VALU"] * 64.0)
    util = _means(a.util)
    sha = source_sha256()
    rl = bench["roofline"]
    lines = [f"# {a.title}", "",
             "One bench step = one lik_ode_eval call: input copies, lik_ode_spec (the model "
             "compiled with hipRTC; every lane takes (theta, pattern) pairs from a shared "
             "counter and integrates them) and k_ode_finish (per-theta sums).", "",
             "Commands (repository root on one MI355X, `R` = its path):", "", "```"]
    lines += open(a.commands).read().strip().splitlines() + ["```", "",
              "Kernel statistics (rocprofv3 --kernel-trace --stats):", "",
              "| kernel | calls | total ms | average us | min us | max us | % |",
              "|---|---|---|---|---|---|---|"]
    for s in stats:
        lines.append(f"| {s['kernel']} | {s['calls']} | {s['total_ms']:.2f} | {s['avg_us']:.1f} | "
                     f"{s['min_us']:.1f} | {s['max_us']:.1f} | {s['pct']:.3f} |")
    lines += ["", f"bench.py, same configuration: {bench['value']:.0f} evals/s, "
                  f"{bench['ms_per_step']:.2f} ms per step; {KERNEL} average per launch "
                  f"{rl['avg_launch_ms']:.3f} ms (HIP events on the launch stream); "
                  f"{bench['solver_steps_per_eval']:.1f} step attempts per theta; VALU fraction "
                  f"{rl['frac']:.3f} of {rl['peak']:.2f} T lane-op/s by the model count; "
                  f"{rl['fp64_tflops']:.2f} TFLOP/s of binary64 arithmetic.", "",
              f"HBM traffic of {KERNEL} (rocprofv3 --pmc, one pass per counter):", "",
              f"- copy calibration (1 GiB device-to-device): FETCH_SIZE read "
              f"{tr['fetch_copy_kib']:.0f} KiB -> scale {tr['fetch_scale']:.4f}; WRITE_SIZE read "
              f"{tr['write_copy_kib']:.0f} KiB -> scale {tr['write_scale']:.4f}",
              f"- per launch ({tr['launches']} launches): FETCH_SIZE {tr['fetch_kib_per_launch']:.0f}"
              f" KiB -> {tr['fetch_bytes_per_launch'] / 1e6:.2f} MB; WRITE_SIZE "
              f"{tr['write_kib_per_launch']:.0f} KiB -> {tr['write_bytes_per_launch'] / 1e6:.2f} MB;"
              f" total {tr['hbm_bytes_per_launch'] / 1e6:.2f} MB", "",
              f"VALU work of {KERNEL} (rocprofv3 --pmc {' '.join(P.VALU_COUNTERS)}, one bench "
              "step):", "",
              f"- step attempts in the launch: {attempts:.6g}",
              f"- SQ_THREAD_CYCLES_VALU {c['SQ_THREAD_CYCLES_VALU']:.6g}, SQ_ACTIVE_INST_VALU "
              f"{c['SQ_ACTIVE_INST_VALU']:.6g}, SQ_INSTS_VALU {c['SQ_INSTS_VALU']:.6g}, "
              f"GRBM_GUI_ACTIVE {c.get('GRBM_GUI_ACTIVE', 0):.6g}",
              f"- lane-op issue slots per step attempt (SQ_THREAD_CYCLES_VALU / attempts): "
              f"{slots:.1f} (model count {rl['basis'].split('(model count, ')[-1].split(' ')[0]})",
              f"- active lanes per VALU issue slot: {lane_util:.3f}", "",
              "Utilisation counters (mean per dispatch):", ""]
    for (k, cn), (v, n) in sorted(util.items()):
        if k == KERNEL:
            lines.append(f"- {k} {cn}: {v:.2f} ({n} dispatches)")
    lines += ["", f"Solver sources fingerprint (sha256): {sha}", ""]
    open(a.out, "w").write("\n".join(lines))
    with open(a.traffic, "w") as f:
        f.write(f"# HBM traffic of {KERNEL} per launch, {a.title};\n"
                "# read by bench.py while the solver sources match.\n")
        f.write(f"source_sha256: {sha}\n")
        for k in ("fetch_scale", "write_scale", "fetch_bytes_per_launch",
                  "write_bytes_per_launch", "hbm_bytes_per_launch"):
            f.write(f"{k}: {tr[k]:.6g}\n")
        f.write(f"lane_slots_per_attempt: {slots:.6g}\n")
        f.write(f"lane_utilisation: {lane_util:.6g}\n")
    print(a.out, a.traffic)


if __name__ == "__main__":
    main()
