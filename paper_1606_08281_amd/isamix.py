"""Instruction mix of a network-specialised SSA kernel's event loop, priced
with the issue costs that microbench/isa_cost.hip measures, for the
profiles/ folder.

  python -m paper_1606_08281_amd.isamix --workload telegraph --precision 0 \\
      --kernel lik_flow_spec --costs gpurun_out/isa_cost.txt --out MIX.json
  python -m paper_1606_08281_amd.isamix calibration --costs gpurun_out/isa_cost.txt \\
      --types DIR_A DIR_B --commands FILE --out profiles/NAME.md

Why: SQ_THREAD_CYCLES_VALU credits each wave64 VALU instruction with 64
lane-cycles per issue pass, whatever the instruction: one pass for every
instruction but the transcendental ones (v_rcp_f64 four, v_rcp_f32 two).
On gfx950 the plain 32-bit moves, additions, logic and shifts and the
binary32 additions, multiplies and fmas issue in about 0.6 of a pass, while
64-bit operations, conversions, compares and selects take a full pass or a
little more.  The counter is then a count of issue passes, and its ratio to
issue time depends on the mix of instructions.

What: the kernel is compiled with hipRTC into a private cache folder (no GPU
needed) and disassembled with llvm-objdump.  The event loop is the loop that
draws one Philox block (16 to 24 32 x 32 -> 64 multiplies), takes a log and
holds the most VALU instructions.  Each of its instructions gets the class rocprofv3's
SQ_INSTS_VALU_* counters file it under (INT32, INT64, CVT, ADD/MUL/FMA/TRANS
per precision, "other" for the rest: moves, logic, shifts, selects,
floating-point compares, the divide's scale and fix-up), its issue passes and
its issue time in full-rate slots.  The JSON output holds, per class, the
loop's instruction count, passes and time; profsum combines the per-class
time per pass with the kernel's own per-class counter totals.

Instructions the microbenchmark does not time take the cost of the closest
timed form: SDWA forms and three-operand 32-bit integer operations (add3,
lshl_add, max3, the carry forms, mbcnt) the cost of v_alignbit_b32, a 32-bit
operation that takes a full pass; 24-bit multiplies the cost of
v_mul_lo_u32; frexp/ldexp/trunc the cost of v_frexp_mant_f32; the divide's
scale, fix-up and fused step the cost of v_div_scale_f64.  Any other is
priced at one slot and listed under "unpriced".
"""
import argparse
import collections
import json
import os
import re
import shutil
import subprocess
import sys
import tempfile

OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"

F_TYPES = {"fma": "FMA", "fmac": "FMA", "fmamk": "FMA", "fmaak": "FMA", "mac": "FMA",
           "add": "ADD", "sub": "ADD", "subrev": "ADD", "mul": "MUL"}


def read_costs(path):
    """{microbenchmark name: issue slots} from isa_cost's table."""
    out = {}
    for line in open(path):
        if line.startswith("#") or line.startswith("instruction"):
            continue
        parts = line.rsplit(None, 3)
        if len(parts) == 4:
            try:
                out[parts[0].strip()] = float(parts[3])
            except ValueError:
                pass
    return out


def classify(op, k):
    """(counter class, issue passes, issue time in slots, priced) of one
    mnemonic, with k the microbenchmark's costs."""
    enc = "sdwa" if op.endswith("_sdwa") else ""
    o = re.sub(r"_(e32|e64|sdwa|dpp)$", "", op)
    vop3_32 = k["v_alignbit_b32"]
    sdwa = vop3_32
    m = re.match(r"v_(fma|fmac|fmamk|fmaak|mac|add|sub|subrev|mul)_f(32|64)$", o)
    if m:
        prec = m.group(2)
        cost = k["v_fma_f64"] if prec == "64" else (k["v_fma_f32"] if not enc else sdwa)
        return f"{F_TYPES[m.group(1)]}_F{prec}", 1, cost, True
    if re.match(r"v_(rcp|rsq|sqrt|log|exp|sin|cos)(_iflag)?_f64$", o):
        return "TRANS_F64", 4, k["v_rcp_f64"], True
    if re.match(r"v_(rcp|rsq|sqrt|log|exp|sin|cos)(_iflag)?_f32$", o):
        return "TRANS_F32", 2, k["v_rcp_f32"], True
    if o == "v_mad_u64_u32" or o == "v_mad_i64_i32":
        return "INT64", 1, k["v_mad_u64_u32"], True
    if re.match(r"v_mul_(hi|lo)_[ui]32$", o):
        return "INT32", 1, k["v_mul_lo_u32"], True
    if re.match(r"v_mul_(hi_)?[ui]32_[ui]24$", o):
        return "INT32", 1, k["v_mul_lo_u32"], True
    if re.match(r"v_cmpx?_\w+_[ui](16|32|64)$", o):
        return "INT32", 1, k["v_cmp_gt_u32"], True
    if re.match(r"v_cmpx?_\w+_f(16|32|64)$", o) or o.startswith("v_cmp_class"):
        return "other", 1, k["v_cmp_gt_f64"], True
    if o.startswith("v_cvt_"):
        return "CVT", 1, k["v_cvt_f64_u32"], True
    if o in ("v_add_u32", "v_sub_u32", "v_subrev_u32", "v_max_i32", "v_min_i32",
             "v_max_u32", "v_min_u32"):
        return "INT32", 1, (k["v_add_u32"] if not enc else sdwa), True
    if o in ("v_addc_co_u32", "v_subb_co_u32", "v_subbrev_co_u32", "v_add_co_u32",
             "v_sub_co_u32", "v_subrev_co_u32", "v_add3_u32", "v_lshl_add_u32", "v_max3_i32",
             "v_min3_i32", "v_max3_u32", "v_min3_u32", "v_mbcnt_lo_u32_b32", "v_mbcnt_hi_u32_b32",
             "v_mad_u32_u24", "v_mad_i32_i24", "v_xad_u32", "v_add_lshl_u32"):
        return "INT32", 1, vop3_32, True
    if o == "v_bitop3_b32":
        return "other", 1, k["v_bitop3_b32"], True
    if o in ("v_xor_b32", "v_and_b32", "v_or_b32", "v_not_b32"):
        return "other", 1, (k["v_xor_b32"] if not enc else sdwa), True
    if o in ("v_lshrrev_b32", "v_lshlrev_b32", "v_ashrrev_i32"):
        return "other", 1, (k["v_lshrrev_b32"] if not enc else sdwa), True
    if o == "v_mov_b32":
        return "other", 1, (k["v_mov_b32"] if not enc else sdwa), True
    if o == "v_mov_b64":
        return "other", 1, k["v_mov_b64"], True
    if o == "v_cndmask_b32":
        return "other", 1, k["v_cndmask_b32"], True
    if re.match(r"v_div_(scale|fixup)_f(32|64)$", o):
        return "other", 1, k["v_div_scale_f64"], True
    if re.match(r"v_div_fmas_f(32|64)$", o):
        return f"FMA_F{o[-2:]}", 1, k["v_div_scale_f64"], True
    if re.match(r"v_(frexp_mant|frexp_exp_i32|ldexp|trunc|floor|ceil|fract|rndne)_f(32|64)$", o):
        return "other", 1, k["v_frexp_mant_f32"], True
    if o in ("v_alignbit_b32", "v_alignbyte_b32", "v_bfe_u32", "v_bfe_i32", "v_bfi_b32",
             "v_perm_b32", "v_lshl_or_b32", "v_and_or_b32", "v_or3_b32", "v_xor3_b32",
             "v_readfirstlane_b32"):
        return "other", 1, vop3_32, True
    return "other", 1, 1.0, False


def parse(dis, kernel):
    """[(address, mnemonic, branch target or None)] of `kernel`."""
    out, inside, base = [], False, None
    for line in dis.splitlines():
        if line.endswith(">:"):
            inside = line.split("<", 1)[1].rstrip(">:") == kernel
            continue
        if not inside:
            continue
        m = re.match(r"\s+(\S+)(.*?)//\s*([0-9A-F]+):", line)
        if not m:
            continue
        addr = int(m.group(3), 16)
        if base is None:
            base = addr
        t = re.search(r"<[\w.]+\+0x([0-9a-f]+)>", line)
        out.append((addr, m.group(1), base + int(t.group(1), 16) if t else None))
    return out


def event_loop(insts):
    """The loop (first, last address) that draws one Philox block, takes the
    log of a uniform (v_frexp_*: the log's argument reduction) and holds the
    most VALU instructions; loops with cross-lane scans (ds_bpermute: the
    weighing and resampling) are not event loops."""
    best = None
    for a, op, t in insts:
        if t is None or t > a or not (op.startswith("s_cbranch") or op == "s_branch"):
            continue
        body = [x for x in insts if t <= x[0] <= a]
        n_mul = sum(1 for x in body if x[1] == "v_mad_u64_u32")
        n_valu = sum(1 for x in body if x[1].startswith("v_"))
        n_log = sum(1 for x in body if x[1].startswith("v_frexp_"))
        n_scan = sum(1 for x in body if x[1] == "ds_bpermute_b32")
        if 16 <= n_mul <= 24 and n_log and not n_scan and (best is None or n_valu > best[0]):
            best = (n_valu, t, a)
    if best is None:
        raise SystemExit("no loop with one Philox block found")
    return best[1], best[2]


def compile_kernel(workload, precision, cache):
    from paper_1606_08281_amd import lik
    from paper_1606_08281_amd import workloads as W
    net = {"telegraph": W.telegraph, "random": W.random_network, "lacgfp": W.lacgfp}[workload]()
    os.environ["LIK_KERNEL_CACHE"] = cache
    lik.Network(net.orders, net.stoich).precompile(precision)
    objs = [os.path.join(cache, f) for f in os.listdir(cache) if f.endswith(".co")]
    if len(objs) != 1:
        raise SystemExit(f"expected one code object in {cache}, found {objs}")
    return objs[0]


def mix(code_object, kernel, costs):
    dis = subprocess.run([OBJDUMP, "-d", code_object], check=True, capture_output=True,
                         text=True).stdout
    insts = parse(dis, kernel)
    lo, hi = event_loop(insts)
    per = collections.defaultdict(lambda: {"n": 0, "passes": 0, "time": 0.0})
    unpriced = collections.Counter()
    for a, op, _ in insts:
        if lo <= a <= hi and op.startswith("v_"):
            cls, p, w, priced = classify(op, costs)
            per[cls]["n"] += 1
            per[cls]["passes"] += p
            per[cls]["time"] += w
            if not priced:
                unpriced[op] += 1
    n = sum(v["n"] for v in per.values())
    passes = sum(v["passes"] for v in per.values())
    time = sum(v["time"] for v in per.values())
    return {"kernel": kernel, "loop": [hex(lo), hex(hi)], "valu_instructions": n,
            "passes": passes, "time_slots": round(time, 3),
            "time_per_pass": round(time / passes, 4),
            "per_class": {k: {"n": v["n"], "passes": v["passes"], "time": round(v["time"], 3)}
                          for k, v in sorted(per.items())},
            "unpriced": dict(unpriced)}


MICRO_OPS = ["v_mad_u64_u32", "v_mul_hi_u32", "v_mul_lo_u32", "v_fma_f64", "v_add_f64",
             "v_mul_f64", "v_rcp_f64", "f64 divide", "f32 divide", "v_bitop3_b32", "v_add_u32",
             "v_cvt_f64_u32", "cmp+select f64", "v_fma_f32", "v_cvt_f32_i32", "v_rcp_f32",
             "v_frexp_mant_f32", "v_cvt_f64_f32", "v_cndmask_b32", "v_mov_b32", "v_mov_b64",
             "v_cmp_gt_f64", "v_cmp_gt_u32", "v_xor_b32", "v_lshrrev_b32", "v_alignbit_b32",
             "v_div_scale_f64"]
CLASSES = ("INT32", "INT64", "CVT", "FMA_F32", "ADD_F32", "MUL_F32", "TRANS_F32", "FMA_F64",
           "ADD_F64", "MUL_F64", "TRANS_F64")


def calibration(costs_file, type_dirs, commands, out):
    """Summary of the microbenchmark under the VALU counters: per instruction,
    its issue time and what the counters credit it with."""
    import csv
    import glob
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for d in type_dirs:
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        for r in csv.DictReader(open(path)):
            per[int(r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
            names[int(r["Dispatch_Id"])] = r["Kernel_Name"]
    # the throughput kernels k_cost<op, 8> of the two passes, by op
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    for dsp, c in per.items():
        m = re.search(r"k_cost<\(?(-?\d+)\)?, 8>", names[dsp])
        if m and int(m.group(1)) >= 0:
            for k, v in c.items():
                acc[int(m.group(1))][k] += v
    lines = ["# VALU issue cost and VALU counters on gfx950 (microbench/isa_cost.hip)", "",
             "Each instruction class runs in its own kernel: 1,024 threads on one compute unit "
             "(four wavefronts per SIMD), 4,112 iterations of eight independent chains.  "
             "`slots` = throughput cycles per wave64 instruction per SIMD / 4 (the microbenchmark's"
             " clock).  From two rocprofv3 --pmc passes over the same program: the counter class "
             "SQ_INSTS_VALU_<class> files the instruction under (\"other\": none of them), and "
             "SQ_THREAD_CYCLES_VALU / (64 x SQ_INSTS_VALU), the issue passes the counter credits "
             "one instruction with.", "", "Commands (`R` = the repository root on one MI355X):", "",
             "```"] + open(commands).read().strip().splitlines() + ["```", "",
             "The divide and cmp+select rows are sequences: slots per sequence, passes per "
             "instruction of it.", "",
             "| instruction | slots (time) | counter class | passes credited |",
             "|---|---|---|---|"]
    costs = read_costs(costs_file)
    for i, name in enumerate(MICRO_OPS):
        c = acc.get(i)
        if not c or name not in costs:
            continue
        tot = c["SQ_INSTS_VALU"] / 2.0  # counted in both passes
        shares = {t: c.get("SQ_INSTS_VALU_" + t, 0.0) / tot for t in CLASSES}
        shares["other"] = 1.0 - sum(shares.values())
        cls = ", ".join(f"{t} {v:.2f}" if v < 0.99 else t
                        for t, v in sorted(shares.items(), key=lambda kv: -kv[1]) if v > 0.05)
        passes = c["SQ_THREAD_CYCLES_VALU"] / (64.0 * tot)
        lines.append(f"| {name} | {costs[name]:.2f} | {cls} | {passes:.2f} |")
    lines += ["", "The counter credits a plain 32-bit operation (0.6 slots of issue time) with "
                  "the same pass as a binary64 fma (1.08): a count of passes is a count of issue "
                  "time only for a mix without the fast 32-bit operations.", ""]
    open(out, "w").write("\n".join(lines))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "calibration":
        ap = argparse.ArgumentParser()
        ap.add_argument("mode")
        ap.add_argument("--costs", required=True)
        ap.add_argument("--types", nargs=2, required=True)
        ap.add_argument("--commands", required=True)
        ap.add_argument("--out", required=True)
        a = ap.parse_args()
        calibration(a.costs, a.types, a.commands, a.out)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True, choices=["telegraph", "random", "lacgfp"])
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--kernel", default="lik_flow_spec")
    ap.add_argument("--costs", required=True, help="output of microbench/isa_cost.hip")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    cache = tempfile.mkdtemp(prefix="lik-mix-")
    try:
        res = mix(compile_kernel(a.workload, a.precision, cache), a.kernel, read_costs(a.costs))
    finally:
        shutil.rmtree(cache, ignore_errors=True)
    res.update({"workload": a.workload, "precision": a.precision})
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({k: res[k] for k in ("loop", "valu_instructions", "passes", "time_slots",
                                           "time_per_pass", "unpriced")}), file=sys.stderr)


if __name__ == "__main__":
    main()
