"""Host logic of the profile tools: the instruction classes and issue costs
isamix gives, its choice of the event loop, profsum's pricing of issue passes
and its refusal of counter folders that hold other launches of the kernel."""
import csv
import os

import pytest

from paper_1606_08281_amd import isamix, profsum

COSTS = {"v_mad_u64_u32": 1.14, "v_mul_lo_u32": 1.09, "v_fma_f64": 1.08, "v_rcp_f64": 4.07,
         "v_bitop3_b32": 0.64, "v_add_u32": 0.63, "v_cvt_f64_u32": 1.11, "v_fma_f32": 0.65,
         "v_rcp_f32": 2.06, "v_frexp_mant_f32": 1.05, "v_cndmask_b32": 1.08, "v_mov_b32": 0.61,
         "v_mov_b64": 1.07, "v_cmp_gt_f64": 1.22, "v_cmp_gt_u32": 1.21, "v_xor_b32": 0.63,
         "v_lshrrev_b32": 0.59, "v_alignbit_b32": 1.09, "v_div_scale_f64": 1.22}


@pytest.mark.parametrize("op,cls,passes,cost", [
    ("v_fma_f64", "FMA_F64", 1, 1.08),
    ("v_fmac_f64_e32", "FMA_F64", 1, 1.08),
    ("v_add_f64", "ADD_F64", 1, 1.08),
    ("v_mul_f32_e32", "MUL_F32", 1, 0.65),
    ("v_fmamk_f32", "FMA_F32", 1, 0.65),
    ("v_rcp_f64_e32", "TRANS_F64", 4, 4.07),
    ("v_rcp_iflag_f32_e32", "TRANS_F32", 2, 2.06),
    ("v_mad_u64_u32", "INT64", 1, 1.14),
    ("v_mul_lo_u32", "INT32", 1, 1.09),
    ("v_cmp_gt_u32_e32", "INT32", 1, 1.21),
    ("v_cmp_ne_u16_sdwa", "INT32", 1, 1.21),
    ("v_cmp_ngt_f64_e32", "other", 1, 1.22),
    ("v_add_u32_e32", "INT32", 1, 0.63),
    ("v_add_u32_sdwa", "INT32", 1, 1.09),
    ("v_cvt_f64_i32_e32", "CVT", 1, 1.11),
    ("v_bitop3_b32", "other", 1, 0.64),
    ("v_xor_b32_e32", "other", 1, 0.63),
    ("v_lshrrev_b32_e32", "other", 1, 0.59),
    ("v_mov_b32_e32", "other", 1, 0.61),
    ("v_mov_b64_e32", "other", 1, 1.07),
    ("v_cndmask_b32_e32", "other", 1, 1.08),
    ("v_div_scale_f64", "other", 1, 1.22),
    ("v_div_fmas_f64", "FMA_F64", 1, 1.22),
    ("v_frexp_exp_i32_f64_e32", "other", 1, 1.05),
    ("v_subbrev_co_u32_e32", "INT32", 1, 1.09),
])
def test_classify(op, cls, passes, cost):
    c, p, w, priced = isamix.classify(op, COSTS)
    assert (c, p, priced) == (cls, passes, True)
    assert w == pytest.approx(cost)


def test_unknown_instruction_is_listed_at_one_slot():
    assert isamix.classify("v_some_future_op_b32", COSTS) == ("other", 1, 1.0, False)


def _line(addr, text, target=None):
    t = f" <k+0x{target:x}>" if target is not None else ""
    return f"\t{text}{t} // {addr + 0x1000:012X}: 00000000"


def _dis(blocks):
    """A disassembly of kernel k: blocks of (instructions, back-edge target
    index or None)."""
    lines, addr = ["0000000000001000 <k>:"], 0
    for insts, back in blocks:
        start = addr
        for op in insts:
            lines.append(_line(addr, op))
            addr += 4
        if back is not None:
            lines.append(_line(addr, "s_cbranch_scc1 1", start))
            addr += 4
    return "\n".join(lines)


def test_event_loop_is_the_drawing_loop_with_a_log():
    philox = ["v_mad_u64_u32 v[0:1], s[0:1], v2, s3, 0"] * 20 + ["v_bitop3_b32 v1, v2, v3, s4"]
    log = ["v_frexp_mant_f64_e32 v[4:5], v[6:7]", "v_fma_f64 v[4:5], v[4:5], v[6:7], v[8:9]"]
    scan = philox + ["ds_bpermute_b32 v1, v2, v3"] + ["v_add_u32_e32 v1, v2, v3"] * 80
    dis = _dis([(["s_mov_b32 s0, 0"], None),
                (philox + log + ["v_add_f64 v[0:1], v[2:3], v[4:5]"] * 10, True),   # event loop
                (["v_mov_b32_e32 v0, 0"], None),
                (philox, True),                   # draws without a log: not the event loop
                (scan, True)])                    # a scan: not the event loop
    insts = isamix.parse(dis, "k")
    lo, hi = isamix.event_loop(insts)
    body = [op for a, op, _ in insts if lo <= a <= hi]
    assert body.count("v_mad_u64_u32") == 20 and "v_frexp_mant_f64_e32" in body
    assert "ds_bpermute_b32" not in body and body.count("v_add_f64") == 10


def _write_pmc(folder, rows):
    os.makedirs(folder, exist_ok=True)
    with open(os.path.join(folder, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_issue_time_prices_passes_by_class(tmp_path):
    # one dispatch: 100 INT32, 50 FMA_F64, 10 TRANS_F64 and 40 other instructions
    a, b = str(tmp_path / "a"), str(tmp_path / "b")
    _write_pmc(a, [(1, "lik_flow_spec", "SQ_INSTS_VALU", 200),
                   (1, "lik_flow_spec", "SQ_INSTS_VALU_INT32", 100),
                   (1, "lik_flow_spec", "SQ_INSTS_VALU_FMA_F64", 50),
                   (1, "lik_flow_spec", "SQ_INSTS_VALU_TRANS_F64", 10)])
    _write_pmc(b, [(1, "lik_flow_spec", "SQ_INSTS_VALU", 200),
                   (1, "lik_flow_spec", "SQ_INSTS_VALU_ADD_F64", 0)])
    mix = {"per_class": {"INT32": {"n": 4, "passes": 4, "time": 3.0},
                         "FMA_F64": {"n": 2, "passes": 2, "time": 2.2},
                         "TRANS_F64": {"n": 1, "passes": 4, "time": 4.0},
                         "other": {"n": 5, "passes": 5, "time": 4.0}}}
    it = profsum.issue_time([a, b], "lik_flow_spec", mix, events=10.0)
    time = 100 * 0.75 + 50 * 1.1 + 10 * 4.0 + 40 * 0.8
    passes = 100 + 50 + 10 * 4 + 40
    assert it["time_per_pass"] == pytest.approx(time / passes)
    assert it["passes_per_event"] == pytest.approx(passes / 10.0)
    assert it["insts_per_event"] == pytest.approx(20.0)


def test_counter_folder_with_other_launches_is_refused(tmp_path):
    d = str(tmp_path / "p")
    _write_pmc(d, [(1, "lik_flow_spec", "SQ_INSTS_VALU", 5),
                   (2, "lik_flow_spec", "SQ_INSTS_VALU", 7),
                   (3, "__amd_rocclr_copyBuffer", "SQ_INSTS_VALU", 1)])
    assert profsum.dispatches(d, "lik_flow_spec") == 2
    profsum.check_dispatches(d, "lik_flow_spec", 2)
    with pytest.raises(SystemExit):
        profsum.check_dispatches(d, "lik_flow_spec", 1)
