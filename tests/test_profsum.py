"""Host logic of the profile summaries: the kernel-source fingerprint that
decides whether bench.py may quote a stored HBM-traffic figure (a figure is
quoted only while the kernel code it was measured on is unchanged)."""
import os

from paper_1606_08281_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fingerprint_ignores_comments_and_layout():
    a = "int f(int x) {\n    return x + 1;  // one\n}\n"
    b = "/* what f does */ int f(int x)\n{ return x + 1; }   // another note\n\n"
    assert profsum._code_only(a) == profsum._code_only(b)


def test_fingerprint_follows_code():
    assert profsum._code_only("return x + 1;") != profsum._code_only("return x + 2;")
    assert profsum._code_only("a = b; // c") != profsum._code_only("a = b; c")


def test_comment_markers_inside_literals_are_code():
    s = 'const char *p = "a // b /* c */"; char q = \'/\'; int d = 1; /* gone */ int e;'
    out = profsum._code_only(s)
    assert '"a // b /* c */"' in out
    assert "char q = '/';" in out
    assert "int d = 1; int e;" in out
    assert "gone" not in out
    # an escaped quote does not end the literal
    assert profsum._code_only(r'x = "q\" // kept"; // dropped') == r'x = "q\" // kept";'


def test_source_fingerprint_covers_every_kernel_source():
    assert len(profsum.source_sha256()) == 64
    for rel in profsum.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, rel)), rel
    for name in ("propagate.hpp", "flow.hpp", "weigh.hpp", "devmath.hpp", "kernels.hip"):
        assert any(r.endswith(name) for r in profsum.KERNEL_SOURCES), name


def test_traffic_record_is_read_only_for_matching_sources(tmp_path):
    body = ("# HBM traffic per launch\nsource_sha256: {}\nfetch_scale: 2.0\n"
            "hbm_bytes_per_launch: 1.5e+09\n")
    good = tmp_path / "good.txt"
    good.write_text(body.format(profsum.source_sha256()))
    rec = profsum.read_traffic(str(good))
    assert rec is not None and float(rec["hbm_bytes_per_launch"]) == 1.5e9
    stale = tmp_path / "stale.txt"
    stale.write_text(body.format("0" * 64))
    assert profsum.read_traffic(str(stale)) is None
    assert profsum.read_traffic(str(tmp_path / "absent.txt")) is None


def test_committed_traffic_records_are_well_formed():
    names = [n for n in os.listdir(os.path.join(ROOT, "profiles")) if "_traffic_" in n]
    assert names
    for n in names:
        rec = {}
        for line in open(os.path.join(ROOT, "profiles", n)):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
        assert len(rec["source_sha256"]) == 64, n
        total = float(rec["hbm_bytes_per_launch"])
        assert abs(total - float(rec["fetch_bytes_per_launch"])
                   - float(rec["write_bytes_per_launch"])) <= 1e-4 * total, n


def test_valu_work_per_event_from_counters(tmp_path):
    # SQ_THREAD_CYCLES_VALU / events of the launch is the measured lane-op
    # issue slots per event; a record is read only for matching sources
    d = tmp_path / "pmc"
    d.mkdir()
    rows = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value",
            "1,lik_flow_spec.kd,SQ_THREAD_CYCLES_VALU,6400",
            "1,lik_flow_spec.kd,SQ_ACTIVE_INST_VALU,125",
            "1,lik_flow_spec.kd,SQ_INSTS_VALU,120",
            "1,lik_flow_spec.kd,GRBM_GUI_ACTIVE,999",
            "2,lik::k_admit(),SQ_THREAD_CYCLES_VALU,5"]
    (d / "x_counter_collection.csv").write_text("\n".join(rows) + "\n")
    bench = {"events_per_step": 40, "steps": 1, "roofline": {"launches": 1}}
    vw = profsum.valu_work(str(d), bench, "lik_flow_spec")
    assert vw["lane_slots_per_event"] == 160.0
    assert vw["wave_insts_per_event"] == 3.0
    assert vw["lane_utilisation"] == 6400 / (125 * 64)
    rec = tmp_path / "valu.txt"
    rec.write_text(f"source_sha256: {profsum.source_sha256()}\nlane_slots_per_event: 160\n")
    assert float(profsum.read_record(str(rec))["lane_slots_per_event"]) == 160.0
