"""Host logic of bench.py that needs no GPU: the per-step summary and the
reading of rocm-smi's clocks and power."""
import json
import shutil
import subprocess
import sys
import types

import bench


class _FakeEvent:
    """Stands in for torch.cuda.Event: record() stores a time taken from a
    list, elapsed_time() subtracts (milliseconds)."""
    times = []

    def __init__(self, enable_timing=True):
        self.t = None

    def record(self, stream):
        self.t = _FakeEvent.times.pop(0)

    def elapsed_time(self, end):
        return end.t - self.t


def test_step_clock_summary():
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(Event=_FakeEvent))
    _FakeEvent.times = [0.0, 10.0, 21.0, 30.0, 42.0]
    mark, summary = bench.step_clock(fake_torch, 4, stream=None)
    for _ in range(5):
        mark()
    s = summary()
    assert s["each"] == [10.0, 11.0, 9.0, 12.0]
    assert (s["median"], s["min"], s["max"]) == (10.5, 9.0, 12.0)
    assert abs(s["spread"] - 3.0 / 10.5) < 1e-12


def test_device_state_keeps_clocks_and_power(monkeypatch):
    report = {"card0": {"sclk clock speed:": "(2400Mhz)", "mclk clock speed:": "(1900Mhz)",
                        "Current Socket Graphics Package Power (W)": "812.0",
                        "Max Graphics Package Power (W)": "1400.0", "Card series": "x"}}
    out = "WARNING: something\n" + json.dumps(report)

    def fake_run(cmd, **kw):
        # the script under this interpreter: no `env` launcher in between
        assert cmd[0] == sys.executable and cmd[1].endswith("rocm_smi.py") and "--json" in cmd
        return types.SimpleNamespace(stdout=out, returncode=0)

    monkeypatch.setattr(subprocess, "run", fake_run)
    monkeypatch.setattr(shutil, "which", lambda name: "/opt/rocm/libexec/rocm_smi/rocm_smi.py")
    monkeypatch.delenv("LD_PRELOAD", raising=False)
    got = bench.device_state()["rocm_smi"]
    assert set(got) == {"sclk clock speed:", "mclk clock speed:",
                        "Current Socket Graphics Package Power (W)",
                        "Max Graphics Package Power (W)"}


def test_device_state_without_the_tool(monkeypatch):
    monkeypatch.setattr(shutil, "which", lambda name: None)
    monkeypatch.delenv("LD_PRELOAD", raising=False)
    got = bench.device_state()
    assert got["rocm_smi"] is None and "rocm-smi" in got["error"]


def test_device_state_not_read_under_a_profiler(monkeypatch):
    def never(cmd, **kw):
        raise AssertionError("no child process under a profiler")

    monkeypatch.setattr(subprocess, "run", never)
    monkeypatch.setenv("LD_PRELOAD", "/opt/rocm/lib/rocprofiler-sdk/librocprofiler-sdk-tool.so")
    assert bench.device_state()["rocm_smi"] is None
