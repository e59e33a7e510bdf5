"""Pins of the oracle's random streams and elementary functions.

* Philox4x32-10 against rocRAND's independent implementation of the same
  generator (Salmon et al., SC'11), run on the host.
* log, exp (binary64) and log (binary32) against mpmath at 60 digits: at most
  2 units in the last place everywhere they are used, exact at the special
  points (log 1 = 0, exp 0 = 1).
"""
import math
import os
import shutil
import subprocess
import tempfile

import mpmath
import numpy as np
import pytest

mpmath.mp.dps = 60
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "philox_ref")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp")],
                   check=True, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(11)
    cases = [[0, 0, 0, 0, 0, 0], [1, 2, 3, 4, 5, 6],
             [0xFFFFFFFF] * 6, [7, 0, (3 << 16) | 9, (5 << 2) | 1, 5, 0]]
    cases += rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64).tolist()
    inp = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        got = orc.philox(c[:4], c[4:]).tolist()
        assert got == r, (c, got, r)


def ulp(x):
    return math.ulp(x) if x != 0 else 5e-324


def _log_err_ulps(orc, x):
    got = orc.log(x)
    exact = mpmath.log(mpmath.mpf(x))
    return float(abs(mpmath.mpf(got) - exact) / ulp(float(exact)))


def test_log_special_points(orc):
    assert orc.log(1.0) == 0.0
    assert orc.log(0.0) == -math.inf
    assert math.isnan(orc.log(-1.0))


def test_log_accuracy_event_uniforms(orc):
    # the event-time argument: u1 = (z + 1) 2^-53, z a 53-bit integer
    rng = np.random.default_rng(1)
    z = rng.integers(0, 2**53, size=3000, dtype=np.int64)
    xs = [(int(v) + 1) * 2.0**-53 for v in z] + [2.0**-53, 1.0 - 2.0**-53, 0.5, 0.75]
    worst = max(_log_err_ulps(orc, x) for x in xs if x != 1.0)
    assert worst <= 2.0, worst


def test_log_accuracy_counts_and_wide_range(orc):
    rng = np.random.default_rng(2)
    xs = [float(v) for v in rng.integers(1, 2**31, size=1500)] + [1.0, 2.0, 3.0, 4.0]
    # log-uniform over the whole binary64 range, subnormals included
    e = rng.uniform(-1074, 1023, size=1500)
    xs += [float(2.0**v) for v in e if 2.0**v > 0]
    xs += [5e-324, 2.2250738585072014e-308, 1.7976931348623157e308, math.sqrt(2.0), math.sqrt(0.5)]
    worst = max(_log_err_ulps(orc, x) for x in xs if x != 1.0)
    assert worst <= 2.0, worst


def test_exp_accuracy(orc):
    rng = np.random.default_rng(3)
    ds = list(-rng.uniform(0, 708, size=3000)) + list(-rng.uniform(0, 1, size=1000))
    ds += [-1e-300, -1e-10, -0.34657359, -0.34657360, -707.99]
    worst = 0.0
    for d in ds:
        got = orc.exp(d)
        exact = mpmath.exp(mpmath.mpf(d))
        worst = max(worst, float(abs(mpmath.mpf(got) - exact) / ulp(float(exact))))
    assert worst <= 2.0, worst
    assert orc.exp(0.0) == 1.0
    assert orc.exp(-math.inf) == 0.0
    assert orc.exp(-708.5) == 0.0


def test_logf_accuracy(orc):
    rng = np.random.default_rng(4)
    z = rng.integers(0, 2**24, size=4000)
    worst = 0.0
    for v in list(z) + [0, 2**24 - 1, 2**23]:
        x = float(np.float32((int(v) + 1) * 2.0**-24))
        if x == 1.0:
            assert orc.logf(x) == 0.0
            continue
        got = orc.logf(x)
        exact = mpmath.log(mpmath.mpf(x))
        u = float(np.spacing(np.float32(abs(float(exact)))))
        worst = max(worst, float(abs(mpmath.mpf(got) - exact)) / u)
    assert worst <= 2.0, worst
