"""The level-set sampler driving the server on the GPU: every served result
equals the same request evaluated alone, and the sampler's levels rise."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_sampler_stream_served_equals_alone():
    from paper_1606_08281_amd import serve_lns
    print("[case] sampler closed loop: N 40, 2 levels, H 128 and 512, batches of 16", flush=True)
    rep, recs, nets = serve_lns.closed_loop(H_list=(128, 512), N=40, levels=2, batch=16,
                                            inflight=3, check=16)
    assert rep["requests"] >= 16
    assert rep["served_equals_alone"] and rep["checked_alone"] == 16
    for run in rep["samplers"]:
        assert run["levels"] == 2 and run["eps"][1] > run["eps"][0]
    assert all(r["result"] is not None and r["t_done"] >= r["t_submit"] for r in recs)
    assert {r["tag"] for r in recs} == {"telegraph-H128", "telegraph-H512", "random-20x40"}
    assert rep["server_stats"]["completed"] == len(recs)
    print("[case] replay of the emitted stream: 60 requests, load 0.5", flush=True)
    out = serve_lns.replay(recs, nets, 60, loads=(0.5,))
    assert out["requests"] == 60 and out["saturated"]["evals_per_s"] > 0
    assert out["at_load"][0]["p99_ms"] >= out["at_load"][0]["p50_ms"] > 0
