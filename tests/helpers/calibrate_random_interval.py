"""Observation interval of the 20-species, 40-reaction benchmark network at
which the median rate vector of its prior realises 1e4 direct-method SSA
events per particle per interval.

A pilot: one exact SSA path (the oracle's direct method, one particle, so no
resampling) per rate vector for 256 of the 4096 prior draws (every 16th),
from the network's x0 over 100 intervals; the interval is rescaled until the
median over the rate vectors of events per interval is within 1 % of 1e4.
Prints the interval and the spread of events per interval.  The result is
the constant workloads.RANDOM_DT_1E4 (an input of the workload, not an
expected value).

  python tests/helpers/calibrate_random_interval.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_1606_08281_amd import workloads as W  # noqa: E402


def realised_events(net, x0, theta, ids, dt, T=100):
    traj = {"t_obs": dt * np.arange(1, T + 1), "y": np.full((T, 2), 100.0), "t0": 0.0,
            "x0": x0}
    P = orc.Problem(net.orders, net.stoich, W.OBS_GAUSSIAN, [0, 1], 10.0, theta, [traj], 1,
                    W.SEED_FILTER, theta_ids=ids, event_cap=10_000_000)
    out = orc.evaluate(P)
    assert np.all(out["status"] == 0)
    return out["events"] / T


def main():
    net = W.random_network()
    x0 = W.random_network_x0(net)
    theta = W.random_network_theta(net, 4096)
    ids = np.arange(0, 4096, 16)
    dt = 1.0
    for _ in range(12):
        per = realised_events(net, x0, theta[ids], ids, dt)
        med = float(np.median(per))
        print(f"dt {dt:.6g}: median {med:.6g}, mean {per.mean():.6g}, "
              f"p99 {np.percentile(per, 99):.6g}, max {per.max():.6g} events per interval",
              flush=True)
        if abs(med / 1e4 - 1.0) < 0.01:
            break
        dt *= (1e4 / med) ** 0.9
    print(f"RANDOM_DT_1E4 = {dt:.6g}")


if __name__ == "__main__":
    main()
