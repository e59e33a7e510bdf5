"""lik_eval_batch_device_noalloc (the entry point for callers that cannot
allocate device memory) against lik_eval_batch_device on the same inputs:
bit-identical results on two calls in a row, the second with a smaller
batch (the static scratch keeps the first call's contents), in both kernel
variants; batches beyond its scratch and graph mode are rejected on the
host."""
import numpy as np
import pytest

from paper_1606_08281_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _pair(lik, torch, wl, n_theta, precision, kernel, seed, schedule):
    net = lik.Network(wl.net.orders, wl.net.stoich)
    net.set_tuning(schedule=schedule)
    theta = torch.from_numpy(np.ascontiguousarray(wl.theta[:n_theta])).cuda()
    db = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories, n_theta,
                         wl.n_particles, precision=precision, kernel=kernel)
    F = n_theta * len(wl.trajectories)
    fs = torch.empty((F, wl.net.U, wl.n_particles), dtype=torch.int32, device="cuda")
    ll, st = db.run(theta, seed, final_state=fs)
    ref = {"ll": ll.clone(), "st": st.clone(), "ev": db.events.clone(),
           "fll": db.filter_loglik.clone(), "fs": fs.clone()}
    fs.fill_(-7)
    db.loglik.fill_(0.0)
    db.events.fill_(0)
    ll, st = db.run_noalloc(theta, seed, final_state=fs)
    torch.cuda.synchronize()
    assert torch.equal(ll, ref["ll"]) and torch.equal(st, ref["st"])
    assert torch.equal(db.events, ref["ev"]) and torch.equal(db.filter_loglik, ref["fll"])
    assert torch.equal(fs, ref["fs"])
    assert bool(torch.all(st == 0))
    return net


@pytest.mark.parametrize("kernel", [1, 2])   # generic, network-specialised
def test_no_alloc_entry_point_matches_device_entry_point(kernel):
    import torch
    from paper_1606_08281_amd import lik
    big = W.telegraph_workload(n_theta=96, n_traj=2, n_obs=20, n_particles=1000)
    small = W.immigration_death_workload(n_theta=24, n_particles=200)
    _say("no-alloc: telegraph 96x2x1000x20, flow schedule, kernel", kernel)
    _pair(lik, torch, big, 96, 0, kernel, 5, 1)
    _say("no-alloc: immigration-death 24x1x200x20 (second, smaller call), per-interval, kernel",
         kernel)
    _pair(lik, torch, small, 24, 1, kernel, 6, 0)


def test_no_alloc_entry_point_rejects_what_needs_allocation():
    import torch
    from paper_1606_08281_amd import lik
    wl = W.telegraph_workload(n_theta=256, n_traj=10, n_obs=5, n_particles=1000)
    net = lik.Network(wl.net.orders, wl.net.stoich)
    db = lik.DeviceBatch(net, wl.obs_kind, wl.observed, wl.sigma, wl.trajectories, wl.n_theta,
                         wl.n_particles)
    assert db.ws_bytes > (64 << 20)
    theta = torch.from_numpy(wl.theta).cuda()
    _say("no-alloc: batch above the scratch size is rejected")
    with pytest.raises(lik.LikError):
        db.run_noalloc(theta, 1)
    small = W.immigration_death_workload(n_theta=4, n_particles=64)
    snet = lik.Network(small.net.orders, small.net.stoich)
    g = lik.DeviceBatch(snet, small.obs_kind, small.observed, small.sigma, small.trajectories, 4,
                        64, graph=True)
    with pytest.raises(lik.LikError):
        g.run_noalloc(torch.from_numpy(small.theta).cuda(), 1)
