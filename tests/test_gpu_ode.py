"""Deterministic-model likelihood on the GPU against the oracle (Sec.
"Chemical Reaction Networks", deterministic formulation; Results,
deterministic models; Supplementary "Egf-Ras-Raf-Mek-Erk model").

Both sides take the same Dormand-Prince steps under the same step rule, with
every operation in the same order and the same log and exp, so the
log-likelihoods and statuses agree bit for bit."""
import numpy as np
import pytest

from paper_1606_08281_amd import workloads as W
from tests.test_oracle_ode import every_factor_model, imm_death_model

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def both(orc, spec, theta, trajs, **kw):
    """The generic and the model-specialised kernel against the oracle: both
    must give the same results; returns the specialised one's."""
    from paper_1606_08281_amd import lik
    model = lik.OdeModel(spec)
    ref = orc.ode_eval(orc.OdeProblem(spec, theta, trajs, **kw))
    outs = []
    for kernel in (lik.KERNEL_GENERIC, lik.KERNEL_SPECIALIZED):
        ll, st, steps = lik.ode_eval(model, theta, trajs, steps=True, kernel=kernel, **kw)
        # the same step sequence: equal step counts per trajectory
        assert np.array_equal(steps.ravel(), ref["traj_steps"]), kernel
        outs.append((ll, st))
    assert np.array_equal(outs[0][0], outs[1][0], equal_nan=True)
    assert np.array_equal(outs[0][1], outs[1][1])
    return outs[1][0], outs[1][1], ref


def assert_same(ll, st, ref):
    assert np.array_equal(st, ref["status"]), (st, ref["status"])
    bad = ~np.isfinite(ref["loglik"])
    assert np.array_equal(np.isnan(ll), np.isnan(ref["loglik"]))
    diff = np.abs(ll[~bad] - ref["loglik"][~bad])
    assert np.all(ll[~bad] == ref["loglik"][~bad]), diff.max()


def test_small_models_bit_exact(orc):
    rng = np.random.default_rng(3)
    _say("immigration-death rate equations, 200 theta, 3 trajectories")
    t = np.linspace(0.5, 12.0, 24)
    trajs = [{"t_obs": t + 0.1 * m, "y": rng.normal(10, 3, len(t)), "x0": [m * 2.0]} for m in range(3)]
    theta = np.exp(rng.normal(0.0, 1.0, (200, 2)))
    assert_same(*both(orc, imm_death_model(), theta, trajs, rtol=1e-7, atol=1e-10))
    _say("every factor kind, inputs, FRET read-out, 300 theta")
    tin, uin = np.array([0.0, 3.0, 5.0]), np.array([1.0, 0.2, 2.0])
    t = np.linspace(0.4, 8.0, 20)
    trajs = [{"t_obs": t, "y": rng.normal(1.0, 0.05, len(t)), "x0": [0, 0, 0.4, 0.1],
              "t_in": tin, "u_in": uin},
             {"t_obs": t[::2], "y": rng.normal(1.0, 0.05, 10), "x0": [0, 0.1, 0.2, 0.0]}]
    base = np.array([1.3, 0.8, 0.4, 2.0, 0.3, 0.7, 1.1, 0.5, 0.2, 2.5])
    theta = base * np.exp(rng.normal(0.0, 0.7, (300, 10)))
    for rtol in (1e-4, 1e-8):
        assert_same(*both(orc, every_factor_model(), theta, trajs, rtol=rtol, atol=rtol * 1e-3))


def test_erk_batch_bit_exact(orc):
    wl = W.erk_workload(n_theta=512, spread=0.5)
    _say("ERK model, 512 theta x 6 input patterns x 60 FRET observations")
    ll, st, ref = both(orc, wl["spec"], wl["theta"], wl["trajectories"], rtol=1e-6, atol=1e-9)
    assert np.mean(st == 0) > 0.9
    assert_same(ll, st, ref)


def test_statuses_agree(orc):
    wl = W.erk_workload(n_theta=64, spread=1.5)
    th = wl["theta"].copy()
    th[1, 3] = -1.0           # a negative Hill constant
    th[2, 0] = np.nan
    th[3, 32] = 0.0           # zero noise sd
    _say("ERK statuses: bad parameters and a step limit")
    ll, st, ref = both(orc, wl["spec"], th, wl["trajectories"], rtol=1e-6, atol=1e-9,
                       max_steps=400)
    assert list(st[1:4]) == [3, 3, 3]
    assert np.any(st == 7)
    assert_same(ll, st, ref)


def test_erk_bench_batch_sampled(orc):
    """The bench's ERK batch at full size (65,536 theta x 6 input patterns) on
    the GPU; 256 theta of it recomputed by the oracle, step counts included."""
    from paper_1606_08281_amd import lik
    wl = W.erk_workload(n_theta=65536, spread=0.3)
    _say("ERK bench batch 65536 x 6 on the GPU")
    ll, st, steps = lik.ode_eval(lik.OdeModel(wl["spec"]), wl["theta"], wl["trajectories"],
                                 steps=True)
    pick = np.random.default_rng(9).choice(65536, 256, replace=False)
    ref = orc.ode_eval(orc.OdeProblem(wl["spec"], wl["theta"][pick], wl["trajectories"]))
    assert np.array_equal(st[pick], ref["status"])
    assert np.array_equal(ll[pick], ref["loglik"])
    assert np.array_equal(steps[pick].ravel(), ref["traj_steps"])


@pytest.mark.parametrize("n_theta", [1, 7, 13, 300])
def test_pair_queue_order_and_ragged_sizes(orc, n_theta):
    """Lanes take (theta, trajectory) pairs from a shared counter, the
    trajectories with the most stops first: trajectories whose stop counts
    rise with their index (so the order is reversed), one with input
    breakpoints, and pair counts that leave the last wavefront part-full or
    take one lane; every result lands at its own (theta, trajectory)."""
    rng = np.random.default_rng(31 + n_theta)
    trajs = []
    for m in range(5):
        t = np.linspace(0.3, 10.0, 4 + 5 * m)
        tr = {"t_obs": t, "y": rng.normal(20, 4, len(t)), "x0": [1.0 + m]}
        if m == 3:
            tr.update(t_in=np.array([0.0, 2.0, 6.5]), u_in=np.array([1.0, 0.0, 2.0]))
        trajs.append(tr)
    spec = dict(imm_death_model(), terms=[{"to": 0, "rate_param": 0, "factors": [(4, 0, 0)]},
                                          {"frm": 0, "rate_param": 1, "factors": [(0, 0, 0)]}])
    theta = np.exp(rng.normal(0.0, 1.0, (n_theta, 2))) * np.array([8.0, 0.5])
    _say("pair queue: immigration-death with input, 5 trajectories,", n_theta, "theta")
    assert_same(*both(orc, spec, theta, trajs, rtol=1e-7, atol=1e-10))


def test_device_entry_point_equals_host_entry_point(orc):
    """lik_ode_eval_device on resident buffers (torch tensors, the current
    stream, one workspace reused by consecutive calls) gives lik_ode_eval's
    results bit for bit, with and without inputs, for both kernels; the
    oracle agrees."""
    import torch
    from paper_1606_08281_amd import lik
    wl = W.erk_workload(n_theta=200, spread=0.5)
    model = lik.OdeModel(wl["spec"])
    for kernel in (lik.KERNEL_GENERIC, lik.KERNEL_SPECIALIZED):
        db = lik.OdeDeviceBatch(model, wl["trajectories"], 200, steps=True, kernel=kernel)
        for rep in range(2):
            theta = wl["theta"] * (1.0 + 0.1 * rep)
            _say("ODE device entry point, kernel", kernel, "call", rep)
            ll_d, st_d = db.run(torch.from_numpy(np.ascontiguousarray(theta)).cuda())
            torch.cuda.synchronize()
            ll, st, steps = lik.ode_eval(model, theta, wl["trajectories"], steps=True,
                                         kernel=kernel)
            assert np.array_equal(ll_d.cpu().numpy(), ll, equal_nan=True)
            assert np.array_equal(st_d.cpu().numpy(), st)
            assert np.array_equal(db.steps[:200 * 6].cpu().numpy().reshape(200, 6), steps)
    ref = orc.ode_eval(orc.OdeProblem(wl["spec"], theta[:16], wl["trajectories"]))
    assert np.array_equal(ll[:16], ref["loglik"], equal_nan=True)
    _say("ODE device entry point without inputs")
    t = np.linspace(0.5, 12.0, 24)
    trajs = [{"t_obs": t, "y": np.full(24, 10.0), "x0": [1.0]}, {"t_obs": t[:5], "y": np.ones(5),
                                                               "x0": [3.0]}]
    m2 = lik.OdeModel(imm_death_model())
    th2 = np.exp(np.random.default_rng(4).normal(0.0, 1.0, (70, 2)))
    db2 = lik.OdeDeviceBatch(m2, trajs, 70)
    ll_d, st_d = db2.run(torch.from_numpy(th2).cuda())
    ll, st = lik.ode_eval(m2, th2, trajs)
    assert np.array_equal(ll_d.cpu().numpy(), ll) and np.array_equal(st_d.cpu().numpy(), st)
