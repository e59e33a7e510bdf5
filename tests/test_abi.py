"""C ABI checks that need no GPU: the library loads, exports every function
include/lik.h declares, and rejects invalid networks and arguments on the
host before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1606_08281_amd import lik
from paper_1606_08281_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lik.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*(lik_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_function():
    L = lik.lib()
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lik.EXPORTED)
    assert lik.lib().lik_version().startswith(b"lik")


def test_compiled_for_gfx950_only():
    # the device code in the library is built for gfx950
    data = open(lik.LIB_PATH, "rb").read()
    assert b"gfx950" in data


@pytest.mark.parametrize("orders,stoich,code", [
    ([[3]], [[-1]], lik.LIK_EINVAL),          # order 3
    ([[1, 1]], [[-1, -2]], lik.LIK_EINVAL),   # consumes more than it uses
    ([[-1]], [[1]], lik.LIK_EINVAL),          # negative order
    ([[0]], [[9]], lik.LIK_EUNSUPPORTED),     # |net change| > 7
    ([[2, 0]], [[-2, 1]], lik.LIK_OK),        # dimerisation
    ([[1, 1]], [[-1, -1]], lik.LIK_OK),       # hetero second order
])
def test_network_validation(orders, stoich, code):
    if code == lik.LIK_OK:
        net = lik.Network(orders, stoich)
        assert net.U == len(orders[0])
    else:
        with pytest.raises(lik.LikError) as e:
            lik.Network(orders, stoich)
        assert e.value.code == code


def test_network_size_limits():
    with pytest.raises(lik.LikError):
        lik.Network(np.zeros((65, 1)), np.zeros((65, 1)))
    with pytest.raises(lik.LikError):
        lik.Network(np.zeros((1, 33)), np.zeros((1, 33)))
    lik.Network(np.zeros((64, 32)), np.zeros((64, 32)))


def _args(**kw):
    from paper_1606_08281_amd import workloads as W
    wl = W.immigration_death_workload(n_theta=2, n_particles=8)
    a = dict(obs_kind=0, observed=[0], sigma=2.0, theta=wl.theta,
             trajectories=wl.trajectories, n_particles=8, seed=1)
    a.update(kw)
    return wl, a


@pytest.mark.parametrize("bad", [
    dict(sigma=0.0), dict(sigma=-1.0), dict(observed=[1]), dict(obs_kind=7),
    dict(n_particles=0), dict(n_particles=4097), dict(precision=5),
    # fluorescence model: (sigma, gain, bg_mean, bg_sd)
    dict(obs_kind=2, sigma=(1.0, 2.0, 0.0, 0.0)), dict(obs_kind=2, sigma=(-1.0, 2.0, 0.0, 1.0)),
    dict(obs_kind=2, sigma=(1.0, float("inf"), 0.0, 1.0)),
    dict(obs_kind=2, sigma=(1.0, 2.0, float("nan"), 1.0)),
])
def test_host_validation_rejects_before_device_work(bad):
    wl, a = _args(**bad)
    net = lik.Network(wl.net.orders, wl.net.stoich)
    with pytest.raises(lik.LikError) as e:
        lik.eval_batch(net, **a)
    assert e.value.code == lik.LIK_EINVAL


def test_observation_checks():
    wl, a = _args()
    net = lik.Network(wl.net.orders, wl.net.stoich)
    tr = dict(wl.trajectories[0])
    tr["t_obs"] = tr["t_obs"][::-1].copy()
    with pytest.raises(lik.LikError):
        lik.eval_batch(net, **dict(a, trajectories=[tr]))
    tr = dict(wl.trajectories[0])
    tr["y"] = -np.abs(tr["y"])
    with pytest.raises(lik.LikError):   # log-normal needs y > 0
        lik.eval_batch(net, **dict(a, trajectories=[tr], obs_kind=1))
    tr = dict(wl.trajectories[0])
    tr["x0"] = np.array([-1], np.int32)
    with pytest.raises(lik.LikError):
        lik.eval_batch(net, **dict(a, trajectories=[tr]))
    for hi in (-1, (1 << 30) + 1):     # random initial counts: x0 <= x0_hi <= 2^30
        tr = dict(wl.trajectories[0], x0=np.array([0], np.int32), x0_hi=np.array([hi], np.int32))
        with pytest.raises(lik.LikError):
            lik.eval_batch(net, **dict(a, trajectories=[tr]))


def test_empty_batch_is_ok_without_device():
    wl, a = _args(theta=np.zeros((0, 2)))
    net = lik.Network(wl.net.orders, wl.net.stoich)
    out = lik.eval_batch(net, **a)
    assert out["loglik"].shape == (0,)


def test_precompile_specialized_kernels_without_gpu(tmp_path, monkeypatch):
    # run-time specialisation compiles with hipRTC for gfx950; no device needed
    monkeypatch.setenv("LIK_KERNEL_CACHE", str(tmp_path))
    from paper_1606_08281_amd import workloads as W
    for net in [W.immigration_death(), W.telegraph(), W.random_network()]:
        n = lik.Network(net.orders, net.stoich)
        for precision in (lik.FP64, lik.FP32_MIXED):
            n.precompile(precision)
    files = sorted(os.listdir(tmp_path))
    assert len([f for f in files if f.endswith(".co")]) == 6
    for f in files:
        assert b"gfx950" in open(os.path.join(tmp_path, f), "rb").read()


def test_tuning_set_get_and_bounds():
    net = lik.Network(*[np.asarray(a) for a in (W.telegraph().orders, W.telegraph().stoich)])
    default = {"pool_min": 1, "pool_max": 6, "pool_events": 1536, "pool_first": 1,
               "refill_min": 1, "priority": 0, "items_per_cu": 160, "persistent": 0,
               "schedule": 1, "urgent_events": 16000, "backlog_per_cu": 60}
    assert net.tuning() == default
    assert net.set_tuning(pool_min=1, pool_max=16, pool_events=100, pool_first=3,
                          refill_min=9, priority=1, items_per_cu=0, persistent=1,
                          schedule=1, urgent_events=0, backlog_per_cu=7) == {
        "pool_min": 1, "pool_max": 16, "pool_events": 100, "pool_first": 3, "refill_min": 9,
        "priority": 1, "items_per_cu": 0, "persistent": 1, "schedule": 1, "urgent_events": 0,
        "backlog_per_cu": 7}
    for bad in ({"pool_min": 0}, {"pool_min": 17}, {"pool_max": 65}, {"pool_first": 0},
                {"pool_first": 65}, {"refill_min": 0}, {"refill_min": 65}, {"priority": 2},
                {"items_per_cu": -1}, {"persistent": 2}, {"schedule": 2},
                {"backlog_per_cu": 0}):
        with pytest.raises(lik.LikError):
            net.set_tuning(**bad)
    assert net.tuning()["pool_max"] == 16  # a rejected call changes nothing
    assert net.set_tuning(default=True) == default


def test_eval_requests_rejects_on_the_host():
    # every check runs before any device work
    imm = W.immigration_death_workload(n_theta=4, n_particles=16)
    net = lik.Network(imm.net.orders, imm.net.stoich)
    base = dict(net=net, obs_kind=imm.obs_kind, observed=imm.observed, sigma=imm.sigma,
                theta=imm.theta[:2], trajectories=imm.trajectories, n_particles=16, seed=1)
    with pytest.raises(lik.LikError) as e:   # mixed precisions
        lik.eval_requests([base, dict(base, precision=lik.FP32_MIXED)])
    assert e.value.code == lik.LIK_EINVAL
    with pytest.raises(lik.LikError) as e:   # an invalid request is named
        lik.eval_requests([base, dict(base, n_particles=0)])
    assert e.value.code == lik.LIK_EINVAL and "request 1" in str(e.value)
    nets = [lik.Network(imm.net.orders, imm.net.stoich) for _ in range(17)]
    with pytest.raises(lik.LikError) as e:   # more than 16 networks
        lik.eval_requests([dict(base, net=n) for n in nets])
    assert e.value.code == lik.LIK_EUNSUPPORTED
    with pytest.raises(lik.LikError):
        lik.precompile_requests(nets)


def test_ode_model_validation_and_empty_batch():
    # every check runs on the host; an empty batch needs no device
    good = {"U": 1, "V": 2, "terms": [{"to": 0, "rate_param": 0},
                                      {"frm": 0, "rate_param": 1, "factors": [(0, 0, 0)]}],
            "x0_param": [-1], "sd_const": 1.0}
    m = lik.OdeModel(good)
    ll, st = lik.ode_eval(m, np.zeros((0, 2)), [{"t_obs": [1.0], "y": [0.0], "x0": [0.0]}])
    assert ll.shape == (0,)
    for bad in (dict(good, U=0), dict(good, V=0), dict(good, sd_const=0.0),
                dict(good, terms=[{"frm": 1, "rate_param": 0}]),
                dict(good, terms=[{"to": 0, "rate_param": 2}]),
                dict(good, terms=[{"to": 0, "rate_param": 0, "factors": [(1, 0, 5)]}]),
                dict(good, terms=[{"to": 0, "rate_param": 0, "factors": [(9, 0, 0)]}]),
                dict(good, x0_param=[3]), dict(good, obs_kind=1, fret_param=[0, 1, 2, 3, 4])):
        with pytest.raises(lik.LikError) as e:
            lik.OdeModel(bad)
        assert e.value.code == lik.LIK_EINVAL
    tr = {"t_obs": [1.0, 0.5], "y": [0.0, 0.0], "x0": [0.0]}
    with pytest.raises(lik.LikError):          # times must increase
        lik.ode_eval(m, np.ones((1, 2)), [tr])
    with pytest.raises(lik.LikError):          # tolerances
        lik.ode_eval(m, np.ones((1, 2)), [dict(tr, t_obs=[1.0, 2.0])], rtol=0.0)


def test_ode_device_entry_point_checks_on_the_host():
    # lik_ode_eval_device: argument checks that run before any device work
    m = lik.OdeModel({"U": 1, "V": 2, "terms": [{"to": 0, "rate_param": 0},
                                                {"frm": 0, "rate_param": 1,
                                                 "factors": [(0, 0, 0)]}],
                      "x0_param": [-1], "sd_const": 1.0})
    L = lik.lib()
    assert L.lik_ode_workspace_size(m.handle, 100, 3) >= 100 * 3 * 16
    assert L.lik_ode_workspace_size(None, 100, 3) == 0
    assert L.lik_ode_workspace_size(m.handle, 100, 0) == 0
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails its checks
    offs = np.array([0, 2], np.int32)
    d = lik.OdeData(1, fake, fake, fake, fake, fake, None, None, None)

    def call(data=d, offs_host=offs, ioff_host=None, ws=None, wsb=0, n=4, rtol=1e-6):
        return L.lik_ode_eval_device(m.handle, n, fake, ctypes.byref(data),
                                     None if offs_host is None else offs_host.ctypes.data,
                                     None if ioff_host is None else ioff_host.ctypes.data,
                                     rtol, 1e-9, 1000, lik.KERNEL_AUTO, fake, None, None,
                                     ws, wsb, None)
    assert call() == lik.LIK_EINVAL                       # no workspace
    assert call(wsb=1 << 30) == lik.LIK_EINVAL            # workspace NULL
    assert call(offs_host=None, ws=fake, wsb=1 << 30) == lik.LIK_EINVAL
    assert call(offs_host=np.array([1, 2], np.int32), ws=fake, wsb=1 << 30) == lik.LIK_EINVAL
    assert call(ioff_host=np.array([0, 1], np.int32), ws=fake, wsb=1 << 30) == lik.LIK_EINVAL
    assert call(rtol=0.0, ws=fake, wsb=1 << 30) == lik.LIK_EINVAL
    assert call(n=0) == lik.LIK_OK                        # an empty batch does nothing


def test_ode_specialised_kernels_compile_without_gpu(tmp_path, monkeypatch):
    monkeypatch.setenv("LIK_KERNEL_CACHE", str(tmp_path))
    from paper_1606_08281_amd import workloads as W
    lik.OdeModel(W.erk_model()).precompile()
    from tests.test_oracle_ode import every_factor_model, imm_death_model
    lik.OdeModel(every_factor_model()).precompile()
    lik.OdeModel(imm_death_model()).precompile()
    assert len(list(tmp_path.iterdir())) == 3
