"""ctypes binding of liblik.so (include/lik.h): argument marshalling only.

Every step of the likelihood runs in the library's HIP kernels.  There is no
fallback: if the library or a GPU is missing, calls raise.  PyTorch is used
only to hold device buffers and to name the stream work is enqueued on.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblik.so")

LIK_OK, LIK_EINVAL, LIK_ENOMEM, LIK_EDEVICE, LIK_EUNSUPPORTED, LIK_ETIMEOUT = 0, -1, -2, -3, -4, -5
STATUS_OK, STATUS_EVENT_CAP, STATUS_COUNT_OVERFLOW, STATUS_BAD_THETA = 0, 1, 2, 3
STATUS_SCHEDULER, STATUS_CANCELLED, STATUS_TIMED_OUT = 4, 5, 6
STATUS_STEP_LIMIT, STATUS_NONFINITE = 7, 8
ODE_SPECIES, ODE_SATURATING, ODE_HILL2, ODE_REPRESS2, ODE_INPUT = 0, 1, 2, 3, 4
ODE_OBS_SPECIES, ODE_OBS_FRET = 0, 1
OBS_GAUSSIAN, OBS_LOGNORMAL, OBS_FLUORESCENCE = 0, 1, 2
FP64, FP32_MIXED = 0, 1
KERNEL_AUTO, KERNEL_GENERIC, KERNEL_SPECIALIZED = 0, 1, 2
FLAG_GRAPH = 1
MAX_OBSERVED = 8

EXPORTED = ["lik_create_network", "lik_destroy_network", "lik_network_precompile", "lik_eval_batch",
            "lik_workspace_size", "lik_eval_batch_device", "lik_eval_batch_device_noalloc",
            "lik_server_create",
            "lik_server_submit", "lik_server_wait", "lik_server_cancel", "lik_server_stats_get",
            "lik_server_destroy",
            "lik_timing_enable", "lik_timing_read", "lik_last_error", "lik_version",
            "lik_network_set_tuning", "lik_network_get_tuning", "lik_autotune_device",
            "lik_eval_requests", "lik_precompile_requests", "lik_autotune_requests",
            "lik_ode_create", "lik_ode_destroy", "lik_ode_eval", "lik_ode_precompile",
            "lik_ode_workspace_size", "lik_ode_eval_device"]


class LikError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblik error {code}: {msg}")
        self.code = code


class ObsModel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_observed", ctypes.c_int32),
                ("species", ctypes.c_int32 * MAX_OBSERVED), ("sigma", ctypes.c_double),
                ("gain", ctypes.c_double), ("bg_mean", ctypes.c_double),
                ("bg_sd", ctypes.c_double)]


class Data(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_int32), ("obs_offsets", ctypes.c_void_p),
                ("t_obs", ctypes.c_void_p), ("y", ctypes.c_void_p), ("t0", ctypes.c_void_p),
                ("x0", ctypes.c_void_p), ("x0_hi", ctypes.c_void_p)]


class EvalOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("event_cap", ctypes.c_uint64), ("theta_ids", ctypes.c_void_p),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Timing(ctypes.Structure):
    _fields_ = [("propagate_ms", ctypes.c_double), ("propagate_launches", ctypes.c_int64),
                ("weigh_ms", ctypes.c_double), ("weigh_launches", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("pool_min", ctypes.c_int32), ("pool_max", ctypes.c_int32),
                ("pool_events", ctypes.c_uint32), ("pool_first", ctypes.c_int32),
                ("refill_min", ctypes.c_int32), ("priority", ctypes.c_int32),
                ("items_per_cu", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("urgent_events", ctypes.c_uint32),
                ("backlog_per_cu", ctypes.c_uint32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_size_t), ("staging_bytes", ctypes.c_size_t),
                ("max_filters", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tuning", ctypes.c_void_p)]


class Request(ctypes.Structure):
    _fields_ = [("net", ctypes.c_void_p), ("obs", ObsModel), ("precision", ctypes.c_int32),
                ("n_theta", ctypes.c_int32), ("theta", ctypes.c_void_p),
                ("theta_ids", ctypes.c_void_p), ("data", Data), ("n_particles", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("event_cap", ctypes.c_uint64), ("timeout_us", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("evals", ctypes.c_uint64), ("iterations", ctypes.c_uint64),
                ("p50_latency_us", ctypes.c_double), ("p99_latency_us", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("cancelled", ctypes.c_uint64)]


class Aux(ctypes.Structure):
    _fields_ = [("filter_events", ctypes.c_void_p), ("filter_loglik", ctypes.c_void_p),
                ("final_state", ctypes.c_void_p)]


_lib = None


def lib():
    """Load liblik.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1606_08281_amd.build`")
        # liblik is linked against the HIP runtime bundled with PyTorch-ROCm.
        # Loading torch first makes the dynamic loader resolve liblik's HIP
        # dependency to that same, already loaded copy, so the process has one
        # HIP runtime shared by torch's allocator/streams and our kernels.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t
        L.lik_create_network.argtypes = [i32, i32, vp, vp, ctypes.POINTER(vp)]
        L.lik_create_network.restype = ctypes.c_int
        L.lik_network_precompile.argtypes = [vp, i32]
        L.lik_network_precompile.restype = ctypes.c_int
        L.lik_network_set_tuning.argtypes = [vp, vp]
        L.lik_network_set_tuning.restype = ctypes.c_int
        L.lik_network_get_tuning.argtypes = [vp, vp]
        L.lik_network_get_tuning.restype = ctypes.c_int
        L.lik_autotune_device.argtypes = [vp, vp, vp, i32, vp, vp, vp, i32, u64, vp, vp, vp, sz,
                                          vp, vp]
        L.lik_autotune_device.restype = ctypes.c_int
        L.lik_destroy_network.argtypes = [vp]
        L.lik_destroy_network.restype = ctypes.c_int
        L.lik_eval_batch.argtypes = [vp, vp, vp, i32, vp, vp, i32, u64, vp, vp, vp]
        L.lik_eval_batch.restype = ctypes.c_int
        L.lik_workspace_size.argtypes = [vp, i32, i32, i32]
        L.lik_workspace_size.restype = sz
        L.lik_eval_batch_device.argtypes = [vp, vp, vp, i32, vp, vp, vp, i32, u64, vp, vp, vp,
                                            vp, sz, vp]
        L.lik_eval_batch_device.restype = ctypes.c_int
        L.lik_eval_batch_device_noalloc.argtypes = [vp, vp, vp, i32, vp, vp, vp, i32, u64, vp, vp,
                                                    vp, vp]
        L.lik_eval_batch_device_noalloc.restype = ctypes.c_int
        L.lik_server_create.argtypes = [vp, ctypes.POINTER(vp)]
        L.lik_server_create.restype = ctypes.c_int
        L.lik_server_submit.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_uint64)]
        L.lik_server_submit.restype = ctypes.c_int
        L.lik_server_wait.argtypes = [vp, ctypes.c_uint64, vp, vp, ctypes.c_int64]
        L.lik_server_wait.restype = ctypes.c_int
        L.lik_server_cancel.argtypes = [vp, ctypes.c_uint64]
        L.lik_server_cancel.restype = ctypes.c_int
        L.lik_server_stats_get.argtypes = [vp, vp]
        L.lik_server_stats_get.restype = ctypes.c_int
        L.lik_server_destroy.argtypes = [vp]
        L.lik_server_destroy.restype = ctypes.c_int
        L.lik_eval_requests.argtypes = [vp, i32, vp, i32, vp, vp, vp]
        L.lik_eval_requests.restype = ctypes.c_int
        L.lik_precompile_requests.argtypes = [vp, i32, i32]
        L.lik_precompile_requests.restype = ctypes.c_int
        L.lik_autotune_requests.argtypes = [vp, i32, i32, vp]
        L.lik_autotune_requests.restype = ctypes.c_int
        L.lik_ode_create.argtypes = [vp, ctypes.POINTER(vp)]
        L.lik_ode_create.restype = ctypes.c_int
        L.lik_ode_precompile.argtypes = [vp]
        L.lik_ode_precompile.restype = ctypes.c_int
        L.lik_ode_destroy.argtypes = [vp]
        L.lik_ode_destroy.restype = ctypes.c_int
        L.lik_ode_eval.argtypes = [vp, i32, vp, vp, ctypes.c_double, ctypes.c_double, i32, i32,
                                   vp, vp, vp]
        L.lik_ode_eval.restype = ctypes.c_int
        L.lik_ode_workspace_size.argtypes = [vp, i32, i32]
        L.lik_ode_workspace_size.restype = ctypes.c_size_t
        L.lik_ode_eval_device.argtypes = [vp, i32, vp, vp, vp, vp, ctypes.c_double,
                                          ctypes.c_double, i32, i32, vp, vp, vp, vp,
                                          ctypes.c_size_t, vp]
        L.lik_ode_eval_device.restype = ctypes.c_int
        L.lik_timing_enable.argtypes = [ctypes.c_int]
        L.lik_timing_enable.restype = ctypes.c_int
        L.lik_timing_read.argtypes = [vp]
        L.lik_timing_read.restype = ctypes.c_int
        L.lik_last_error.restype = ctypes.c_char_p
        L.lik_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != LIK_OK:
        raise LikError(rc, lib().lik_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data


def timing_enable(on=True):
    _check(lib().lik_timing_enable(1 if on else 0))


def timing_read():
    """Summed kernel durations (ms) and launch counts since the last read."""
    t = Timing()
    _check(lib().lik_timing_read(ctypes.byref(t)))
    return {"propagate_ms": t.propagate_ms, "propagate_launches": t.propagate_launches,
            "weigh_ms": t.weigh_ms, "weigh_launches": t.weigh_launches}


def _tuning_dict(t):
    return {k: getattr(t, k) for k, _ in Tuning._fields_}


class Network:
    """A validated reaction network (reactant orders p_ru, net changes nu_ru)."""

    def __init__(self, reactant_orders, stoichiometry):
        self.orders = np.ascontiguousarray(reactant_orders, dtype=np.int32)
        self.stoich = np.ascontiguousarray(stoichiometry, dtype=np.int32)
        self.R, self.U = self.orders.shape
        h = ctypes.c_void_p()
        _check(lib().lik_create_network(self.U, self.R, self.orders.ctypes.data,
                                        self.stoich.ctypes.data, ctypes.byref(h)))
        self.handle = h

    def precompile(self, precision=FP64):
        """Compile the network-specialised kernel into the disk cache (no GPU)."""
        _check(lib().lik_network_precompile(self.handle, int(precision)))

    def set_tuning(self, pool_min=None, pool_max=None, pool_events=None, pool_first=None,
                   refill_min=None, priority=None, items_per_cu=None, persistent=None,
                   schedule=None, urgent_events=None, backlog_per_cu=None,
                   default=False):
        """Work partitioning of the propagation kernels (never changes results)."""
        if default:
            _check(lib().lik_network_set_tuning(self.handle, None))
            return self.tuning()
        t = Tuning(**self.tuning())
        for k, v in (("pool_min", pool_min), ("pool_max", pool_max),
                     ("pool_events", pool_events), ("pool_first", pool_first),
                     ("refill_min", refill_min), ("priority", priority),
                     ("items_per_cu", items_per_cu), ("persistent", persistent),
                     ("schedule", schedule), ("urgent_events", urgent_events),
                     ("backlog_per_cu", backlog_per_cu)):
            if v is not None:
                setattr(t, k, int(v))
        _check(lib().lik_network_set_tuning(self.handle, ctypes.byref(t)))
        return self.tuning()

    def tuning(self):
        t = Tuning()
        _check(lib().lik_network_get_tuning(self.handle, ctypes.byref(t)))
        return _tuning_dict(t)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.lik_destroy_network(h)
            self.handle = None


def obs_model(kind, observed, sigma):
    """sigma: the noise scale, or for OBS_FLUORESCENCE the tuple
    (sigma, gain, bg_mean, bg_sd)."""
    o = ObsModel()
    o.kind = int(kind)
    o.n_observed = len(observed)
    for k, s in enumerate(observed):
        o.species[k] = int(s)
    if isinstance(sigma, (tuple, list)):
        o.sigma, o.gain, o.bg_mean, o.bg_sd = (float(v) for v in sigma)
    else:
        o.sigma = float(sigma)
    return o


def pack_trajectories(trajectories, P):
    offs = [0]
    for tr in trajectories:
        offs.append(offs[-1] + len(tr["t_obs"]))
    return {
        "obs_offsets": np.array(offs, dtype=np.int32),
        "t_obs": np.ascontiguousarray(np.concatenate([np.asarray(tr["t_obs"], np.float64)
                                                      for tr in trajectories])),
        "y": np.ascontiguousarray(np.concatenate([np.asarray(tr["y"], np.float64).reshape(-1, P)
                                                  for tr in trajectories])),
        "t0": np.array([float(tr.get("t0", 0.0)) for tr in trajectories], dtype=np.float64),
        "x0": np.ascontiguousarray(np.stack([np.asarray(tr["x0"], np.int32)
                                             for tr in trajectories])),
    } | ({"x0_hi": np.ascontiguousarray(np.stack([np.asarray(tr.get("x0_hi", tr["x0"]), np.int32)
                                                  for tr in trajectories]))}
         if any("x0_hi" in tr for tr in trajectories) else {})


def _data(M, d, ptr):
    """Data struct over the arrays of a pack_trajectories dict d (ptr: the
    address of one of its arrays)."""
    return Data(M, ptr(d["obs_offsets"]), ptr(d["t_obs"]), ptr(d["y"]), ptr(d["t0"]),
                ptr(d["x0"]), ptr(d["x0_hi"]) if "x0_hi" in d else None)


def eval_batch(net, obs_kind, observed, sigma, theta, trajectories, n_particles, seed,
               precision=FP64, event_cap=0, theta_ids=None, aux=False, kernel=KERNEL_AUTO):
    """Host-pointer entry point lik_eval_batch.  Returns a dict with loglik
    [n_theta], status [n_theta] and, if aux, filter_events, filter_loglik
    [n_theta*M] and final_state [n_theta*M, U, H]."""
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, net.R))
    n_theta = theta.shape[0]
    P = len(observed)
    d = pack_trajectories(trajectories, P)
    M = len(trajectories)
    data = _data(M, d, _ptr)
    ids = None if theta_ids is None else np.ascontiguousarray(theta_ids, dtype=np.uint32)
    opts = EvalOpts(int(precision), int(kernel), int(event_cap), _ptr(ids))
    om = obs_model(obs_kind, observed, sigma)
    ll = np.zeros(n_theta, dtype=np.float64)
    st = np.zeros(n_theta, dtype=np.int32)
    out = {"loglik": ll, "status": st}
    aux_s = None
    if aux:
        F = n_theta * M
        out["filter_events"] = np.zeros(F, dtype=np.uint64)
        out["filter_loglik"] = np.zeros(F, dtype=np.float64)
        out["final_state"] = np.zeros((F, net.U, int(n_particles)), dtype=np.int32)
        aux_s = Aux(_ptr(out["filter_events"]), _ptr(out["filter_loglik"]),
                    _ptr(out["final_state"]))
    _check(lib().lik_eval_batch(net.handle, ctypes.byref(om), ctypes.byref(opts), n_theta,
                                theta.ctypes.data, ctypes.byref(data), int(n_particles),
                                int(seed) & (2**64 - 1), ll.ctypes.data, st.ctypes.data,
                                None if aux_s is None else ctypes.byref(aux_s)))
    return out


def eval_batch_device(net, obs_kind, observed, sigma, theta_dev, data_dev, offsets_host,
                      n_particles, seed, loglik_dev, status_dev, workspace_dev, workspace_bytes,
                      stream, precision=FP64, kernel=KERNEL_AUTO, event_cap=0,
                      theta_ids_dev=None):
    """lik_eval_batch_device on caller-owned device tensors: theta_dev
    [n_theta * R] float64; data_dev a dict of device tensors obs_offsets,
    t_obs, y, t0, x0 and, for random initial counts, x0_hi (as
    pack_trajectories lays them out); offsets_host the host copy of
    obs_offsets; loglik_dev / status_dev outputs; workspace_dev at least
    lik_workspace_size bytes; stream a torch stream.  Enqueues and
    returns."""
    n_theta = theta_dev.numel() // net.R
    data = _data(len(offsets_host) - 1, data_dev, lambda t: t.data_ptr())
    opts = EvalOpts(int(precision), int(kernel), int(event_cap),
                    None if theta_ids_dev is None else theta_ids_dev.data_ptr(), 0, 0)
    om = obs_model(obs_kind, observed, sigma)
    offs = np.ascontiguousarray(offsets_host, dtype=np.int32)
    _check(lib().lik_eval_batch_device(
        net.handle, ctypes.byref(om), ctypes.byref(opts), n_theta, theta_dev.data_ptr(),
        ctypes.byref(data), offs.ctypes.data, int(n_particles), int(seed) & (2**64 - 1),
        loglik_dev.data_ptr(), None if status_dev is None else status_dev.data_ptr(), None,
        workspace_dev.data_ptr(), int(workspace_bytes), ctypes.c_void_p(stream.cuda_stream)))


def workspace_size(net, n_theta, n_traj, n_particles):
    return int(lib().lik_workspace_size(net.handle, int(n_theta), int(n_traj), int(n_particles)))


class DeviceBatch:
    """Device-resident inputs + workspace for repeated lik_eval_batch_device
    calls (torch tensors on the current CUDA/HIP device)."""

    def __init__(self, net, obs_kind, observed, sigma, trajectories, n_theta, n_particles,
                 precision=FP64, event_cap=0, device="cuda", kernel=KERNEL_AUTO, graph=False):
        import torch
        self.torch = torch
        self.net = net
        self.P = len(observed)
        d = pack_trajectories(trajectories, self.P)
        self.offsets_host = d["obs_offsets"]
        self.dev = {k: torch.from_numpy(v).to(device) for k, v in d.items()}
        self.M = len(trajectories)
        self.n_theta = int(n_theta)
        self.H = int(n_particles)
        self.om = obs_model(obs_kind, observed, sigma)
        self.precision = int(precision)
        self.event_cap = int(event_cap)
        self.kernel = int(kernel)
        self.flags = FLAG_GRAPH if graph else 0
        self.data = _data(self.M, self.dev, lambda t: t.data_ptr())
        self.ws_bytes = int(lib().lik_workspace_size(net.handle, self.n_theta, self.M, self.H))
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        self.loglik = torch.empty(self.n_theta, dtype=torch.float64, device=device)
        self.status = torch.empty(self.n_theta, dtype=torch.int32, device=device)
        F = self.n_theta * self.M
        self.events = torch.empty(F, dtype=torch.int64, device=device)
        self.filter_loglik = torch.empty(F, dtype=torch.float64, device=device)

    def run(self, theta_dev, seed, theta_ids_dev=None, stream=None, final_state=None):
        """Enqueue one evaluation on `stream` (default: torch's current stream)."""
        torch = self.torch
        assert theta_dev.dtype == torch.float64 and theta_dev.is_contiguous()
        assert theta_dev.numel() == self.n_theta * self.net.R
        s = stream if stream is not None else torch.cuda.current_stream()
        opts = EvalOpts(self.precision, self.kernel, self.event_cap,
                        None if theta_ids_dev is None else theta_ids_dev.data_ptr(), self.flags, 0)
        aux = Aux(self.events.data_ptr(), self.filter_loglik.data_ptr(),
                  None if final_state is None else final_state.data_ptr())
        ws = self.workspace.data_ptr()
        _check(lib().lik_eval_batch_device(
            self.net.handle, ctypes.byref(self.om), ctypes.byref(opts), self.n_theta,
            theta_dev.data_ptr(), ctypes.byref(self.data), self.offsets_host.ctypes.data,
            self.H, int(seed) & (2**64 - 1), self.loglik.data_ptr(), self.status.data_ptr(),
            ctypes.byref(aux), ws, self.ws_bytes + 256, ctypes.c_void_p(s.cuda_stream)))
        return self.loglik, self.status

    def run_noalloc(self, theta_dev, seed, theta_ids_dev=None, stream=None, final_state=None):
        """The same evaluation through lik_eval_batch_device_noalloc: the
        library's static scratch instead of this batch's workspace."""
        torch = self.torch
        assert theta_dev.dtype == torch.float64 and theta_dev.is_contiguous()
        assert theta_dev.numel() == self.n_theta * self.net.R
        s = stream if stream is not None else torch.cuda.current_stream()
        opts = EvalOpts(self.precision, self.kernel, self.event_cap,
                        None if theta_ids_dev is None else theta_ids_dev.data_ptr(), self.flags, 0)
        aux = Aux(self.events.data_ptr(), self.filter_loglik.data_ptr(),
                  None if final_state is None else final_state.data_ptr())
        _check(lib().lik_eval_batch_device_noalloc(
            self.net.handle, ctypes.byref(self.om), ctypes.byref(opts), self.n_theta,
            theta_dev.data_ptr(), ctypes.byref(self.data), self.offsets_host.ctypes.data,
            self.H, int(seed) & (2**64 - 1), self.loglik.data_ptr(), self.status.data_ptr(),
            ctypes.byref(aux), ctypes.c_void_p(s.cuda_stream)))
        return self.loglik, self.status

    def autotune(self, theta_dev, seed, theta_ids_dev=None, stream=None):
        """Time the candidate tunings on this batch (synchronous) and keep the
        fastest as the network's tuning; returns it."""
        torch = self.torch
        assert theta_dev.dtype == torch.float64 and theta_dev.is_contiguous()
        assert theta_dev.numel() == self.n_theta * self.net.R
        s = stream if stream is not None else torch.cuda.current_stream()
        opts = EvalOpts(self.precision, self.kernel, self.event_cap,
                        None if theta_ids_dev is None else theta_ids_dev.data_ptr(), 0, 0)
        t = Tuning()
        _check(lib().lik_autotune_device(
            self.net.handle, ctypes.byref(self.om), ctypes.byref(opts), self.n_theta,
            theta_dev.data_ptr(), ctypes.byref(self.data), self.offsets_host.ctypes.data,
            self.H, int(seed) & (2**64 - 1), self.loglik.data_ptr(), self.status.data_ptr(),
            self.workspace.data_ptr(), self.ws_bytes + 256, ctypes.c_void_p(s.cuda_stream),
            ctypes.byref(t)))
        return _tuning_dict(t)


def _request(net, obs_kind, observed, sigma, theta, trajectories, n_particles, seed,
             precision=FP64, event_cap=0, theta_ids=None, timeout_s=None, keep=None):
    """A Request struct over numpy copies (appended to `keep`, which must
    outlive the struct's use)."""
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, net.R))
    P = len(observed)
    d = pack_trajectories(trajectories, P)
    ids = None if theta_ids is None else np.ascontiguousarray(theta_ids, dtype=np.uint32)
    if keep is not None:
        keep.append((theta, d, ids))
    q = Request()
    q.net = net.handle.value
    q.obs = obs_model(obs_kind, observed, sigma)
    q.precision = int(precision)
    q.n_theta = theta.shape[0]
    q.theta = theta.ctypes.data
    q.theta_ids = _ptr(ids)
    q.data = _data(len(trajectories), d, _ptr)
    q.n_particles = int(n_particles)
    q.reserved = 0
    q.seed = int(seed) & (2**64 - 1)
    q.event_cap = int(event_cap)
    q.timeout_us = 0 if timeout_s is None else max(1, int(timeout_s * 1e6))
    return q


def _request_array(requests, keep):
    arr = (Request * len(requests))()
    for k, r in enumerate(requests):
        arr[k] = _request(keep=keep, **r)
    return arr


def eval_requests(requests, tuning=None, kernel=KERNEL_AUTO):
    """lik_eval_requests over a list of request dicts (keys: net, obs_kind,
    observed, sigma, theta, trajectories, n_particles, seed and optionally
    precision, event_cap, theta_ids).  Returns (list of loglik arrays, list
    of status arrays, done_ms array)."""
    keep = []
    arr = _request_array(requests, keep)
    n = [arr[k].n_theta for k in range(len(requests))]
    ll = np.zeros(max(sum(n), 1), dtype=np.float64)
    st = np.zeros(max(sum(n), 1), dtype=np.int32)
    done = np.zeros(max(len(requests), 1), dtype=np.float64)
    tp = None
    if tuning is not None:
        t = dict(pool_min=1, pool_max=6, pool_events=1536, pool_first=1, refill_min=1,
                 priority=0, items_per_cu=160, persistent=0, schedule=1, urgent_events=16000,
                 backlog_per_cu=60)
        t.update(tuning)
        tp = Tuning(**{k: int(v) for k, v in t.items()})
    _check(lib().lik_eval_requests(arr, len(requests), None if tp is None else ctypes.byref(tp),
                                   int(kernel), ll.ctypes.data, st.ctypes.data, done.ctypes.data))
    offs = np.cumsum([0] + n)
    return ([ll[offs[k]:offs[k + 1]].copy() for k in range(len(requests))],
            [st[offs[k]:offs[k + 1]].copy() for k in range(len(requests))], done[:len(requests)])


def precompile_requests(nets, precision=FP64):
    """Compile the multi-network flow kernel for these networks (in the order
    they first appear in the requests) into the disk cache (no GPU)."""
    arr = (ctypes.c_void_p * len(nets))(*[n.handle.value for n in nets])
    _check(lib().lik_precompile_requests(arr, len(nets), int(precision)))


def autotune_requests(requests, kernel=KERNEL_AUTO):
    """The fastest candidate tuning for lik_eval_requests on these requests."""
    keep = []
    arr = _request_array(requests, keep)
    t = Tuning()
    _check(lib().lik_autotune_requests(arr, len(requests), int(kernel), ctypes.byref(t)))
    return _tuning_dict(t)


class Server:
    """Continuous-batching server (lik_server_*): requests of any network,
    particle count and trajectory length share the GPU as they arrive."""

    def __init__(self, arena_bytes=0, staging_bytes=0, max_filters=0, kernel=0, max_inflight=0,
                 tuning=None):
        """tuning: dict of lik_tuning fields (missing ones take the defaults)."""
        self._tuning = None
        tp = None
        if tuning is not None:
            t = dict(pool_min=1, pool_max=6, pool_events=1536, pool_first=1, refill_min=1,
                     priority=0, items_per_cu=160, persistent=0, schedule=1,
                     urgent_events=16000, backlog_per_cu=60)
            t.update(tuning)
            self._tuning = Tuning(**{k: int(v) for k, v in t.items()})
            tp = ctypes.addressof(self._tuning)
        o = ServerOpts(int(arena_bytes), int(staging_bytes), int(max_filters), int(kernel),
                       int(max_inflight), 0, tp)
        h = ctypes.c_void_p()
        _check(lib().lik_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self._n_theta = {}

    def submit(self, net, obs_kind, observed, sigma, theta, trajectories, n_particles, seed,
               precision=FP64, event_cap=0, theta_ids=None, timeout_s=None):
        """Copies the request's inputs; returns a ticket.  timeout_s: the
        request's own time limit (withdrawn with STATUS_TIMED_OUT)."""
        theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, net.R))
        P = len(observed)
        d = pack_trajectories(trajectories, P)
        ids = None if theta_ids is None else np.ascontiguousarray(theta_ids, dtype=np.uint32)
        q = Request()
        q.net = net.handle.value
        q.obs = obs_model(obs_kind, observed, sigma)
        q.precision = int(precision)
        q.n_theta = theta.shape[0]
        q.theta = theta.ctypes.data
        q.theta_ids = _ptr(ids)
        q.data = _data(len(trajectories), d, _ptr)
        q.n_particles = int(n_particles)
        q.reserved = 0
        q.seed = int(seed) & (2**64 - 1)
        q.event_cap = int(event_cap)
        q.timeout_us = 0 if timeout_s is None else max(1, int(timeout_s * 1e6))
        t = ctypes.c_uint64()
        _check(lib().lik_server_submit(self.handle, ctypes.byref(q), ctypes.byref(t)))
        self._n_theta[t.value] = theta.shape[0]
        return t.value

    def wait(self, ticket, timeout_s=None):
        """(loglik, status) of a finished request; None on timeout."""
        n = self._n_theta[ticket]
        ll = np.zeros(n, dtype=np.float64)
        st = np.zeros(n, dtype=np.int32)
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        rc = lib().lik_server_wait(self.handle, ticket, ll.ctypes.data, st.ctypes.data, us)
        if rc == LIK_ETIMEOUT:
            return None
        _check(rc)
        del self._n_theta[ticket]
        return ll, st

    def cancel(self, ticket):
        """Withdraws a request (its wait then reports STATUS_CANCELLED)."""
        _check(lib().lik_server_cancel(self.handle, ticket))

    def stats(self):
        s = ServerStats()
        _check(lib().lik_server_stats_get(self.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(lib().lik_server_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# -- deterministic models (lik_ode_*) ----------------------------------------

class OdeTerm(ctypes.Structure):
    _fields_ = [("frm", ctypes.c_int32), ("to", ctypes.c_int32), ("rate_param", ctypes.c_int32),
                ("n_factors", ctypes.c_int32), ("rate_scale", ctypes.c_double),
                ("kind", ctypes.c_int32 * 3), ("species", ctypes.c_int32 * 3),
                ("param", ctypes.c_int32 * 3)]


class OdeModelC(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_params", ctypes.c_int32),
                ("n_terms", ctypes.c_int32), ("terms", ctypes.c_void_p),
                ("x0_param", ctypes.c_void_p), ("obs_kind", ctypes.c_int32),
                ("obs_species", ctypes.c_int32), ("obs_species2", ctypes.c_int32),
                ("sd_param", ctypes.c_int32), ("sd_const", ctypes.c_double),
                ("fret_param", ctypes.c_int32 * 5)]


class OdeData(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_int32), ("obs_offsets", ctypes.c_void_p),
                ("t_obs", ctypes.c_void_p), ("y", ctypes.c_void_p), ("t0", ctypes.c_void_p),
                ("x0", ctypes.c_void_p), ("in_offsets", ctypes.c_void_p),
                ("t_in", ctypes.c_void_p), ("u_in", ctypes.c_void_p)]


class OdeModel:
    """A deterministic model (lik_ode_create).  spec: dict with U, V, terms
    (dicts frm, to, rate_param, rate_scale, factors [(kind, species,
    param)]), x0_param [U], obs_kind, obs_species, obs_species2, sd_param,
    sd_const, fret_param [5]."""

    def __init__(self, spec):
        U, V = int(spec["U"]), int(spec["V"])
        terms = spec["terms"]
        arr = (OdeTerm * len(terms))()
        for k, t in enumerate(terms):
            T = arr[k]
            T.frm, T.to = int(t.get("frm", -1)), int(t.get("to", -1))
            T.rate_param = int(t.get("rate_param", -1))
            T.rate_scale = float(t.get("rate_scale", 1.0))
            fs = t.get("factors", [])
            T.n_factors = len(fs)
            for j, (kind, sp, par) in enumerate(fs):
                T.kind[j], T.species[j], T.param[j] = int(kind), int(sp), int(par)
        x0p = np.ascontiguousarray(spec.get("x0_param", [-1] * U), dtype=np.int32)
        m = OdeModelC(U, V, len(terms), ctypes.addressof(arr), x0p.ctypes.data,
                      int(spec.get("obs_kind", 0)), int(spec.get("obs_species", 0)),
                      int(spec.get("obs_species2", 0)), int(spec.get("sd_param", -1)),
                      float(spec.get("sd_const", 1.0)),
                      (ctypes.c_int32 * 5)(*[int(v) for v in spec.get("fret_param", [0] * 5)]))
        h = ctypes.c_void_p()
        _check(lib().lik_ode_create(ctypes.byref(m), ctypes.byref(h)))   # copies the arrays
        self.handle = h
        self.U, self.V = U, V

    def precompile(self):
        """Compile the model-specialised kernel into the disk cache (no GPU)."""
        _check(lib().lik_ode_precompile(self.handle))

    def __del__(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().lik_ode_destroy(self.handle)
            self.handle = None


def _ode_arrays(model, trajectories):
    """The trajectories as lik_ode_data's arrays (numpy): offs, t_obs, y, t0,
    x0, and ioff, t_in, u_in (None without inputs)."""
    offs, tin, ioff = [0], [], [0]
    for tr in trajectories:
        offs.append(offs[-1] + len(tr["t_obs"]))
        tin.append(len(tr.get("t_in", [])))
        ioff.append(ioff[-1] + tin[-1])
    offs = np.array(offs, np.int32)
    t_obs = np.ascontiguousarray(np.concatenate([np.asarray(tr["t_obs"], np.float64)
                                                 for tr in trajectories]))
    y = np.ascontiguousarray(np.concatenate([np.asarray(tr["y"], np.float64).ravel()
                                             for tr in trajectories]))
    t0 = np.array([float(tr.get("t0", 0.0)) for tr in trajectories], np.float64)
    x0 = np.ascontiguousarray(np.stack([np.asarray(tr.get("x0", np.zeros(model.U)), np.float64)
                                        for tr in trajectories]))
    has_in = ioff[-1] > 0
    ioff = np.array(ioff, np.int32)
    t_in = np.ascontiguousarray(np.concatenate([np.asarray(tr.get("t_in", []), np.float64)
                                                for tr in trajectories])) if has_in else None
    u_in = np.ascontiguousarray(np.concatenate([np.asarray(tr.get("u_in", []), np.float64)
                                                for tr in trajectories])) if has_in else None
    return offs, t_obs, y, t0, x0, (ioff if has_in else None), t_in, u_in


def ode_eval(model, theta, trajectories, rtol=1e-6, atol=1e-9, max_steps=100000, steps=False,
             kernel=KERNEL_AUTO):
    """lik_ode_eval: (loglik [n_theta], status [n_theta]) and, with steps,
    the step attempts [n_theta, M].  trajectories:
    dicts t_obs, y, t0, x0 [U] (the species not set by theta) and optionally
    t_in, u_in (piecewise-constant input)."""
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, model.V))
    offs, t_obs, y, t0, x0, ioff, t_in, u_in = _ode_arrays(model, trajectories)
    d = OdeData(len(trajectories), offs.ctypes.data, t_obs.ctypes.data, y.ctypes.data,
                t0.ctypes.data, x0.ctypes.data, _ptr(ioff), _ptr(t_in), _ptr(u_in))
    n = theta.shape[0]
    ll = np.zeros(max(n, 1))
    st = np.zeros(max(n, 1), np.int32)
    ns = np.zeros(max(n * len(trajectories), 1), np.int32)
    _check(lib().lik_ode_eval(model.handle, n, theta.ctypes.data, ctypes.byref(d), float(rtol),
                              float(atol), int(max_steps), int(kernel), ll.ctypes.data,
                              st.ctypes.data,
                              ns.ctypes.data if steps else None))
    if steps:
        return ll[:n], st[:n], ns[:n * len(trajectories)].reshape(n, len(trajectories))
    return ll[:n], st[:n]


class OdeDeviceBatch:
    """Trajectories and workspace resident on the device for repeated
    lik_ode_eval_device calls (torch tensors, torch's current stream): the
    deterministic counterpart of DeviceBatch."""

    def __init__(self, model, trajectories, n_theta, steps=False, kernel=KERNEL_AUTO):
        import torch
        self.torch, self.model, self.n_theta, self.kernel = torch, model, int(n_theta), kernel
        self.M = len(trajectories)
        offs, t_obs, y, t0, x0, ioff, t_in, u_in = _ode_arrays(model, trajectories)
        self.offs_host, self.ioff_host = offs, ioff
        dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
        self.arrays = [dev(a) for a in (offs, t_obs, y, t0, x0, ioff, t_in, u_in)]
        p = [None if a is None else a.data_ptr() for a in self.arrays]
        self.data = OdeData(self.M, *p)
        ws = lib().lik_ode_workspace_size(model.handle, self.n_theta, self.M)
        if ws == 0:
            raise LikError(-1, "lik_ode_workspace_size: bad arguments")
        self.workspace = torch.empty(ws, dtype=torch.uint8, device="cuda")
        self.loglik = torch.empty(max(self.n_theta, 1), dtype=torch.float64, device="cuda")
        self.status = torch.empty(max(self.n_theta, 1), dtype=torch.int32, device="cuda")
        self.steps = (torch.empty(max(self.n_theta * self.M, 1), dtype=torch.int32, device="cuda")
                      if steps else None)

    def run(self, theta_dev, rtol=1e-6, atol=1e-9, max_steps=100000, stream=None):
        """Enqueue one evaluation of theta_dev [n_theta, V] (float64, device)."""
        torch = self.torch
        assert theta_dev.dtype == torch.float64 and theta_dev.is_contiguous()
        assert theta_dev.numel() == self.n_theta * self.model.V
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().lik_ode_eval_device(
            self.model.handle, self.n_theta, theta_dev.data_ptr(), ctypes.byref(self.data),
            self.offs_host.ctypes.data, _ptr(self.ioff_host), float(rtol), float(atol),
            int(max_steps), int(self.kernel), self.loglik.data_ptr(), self.status.data_ptr(),
            None if self.steps is None else self.steps.data_ptr(), self.workspace.data_ptr(),
            self.workspace.numel(), ctypes.c_void_p(s.cuda_stream)))
        return self.loglik[:self.n_theta], self.status[:self.n_theta]
