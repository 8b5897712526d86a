"""ctypes binding of include/chanenv.h: argument marshalling only.

Every function here has the name of the C entry point it calls.  Device
buffers are passed as raw pointers (``tensor.data_ptr()``) on the stream the env
was created with; PyTorch serves only as the allocator of device memory and the
owner of the stream.
"""
import ctypes
import weakref
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

CHAN_OK, CHAN_EINVAL, CHAN_ENOMEM, CHAN_EDEVICE, CHAN_ENONFINITE, CHAN_ESTATE, CHAN_EBUSY = 0, -1, -2, -3, -4, -5, -6
CHAN_TOP_WALL, CHAN_TOP_FREESLIP = 0, 1
CHAN_CFR, CHAN_CPG = 0, 1
CHAN_CTRL_EXTERNAL, CHAN_CTRL_OPPOSITION = 0, 1
CHAN_RAMP, CHAN_HOLD = 0, 1
CHAN_IC_LAMINAR, CHAN_IC_REICHARDT = 0, 1
CHAN_OBS_U, CHAN_OBS_V, CHAN_OBS_W, CHAN_OBS_P = 1, 2, 4, 8

EXPORTED = ["chan_opts_default", "chan_env_create", "chan_env_reset", "chan_env_step",
            "chan_env_get_state", "chan_env_set_state", "chan_env_query",
            "chan_env_footprint_bytes", "chan_env_destroy", "chan_strerror", "chan_last_error",
            "chan_env_set_timing", "chan_env_timing_read", "chan_kernel_class_name"]


class ChanGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("lz", ctypes.c_double), ("re_tau", ctypes.c_double),
                ("dt_plus", ctypes.c_double), ("obs_y_plus", ctypes.c_double)]


class ChanOpts(ctypes.Structure):
    _fields_ = [("top_bc", ctypes.c_int32), ("forcing", ctypes.c_int32),
                ("ub_plus", ctypes.c_double), ("px", ctypes.c_double),
                ("nu_override", ctypes.c_double), ("dt_override", ctypes.c_double),
                ("controller", ctypes.c_int32), ("opp_alpha", ctypes.c_double),
                ("action_mode", ctypes.c_int32), ("clip", ctypes.c_double),
                ("obs_mask", ctypes.c_uint32), ("ic_profile", ctypes.c_int32),
                ("ic_amp", ctypes.c_double), ("n_extra_planes", ctypes.c_int32),
                ("extra_obs_y_plus", ctypes.c_double * 3)]


class ChanInfo(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("js", ctypes.c_int32), ("y_plus_node", ctypes.c_double), ("nu", ctypes.c_double),
                ("dt", ctypes.c_double), ("ub", ctypes.c_double), ("t", ctypes.c_double),
                ("nstep", ctypes.c_int64), ("state_doubles", ctypes.c_size_t),
                ("obs_doubles", ctypes.c_size_t), ("footprint_bytes", ctypes.c_size_t),
                ("n_planes", ctypes.c_int32), ("js_planes", ctypes.c_int32 * 4),
                ("y_plus_planes", ctypes.c_double * 4)]


class ChanError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        detail = chan_last_error()
        super().__init__(f"{where}: {chan_strerror(code)} ({code})" + (f" [{detail}]" if detail else ""))


_LIB = None


def library_path():
    return os.path.join(HERE, "libchanenv.so")


def load_library():
    """Load libchanenv.so; raises if it has not been built (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2301_09889_amd/build.py")
    # PyTorch ships its own HIP runtime.  Load it first, so that the library's
    # libamdhip64.so.7 dependency resolves to the same runtime (one device
    # context; streams and device pointers from torch are valid in the library).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.chan_opts_default.argtypes = [P(ChanOpts)]
    lib.chan_opts_default.restype = None
    lib.chan_env_create.argtypes = [P(ChanGrid), P(ChanOpts), vp, P(vp)]
    lib.chan_env_create.restype = ctypes.c_int
    lib.chan_env_reset.argtypes = [vp, ctypes.c_uint64]
    lib.chan_env_reset.restype = ctypes.c_int
    lib.chan_env_step.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
    lib.chan_env_step.restype = ctypes.c_int
    lib.chan_env_get_state.argtypes = [vp, P(ctypes.c_double), ctypes.c_size_t]
    lib.chan_env_get_state.restype = ctypes.c_int
    lib.chan_env_set_state.argtypes = [vp, P(ctypes.c_double), ctypes.c_size_t]
    lib.chan_env_set_state.restype = ctypes.c_int
    lib.chan_env_query.argtypes = [vp, P(ChanInfo)]
    lib.chan_env_query.restype = ctypes.c_int
    lib.chan_env_footprint_bytes.argtypes = [P(ChanGrid), P(ChanOpts)]
    lib.chan_env_footprint_bytes.restype = ctypes.c_size_t
    lib.chan_env_destroy.argtypes = [vp]
    lib.chan_env_destroy.restype = None
    lib.chan_strerror.argtypes = [ctypes.c_int]
    lib.chan_strerror.restype = ctypes.c_char_p
    lib.chan_last_error.argtypes = []
    lib.chan_last_error.restype = ctypes.c_char_p
    lib.chan_env_set_timing.argtypes = [vp, ctypes.c_int32]
    lib.chan_env_set_timing.restype = ctypes.c_int
    lib.chan_env_timing_read.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_double)]
    lib.chan_env_timing_read.restype = ctypes.c_int
    lib.chan_kernel_class_name.argtypes = [ctypes.c_int32]
    lib.chan_kernel_class_name.restype = ctypes.c_char_p
    lib.chan_batch_create.argtypes = [ctypes.c_int32, P(vp), P(vp)]
    lib.chan_batch_create.restype = ctypes.c_int
    lib.chan_batch_step.argtypes = [vp, P(vp), ctypes.c_int32, P(vp), P(vp), P(vp), P(ctypes.c_int32)]
    lib.chan_batch_step.restype = ctypes.c_int
    lib.chan_batch_step_subset.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int32), P(vp), ctypes.c_int32, P(vp),
                                           P(vp), P(vp), P(ctypes.c_int32)]
    lib.chan_batch_step_subset.restype = ctypes.c_int
    lib.chan_batch_destroy.argtypes = [vp]
    lib.chan_batch_destroy.restype = None
    lib.chan_batch_size.argtypes = [vp]
    lib.chan_batch_size.restype = ctypes.c_int32
    lib.chan_batch_set_timing.argtypes = [vp, ctypes.c_int32]
    lib.chan_batch_set_timing.restype = ctypes.c_int
    lib.chan_batch_timing_read.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_double)]
    lib.chan_batch_timing_read.restype = ctypes.c_int
    lib.chan_batch_launch.argtypes = [vp, vp, ctypes.c_int32, P(vp), P(vp), ctypes.c_int32, P(vp), P(vp), P(vp),
                                      P(vp)]
    lib.chan_batch_launch.restype = ctypes.c_int
    lib.chan_call_query.argtypes = [vp]
    lib.chan_call_query.restype = ctypes.c_int
    lib.chan_call_finish.argtypes = [vp, P(ctypes.c_int32)]
    lib.chan_call_finish.restype = ctypes.c_int
    lib.chan_batch_add.argtypes = [vp, vp]
    lib.chan_batch_add.restype = ctypes.c_int
    lib.chan_batch_remove.argtypes = [vp, vp]
    lib.chan_batch_remove.restype = ctypes.c_int
    lib.chan_batch_tuning.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int32)]
    lib.chan_batch_tuning.restype = ctypes.c_int
    lib.chan_batch_capture.argtypes = [vp, ctypes.c_int32, P(vp), P(vp), ctypes.c_int32, P(vp), P(vp), P(vp), P(vp)]
    lib.chan_batch_capture.restype = ctypes.c_int
    lib.chan_env_capture.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp, P(vp)]
    lib.chan_env_capture.restype = ctypes.c_int
    lib.chan_graph_launch.argtypes = [vp, vp, P(vp)]
    lib.chan_graph_launch.restype = ctypes.c_int
    lib.chan_graph_destroy.argtypes = [vp]
    lib.chan_graph_destroy.restype = None
    lib.chan_step_static.argtypes = [P(ChanGrid), P(ChanOpts), vp, vp, vp, ctypes.c_int32, vp, vp, vp]
    lib.chan_step_static.restype = ctypes.c_int
    _LIB = lib
    return lib


def chan_strerror(code):
    return load_library().chan_strerror(int(code)).decode()


def chan_last_error():
    return load_library().chan_last_error().decode()


def chan_opts_default():
    o = ChanOpts()
    load_library().chan_opts_default(ctypes.byref(o))
    return o


def chan_env_create(grid, opts=None, stream=0):
    h = ctypes.c_void_p()
    rc = load_library().chan_env_create(ctypes.byref(grid), ctypes.byref(opts) if opts is not None else None,
                                        ctypes.c_void_p(stream), ctypes.byref(h))
    if rc != CHAN_OK:
        raise ChanError(rc, "chan_env_create")
    return h


def chan_step_static(grid, opts, stream, state_ptr, action_ptr, n_substeps, obs_ptr, tau_ptr, drag_ptr):
    """One env step of the flow state at state_ptr (device, exchange layout) with no allocation;
    returns the library's code."""
    return load_library().chan_step_static(ctypes.byref(grid), ctypes.byref(opts) if opts is not None else None,
                                           ctypes.c_void_p(stream), ctypes.c_void_p(state_ptr),
                                           ctypes.c_void_p(action_ptr or None), int(n_substeps),
                                           ctypes.c_void_p(obs_ptr or None), ctypes.c_void_p(tau_ptr or None),
                                           ctypes.c_void_p(drag_ptr or None))


def chan_env_reset(h, seed):
    return load_library().chan_env_reset(h, ctypes.c_uint64(seed))


def chan_env_step(h, action_ptr, n_substeps, obs_ptr, tau_ptr, drag_ptr):
    return load_library().chan_env_step(h, ctypes.c_void_p(action_ptr or None), int(n_substeps),
                                        ctypes.c_void_p(obs_ptr or None), ctypes.c_void_p(tau_ptr or None),
                                        ctypes.c_void_p(drag_ptr or None))


def chan_env_get_state(h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.float64)
    return load_library().chan_env_get_state(h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), buf.size)


def chan_env_set_state(h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.float64)
    return load_library().chan_env_set_state(h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), buf.size)


def chan_env_query(h):
    info = ChanInfo()
    rc = load_library().chan_env_query(h, ctypes.byref(info))
    if rc != CHAN_OK:
        raise ChanError(rc, "chan_env_query")
    return info


def chan_env_footprint_bytes(grid, opts=None):
    return load_library().chan_env_footprint_bytes(ctypes.byref(grid),
                                                   ctypes.byref(opts) if opts is not None else None)


def chan_env_set_timing(h, enable):
    return load_library().chan_env_set_timing(h, int(bool(enable)))


def chan_env_timing_read(h, nclass=16):
    """Returns {class name: (launches, total ms)}."""
    launches = (ctypes.c_int64 * nclass)()
    ms = (ctypes.c_double * nclass)()
    n = load_library().chan_env_timing_read(h, nclass, launches, ms)
    if n < 0:
        raise ChanError(n, "chan_env_timing_read")
    return {chan_kernel_class_name(k): (launches[k], ms[k]) for k in range(min(n, nclass))}


def chan_kernel_class_name(cls):
    return load_library().chan_kernel_class_name(int(cls)).decode()


def chan_env_destroy(h):
    load_library().chan_env_destroy(h)


def _ptr_array(ptrs):
    """ctypes array of device pointers (0 / None -> NULL), or None for an absent list."""
    if ptrs is None:
        return None
    return (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(p or None) for p in ptrs])


def chan_batch_create(env_handles):
    hs = (ctypes.c_void_p * len(env_handles))(*env_handles)
    h = ctypes.c_void_p()
    rc = load_library().chan_batch_create(len(env_handles), hs, ctypes.byref(h))
    if rc != CHAN_OK:
        raise ChanError(rc, "chan_batch_create")
    return h


def chan_batch_step(h, action_ptrs, n_substeps, obs_ptrs, tau_ptrs, drag_ptrs, results=None):
    """Pointer lists hold one device address (or 0) per env; results, if given, is a ctypes
    int32 array of the batch size."""
    return load_library().chan_batch_step(h, _ptr_array(action_ptrs), int(n_substeps), _ptr_array(obs_ptrs),
                                          _ptr_array(tau_ptrs), _ptr_array(drag_ptrs), results)


def chan_batch_step_subset(h, idx, action_ptrs, n_substeps, obs_ptrs, tau_ptrs, drag_ptrs, results=None):
    """Like chan_batch_step for the envs idx (positions at creation); pointer lists are indexed
    like idx."""
    ia = (ctypes.c_int32 * len(idx))(*[int(i) for i in idx])
    return load_library().chan_batch_step_subset(h, len(idx), ia, _ptr_array(action_ptrs), int(n_substeps),
                                                 _ptr_array(obs_ptrs), _ptr_array(tau_ptrs), _ptr_array(drag_ptrs),
                                                 results)


def chan_batch_launch(h, stream, env_handles, action_ptrs, n_substeps, obs_ptrs, tau_ptrs, drag_ptrs):
    """Queue one env step of the listed envs on stream; returns (code, call handle)."""
    call = ctypes.c_void_p()
    hs = (ctypes.c_void_p * len(env_handles))(*env_handles)
    rc = load_library().chan_batch_launch(h, ctypes.c_void_p(stream), len(env_handles), hs,
                                          _ptr_array(action_ptrs), int(n_substeps), _ptr_array(obs_ptrs),
                                          _ptr_array(tau_ptrs), _ptr_array(drag_ptrs), ctypes.byref(call))
    return rc, call


def chan_batch_tuning(h):
    """The batch's tuned launch shapes: a list of dicts per grid shape."""
    lib = load_library()
    n = lib.chan_batch_tuning(h, 0, None)
    if n < 0:
        raise ChanError(n, "chan_batch_tuning")
    buf = (ctypes.c_int32 * (7 * max(n, 1)))()
    lib.chan_batch_tuning(h, n, buf)
    keys = ("nx", "ny", "nz", "z_pencils_per_block", "x_pairs_per_block", "columns_per_block", "plane_fused")
    return [dict(zip(keys, buf[7 * k:7 * k + 7])) for k in range(n)]


def chan_batch_capture(h, env_handles, action_ptrs, n_substeps, obs_ptrs, tau_ptrs, drag_ptrs):
    """Capture one env step of the listed envs as a graph; returns (code, graph handle)."""
    graph = ctypes.c_void_p()
    hs = (ctypes.c_void_p * len(env_handles))(*env_handles)
    rc = load_library().chan_batch_capture(h, len(env_handles), hs, _ptr_array(action_ptrs), int(n_substeps),
                                           _ptr_array(obs_ptrs), _ptr_array(tau_ptrs), _ptr_array(drag_ptrs),
                                           ctypes.byref(graph))
    return rc, graph


def chan_env_capture(h, action_ptr, n_substeps, obs_ptr, tau_ptr, drag_ptr):
    graph = ctypes.c_void_p()
    rc = load_library().chan_env_capture(h, ctypes.c_void_p(action_ptr), int(n_substeps), ctypes.c_void_p(obs_ptr),
                                         ctypes.c_void_p(tau_ptr), ctypes.c_void_p(drag_ptr), ctypes.byref(graph))
    return rc, graph


def chan_graph_launch(graph, stream):
    call = ctypes.c_void_p()
    rc = load_library().chan_graph_launch(graph, ctypes.c_void_p(stream), ctypes.byref(call))
    return rc, call


def chan_graph_destroy(graph):
    load_library().chan_graph_destroy(graph)


def chan_call_query(call):
    return load_library().chan_call_query(call)


def chan_call_finish(call, results):
    return load_library().chan_call_finish(call, results)


def chan_batch_add(h, env_handle):
    return load_library().chan_batch_add(h, env_handle)


def chan_batch_remove(h, env_handle):
    return load_library().chan_batch_remove(h, env_handle)


def chan_batch_destroy(h):
    load_library().chan_batch_destroy(h)


def chan_batch_size(h):
    return load_library().chan_batch_size(h)


def chan_batch_set_timing(h, enable):
    return load_library().chan_batch_set_timing(h, int(bool(enable)))


def chan_batch_timing_read(h, nclass=16):
    """Returns {class name: (launches, total ms)}."""
    launches = (ctypes.c_int64 * nclass)()
    ms = (ctypes.c_double * nclass)()
    n = load_library().chan_batch_timing_read(h, nclass, launches, ms)
    if n < 0:
        raise ChanError(n, "chan_batch_timing_read")
    return {chan_kernel_class_name(k): (launches[k], ms[k]) for k in range(min(n, nclass))}


def make_grid(nx, ny, nz, lx, lz, re_tau, dt_plus, obs_y_plus):
    return ChanGrid(nx, ny, nz, lx, lz, re_tau, dt_plus, obs_y_plus)


def make_opts(**kw):
    """chan_opts_t with the defaults, then the given fields; ``extra_obs_y_plus`` takes a sequence
    of heights and sets ``n_extra_planes`` to its length."""
    o = chan_opts_default()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k == "extra_obs_y_plus":
            v = list(v)
            if len(v) > len(o.extra_obs_y_plus):
                raise ValueError(f"at most {len(o.extra_obs_y_plus)} extra observation planes")
            for i, y in enumerate(v):
                o.extra_obs_y_plus[i] = float(y)
            o.n_extra_planes = len(v)
            continue
        setattr(o, k, v)
    return o


def _action_ptr(env, a):
    """Device pointer of an action tensor for env (0 for None), after checking that the kernels
    can read it: float64, contiguous, (nz, nx), on the env's device."""
    if a is None:
        return 0
    if a.dtype != env.torch.float64 or not a.is_contiguous():
        raise ValueError("action must be a contiguous float64 tensor")
    if tuple(a.shape) != (env.grid.nz, env.grid.nx):
        raise ValueError(f"action shape {tuple(a.shape)} != (nz, nx) = {(env.grid.nz, env.grid.nx)}")
    if a.device != env.obs.device:
        raise ValueError(f"action on {a.device}, env on {env.obs.device}")
    return a.data_ptr()


class ChanEnv:
    """One channel on the current HIP device; tensors come from PyTorch."""

    def __init__(self, grid, opts=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("ChanEnv needs a HIP device")
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.grid = grid
        self.opts = opts if opts is not None else chan_opts_default()
        self.handle = chan_env_create(grid, self.opts, self.stream.cuda_stream)
        self.info = chan_env_query(self.handle)
        dev = torch.device("cuda", torch.cuda.current_device())
        nobs = bin(self.opts.obs_mask).count("1") * self.info.n_planes   # [plane][component] flattened
        self.obs = torch.zeros((nobs, grid.nz, grid.nx), dtype=torch.float64, device=dev)
        self.tau_w = torch.zeros((grid.nz, grid.nx), dtype=torch.float64, device=dev)
        self.drag = torch.zeros(1, dtype=torch.float64, device=dev)

    def _check(self, rc, where):
        if rc != CHAN_OK:
            raise ChanError(rc, where)

    def reset(self, seed):
        self._check(chan_env_reset(self.handle, seed), "chan_env_reset")

    def set_state(self, flat):
        self._check(chan_env_set_state(self.handle, flat), "chan_env_set_state")

    def get_state(self):
        buf = np.zeros(self.info.state_doubles)
        self._check(chan_env_get_state(self.handle, buf), "chan_env_get_state")
        return buf

    def step(self, action, n_substeps):
        """action: float64 device tensor (nz, nx) or None.  Returns (obs, tau_w, drag) tensors."""
        ptr = _action_ptr(self, action)
        rc = chan_env_step(self.handle, ptr, n_substeps, self.obs.data_ptr(), self.tau_w.data_ptr(),
                           self.drag.data_ptr())
        self._check(rc, "chan_env_step")
        return self.obs, self.tau_w, self.drag

    def query(self):
        return chan_env_query(self.handle)

    def capture(self, action, n_substeps):
        """Capture one env step with this action tensor (or None) and the env's own output tensors
        as a graph; ChanGraph.launch replays it (refill the action tensor between replays)."""
        rc, g = chan_env_capture(self.handle, _action_ptr(self, action), n_substeps, self.obs.data_ptr(),
                                 self.tau_w.data_ptr(), self.drag.data_ptr())
        self._check(rc, "chan_env_capture")
        graph = ChanGraph(g, 1, keep=(action,))
        if not hasattr(self, "_graphs"):
            self._graphs = weakref.WeakSet()
        self._graphs.add(graph)
        return graph

    def close(self):
        """Destroy the env: the library waits for a call that holds it and removes it from every
        batch; the Python batches that list it drop it too.  Replays of the env's own graphs
        (capture) are finished by the library."""
        if self.handle:
            for b in list(getattr(self, "_batches", ())):
                b._drop(self)
            for g in list(getattr(self, "_graphs", ())):
                g._abandon_calls()
            chan_env_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ChanBatch:
    """Several ChanEnv (same stream) advanced together; each env's step outputs land in that
    env's own obs / tau_w / drag tensors, exactly as ChanEnv.step would write them."""

    def __init__(self, envs):
        self.envs = list(envs)
        self.handle = chan_batch_create([e.handle for e in self.envs])
        self.results = (ctypes.c_int32 * len(self.envs))()
        self._calls = weakref.WeakSet()
        self._graphs = weakref.WeakSet()
        for e in self.envs:
            _member_of(e).add(self)

    def _drop(self, env):
        """env is being destroyed (the library removes it from the batch itself)."""
        if env in self.envs:
            self.envs.remove(env)
            self.results = (ctypes.c_int32 * max(1, len(self.envs)))()

    def step(self, actions, n_substeps):
        """actions: list of float64 device tensors (nz, nx) or None per env (or None for all).
        Returns the per-env result codes; raises if the call itself failed before running."""
        aptrs = [_action_ptr(e, actions[k] if actions is not None else None) for k, e in enumerate(self.envs)]
        for k in range(len(self.envs)):
            self.results[k] = CHAN_OK
        rc = chan_batch_step(self.handle, aptrs, n_substeps, [e.obs.data_ptr() for e in self.envs],
                             [e.tau_w.data_ptr() for e in self.envs], [e.drag.data_ptr() for e in self.envs],
                             self.results)
        codes = list(self.results)
        if rc != CHAN_OK and all(c == CHAN_OK for c in codes):
            raise ChanError(rc, "chan_batch_step")
        return codes

    def step_subset(self, idx, actions, n_substeps):
        """Advance only the envs idx (positions in this batch); actions indexed like idx (or None).
        Returns the result codes, indexed like idx."""
        if any(not 0 <= i < len(self.envs) for i in idx):
            raise ValueError("env index out of range")
        aptrs = [_action_ptr(self.envs[i], actions[k] if actions is not None else None) for k, i in enumerate(idx)]
        res = (ctypes.c_int32 * len(idx))()
        sel = [self.envs[i] for i in idx]
        rc = chan_batch_step_subset(self.handle, idx, aptrs, n_substeps, [e.obs.data_ptr() for e in sel],
                                    [e.tau_w.data_ptr() for e in sel], [e.drag.data_ptr() for e in sel], res)
        codes = list(res)
        if rc != CHAN_OK and all(c == CHAN_OK for c in codes):
            raise ChanError(rc, "chan_batch_step_subset")
        return codes

    def launch(self, envs, actions, n_substeps, obs, tau_w, drag, stream=None):
        """Queue one env step of envs (members of this batch) on stream (a torch stream; None: the
        current one) and return at once.  actions: float64 device tensors (nz, nx) or None per
        env; obs, tau_w, drag: per-env output tensors (or None) written by the stream.  Returns a
        ChanCall; the envs are held by it until its finish()."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        aptrs = [_action_ptr(e, actions[k] if actions is not None else None) for k, e in enumerate(envs)]

        def ptrs(ts):
            return [t.data_ptr() if t is not None else 0 for t in ts] if ts is not None else [0] * len(envs)

        rc, call = chan_batch_launch(self.handle, st.cuda_stream, [e.handle for e in envs], aptrs, n_substeps,
                                     ptrs(obs), ptrs(tau_w), ptrs(drag))
        if rc != CHAN_OK:
            raise ChanError(rc, "chan_batch_launch")
        c = ChanCall(call, len(envs), keep=(actions, obs, tau_w, drag))
        self._calls.add(c)
        return c

    def capture(self, envs, actions, n_substeps, obs, tau_w, drag):
        """Capture one env step of envs with these tensors (as for launch) as a graph;
        ChanGraph.launch replays it."""
        aptrs = [_action_ptr(e, actions[k] if actions is not None else None) for k, e in enumerate(envs)]

        def ptrs(ts):
            return [t.data_ptr() if t is not None else 0 for t in ts] if ts is not None else [0] * len(envs)

        rc, g = chan_batch_capture(self.handle, [e.handle for e in envs], aptrs, n_substeps, ptrs(obs), ptrs(tau_w),
                                   ptrs(drag))
        if rc != CHAN_OK:
            raise ChanError(rc, "chan_batch_capture")
        graph = ChanGraph(g, len(envs), keep=(actions, obs, tau_w, drag))
        self._graphs.add(graph)
        return graph

    def add(self, env):
        rc = chan_batch_add(self.handle, env.handle)
        if rc != CHAN_OK:
            raise ChanError(rc, "chan_batch_add")
        self.envs.append(env)
        _member_of(env).add(self)
        self.results = (ctypes.c_int32 * len(self.envs))()

    def remove(self, env):
        rc = chan_batch_remove(self.handle, env.handle)
        if rc != CHAN_OK:
            raise ChanError(rc, "chan_batch_remove")
        self.envs.remove(env)
        _member_of(env).discard(self)
        self.results = (ctypes.c_int32 * max(1, len(self.envs)))()

    def close(self):
        """Destroy the batch: the library finishes its unfinished calls itself (the envs'
        outcomes applied; finish() then reports CHAN_EINVAL for every env of such a call)."""
        if self.handle:
            for c in list(self._calls):
                c._abandon()
            for g in list(self._graphs):
                g._abandon_calls()
            for e in self.envs:
                _member_of(e).discard(self)
            chan_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _member_of(env):
    if not hasattr(env, "_batches"):
        env._batches = weakref.WeakSet()
    return env._batches


class ChanCall:
    """An asynchronous batch call (chan_batch_launch); keeps its tensors alive until finished."""

    def __init__(self, handle, n, keep=None):
        self.handle = handle
        self.n = n
        self.keep = keep
        self.codes = None

    def done(self):
        """True once the call's work has finished (does not block)."""
        if self.codes is not None:
            return True
        rc = chan_call_query(self.handle)
        if rc < 0:
            raise ChanError(rc, "chan_call_query")
        return rc == 0

    def _abandon(self):
        """Its batch is being destroyed (the library finishes the call and frees it)."""
        if self.codes is None:
            self.handle = None
            self.codes = [CHAN_EINVAL] * self.n
            self.keep = None

    def finish(self):
        """Wait for the call, apply its outcome to the envs and return the per-env codes."""
        if self.codes is None:
            res = (ctypes.c_int32 * self.n)()
            chan_call_finish(self.handle, res)
            self.handle = None
            self.codes = list(res)
            self.keep = None
        return self.codes


class ChanGraph:
    """A captured env step (ChanBatch.capture / ChanEnv.capture): launch() replays it and returns a
    ChanCall; keeps the captured tensors alive."""

    def __init__(self, handle, n, keep=None):
        self.handle = handle
        self.n = n
        self.keep = keep
        self._calls = weakref.WeakSet()

    def launch(self, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        rc, call = chan_graph_launch(self.handle, st.cuda_stream)
        if rc != CHAN_OK:
            raise ChanError(rc, "chan_graph_launch")
        c = ChanCall(call, self.n, keep=self.keep)
        self._calls.add(c)
        return c

    def _abandon_calls(self):
        """The library is about to finish this graph's replay in flight itself."""
        for c in list(self._calls):
            c._abandon()

    def close(self):
        if self.handle:
            self._abandon_calls()
            chan_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
