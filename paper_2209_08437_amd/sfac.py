"""Thin ctypes binding of libsfac.so (argument marshalling only; every step of the solve runs
in the library's HIP kernels). Names mirror the C ABI in include/sfac.h.

States are torch tensors on the GPU: contiguous, float64 or float32, shape (N_d, ..., N_1)
(axis 1 last, i.e. fastest). PyTorch provides device memory and streams only.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfac.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE, EBUDGET = range(6)
FP64, FP32 = 0, 1
METHOD_AUTO, METHOD_DIAG, METHOD_EMBED, METHOD_EXACT = 0, 1, 2, 3
FLAG_NONFINITE, FLAG_ABOVE_ONE = 1, 2
_STATUS = {0: "OK", 1: "EINVAL", 2: "EUNSUPPORTED", 3: "ENOMEM", 4: "EDEVICE", 5: "EBUDGET"}

EXPORTS = [
    "sfac_plan_create", "sfac_step", "sfac_plan_destroy", "sfac_plan_device_bytes",
    "sfac_plan_flags", "sfac_plan_reset_flags", "sfac_plan_method", "sfac_last_error",
    "sfac_batch_create", "sfac_batch_step", "sfac_batch_destroy", "sfac_batch_device_bytes",
    "sfac_axis_tables", "sfac_plan_time_passes", "sfac_group_create", "sfac_group_step",
    "sfac_group_destroy", "sfac_group_device_bytes", "sfac_batch_plan", "sfac_plan_energy",
    "sfac_plan_trace", "sfac_plan_read_trace", "sfac_exact_exponential", "sfac_solve_noalloc",
    "sfac_plan_time_fused",
]


class SfacError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32 * 3), ("use_graph", ctypes.c_int32),
                ("graph_chunk", ctypes.c_int32), ("elems_log2", ctypes.c_int32 * 3),
                ("lines_per_block", ctypes.c_int32 * 3), ("kernel", ctypes.c_int32 * 3)]


class InstanceDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("alpha", ctypes.c_double * 3),
                ("eps", ctypes.c_double), ("tau", ctypes.c_double), ("h", ctypes.c_double * 3)]


_lib = None


def lib():
    """Load libsfac.so (once). Raises if it has not been built: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2209_08437_amd.build_lib` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.sfac_plan_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i32), ctypes.POINTER(dbl),
                                   dbl, dbl, ctypes.POINTER(dbl), ctypes.c_int, vp, ctypes.POINTER(Options)]
    L.sfac_step.argtypes = [vp, vp, i64]
    L.sfac_plan_destroy.argtypes = [vp]
    L.sfac_plan_device_bytes.argtypes = [vp]
    L.sfac_plan_device_bytes.restype = ctypes.c_size_t
    L.sfac_plan_flags.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(dbl)]
    L.sfac_plan_reset_flags.argtypes = [vp]
    L.sfac_plan_method.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.sfac_last_error.restype = ctypes.c_char_p
    L.sfac_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(InstanceDesc), ctypes.c_int, vp,
                                    ctypes.POINTER(Options)]
    L.sfac_batch_step.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i64)]
    L.sfac_batch_destroy.argtypes = [vp]
    L.sfac_batch_device_bytes.argtypes = [vp]
    L.sfac_batch_device_bytes.restype = ctypes.c_size_t
    L.sfac_axis_tables.argtypes = [i32, dbl, dbl, dbl, dbl, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl),
                                   ctypes.POINTER(dbl), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.sfac_plan_time_passes.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_float)]
    L.sfac_plan_time_fused.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_float)]
    L.sfac_plan_energy.argtypes = [vp, vp, ctypes.POINTER(dbl)]
    L.sfac_plan_trace.argtypes = [vp, i64]
    L.sfac_exact_exponential.argtypes = [i32, dbl, dbl, dbl, dbl, ctypes.POINTER(dbl)]
    L.sfac_plan_read_trace.argtypes = [vp, ctypes.POINTER(dbl), i64, ctypes.POINTER(i64)]
    L.sfac_group_create.argtypes = [ctypes.POINTER(vp), vp]
    L.sfac_group_step.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64)]
    L.sfac_group_destroy.argtypes = [vp]
    L.sfac_group_device_bytes.argtypes = [vp]
    L.sfac_group_device_bytes.restype = ctypes.c_size_t
    L.sfac_batch_plan.argtypes = [vp, i32]
    L.sfac_batch_plan.restype = vp
    L.sfac_solve_noalloc.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(dbl), dbl, dbl, ctypes.POINTER(dbl),
                                     ctypes.c_int, vp, i64, vp, ctypes.POINTER(Options),
                                     ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(dbl)]
    L.sfac_solve_noalloc.restype = ctypes.c_int
    for name in ["sfac_group_create", "sfac_group_step", "sfac_group_destroy", "sfac_plan_time_passes", "sfac_plan_time_fused", "sfac_axis_tables", "sfac_plan_create", "sfac_step", "sfac_plan_destroy", "sfac_plan_flags",
                 "sfac_plan_reset_flags", "sfac_plan_method", "sfac_batch_create",
                 "sfac_batch_step", "sfac_batch_destroy", "sfac_plan_energy",
                 "sfac_plan_trace", "sfac_plan_read_trace", "sfac_exact_exponential"]:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != OK:
        msg = lib().sfac_last_error()
        raise SfacError(status, msg.decode() if msg else "")


def _dtype_code(dtype):
    if dtype in ("f64", "float64", FP64):
        return FP64
    if dtype in ("f32", "float32", FP32):
        return FP32
    try:
        import torch
        if dtype == torch.float64:
            return FP64
        if dtype == torch.float32:
            return FP32
    except ImportError:
        pass
    raise ValueError(f"unsupported dtype {dtype!r}")


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _check_state(u, shape, dt):
    import torch
    want = torch.float64 if dt == FP64 else torch.float32
    if not u.is_cuda:
        raise ValueError("state must be a GPU tensor")
    if u.dtype != want:
        raise ValueError(f"state dtype {u.dtype}, plan expects {want}")
    if tuple(u.shape) != tuple(shape):
        raise ValueError(f"state shape {tuple(u.shape)}, plan expects {tuple(shape)}")
    if not u.is_contiguous():
        raise ValueError("state must be contiguous")


TABLES_INCREMENT = 0x100


def axis_tables(n, alpha, eps, tau, h, method=None, increment=False):
    """Host-only: (length, scale_c, scale_s, radices) the library builds for one axis;
    increment=True gives the tables of the factors minus the identity (those FP32 plans use)."""
    import numpy as np
    codes = {None: METHOD_AUTO, "auto": METHOD_AUTO, "diag": METHOD_DIAG, "embed": METHOD_EMBED}
    L = lib()
    length = ctypes.c_int32()
    m = codes[method] | (TABLES_INCREMENT if increment else 0)
    _check(L.sfac_axis_tables(int(n), float(alpha), float(eps), float(tau), float(h), m,
                              ctypes.byref(length), None, None, None, None))
    sc = np.zeros(length.value)
    ss = np.zeros(length.value)
    rad = (ctypes.c_int32 * 12)()
    nst = ctypes.c_int32()
    dp = ctypes.POINTER(ctypes.c_double)
    _check(L.sfac_axis_tables(int(n), float(alpha), float(eps), float(tau), float(h), m,
                              ctypes.byref(length), sc.ctypes.data_as(dp), ss.ctypes.data_as(dp),
                              rad, ctypes.byref(nst)))
    return length.value, sc, ss, list(rad[: nst.value])


def exact_exponential(n, alpha, eps, tau, h):
    """e^{tau B} of one axis (host-only, FP64), an n x n numpy array."""
    import numpy as np
    out = np.zeros((n, n), dtype=np.float64)
    _check(lib().sfac_exact_exponential(int(n), float(alpha), float(eps), float(tau), float(h),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def fill_options(opt, dims, method=None, elems_log2=None, lines_per_block=None, kernel=None):
    """Write a kernel schedule into an Options struct: each argument is None (automatic), one
    value for every axis or a per-axis sequence (method: None, "auto", "diag", "embed" or
    "exact"; "exact" on every axis or none)."""
    def per_axis(v, a):
        return v[a] if isinstance(v, (list, tuple)) else v
    codes = {None: METHOD_AUTO, "auto": METHOD_AUTO, "diag": METHOD_DIAG, "embed": METHOD_EMBED,
             "exact": METHOD_EXACT}
    for a in range(3):
        opt.method[a] = codes[per_axis(method, a)] if a < dims else METHOD_AUTO
    for a in range(min(3, dims)):
        if elems_log2 is not None:
            opt.elems_log2[a] = int(per_axis(elems_log2, a) or 0)
        if lines_per_block is not None:
            opt.lines_per_block[a] = int(per_axis(lines_per_block, a) or 0)
        if kernel is not None:
            opt.kernel[a] = int(per_axis(kernel, a) or 0)
    return opt


def solve_noalloc(u, ns, alphas, eps, tau, hs, nsteps, dtype="f64", stream=None, method=None,
                  elems_log2=None, lines_per_block=None, kernel=None):
    """sfac_solve_noalloc: advance the GPU tensor u in place by nsteps steps without a plan and
    without device allocation; returns (flags, max_abs) of those steps (waits for the work)."""
    dims = len(ns)
    dt = _dtype_code(dtype)
    _check_state(u, tuple(reversed([int(n) for n in ns])), dt)
    opt = Options()
    fill_options(opt, dims, method=method, elems_log2=elems_log2, lines_per_block=lines_per_block, kernel=kernel)
    n_arr = (ctypes.c_int32 * dims)(*[int(n) for n in ns])
    a_arr = (ctypes.c_double * dims)(*[float(a) for a in alphas])
    h_arr = (ctypes.c_double * dims)(*[float(h) for h in hs])
    f = ctypes.c_uint32()
    m = ctypes.c_double()
    _check(lib().sfac_solve_noalloc(dims, n_arr, a_arr, float(eps), float(tau), h_arr, dt,
                                    ctypes.c_void_p(u.data_ptr()), int(nsteps), _stream_handle(stream),
                                    ctypes.byref(opt), ctypes.byref(f), ctypes.byref(m)))
    return f.value, m.value


class Plan:
    """sfac_plan_create / sfac_step / sfac_plan_destroy for one instance.

    ns, alphas, hs: per-axis sequences, axis 1 first. dtype: "f64" or "f32".
    method: None (automatic), "diag" or "embed" (one for all axes) or a per-axis sequence;
    "exact" (every axis, FP64) for the one-level scheme with the exact exponential.
    elems_log2, lines_per_block: kernel schedule per axis (None or 0 = automatic; see
    sfac_options in include/sfac.h and autotune.py)."""

    def __init__(self, ns, alphas, eps, tau, hs, dtype="f64", stream=None, method=None,
                 use_graph=True, graph_chunk=32, elems_log2=None, lines_per_block=None, kernel=None):
        L = lib()
        self.dims = len(ns)
        if not (len(alphas) == len(hs) == self.dims):
            raise ValueError("ns, alphas and hs must have one entry per axis")
        self.ns = tuple(int(n) for n in ns)
        self.dt = _dtype_code(dtype)
        opt = Options()
        fill_options(opt, self.dims, method=method, elems_log2=elems_log2, lines_per_block=lines_per_block,
                     kernel=kernel)
        opt.use_graph = 1 if use_graph else 0
        opt.graph_chunk = int(graph_chunk)
        n_arr = (ctypes.c_int32 * self.dims)(*self.ns)
        a_arr = (ctypes.c_double * self.dims)(*[float(a) for a in alphas])
        h_arr = (ctypes.c_double * self.dims)(*[float(h) for h in hs])
        self._h = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        _check(L.sfac_plan_create(ctypes.byref(self._h), self.dims, n_arr, a_arr, float(eps), float(tau),
                                  h_arr, self.dt, self._stream, ctypes.byref(opt)))

    @property
    def shape(self):
        return tuple(reversed(self.ns))

    def step(self, u, nsteps):
        """Advance the GPU tensor u in place by nsteps steps (asynchronous on the plan's stream)."""
        _check_state(u, self.shape, self.dt)
        _check(lib().sfac_step(self._h, ctypes.c_void_p(u.data_ptr()), int(nsteps)))
        return u

    def time_passes(self, u, reps):
        """Mean duration (ms) of each axis' pass kernel over `reps` steps (advances u)."""
        _check_state(u, self.shape, self.dt)
        ms = (ctypes.c_float * self.dims)()
        _check(lib().sfac_plan_time_passes(self._h, ctypes.c_void_p(u.data_ptr()), int(reps), ms))
        return list(ms)

    def time_fused(self, u, reps):
        """Mean duration (ms) of the launches that cover axis 1 and axis d twice (the last pass of
        a step with the first of the next), [axis 1, axis d]; 0 where the kernel does not fuse
        (advances u)."""
        _check_state(u, self.shape, self.dt)
        ms = (ctypes.c_float * 2)()
        _check(lib().sfac_plan_time_fused(self._h, ctypes.c_void_p(u.data_ptr()), int(reps), ms))
        return list(ms)

    def energy(self, u):
        """Discrete free energy of Sec. 5, Example 5 of the state u (only read); synchronizes the
        plan's stream."""
        _check_state(u, self.shape, self.dt)
        e = ctypes.c_double()
        _check(lib().sfac_plan_energy(self._h, ctypes.c_void_p(u.data_ptr()), ctypes.byref(e)))
        return e.value

    def trace(self, capacity):
        """Record max|u| after each of the next `capacity` steps (0 stops recording)."""
        _check(lib().sfac_plan_trace(self._h, int(capacity)))
        self._trace_cap = int(capacity)

    def read_trace(self):
        """(values recorded so far as a numpy array, steps counted since trace())."""
        import numpy as np
        cap = getattr(self, "_trace_cap", 0)
        out = (ctypes.c_double * max(cap, 1))()
        n = ctypes.c_int64()
        _check(lib().sfac_plan_read_trace(self._h, out, cap, ctypes.byref(n)))
        return np.array(out[:min(n.value, cap)], dtype=np.float64), n.value

    def flags(self):
        """(flags, max_abs) since the last reset; synchronizes the plan's stream."""
        f = ctypes.c_uint32()
        m = ctypes.c_double()
        _check(lib().sfac_plan_flags(self._h, ctypes.byref(f), ctypes.byref(m)))
        return f.value, m.value

    def reset_flags(self):
        _check(lib().sfac_plan_reset_flags(self._h))

    def method(self, axis):
        m = ctypes.c_int32()
        n = ctypes.c_int32()
        _check(lib().sfac_plan_method(self._h, int(axis), ctypes.byref(m), ctypes.byref(n)))
        return {METHOD_DIAG: "diag", METHOD_EMBED: "embed", METHOD_EXACT: "exact"}[m.value], n.value

    @property
    def device_bytes(self):
        return lib().sfac_plan_device_bytes(self._h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sfac_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Group:
    """sfac_group_create / sfac_group_step / sfac_group_destroy: step several plans together.
    Plans should be created on the same stream as the group."""

    def __init__(self, stream=None):
        self._h = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        _check(lib().sfac_group_create(ctypes.byref(self._h), self._stream))

    def step(self, plans, states, nsteps):
        """Advance states[i] with plans[i] by nsteps[i] steps (an int applies to all)."""
        n = len(plans)
        if len(states) != n:
            raise ValueError("one state per plan")
        if isinstance(nsteps, int):
            nsteps = [nsteps] * n
        for p, u in zip(plans, states):
            _check_state(u, p.shape, p.dt)
        hs = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
        ptrs = (ctypes.c_void_p * n)(*[u.data_ptr() for u in states])
        steps = (ctypes.c_int64 * n)(*[int(x) for x in nsteps])
        _check(lib().sfac_group_step(self._h, n, hs, ptrs, steps))
        return states

    @property
    def device_bytes(self):
        return lib().sfac_group_device_bytes(self._h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sfac_group_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """sfac_batch_create / sfac_batch_step / sfac_batch_destroy.

    instances: sequence of objects with ns, alphas, eps, tau, hs (e.g. workloads.Instance).
    schedules: None (automatic) or one entry per instance, each None or a dict with any of the
    keys method, elems_log2, lines_per_block, kernel (as for Plan; autotune.schedules returns
    them)."""

    def __init__(self, instances, dtype="f64", stream=None, schedules=None):
        L = lib()
        self.count = len(instances)
        self.dt = _dtype_code(dtype)
        opts = None
        if schedules is not None:
            if len(schedules) != self.count:
                raise ValueError("one schedule (or None) per instance")
            opts = (Options * self.count)()
            for i, (inst, sch) in enumerate(zip(instances, schedules)):
                fill_options(opts[i], len(inst.ns), **(sch or {}))
        arr = (InstanceDesc * self.count)()
        self.shapes = []
        for i, inst in enumerate(instances):
            d = arr[i]
            d.dims = len(inst.ns)
            for a in range(d.dims):
                d.n[a] = int(inst.ns[a])
                d.alpha[a] = float(inst.alphas[a])
                d.h[a] = float(inst.hs[a])
            d.eps = float(inst.eps)
            d.tau = float(inst.tau)
            self.shapes.append(tuple(reversed([int(n) for n in inst.ns])))
        self._h = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        _check(L.sfac_batch_create(ctypes.byref(self._h), self.count, arr, self.dt, self._stream, opts))

    def step(self, states, nsteps):
        """Advance states[i] by nsteps[i] steps (an int applies to all)."""
        if len(states) != self.count:
            raise ValueError("one state per instance")
        if isinstance(nsteps, int):
            nsteps = [nsteps] * self.count
        for u, shp in zip(states, self.shapes):
            _check_state(u, shp, self.dt)
        ptrs = (ctypes.c_void_p * self.count)(*[u.data_ptr() for u in states])
        steps = (ctypes.c_int64 * self.count)(*[int(s) for s in nsteps])
        _check(lib().sfac_batch_step(self._h, ptrs, steps))
        return states

    def reset_flags(self):
        """Clear every instance's sticky status (sfac_plan_reset_flags on each plan of the batch)."""
        for i in range(self.count):
            _check(lib().sfac_plan_reset_flags(lib().sfac_batch_plan(self._h, i)))

    def flags(self, i):
        """(flags, max_abs) of instance i; synchronizes the batch's stream."""
        h = lib().sfac_batch_plan(self._h, int(i))
        if not h:
            raise IndexError(i)
        f = ctypes.c_uint32()
        m = ctypes.c_double()
        _check(lib().sfac_plan_flags(ctypes.c_void_p(h), ctypes.byref(f), ctypes.byref(m)))
        return f.value, m.value

    @property
    def device_bytes(self):
        return lib().sfac_batch_device_bytes(self._h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sfac_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
