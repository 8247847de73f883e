"""ctypes binding of libdgmi.so: the C-ABI calls under the same names.

Argument marshalling only -- every step of the right-hand side, the RK stage
and the force integral runs in the library's HIP kernels.  torch is imported
first so that the library binds to the HIP runtime torch already loaded (one
runtime per process); device arrays are passed as torch tensors and their
data pointers, streams as torch streams or raw hipStream_t integers.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgmi.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EHIP, DG_EMESH, DG_EUNSUPPORTED, DG_ENONFINITE, DG_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
DG_FP64, DG_FP64_PERT, DG_FP32_PERT, DG_FP32_PERT_BF16OPS = 0, 1, 2, 3
DG_PENALTY_PAPER, DG_PENALTY_STANDARD = 0, 1
DG_WALL_ADIABATIC, DG_WALL_PRINTED = 0, 1

STATUS_NAMES = {0: "DG_OK", -1: "DG_EINVAL", -2: "DG_ENOMEM", -3: "DG_EHIP", -4: "DG_EMESH",
                -5: "DG_EUNSUPPORTED", -6: "DG_ENONFINITE", -7: "DG_ESTATE"}

# exported symbol -> (restype, argtypes)
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_L = ctypes.c_int64
_DP = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "dg_create": (_I, [_I, _I, ctypes.POINTER(_P)]),
    "dg_set_physics": (_I, [_P, _D, _D, _D, _D, _I, _D, _DP]),
    "dg_set_wall_flux": (_I, [_P, _I]),
    "dg_set_curved_elements": (_I, [_P, _L, ctypes.POINTER(ctypes.c_int32), _DP]),
    "dg_batch_rk_step_states": (_I, [_P, _P, _P, _DP, _DP, _P]),
    "dg_mlp_set_schedule": (_I, [_P, _I]),
    "dg_set_mesh": (_I, [_P, _L, _DP, _DP, _L, ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int8), _DP]),
    "dg_setup_host": (_I, [_P]),
    "dg_setup": (_I, [_P]),
    "dg_num_elements": (_L, [_P]),
    "dg_num_nodes": (_I, [_P]),
    "dg_num_face_nodes": (_I, [_P]),
    "dg_get_host_table": (_I, [_P, ctypes.c_char_p, _DP, _L]),
    "dg_set_overintegration": (_I, [_P, _I]),
    "dg_get_nodes": (_I, [_P, _DP, _DP]),
    "dg_rhs": (_I, [_P, _P, _P, _DP, _P]),
    "dg_rk_step": (_I, [_P, _P, _P, _D, _DP, _P]),
    "dg_rk_steps": (_I, [_P, _P, _P, _I, _D, _DP, _P, _P]),
    "dg_rk_steps_noalloc": (_I, [_P, _P, _P, _I, _D, _DP, _P, _P]),
    "dg_rk_stage": (_I, [_P, _P, _P, _P, _D, _D, _D, _DP, _P]),
    "dg_force": (_I, [_P, _P, _DP, _DP, _P]),
    "dg_force_device": (_I, [_P, _P, _DP, _P, _P]),
    "dg_cfl_time_step": (_I, [_P, _P, _DP, _D, _D, _DP, _P]),
    "dg_newmark_step": (_I, [_DP, _D, _D, _D, _D, _D]),
    "dg_set_tuning": (_I, [_P, _I, _I]),
    "dg_get_tuning": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "dg_autotune": (_I, [_P, _P, _I, ctypes.c_char_p, _P, _DP]),
    "dg_batch_create": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(_P)]),
    "dg_batch_set_state": (_I, [_P, _I, _P, _P]),
    "dg_batch_get_state": (_I, [_P, _I, _P, _P]),
    "dg_batch_rk_step": (_I, [_P, _DP, _DP, _P]),
    "dg_batch_force": (_I, [_P, _DP, _DP, _P]),
    "dg_batch_coupled_step": (_I, [_P, _DP, _DP, _DP, _DP, _DP, _P]),
    "dg_batch_get_config": (_I, [_P] + [ctypes.POINTER(_I)] * 4),
    "dg_batch_configure": (_I, [_P, _I, _I, _I, _I]),
    "dg_batch_autotune": (_I, [_P, _I, _P, _DP]),
    "dg_batch_last_error": (ctypes.c_char_p, [_P]),
    "dg_batch_destroy": (None, [_P]),
    "dg_mlp_create": (_I, [_I, _I, _I, _L, ctypes.POINTER(_P)]),
    "dg_mlp_num_params": (_L, [_P]),
    "dg_mlp_set_params": (_I, [_P, ctypes.POINTER(ctypes.c_float), _L]),
    "dg_mlp_get_params": (_I, [_P, ctypes.POINTER(ctypes.c_float), _L]),
    "dg_mlp_get_grad": (_I, [_P, ctypes.POINTER(ctypes.c_float), _L]),
    "dg_mlp_set_normalization": (_I, [_P] + [ctypes.POINTER(ctypes.c_float)] * 4),
    "dg_mlp_forward": (_I, [_P, _P, _L, _L, _P, _L, _P]),
    "dg_mlp_backward": (_I, [_P, _P, _L, _P, _L, _L, _DP, _P]),
    "dg_mlp_adam": (_I, [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
    "dg_mlp_last_error": (ctypes.c_char_p, [_P]),
    "dg_mlp_destroy": (None, [_P]),
    "dg_column_stats": (_I, [_P, _L, _L, _I, _DP, _DP, _P]),
    "dg_closure_create": (_I, [_P, _P, ctypes.POINTER(_P)]),
    "dg_closure_sizes": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "dg_closure_features": (_I, [_P, _P, _I, _P, _L, _P]),
    "dg_closure_targets": (_I, [_P, _P, _P, _L, _P]),
    "dg_closure_apply": (_I, [_P, _P, _P, _P, _L, _P, _P]),
    "dg_closure_restrict": (_I, [_P, _P, _P, _P]),
    "dg_closure_drift_targets": (_I, [_P, _P, _P, _P, _L, _P]),
    "dg_closure_correct": (_I, [_P, _P, _P, _L, _P, _P]),
    "dg_closure_last_error": (ctypes.c_char_p, [_P]),
    "dg_closure_destroy": (None, [_P]),
    "dg_last_error": (ctypes.c_char_p, [_P]),
    "dg_destroy": (None, [_P]),
}

_lib = None


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


def load():
    """Load the library (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (binds the library to torch's HIP runtime)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdgmi.so is not built; run `python -m paper_2508_17917_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    _check_single_hip_runtime()
    return lib


def _check_single_hip_runtime():
    try:
        with open("/proc/self/maps") as fh:
            paths = {line.split()[-1] for line in fh if "libamdhip64" in line}
    except OSError:
        return
    real = {os.path.realpath(p) for p in paths}
    if len(real) > 1:
        raise RuntimeError("two HIP runtimes are mapped in this process: %s" % sorted(real))


def _dp(a):
    return a.ctypes.data_as(_DP)


def _check(code, handle=None):
    if code != DG_OK:
        msg = load().dg_last_error(handle)
        raise DGError(code, msg.decode() if msg else "")
    return code


# ---- argument checks --------------------------------------------------------
# Every device array is checked on the host before its address reaches the
# library: a tensor of the wrong type, on the host, non-contiguous or too short
# would make a kernel read or write outside it.
def _dtype(name):
    import torch
    return {"f64": torch.float64, "f32": torch.float32}[name]


def _dev(t, dtype, count, what, optional=False):
    """Address of a device array: a GPU tensor of `dtype` ("f64"/"f32"),
    contiguous, with at least `count` elements (ValueError otherwise)."""
    if t is None:
        if optional:
            return None
        raise ValueError("%s: a device array is required" % what)
    if not hasattr(t, "data_ptr") or not getattr(t, "is_cuda", False):
        raise ValueError("%s must be a GPU tensor" % what)
    if t.dtype != _dtype(dtype):
        raise ValueError("%s must be %s, got %s" % (what, _dtype(dtype), t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.numel() < count:
        raise ValueError("%s has %d elements, the call needs %d" % (what, t.numel(), count))
    return ctypes.c_void_p(t.data_ptr())


def _rows(t, rows, cols, what, dtype="f32"):
    """(address, row stride) of a 2-D device array of at least `rows` rows of
    at least `cols` contiguous values (ValueError otherwise)."""
    if t is None or not hasattr(t, "data_ptr") or not getattr(t, "is_cuda", False):
        raise ValueError("%s must be a GPU tensor" % what)
    if t.dtype != _dtype(dtype):
        raise ValueError("%s must be %s, got %s" % (what, _dtype(dtype), t.dtype))
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("%s must be a 2-D array with contiguous rows" % what)
    if t.shape[0] < rows or t.shape[1] < cols:
        raise ValueError("%s has shape %s, the call needs at least (%d, %d)"
                         % (what, tuple(t.shape), rows, cols))
    return ctypes.c_void_p(t.data_ptr()), t.stride(0)


def state_len(h):
    """Values of one state [K][4][Np] of context h."""
    return dg_num_elements(h) * 4 * dg_num_nodes(h)


def _st(h, t, what):
    return _dev(t, "f64", state_len(h), what)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _vw(v_w):
    return np.ascontiguousarray(np.asarray(v_w if v_w is not None else (0.0, 0.0), dtype=np.float64))


# ---- the C-ABI calls ------------------------------------------------------
def dg_set_overintegration(h, on):
    return _check(load().dg_set_overintegration(h, 1 if on else 0), h)


def dg_create(p, precision=DG_FP64):
    h = ctypes.c_void_p()
    _check(load().dg_create(int(p), int(precision), ctypes.byref(h)))
    return h


def dg_set_physics(h, gamma, Pr, mu, theta, penalty_mode, C_pen, U_inf):
    u = np.ascontiguousarray(np.asarray(U_inf, dtype=np.float64))
    return _check(load().dg_set_physics(h, gamma, Pr, mu, theta, int(penalty_mode), C_pen, _dp(u)), h)


def dg_set_wall_flux(h, mode):
    return _check(load().dg_set_wall_flux(h, int(mode)), h)


def dg_set_mesh(h, VX, VY, EToV, face_tag=None, period=(0.0, 0.0)):
    VX = np.ascontiguousarray(np.asarray(VX, dtype=np.float64))
    VY = np.ascontiguousarray(np.asarray(VY, dtype=np.float64))
    E = np.ascontiguousarray(np.asarray(EToV, dtype=np.int32))
    K = E.shape[0]
    ft = None if face_tag is None else np.ascontiguousarray(np.asarray(face_tag, dtype=np.int8))
    per = np.ascontiguousarray(np.asarray(period, dtype=np.float64))
    return _check(load().dg_set_mesh(
        h, VX.size, _dp(VX), _dp(VY), K, E.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        None if ft is None else ft.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), _dp(per)), h)


def dg_set_curved_elements(h, elems, xy):
    """Isoparametric elements: indices (n,) and node positions (n, 2, Np),
    x then y per element in the library's node order (host arrays)."""
    E = np.ascontiguousarray(np.asarray(elems, dtype=np.int32).ravel())
    n = E.size
    X = np.ascontiguousarray(np.asarray(xy, dtype=np.float64))
    if n and X.ndim != 3:
        raise ValueError("xy must have shape (n, 2, Np)")
    if n and (X.shape[0] != n or X.shape[1] != 2):
        raise ValueError("xy has shape %s for %d elements" % (X.shape, n))
    if n and X.shape[2] != load().dg_num_nodes(h):
        raise ValueError("xy has %d nodes per element, the context's order %d"
                         % (X.shape[2], load().dg_num_nodes(h)))
    return _check(load().dg_set_curved_elements(
        h, n, E.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if n else None,
        _dp(X) if n else None), h)


def dg_setup_host(h):
    return _check(load().dg_setup_host(h), h)


def dg_setup(h):
    return _check(load().dg_setup(h), h)


def dg_num_elements(h):
    return int(load().dg_num_elements(h))


def dg_num_nodes(h):
    return int(load().dg_num_nodes(h))


def dg_num_face_nodes(h):
    return int(load().dg_num_face_nodes(h))


def dg_get_host_table(h, name, count):
    out = np.zeros(int(count))
    _check(load().dg_get_host_table(h, name.encode(), _dp(out), int(count)), h)
    return out


def dg_get_nodes(h):
    n = dg_num_elements(h) * dg_num_nodes(h)
    x, y = np.zeros(n), np.zeros(n)
    _check(load().dg_get_nodes(h, _dp(x), _dp(y)), h)
    return x, y


def dg_rhs(h, U, R, v_w=(0.0, 0.0), stream=None):
    vw = _vw(v_w)
    return _check(load().dg_rhs(h, _st(h, U, "U"), _st(h, R, "R"), _dp(vw), _stream(stream)), h)


def dg_rk_step(h, U, K1, dt, v_w=(0.0, 0.0), stream=None):
    vw = _vw(v_w)
    return _check(load().dg_rk_step(h, _st(h, U, "U"), _st(h, K1, "K1"), float(dt), _dp(vw),
                                    _stream(stream)), h)


def dg_rk_steps(h, U, K1, nsteps, dt, v_w=(0.0, 0.0), force=None, stream=None):
    vw = _vw(v_w)
    nsteps = int(nsteps)
    f = _dev(force, "f64", 3 * max(nsteps, 0), "force", optional=True)
    return _check(load().dg_rk_steps(h, _st(h, U, "U"), _st(h, K1, "K1"), nsteps, float(dt),
                                     _dp(vw), f, _stream(stream)), h)


def dg_rk_steps_noalloc(h, U, K1, nsteps, dt, v_w=(0.0, 0.0), force=None, stream=None):
    vw = _vw(v_w)
    nsteps = int(nsteps)
    f = _dev(force, "f64", 3 * max(nsteps, 0), "force", optional=True)
    return _check(load().dg_rk_steps_noalloc(h, _st(h, U, "U"), _st(h, K1, "K1"), nsteps,
                                             float(dt), _dp(vw), f, _stream(stream)), h)


def dg_rk_stage(h, U_in, U_out, K1, a, b, dt, v_w=(0.0, 0.0), stream=None):
    vw = _vw(v_w)
    return _check(load().dg_rk_stage(h, _st(h, U_in, "U_in"), _st(h, U_out, "U_out"),
                                     _st(h, K1, "K1"), float(a), float(b), float(dt), _dp(vw),
                                     _stream(stream)), h)


def dg_force(h, U, v_w=(0.0, 0.0), stream=None):
    vw = _vw(v_w)
    out = np.zeros(3)
    _check(load().dg_force(h, _st(h, U, "U"), _dp(vw), _dp(out), _stream(stream)), h)
    return out


def dg_force_device(h, U, out, v_w=(0.0, 0.0), stream=None):
    vw = _vw(v_w)
    return _check(load().dg_force_device(h, _st(h, U, "U"), _dp(vw), _dev(out, "f64", 3, "out"),
                                         _stream(stream)), h)


def dg_cfl_time_step(h, U, v_w=(0.0, 0.0), C_cfl=1.0, C_grad=1.0, stream=None):
    vw = _vw(v_w)
    out = np.zeros(2)
    _check(load().dg_cfl_time_step(h, _st(h, U, "U"), _dp(vw), C_cfl, C_grad, _dp(out),
                                   _stream(stream)), h)
    return float(out[0]), float(out[1])


def dg_newmark_step(state, F_new, dt, M, C, K):
    st = np.ascontiguousarray(np.asarray(state, dtype=np.float64).copy())
    code = load().dg_newmark_step(_dp(st), float(F_new), float(dt), float(M), float(C), float(K))
    if code != DG_OK:
        raise DGError(code, "invalid Newmark arguments")
    return st


def dg_last_error(h):
    msg = load().dg_last_error(h)
    return msg.decode() if msg else ""


def dg_destroy(h):
    if h is not None and h.value:
        load().dg_destroy(h)


def dg_set_tuning(h, waves, grid):
    return _check(load().dg_set_tuning(h, int(waves), int(grid)), h)


def dg_get_tuning(h):
    w, g = ctypes.c_int(), ctypes.c_int()
    _check(load().dg_get_tuning(h, ctypes.byref(w), ctypes.byref(g)), h)
    return w.value, g.value


def dg_autotune(h, U, reps=20, cache_path=None, stream=None):
    best = ctypes.c_double()
    _check(load().dg_autotune(h, _st(h, U, "U"), int(reps),
                              None if cache_path is None else os.fsencode(cache_path),
                              _stream(stream), ctypes.byref(best)), h)
    return best.value


# ---- batches --------------------------------------------------------------
def _bcheck(code, b=None):
    if code != DG_OK:
        msg = load().dg_batch_last_error(b)
        raise DGError(code, msg.decode() if msg else "")
    return code


# state lengths of each batch's instances, for the argument checks
_BATCH_STATES = {}


def dg_batch_create(handles):
    arr = (ctypes.c_void_p * len(handles))(*[h.value for h in handles])
    b = ctypes.c_void_p()
    _bcheck(load().dg_batch_create(arr, len(handles), ctypes.byref(b)))
    _BATCH_STATES[b.value] = [state_len(h) for h in handles]
    return b


def _batch_state(b, i, U):
    sizes = _BATCH_STATES.get(b.value)
    if sizes is None or not 0 <= int(i) < len(sizes):
        raise ValueError("instance %s is not in the batch" % i)
    return _dev(U, "f64", sizes[int(i)], "U")


def dg_batch_set_state(b, i, U, stream=None):
    return _bcheck(load().dg_batch_set_state(b, int(i), _batch_state(b, i, U), _stream(stream)), b)


def dg_batch_get_state(b, i, U, stream=None):
    return _bcheck(load().dg_batch_get_state(b, int(i), _batch_state(b, i, U), _stream(stream)), b)


def dg_batch_rk_step(b, dt, v_w, stream=None):
    dt = np.ascontiguousarray(np.asarray(dt, dtype=np.float64))
    vw = np.ascontiguousarray(np.asarray(v_w, dtype=np.float64).reshape(-1))
    return _bcheck(load().dg_batch_rk_step(b, _dp(dt), _dp(vw), _stream(stream)), b)


def dg_batch_rk_step_states(b, U, K1, dt, v_w, stream=None):
    """One step on caller-owned states: U, K1 lists of device arrays, one per
    instance (the instance's [K][4][Np] FP64 size)."""
    sizes = _BATCH_STATES.get(b.value)
    if sizes is None:
        raise ValueError("not a live batch")
    n = len(sizes)
    if len(U) != n or len(K1) != n:
        raise ValueError("U and K1 need one array per instance (%d)" % n)
    ua = (ctypes.c_void_p * n)(*[_dev(u, "f64", sizes[i], "U[%d]" % i).value for i, u in enumerate(U)])
    ka = (ctypes.c_void_p * n)(*[_dev(k, "f64", sizes[i], "K1[%d]" % i).value for i, k in enumerate(K1)])
    dt = np.ascontiguousarray(np.asarray(dt, dtype=np.float64))
    vw = np.ascontiguousarray(np.asarray(v_w, dtype=np.float64).reshape(-1))
    if dt.size != n or vw.size != 2 * n:
        raise ValueError("dt needs %d values and v_w %d" % (n, 2 * n))
    return _bcheck(load().dg_batch_rk_step_states(b, ua, ka, _dp(dt), _dp(vw), _stream(stream)), b)


def dg_batch_force(b, n, v_w=None, stream=None):
    vw = np.zeros(2 * n) if v_w is None else np.ascontiguousarray(
        np.asarray(v_w, dtype=np.float64).reshape(-1))
    out = np.zeros(3 * n)
    _bcheck(load().dg_batch_force(b, _dp(vw), _dp(out), _stream(stream)), b)
    return out.reshape(n, 3)


def dg_batch_coupled_step(b, osc, body, F, dt, stream=None):
    """Newmark under the lifts in F, one batch RK step, new forces; body (n x 3)
    and F (n x 3) are float64 C-contiguous arrays updated in place.  Returns
    the wall velocities (n x 2) used for the step."""
    n = body.shape[0]
    for name, a, shape in (("body", body, (n, 3)), ("F", F, (n, 3))):
        if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.shape == shape
                and a.flags.c_contiguous):
            raise ValueError("%s must be a C-contiguous float64 array of shape %s" % (name, shape))
    o = np.ascontiguousarray(np.asarray(osc, dtype=np.float64).reshape(n, 4))
    d = np.ascontiguousarray(np.asarray(dt, dtype=np.float64).reshape(n))
    vw = np.zeros((n, 2))
    _bcheck(load().dg_batch_coupled_step(b, _dp(o), _dp(body), _dp(F), _dp(d), _dp(vw),
                                         _stream(stream)), b)
    return vw


def dg_batch_get_config(b):
    """(mode, waves, grid, use_graph) of the batch's current launch shape."""
    v = [ctypes.c_int() for _ in range(4)]
    _bcheck(load().dg_batch_get_config(b, *[ctypes.byref(x) for x in v]), b)
    return tuple(x.value for x in v)


def dg_batch_configure(b, mode=0, waves=0, grid=0, use_graph=1):
    return _bcheck(load().dg_batch_configure(b, int(mode), int(waves), int(grid), int(use_graph)), b)


def dg_batch_autotune(b, reps=10, stream=None):
    best = ctypes.c_double()
    _bcheck(load().dg_batch_autotune(b, int(reps), _stream(stream), ctypes.byref(best)), b)
    return best.value


def dg_batch_last_error(b):
    msg = load().dg_batch_last_error(b)
    return msg.decode() if msg else ""


def dg_batch_destroy(b):
    if b is not None and b.value:
        _BATCH_STATES.pop(b.value, None)
        load().dg_batch_destroy(b)


# ---- learned closure --------------------------------------------------------
_FP = ctypes.POINTER(ctypes.c_float)


def _fp(a):
    return a.ctypes.data_as(_FP)


def _mcheck(code, m=None):
    if code != DG_OK:
        msg = load().dg_mlp_last_error(m)
        raise DGError(code, msg.decode() if msg else "")
    return code


def _ccheck(code, c=None):
    if code != DG_OK:
        msg = load().dg_closure_last_error(c)
        raise DGError(code, msg.decode() if msg else "")
    return code


# (n_in, n_out) of each network, for the argument checks
_MLP_SIZES = {}


def dg_mlp_create(n_in, n_hidden, n_out, max_batch):
    m = ctypes.c_void_p()
    _mcheck(load().dg_mlp_create(int(n_in), int(n_hidden), int(n_out), int(max_batch),
                                 ctypes.byref(m)))
    _MLP_SIZES[m.value] = (int(n_in), int(n_out))
    return m


def _mlp_sizes(m):
    if m is None or m.value not in _MLP_SIZES:
        raise ValueError("not a network created by dg_mlp_create")
    return _MLP_SIZES[m.value]


def dg_mlp_num_params(m):
    return int(load().dg_mlp_num_params(m))


def dg_mlp_set_params(m, params):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    return _mcheck(load().dg_mlp_set_params(m, _fp(p), p.size), m)


def dg_mlp_get_params(m):
    out = np.zeros(dg_mlp_num_params(m), dtype=np.float32)
    _mcheck(load().dg_mlp_get_params(m, _fp(out), out.size), m)
    return out


def dg_mlp_get_grad(m):
    out = np.zeros(dg_mlp_num_params(m), dtype=np.float32)
    _mcheck(load().dg_mlp_get_grad(m, _fp(out), out.size), m)
    return out


def dg_mlp_set_normalization(m, in_mean, in_std, out_mean, out_std):
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float32))
            for a in (in_mean, in_std, out_mean, out_std)]
    return _mcheck(load().dg_mlp_set_normalization(m, *[_fp(a) for a in arrs]), m)


def dg_mlp_forward(m, X, Y, B=None, stream=None):
    n_in, n_out = _mlp_sizes(m)
    B = X.shape[0] if B is None else int(B)
    x, ldx = _rows(X, B, n_in, "X")
    y, ldy = _rows(Y, B, n_out, "Y")
    return _mcheck(load().dg_mlp_forward(m, x, ldx, B, y, ldy, _stream(stream)), m)


def dg_mlp_set_schedule(m, fused):
    """1: the fused training kernel where built (default); 0: layer by layer."""
    return _mcheck(load().dg_mlp_set_schedule(m, int(fused)), m)


def dg_mlp_backward(m, X, T, B=None, want_loss=True, stream=None):
    n_in, n_out = _mlp_sizes(m)
    B = X.shape[0] if B is None else int(B)
    x, ldx = _rows(X, B, n_in, "X")
    t, ldt = _rows(T, B, n_out, "T")
    loss = ctypes.c_double()
    _mcheck(load().dg_mlp_backward(m, x, ldx, t, ldt, B,
                                   ctypes.byref(loss) if want_loss else None, _stream(stream)), m)
    return loss.value if want_loss else None


def dg_mlp_adam(m, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    return _mcheck(load().dg_mlp_adam(m, float(lr), float(beta1), float(beta2), float(eps),
                                      _stream(stream)), m)


def dg_mlp_last_error(m):
    msg = load().dg_mlp_last_error(m)
    return msg.decode() if msg else ""


def dg_mlp_destroy(m):
    if m is not None and m.value:
        _MLP_SIZES.pop(m.value, None)
        load().dg_mlp_destroy(m)


def dg_column_stats(A, cols=None, rows=None, stream=None):
    rows = A.shape[0] if rows is None else int(rows)
    cols = A.shape[1] if cols is None else int(cols)
    a, lda = _rows(A, rows, cols, "A")
    mean, std = np.zeros(cols), np.zeros(cols)
    code = load().dg_column_stats(a, rows, lda, cols, _dp(mean), _dp(std), _stream(stream))
    if code != DG_OK:
        raise DGError(code, "dg_column_stats failed")
    return mean, std


# (K, state length lo, state length hi, n_features, n_targets) of each
# closure, for the argument checks
_CLOSURE_SIZES = {}


def dg_closure_create(lo, hi):
    c = ctypes.c_void_p()
    _ccheck(load().dg_closure_create(lo, hi, ctypes.byref(c)))
    nf, nt = dg_closure_sizes(c)
    _CLOSURE_SIZES[c.value] = (dg_num_elements(hi), state_len(lo), state_len(hi), nf, nt)
    return c


def _closure_sizes(c):
    if c is None or c.value not in _CLOSURE_SIZES:
        raise ValueError("not a closure created by dg_closure_create")
    return _CLOSURE_SIZES[c.value]


def dg_closure_sizes(c):
    a, b = ctypes.c_int(), ctypes.c_int()
    _ccheck(load().dg_closure_sizes(c, ctypes.byref(a), ctypes.byref(b)), c)
    return a.value, b.value


def dg_closure_features(c, U, X, from_hi, stream=None):
    """from_hi: 1 an order-hi state (restricted), 0 an order-lo state, 2 the
    free stream (U unused, may be None)."""
    K, s_lo, s_hi, nf, _ = _closure_sizes(c)
    mode = int(from_hi)
    if mode not in (0, 1, 2):
        raise ValueError("from_hi must be 0, 1 or 2")
    u = None if mode == 2 else _dev(U, "f64", s_hi if mode == 1 else s_lo, "U")
    x, ldx = _rows(X, K, nf, "X")
    return _ccheck(load().dg_closure_features(c, u, mode, x, ldx, _stream(stream)), c)


def dg_closure_targets(c, U_hi, T, stream=None):
    K, _, s_hi, _, nt = _closure_sizes(c)
    t, ldt = _rows(T, K, nt, "T")
    return _ccheck(load().dg_closure_targets(c, _dev(U_hi, "f64", s_hi, "U_hi"), t, ldt,
                                             _stream(stream)), c)


def dg_closure_restrict(c, U_hi, U_lo, stream=None):
    _, s_lo, s_hi, _, _ = _closure_sizes(c)
    return _ccheck(load().dg_closure_restrict(c, _dev(U_hi, "f64", s_hi, "U_hi"),
                                              _dev(U_lo, "f64", s_lo, "U_lo"), _stream(stream)), c)


def _rows_like(Y0, ldy, K, n, what):
    """Y0 with the same row stride as Y (or None)."""
    if Y0 is None:
        return None
    y0, ld0 = _rows(Y0, K, n, what)
    if ld0 != ldy:
        raise ValueError("%s must have the row stride of Y" % what)
    return y0


def dg_closure_apply(c, U_lo, Y, U_hi, Y0=None, stream=None):
    K, s_lo, s_hi, _, nt = _closure_sizes(c)
    y, ldy = (None, 0) if Y is None else _rows(Y, K, nt, "Y")
    if Y is None and Y0 is not None:
        raise ValueError("Y0 needs Y")
    y0 = _rows_like(Y0, ldy, K, nt, "Y0")
    return _ccheck(load().dg_closure_apply(c, _dev(U_lo, "f64", s_lo, "U_lo"), y, y0, ldy,
                                           _dev(U_hi, "f64", s_hi, "U_hi"), _stream(stream)), c)


def dg_closure_drift_targets(c, U_ref, U_lo, T, stream=None):
    K, s_lo, _, nf, _ = _closure_sizes(c)
    t, ldt = _rows(T, K, nf - 4, "T")
    return _ccheck(load().dg_closure_drift_targets(c, _dev(U_ref, "f64", s_lo, "U_ref"),
                                                   _dev(U_lo, "f64", s_lo, "U_lo"), t, ldt,
                                                   _stream(stream)), c)


def dg_closure_correct(c, Y, U_lo, Y0=None, stream=None):
    K, s_lo, _, nf, _ = _closure_sizes(c)
    y, ldy = _rows(Y, K, nf - 4, "Y")
    y0 = _rows_like(Y0, ldy, K, nf - 4, "Y0")
    return _ccheck(load().dg_closure_correct(c, y, y0, ldy, _dev(U_lo, "f64", s_lo, "U_lo"),
                                             _stream(stream)), c)


def dg_closure_last_error(c):
    msg = load().dg_closure_last_error(c)
    return msg.decode() if msg else ""


def dg_closure_destroy(c):
    if c is not None and c.value:
        _CLOSURE_SIZES.pop(c.value, None)
        load().dg_closure_destroy(c)
