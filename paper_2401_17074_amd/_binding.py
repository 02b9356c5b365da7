"""ctypes binding of libtslb.so (include/tslb.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own: torch tensors supply device memory (their data
pointers) and streams (``torch.cuda.current_stream().cuda_stream``).  If the
HIP library has not been built, importing this module raises ImportError;
there is no fallback path.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtslb.so")

TSLB_D3Q27, TSLB_D3Q19, TSLB_D2Q9 = 27, 19, 9
TSLB_FP32, TSLB_FP16, TSLB_BF16 = 0, 1, 2
TSLB_PERIODIC, TSLB_WALL, TSLB_INLET, TSLB_OUTLET = 0, 1, 2, 3
TSLB_DEVICE, TSLB_RHO_DEVIATION = 1, 2
TSLB_OBJ_KINETIC_ENERGY, TSLB_OBJ_WALL_SHEAR = 0, 1
TSLB_STATS_PROFILE, TSLB_STATS_FIELD = 1, 2
TSLB_REDUCE_VALUES, TSLB_NOALLOC_REDUCE_BLOCKS = 7, 1024
TSLB_OK, TSLB_E_INVALID, TSLB_E_UNSUPPORTED, TSLB_E_NOMEM, TSLB_E_HIP, TSLB_E_UNSTABLE = 0, -1, -2, -3, -4, -5

# every symbol include/tslb.h declares, with (restype, argtypes)
_vp, _i, _f, _d, _sz, _i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double, ctypes.c_size_t, \
    ctypes.c_int64
_fp = ctypes.POINTER(ctypes.c_float)


class tslb_bc(ctypes.Structure):
    _fields_ = [
        ("face", ctypes.c_int * 6),
        ("inlet_u", ctypes.c_float * 3),
        ("inlet_center", ctypes.c_float * 2),
        ("inlet_radius", ctypes.c_float),
        ("inlet_noise", ctypes.c_float),
        ("seed", ctypes.c_uint64),
        ("storage", ctypes.c_int),
        ("scale", ctypes.c_float * 3),
        ("order", ctypes.c_int),
        ("inlet_noise_kind", ctypes.c_int),
    ]


SIGNATURES = {
    "tslb_create": (_i, [_i, _i, _i, _i, _f, _fp, ctypes.POINTER(tslb_bc), ctypes.POINTER(_vp)]),
    "tslb_destroy": (_i, [_vp]),
    "tslb_set_moments": (_i, [_vp, _vp, _vp, _vp, _i, _vp]),
    "tslb_get_moments": (_i, [_vp, _vp, _vp, _vp, _i, _vp]),
    "tslb_set_force_field": (_i, [_vp, _vp, _vp]),
    "tslb_step": (_i, [_vp, _i, _vp]),
    "tslb_bind_state": (_i, [_vp, _vp, _vp, _vp]),
    "tslb_objective": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_double), _vp]),
    "tslb_stats_begin": (_i, [_vp, _i, _i, _vp]),
    "tslb_stats_sample": (_i, [_vp, _vp]),
    "tslb_stats_profile": (_i, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), _vp]),
    "tslb_stats_field": (_i, [_vp, _vp, _vp, _vp]),
    "tslb_stats_jet": (_i, [_vp, _i, _fp, _vp, _vp, _vp]),
    "tslb_set_relaxation_profile": (_i, [_vp, _fp, _vp]),
    "tslb_step_timed": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_double), _vp]),
    "tslb_get_time": (_i64, [_vp]),
    "tslb_set_time": (_i, [_vp, _i64]),
    "tslb_reduce": (_i, [_vp, ctypes.POINTER(_d), _vp]),
    "tslb_reduce_noalloc": (_i, [_vp, _vp, _vp]),
    "tslb_state_bytes": (_sz, [_vp]),
    "tslb_save_state": (_i, [_vp, _vp, _vp]),
    "tslb_load_state": (_i, [_vp, _vp, _vp]),
    "tslb_adjoint_step": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tslb_adjoint_seed": (_i, [_vp, _vp, _i, _vp, _vp]),
    "tslb_rollout_workspace_bytes": (_sz, [_vp, _i, _i]),
    "tslb_rollout_forward": (_i, [_vp, _i, _i, _vp, _sz, _vp]),
    "tslb_rollout_backward": (_i, [_vp, _i, _i, _vp, _sz, _vp, _vp, _vp]),
    "tslb_set_kernel": (_i, [_vp, _i]),
    "tslb_stream_copy": (_i, [_vp, _vp, _sz, _vp]),
    "tslb_last_error": (ctypes.c_char_p, []),
}

if not os.path.exists(LIB_PATH):
    raise ImportError("libtslb.so is not built (run __graft_entry__.build()); there is no fallback path")

# torch first: it loads the HIP runtime the library then binds to, so that
# both use one runtime instance (torch carries its own copy of it)
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)
for _name, (_res, _args) in SIGNATURES.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class TslbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tslb error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != TSLB_OK:
        raise TslbError(rc, lib.tslb_last_error().decode())
    return rc


def _ptr(t):
    """Device (or host) address of a tensor, None for None."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def make_bc(faces=(0,) * 6, inlet_u=(0.0, 0.0, 0.0), inlet_center=(0.0, 0.0), inlet_radius=0.0, inlet_noise=0.0,
            seed=0, storage=TSLB_FP32, scale=(0.0, 0.0, 0.0), order=3, inlet_noise_kind=0):
    b = tslb_bc()
    for k in range(6):
        b.face[k] = faces[k]
    for a in range(3):
        b.inlet_u[a] = inlet_u[a]
        b.scale[a] = scale[a]
    b.inlet_center[0], b.inlet_center[1] = inlet_center
    b.inlet_radius = inlet_radius
    b.inlet_noise = inlet_noise
    b.seed = seed
    b.storage = storage
    b.order = order
    b.inlet_noise_kind = inlet_noise_kind
    return b


def tslb_create(nx, ny, nz, lattice, tau, force=None, bc=None):
    h = ctypes.c_void_p()
    f = (ctypes.c_float * 3)(*force) if force is not None else None
    _check(lib.tslb_create(nx, ny, nz, lattice, tau, f, ctypes.byref(bc) if bc is not None else None,
                           ctypes.byref(h)))
    return h


def tslb_destroy(h):
    return _check(lib.tslb_destroy(h))


def tslb_set_moments(h, rho, u, pineq=None, flags=TSLB_DEVICE, stream=None):
    return _check(lib.tslb_set_moments(h, _ptr(rho), _ptr(u), _ptr(pineq), flags, _stream(stream)))


def tslb_get_moments(h, rho, u, pineq=None, flags=TSLB_DEVICE, stream=None):
    return _check(lib.tslb_get_moments(h, _ptr(rho), _ptr(u), _ptr(pineq), flags, _stream(stream)))


def tslb_set_force_field(h, g, stream=None):
    return _check(lib.tslb_set_force_field(h, _ptr(g), _stream(stream)))


def tslb_step(h, nsteps, stream=None):
    return _check(lib.tslb_step(h, nsteps, _stream(stream)))


def tslb_stats_begin(h, kinds, axis=1, stream=None):
    return _check(lib.tslb_stats_begin(h, kinds, axis, _stream(stream)))


def tslb_stats_sample(h, stream=None):
    return _check(lib.tslb_stats_sample(h, _stream(stream)))


def tslb_stats_profile(h, n_axis, stream=None):
    """Returns (sums as a list of n_axis rows of 13 floats, number of samples)."""
    buf = (ctypes.c_double * (13 * n_axis))()
    ns = ctypes.c_int64()
    _check(lib.tslb_stats_profile(h, buf, ctypes.byref(ns), _stream(stream)))
    return [list(buf[13 * j:13 * j + 13]) for j in range(n_axis)], ns.value


def tslb_stats_field(h, mean_u, cov, stream=None):
    return _check(lib.tslb_stats_field(h, _ptr(mean_u), _ptr(cov), _stream(stream)))


def tslb_stats_jet(h, axis, center, uc, rhalf, stream=None):
    c = (ctypes.c_float * 2)(*[float(v) for v in center])
    return _check(lib.tslb_stats_jet(h, axis, c, _ptr(uc), _ptr(rhalf), _stream(stream)))


def tslb_bind_state(h, buf0, buf1, stream=None):
    return _check(lib.tslb_bind_state(h, _ptr(buf0), _ptr(buf1), _stream(stream)))


def tslb_objective(h, objective, stream=None):
    out = ctypes.c_double()
    _check(lib.tslb_objective(h, objective, ctypes.byref(out), _stream(stream)))
    return out.value


def tslb_set_relaxation_profile(h, tau_z, stream=None):
    """tau_z: sequence of nz floats (host), or None for the uniform tau."""
    arr = None if tau_z is None else (ctypes.c_float * len(tau_z))(*[float(v) for v in tau_z])
    return _check(lib.tslb_set_relaxation_profile(h, arr, _stream(stream)))


def tslb_step_timed(h, nsteps, stream=None):
    ms = (ctypes.c_double * 2)()
    _check(lib.tslb_step_timed(h, nsteps, ms, _stream(stream)))
    return ms[0], ms[1]


def tslb_get_time(h):
    return lib.tslb_get_time(h)


def tslb_set_time(h, t):
    return _check(lib.tslb_set_time(h, t))


def tslb_reduce(h, stream=None, check=True):
    out = (ctypes.c_double * 5)()
    rc = lib.tslb_reduce(h, out, _stream(stream))
    if check:
        _check(rc)
    return list(out), rc


def tslb_reduce_noalloc(h, out, stream=None):
    """out: a float64 CUDA tensor of at least TSLB_REDUCE_VALUES elements."""
    _check(lib.tslb_reduce_noalloc(h, _ptr(out), _stream(stream)))


def tslb_stream_copy(dst, src, stream=None):
    """Copy tensor src into tensor dst (same byte size) with the library's
    streaming copy kernel."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    _check(lib.tslb_stream_copy(_ptr(dst), _ptr(src), nbytes, _stream(stream)))


def tslb_state_bytes(h):
    return lib.tslb_state_bytes(h)


def tslb_save_state(h, dst, stream=None):
    return _check(lib.tslb_save_state(h, _ptr(dst), _stream(stream)))


def tslb_load_state(h, src, stream=None):
    return _check(lib.tslb_load_state(h, _ptr(src), _stream(stream)))


def tslb_adjoint_step(h, state_t, state_t1, lam_t1, lam_t, dg_accum=None, stream=None):
    return _check(lib.tslb_adjoint_step(h, _ptr(state_t), _ptr(state_t1), _ptr(lam_t1), _ptr(lam_t),
                                        _ptr(dg_accum), _stream(stream)))


def tslb_adjoint_seed(h, state, lam, objective=TSLB_OBJ_KINETIC_ENERGY, stream=None):
    return _check(lib.tslb_adjoint_seed(h, _ptr(state), objective, _ptr(lam), _stream(stream)))


def tslb_rollout_workspace_bytes(h, nsteps, every):
    return lib.tslb_rollout_workspace_bytes(h, nsteps, every)


def tslb_rollout_forward(h, nsteps, every, ws, stream=None):
    return _check(lib.tslb_rollout_forward(h, nsteps, every, _ptr(ws), ws.numel() * ws.element_size(),
                                           _stream(stream)))


def tslb_rollout_backward(h, nsteps, every, ws, lam, dg_accum=None, stream=None):
    return _check(lib.tslb_rollout_backward(h, nsteps, every, _ptr(ws), ws.numel() * ws.element_size(), _ptr(lam),
                                            _ptr(dg_accum), _stream(stream)))


def tslb_set_kernel(h, variant):
    return _check(lib.tslb_set_kernel(h, variant))


def tslb_last_error():
    return lib.tslb_last_error().decode()
