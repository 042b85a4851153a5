"""ctypes binding of libcfd (include/cfd.h), with the C ABI's names.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libcfd.so. Arrays are torch tensors on the GPU (float64,
contiguous); streams default to torch's current stream. If libcfd.so is
missing or cannot be loaded, every entry point raises - there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# CFD_LIBRARY names an alternative build of the same library (e.g. for A/B timing)
LIB_PATH = os.environ.get("CFD_LIBRARY") or os.path.join(_HERE, "libcfd.so")

CFD_OK, CFD_EINVAL, CFD_ENOMEM, CFD_EHIP, CFD_ENONFINITE, CFD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
CFD_BC_PERIODIC, CFD_BC_ZERO_GRADIENT, CFD_BC_REFLECT = 0, 1, 2
CFD_F_INVISCID, CFD_F_VISCOUS, CFD_F_HEAT, CFD_F_WENOZ, CFD_F_ROE = 1, 2, 4, 8, 16
CFD_F_WENO3, CFD_F_RUSANOV, CFD_F_RK2, CFD_F_RUSANOV_NN, CFD_F_SAFE_RECON = 32, 64, 128, 256, 512
CFD_NN_PARAMS = 2305
CFD_NOALLOC_MAX_PADDED_CELLS = 386309


class CfdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libcfd error {code}: {msg}")
        self.code = code


class cfd_config(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3),
        ("nh", C.c_int32),
        ("lo", C.c_double * 3),
        ("hi", C.c_double * 3),
        ("gamma", C.c_double),
        ("mu", C.c_double),
        ("prandtl", C.c_double),
        ("cfl", C.c_double),
        ("bc", C.c_int32 * 6),
        ("flags", C.c_uint32),
    ]


EXPORTS = (
    "cfd_create", "cfd_destroy", "cfd_state_numel", "cfd_state_init", "cfd_state_init_adjoint", "cfd_fill_halo", "cfd_rhs",
    "cfd_compute_dt", "cfd_rk3_step", "cfd_advance", "cfd_advance_fixed", "cfd_rhs_adjoint",
    "cfd_rk3_step_adjoint", "cfd_rk3_step_stages", "cfd_rk3_step_adjoint_stages", "cfd_rk3_step_prims",
    "cfd_rk3_step_adjoint_prims", "cfd_profile_stage", "cfd_check", "cfd_last_error",
    "cfd_set_nn_weights", "cfd_rk3_step_noalloc",
    "cfd_batch_create", "cfd_batch_destroy", "cfd_batch_footprint", "cfd_batch_add", "cfd_batch_remove",
    "cfd_batch_state", "cfd_batch_step", "cfd_batch_finish", "cfd_batch_copy_state", "cfd_batch_count",
)

_lib = None


def load():
    """Load libcfd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_2203_13760_amd/build.py "
                           "(or __graft_entry__.build()) first; there is no fallback path")
    lib = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.c_void_p
    cfgp = C.POINTER(cfd_config)
    st = C.c_int
    sig = {
        "cfd_create": ([cfgp, C.POINTER(C.c_void_p)], st),
        "cfd_destroy": ([vp], None),
        "cfd_state_numel": ([vp], C.c_int64),
        "cfd_state_init": ([vp, dp, dp, vp], st),
        "cfd_state_init_adjoint": ([vp, dp, dp, dp, vp], st),
        "cfd_fill_halo": ([vp, dp, vp], st),
        "cfd_rhs": ([vp, dp, dp, vp], st),
        "cfd_compute_dt": ([vp, dp, dp, vp], st),
        "cfd_rk3_step": ([vp, dp, C.c_double, dp, vp], st),
        "cfd_advance": ([vp, dp, C.c_int32, C.c_double, dp, vp], st),
        "cfd_advance_fixed": ([vp, dp, C.c_int32, C.c_double, vp], st),
        "cfd_rhs_adjoint": ([vp, dp, dp, dp, vp], st),
        "cfd_rk3_step_adjoint": ([vp, dp, C.c_double, dp, dp, vp], st),
        "cfd_rk3_step_stages": ([vp, dp, C.c_double, dp, dp, vp], st),
        "cfd_rk3_step_adjoint_stages": ([vp, dp, dp, dp, C.c_double, dp, dp, vp], st),
        "cfd_rk3_step_prims": ([vp, dp, C.c_double, dp, vp], st),
        "cfd_rk3_step_adjoint_prims": ([vp, dp, C.c_double, dp, dp, vp], st),
        "cfd_profile_stage": ([vp, dp, C.c_int32, C.POINTER(C.c_double), vp], st),
        "cfd_set_nn_weights": ([vp, dp, dp], st),
        "cfd_rk3_step_noalloc": ([cfgp, dp, C.c_double, dp, vp], st),
        "cfd_check": ([vp, C.POINTER(C.c_int32)], st),
        "cfd_last_error": ([], C.c_char_p),
        "cfd_batch_create": ([C.c_int32, C.c_int64, C.POINTER(C.c_void_p)], st),
        "cfd_batch_destroy": ([vp], None),
        "cfd_batch_footprint": ([cfgp, C.POINTER(C.c_int64)], st),
        "cfd_batch_add": ([vp, cfgp, dp, C.POINTER(C.c_int32), vp], st),
        "cfd_batch_remove": ([vp, C.c_int32], st),
        "cfd_batch_state": ([vp, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64)], st),
        "cfd_batch_step": ([vp, vp], st),
        "cfd_batch_finish": ([vp, C.c_int32, vp], st),
        "cfd_batch_copy_state": ([vp, C.c_int32, dp, vp], st),
        "cfd_batch_count": ([vp], C.c_int32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != CFD_OK:
        raise CfdError(rc, load().cfd_last_error().decode())


def make_config(case) -> cfd_config:
    c = cfd_config()
    for i in range(3):
        c.n[i] = int(case["n"][i])
        c.lo[i] = float(case["lo"][i])
        c.hi[i] = float(case["hi"][i])
    c.nh = int(case.get("nh", 3))
    c.gamma = float(case["gamma"])
    c.mu = float(case.get("mu", 0.0))
    c.prandtl = float(case.get("prandtl", 0.72))
    c.cfl = float(case.get("cfl", 0.5))
    for i in range(6):
        c.bc[i] = int(case["bc"][i])
    c.flags = int(case["flags"])
    return c


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return C.c_void_p(0)
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), \
        "expected a contiguous float64 CUDA tensor"
    return C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- entry points
def cfd_create(case):
    h = C.c_void_p()
    cfg = make_config(case)
    _check(load().cfd_create(C.byref(cfg), C.byref(h)))
    return h


def cfd_destroy(h):
    if h:
        load().cfd_destroy(h)


def cfd_state_numel(h):
    return int(load().cfd_state_numel(h))


def cfd_state_init(h, W, U, stream=None):
    _check(load().cfd_state_init(h, _ptr(W), _ptr(U), _stream(stream)))


def cfd_state_init_adjoint(h, W, Ubar, Wbar, stream=None):
    _check(load().cfd_state_init_adjoint(h, _ptr(W), _ptr(Ubar), _ptr(Wbar), _stream(stream)))


def cfd_fill_halo(h, U, stream=None):
    _check(load().cfd_fill_halo(h, _ptr(U), _stream(stream)))


def cfd_rhs(h, U, R, stream=None):
    _check(load().cfd_rhs(h, _ptr(U), _ptr(R), _stream(stream)))


def cfd_compute_dt(h, U, dt_dev, stream=None):
    _check(load().cfd_compute_dt(h, _ptr(U), _ptr(dt_dev), _stream(stream)))


def cfd_rk3_step(h, U, dt=0.0, dt_used_dev=None, stream=None):
    _check(load().cfd_rk3_step(h, _ptr(U), float(dt), _ptr(dt_used_dev), _stream(stream)))


def cfd_advance(h, U, n_steps, t_end, t_dev, stream=None):
    _check(load().cfd_advance(h, _ptr(U), int(n_steps), float(t_end), _ptr(t_dev), _stream(stream)))


def cfd_advance_fixed(h, U, n_steps, dt, stream=None):
    _check(load().cfd_advance_fixed(h, _ptr(U), int(n_steps), float(dt), _stream(stream)))


def cfd_rhs_adjoint(h, U, Rbar, Ubar, stream=None):
    _check(load().cfd_rhs_adjoint(h, _ptr(U), _ptr(Rbar), _ptr(Ubar), _stream(stream)))


def cfd_rk3_step_adjoint(h, Un, dt, Ubar_np1, Ubar_n, stream=None):
    _check(load().cfd_rk3_step_adjoint(h, _ptr(Un), float(dt), _ptr(Ubar_np1), _ptr(Ubar_n),
                                       _stream(stream)))


def cfd_rk3_step_stages(h, U, dt, U1_out, U2_out, stream=None):
    _check(load().cfd_rk3_step_stages(h, _ptr(U), float(dt), _ptr(U1_out), _ptr(U2_out), _stream(stream)))


def cfd_rk3_step_adjoint_stages(h, Un, U1, U2, dt, Ubar_np1, Ubar_n, stream=None):
    _check(load().cfd_rk3_step_adjoint_stages(h, _ptr(Un), _ptr(U1), _ptr(U2), float(dt), _ptr(Ubar_np1),
                                              _ptr(Ubar_n), _stream(stream)))


def cfd_rk3_step_prims(h, U, dt, P_out, stream=None):
    _check(load().cfd_rk3_step_prims(h, _ptr(U), float(dt), _ptr(P_out), _stream(stream)))


def cfd_rk3_step_adjoint_prims(h, P, dt, Ubar_np1, Ubar_n, stream=None):
    _check(load().cfd_rk3_step_adjoint_prims(h, _ptr(P), float(dt), _ptr(Ubar_np1), _ptr(Ubar_n),
                                             _stream(stream)))


def cfd_set_nn_weights(h, theta, theta_bar=None):
    """Rusanov-NN weights (device tensor of CFD_NN_PARAMS doubles, kept alive by
    the caller) and the optional weight-gradient accumulator the adjoints add to."""
    _check(load().cfd_set_nn_weights(h, _ptr(theta), _ptr(theta_bar)))


def cfd_rk3_step_noalloc(case, U, dt=0.0, dt_used_dev=None, stream=None):
    """Allocation-free TVD-RK3 step of U in place (no solver handle; the
    library's static device scratch, grids up to CFD_NOALLOC_MAX_PADDED_CELLS)."""
    cfg = make_config(case)
    _check(load().cfd_rk3_step_noalloc(C.byref(cfg), _ptr(U), float(dt), _ptr(dt_used_dev), _stream(stream)))


def cfd_profile_stage(h, U, reps=5, stream=None):
    """Average ms of the stage kernels [prim, sweep_x, sweep_y, sweep_z, prim_halo]."""
    out = (C.c_double * 5)()
    _check(load().cfd_profile_stage(h, _ptr(U), int(reps), out, _stream(stream)))
    return list(out)


def cfd_check(h):
    v = C.c_int32(0)
    _check(load().cfd_check(h, C.byref(v)))
    return int(v.value)


def cfd_last_error():
    return load().cfd_last_error().decode()


# ---------------------------------------------------------------- serving batch
def cfd_batch_create(max_grids, arena_bytes):
    h = C.c_void_p()
    _check(load().cfd_batch_create(int(max_grids), int(arena_bytes), C.byref(h)))
    return h


def cfd_batch_destroy(b):
    if b:
        load().cfd_batch_destroy(b)


def cfd_batch_footprint(case):
    n = C.c_int64(0)
    cfg = make_config(case)
    _check(load().cfd_batch_footprint(C.byref(cfg), C.byref(n)))
    return int(n.value)


def cfd_batch_add(b, case, W, stream=None):
    """Admit a grid; returns its slot, or None when the batch is full (CFD_ENOMEM)."""
    slot = C.c_int32(-1)
    cfg = make_config(case)
    rc = load().cfd_batch_add(b, C.byref(cfg), _ptr(W), C.byref(slot), _stream(stream))
    if rc == CFD_ENOMEM:
        return None
    _check(rc)
    return int(slot.value)


def cfd_batch_remove(b, slot):
    _check(load().cfd_batch_remove(b, int(slot)))


def cfd_batch_state(b, slot):
    """(device pointer, element count) of a resident grid's padded state."""
    p = C.c_void_p()
    n = C.c_int64(0)
    _check(load().cfd_batch_state(b, int(slot), C.byref(p), C.byref(n)))
    return int(p.value), int(n.value)


def cfd_batch_step(b, stream=None):
    _check(load().cfd_batch_step(b, _stream(stream)))


def cfd_batch_finish(b, slot, stream=None):
    _check(load().cfd_batch_finish(b, int(slot), _stream(stream)))


def cfd_batch_copy_state(b, slot, dst, stream=None):
    _check(load().cfd_batch_copy_state(b, int(slot), _ptr(dst), _stream(stream)))


def cfd_batch_count(b):
    return int(load().cfd_batch_count(b))
