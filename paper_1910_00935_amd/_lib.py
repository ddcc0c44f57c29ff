"""ctypes binding of the C ABI in ``include/mpm.h`` (argument marshalling only).

The functions below carry the ABI's names and signatures; every step of the
simulation runs in the HIP kernels of ``libmpm.so``. Loading fails loudly when
the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmpm.so")

MPM_OK = 0
MPM_E_ARG = 1
MPM_E_CAPACITY = 2
MPM_E_TAPE = 3
MPM_E_HIP = 4
MPM_E_DOMAIN = 5
MPM_E_INVERTED = 6
MPM_E_NONFINITE = 7
MPM_E_STATE = 8
MPM_FLAG_DOMAIN = 1
MPM_FLAG_INVERTED = 2
MPM_FLAG_NONFINITE = 4
MPM_LOSS_MEAN_POS = 0
MPM_MODEL_COROTATED = 1
MPM_KERNEL_FWD = 0
MPM_KERNEL_BWD = 1

c_void_p = ctypes.c_void_p
c_int32 = ctypes.c_int32
c_float = ctypes.c_float
c_size_t = ctypes.c_size_t


class mpm_desc(ctypes.Structure):
    _fields_ = [
        ("dim", c_int32), ("n_grid", c_int32), ("bound", c_int32), ("dx", c_float), ("dt", c_float),
        ("gravity", c_float), ("n_scenes", c_int32), ("scene_offsets", ctypes.POINTER(c_int32)),
        ("n_actuators", c_int32), ("act_strength", c_float), ("flags", ctypes.c_uint32),
    ]


class mpm_state(ctypes.Structure):
    _fields_ = [("x", c_void_p), ("v", c_void_p), ("C", c_void_p), ("F", c_void_p)]


class mpm_params(ctypes.Structure):
    _fields_ = [("E", c_void_p), ("nu", c_void_p), ("vol", c_void_p), ("rho", c_void_p), ("act_id", c_void_p),
                ("act", c_void_p), ("mat_id", c_void_p)]


class mpm_param_grad(ctypes.Structure):
    _fields_ = [("E", c_void_p), ("act", c_void_p)]


class smoke_desc(ctypes.Structure):
    _fields_ = [("n", c_int32), ("steps", c_int32), ("iters", c_int32), ("tile", c_int32)]


class MPMError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__(f"{fn} failed: {status_string(status)} (status {status})")


_lib = None

# name -> (restype, argtypes)
_SIGNATURES = {
    "mpm_status_string": (ctypes.c_char_p, [c_int32]),
    "mpm_init": (c_int32, [ctypes.POINTER(mpm_desc), ctypes.POINTER(c_void_p)]),
    "mpm_destroy": (None, [c_void_p]),
    "mpm_workspace_bytes": (c_size_t, [c_void_p]),
    "mpm_bind_workspace": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "mpm_set_knob": (c_int32, [c_void_p, ctypes.c_char_p, ctypes.c_int64]),
    "mpm_step_fwd": (c_int32, [c_void_p, ctypes.POINTER(mpm_params), c_int32, ctypes.POINTER(mpm_state),
                               ctypes.POINTER(mpm_state), c_void_p]),
    "mpm_step_fwd_noalloc": (c_int32, [c_void_p, ctypes.POINTER(mpm_params), c_int32, ctypes.POINTER(mpm_state),
                                       ctypes.POINTER(mpm_state), c_void_p, c_void_p]),
    "mpm_step_bwd": (c_int32, [c_void_p, ctypes.POINTER(mpm_params), c_int32, ctypes.POINTER(mpm_state),
                               ctypes.POINTER(mpm_state), ctypes.POINTER(mpm_state),
                               ctypes.POINTER(mpm_param_grad), c_void_p]),
    "mpm_tape_create": (c_int32, [c_void_p, c_int32, c_int32, ctypes.POINTER(c_void_p)]),
    "mpm_tape_bytes": (c_size_t, [c_void_p]),
    "mpm_tape_bind": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "mpm_tape_destroy": (None, [c_void_p]),
    "mpm_tape_forward": (c_int32, [c_void_p, ctypes.POINTER(mpm_params), ctypes.POINTER(mpm_state),
                                   ctypes.POINTER(mpm_state), c_void_p]),
    "mpm_tape_backward": (c_int32, [c_void_p, ctypes.POINTER(mpm_params), ctypes.POINTER(mpm_state),
                                    ctypes.POINTER(mpm_state), ctypes.POINTER(mpm_param_grad), c_void_p]),
    "mpm_sort_order": (c_int32, [c_void_p, ctypes.POINTER(mpm_state), c_void_p, c_void_p]),
    "mpm_loss": (c_int32, [c_void_p, c_int32, c_int32, c_float, ctypes.POINTER(mpm_state), c_void_p,
                           ctypes.POINTER(mpm_state), c_void_p]),
    "mpm_actuation": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_float, c_int32, c_void_p, c_void_p]),
    "mpm_actuation_bwd": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_float, c_int32, c_void_p, c_void_p,
                                    c_void_p, c_void_p]),
    "mpm_check_errors": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "mpm_kernel_stats": (c_int32, [c_void_p, c_int32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]),
    "mpm_tile_stats": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64)]),
    "mpm_wg_clock_bind": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "mpm_diag_box_atomics": (c_int32, [c_int32, c_void_p, c_int32, c_int32, c_void_p]),
    "mpm_wg_clock_info": (c_int32, [c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                    ctypes.POINTER(c_int32), ctypes.POINTER(c_int32), c_int32,
                                    ctypes.POINTER(c_int32)]),
    # include/smoke.h
    "smoke_tape_bytes": (c_size_t, [ctypes.POINTER(smoke_desc)]),
    "smoke_workspace_bytes": (c_size_t, [ctypes.POINTER(smoke_desc)]),
    "smoke_workspace_init": (c_int32, [ctypes.POINTER(smoke_desc), c_void_p, c_void_p]),
    "smoke_forward": (c_int32, [ctypes.POINTER(smoke_desc), c_void_p, c_void_p, c_void_p, c_void_p]),
    "smoke_loss": (c_int32, [ctypes.POINTER(smoke_desc), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p]),
    "smoke_backward": (c_int32, [ctypes.POINTER(smoke_desc), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "smoke_check_errors": (c_int32, [ctypes.POINTER(smoke_desc), c_void_p, c_void_p,
                                     ctypes.POINTER(ctypes.c_uint32)]),
}


def lib():
    """The loaded library; raises if libmpm.so is missing (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; build it with `python -m paper_1910_00935_amd.build` "
                "(the HIP path has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().mpm_status_string(int(status)).decode()


def check(fn: str, status: int) -> None:
    if status != MPM_OK:
        raise MPMError(fn, status)


def call(name: str, *args) -> int:
    """Calls `name` and raises MPMError on a non-OK status."""
    st = getattr(lib(), name)(*args)
    check(name, st)
    return st


# Thin wrappers with the ABI's names.
def mpm_init(desc):
    h = c_void_p()
    call("mpm_init", ctypes.byref(desc), ctypes.byref(h))
    return h


def mpm_destroy(ctx):
    lib().mpm_destroy(ctx)


def mpm_workspace_bytes(ctx):
    return int(lib().mpm_workspace_bytes(ctx))


def mpm_bind_workspace(ctx, ptr, nbytes):
    call("mpm_bind_workspace", ctx, c_void_p(ptr), c_size_t(nbytes))


def mpm_set_knob(ctx, key: str, value: int):
    call("mpm_set_knob", ctx, key.encode(), int(value))


def mpm_step_fwd(ctx, params, step, st_in, st_out, stream):
    call("mpm_step_fwd", ctx, ctypes.byref(params), int(step), ctypes.byref(st_in), ctypes.byref(st_out),
         c_void_p(stream))


def mpm_step_fwd_noalloc(ctx, params, step, st_in, st_out, err_flags, stream):
    call("mpm_step_fwd_noalloc", ctx, ctypes.byref(params), int(step), ctypes.byref(st_in), ctypes.byref(st_out),
         c_void_p(err_flags), c_void_p(stream))


def mpm_step_bwd(ctx, params, step, st_in, out_grad, in_grad, pg, stream):
    call("mpm_step_bwd", ctx, ctypes.byref(params), int(step), ctypes.byref(st_in), ctypes.byref(out_grad),
         ctypes.byref(in_grad), ctypes.byref(pg), c_void_p(stream))


def mpm_tape_create(ctx, n_steps, ckpt_every):
    h = c_void_p()
    call("mpm_tape_create", ctx, int(n_steps), int(ckpt_every), ctypes.byref(h))
    return h


def mpm_tape_bytes(tape):
    return int(lib().mpm_tape_bytes(tape))


def mpm_tape_bind(tape, ptr, nbytes):
    call("mpm_tape_bind", tape, c_void_p(ptr), c_size_t(nbytes))


def mpm_tape_destroy(tape):
    lib().mpm_tape_destroy(tape)


def mpm_tape_forward(tape, params, init, final, stream):
    call("mpm_tape_forward", tape, ctypes.byref(params), ctypes.byref(init), ctypes.byref(final), c_void_p(stream))


def mpm_tape_backward(tape, params, final_grad, init_grad, pg, stream):
    call("mpm_tape_backward", tape, ctypes.byref(params), ctypes.byref(final_grad), ctypes.byref(init_grad),
         ctypes.byref(pg), c_void_p(stream))


def mpm_sort_order(ctx, state, perm, stream):
    call("mpm_sort_order", ctx, ctypes.byref(state), c_void_p(perm), c_void_p(stream))


def mpm_loss(ctx, kind, axis, sign, final, loss_ptr, seed, stream):
    call("mpm_loss", ctx, int(kind), int(axis), float(sign), ctypes.byref(final), c_void_p(loss_ptr),
         None if seed is None else ctypes.byref(seed), c_void_p(stream))


def mpm_actuation(ctx, W, b, n_sin, omega, n_steps, act, stream):
    call("mpm_actuation", ctx, c_void_p(W), c_void_p(b), int(n_sin), float(omega), int(n_steps), c_void_p(act),
         c_void_p(stream))


def mpm_actuation_bwd(ctx, W, b, n_sin, omega, n_steps, gact, gW, gb, stream):
    call("mpm_actuation_bwd", ctx, c_void_p(W), c_void_p(b), int(n_sin), float(omega), int(n_steps), c_void_p(gact),
         c_void_p(gW), c_void_p(gb), c_void_p(stream))


def mpm_kernel_stats(ctx, kernel):
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    call("mpm_kernel_stats", ctx, int(kernel), ctypes.byref(ms), ctypes.byref(n))
    return float(ms.value), int(n.value)


def mpm_tile_stats(ctx, stream):
    a = ctypes.c_int64(0)
    b = ctypes.c_int64(0)
    call("mpm_tile_stats", ctx, c_void_p(stream), ctypes.byref(a), ctypes.byref(b))
    return int(a.value), int(b.value)


def mpm_wg_clock_bind(ctx, ptr, nbytes):
    call("mpm_wg_clock_bind", ctx, c_void_p(ptr), c_size_t(nbytes))


def mpm_wg_clock_info(ctx):
    """(kinds, workgroups per row, row stride, clock rate in kHz) of the rows
    taken since the last bind."""
    n = c_int32(0)
    call("mpm_wg_clock_info", ctx, ctypes.byref(n), None, None, None, 0, None)
    rows = n.value
    kind = (c_int32 * max(rows, 1))()
    wgs = (c_int32 * max(rows, 1))()
    stride = c_int32(0)
    rate = c_int32(0)
    call("mpm_wg_clock_info", ctx, ctypes.byref(n), ctypes.byref(stride), kind, wgs, rows, ctypes.byref(rate))
    return list(kind)[:rows], list(wgs)[:rows], int(stride.value), int(rate.value)


def mpm_check_errors(ctx, stream):
    flags = ctypes.c_uint32(0)
    st = lib().mpm_check_errors(ctx, c_void_p(stream), ctypes.byref(flags))
    return st, int(flags.value)


def smoke_tape_bytes(desc):
    return int(lib().smoke_tape_bytes(ctypes.byref(desc)))


def smoke_workspace_bytes(desc):
    return int(lib().smoke_workspace_bytes(ctypes.byref(desc)))


def smoke_workspace_init(desc, ws, stream):
    call("smoke_workspace_init", ctypes.byref(desc), c_void_p(ws), c_void_p(stream))


def smoke_forward(desc, init, tape, ws, stream):
    call("smoke_forward", ctypes.byref(desc), c_void_p(init), c_void_p(tape), c_void_p(ws), c_void_p(stream))


def smoke_loss(desc, tape, target, loss, seed, ws, stream):
    call("smoke_loss", ctypes.byref(desc), c_void_p(tape), c_void_p(target), c_void_p(loss), c_void_p(seed),
         c_void_p(ws), c_void_p(stream))


def smoke_backward(desc, tape, seed, grad, ws, stream):
    call("smoke_backward", ctypes.byref(desc), c_void_p(tape), c_void_p(seed), c_void_p(grad), c_void_p(ws),
         c_void_p(stream))


def smoke_check_errors(desc, ws, stream):
    flags = ctypes.c_uint32(0)
    st = lib().smoke_check_errors(ctypes.byref(desc), c_void_p(ws), c_void_p(stream), ctypes.byref(flags))
    return st, int(flags.value)
