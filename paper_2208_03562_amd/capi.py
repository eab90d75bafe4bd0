"""ctypes binding of the C ABI in ``include/prc.h`` (``libprc.so``).

Argument marshalling only: every function here forwards to the entry point of
the same name, and every step of the method runs in the library's HIP
kernels.  Device pointers are plain integers (e.g. ``tensor.data_ptr()``) and
streams are ``hipStream_t`` handles (``torch.cuda.Stream.cuda_stream``; 0 is
the null stream).  A missing or stale library raises at import of
:func:`lib` -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libprc.so")

# prc_status
PRC_OK, PRC_NOT_CONVERGED, PRC_EINVAL, PRC_EHIP, PRC_EDIVERGED, PRC_ENOMEM = 0, 1, -1, -2, -3, -4
STATUS_NAMES = {0: "PRC_OK", 1: "PRC_NOT_CONVERGED", -1: "PRC_EINVAL", -2: "PRC_EHIP",
                -3: "PRC_EDIVERGED", -4: "PRC_ENOMEM"}
# prc_bc
PRC_BC_CAVITY, PRC_BC_PERIODIC, PRC_BC_CHANNEL = 0, 1, 2
# prc_storage
PRC_F64, PRC_F32, PRC_F16, PRC_BF16 = 0, 1, 2, 3
STORAGE_BYTES = {PRC_F64: 8, PRC_F32: 4, PRC_F16: 2, PRC_BF16: 2}
# prc_corrections
PRC_CORR_THETA, PRC_CORR_LAMBDA, PRC_CORR_K11, PRC_CORR_ALL = 1, 2, 4, 7
# prc_frame
PRC_FRAME_CENTRAL, PRC_FRAME_RAW = 0, 1
# prc_member_status
PRC_MEMBER_ACTIVE, PRC_MEMBER_CONVERGED, PRC_MEMBER_MAX_STEPS = 2, 0, 1
PRC_MEMBER_DIVERGED, PRC_MEMBER_REMOVED = -3, -5


class prc_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("r", ctypes.c_double), ("gamma", ctypes.c_double),
        ("omega_nu", ctypes.c_double), ("omega_xi", ctypes.c_double),
        ("omega_1", ctypes.c_double), ("omega_3", ctypes.c_double),
        ("omega_4", ctypes.c_double),
        ("u_lid", ctypes.c_double), ("fx", ctypes.c_double), ("fy", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("bc", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("corrections", ctypes.c_int32), ("frame", ctypes.c_int32),
    ]

    def copy(self) -> "prc_params":
        return prc_params.from_buffer_copy(self)

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class prc_request(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("p", prc_params),
                ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p)]


class prc_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("steps", ctypes.c_int64), ("residual", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class prc_server_result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("steps", ctypes.c_int64),
                ("residual", ctypes.c_double), ("submit_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class prc_serve_config(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int32), ("bc", ctypes.c_int32), ("tol", ctypes.c_double),
                ("check_every", ctypes.c_int64), ("max_steps", ctypes.c_int64),
                ("hbm_budget", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("tile", ctypes.c_int32)]


class PrcError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} -> {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_P = ctypes.POINTER(prc_params)
_VP = ctypes.c_void_p
_DP = ctypes.c_void_p  # double* (device or host, passed as an address)
_I64P = ctypes.POINTER(ctypes.c_int64)

_PROTOS = {
    "prc_params_default": (ctypes.c_int, [_P]),
    "prc_params_from_re": (ctypes.c_int, [_P, ctypes.c_double]),
    "prc_validate": (ctypes.c_int, [_P]),
    "prc_layout": (ctypes.c_int, [_P, _I64P, _I64P]),
    "prc_state_bytes": (ctypes.c_size_t, [_P]),
    "prc_scratch_bytes": (ctypes.c_size_t, [_P]),
    "prc_init": (ctypes.c_int, [_P, _VP, _VP]),
    "prc_step": (ctypes.c_int, [_P, _VP, _VP, ctypes.c_int64, _VP]),
    "prc_step_timed": (ctypes.c_int, [_P, _VP, _VP, ctypes.c_int64, _VP, _VP, ctypes.c_int32,
                                      _VP]),
    "prc_residual": (ctypes.c_int, [_P, _VP, _DP, _VP, ctypes.POINTER(ctypes.c_double), _VP]),
    "prc_residual_noalloc": (ctypes.c_int, [_P, _VP, _DP, ctypes.POINTER(ctypes.c_double), _VP]),
    "prc_convert": (ctypes.c_int, [_P, _VP, ctypes.c_int32, _VP, _VP]),
    "prc_add_density": (ctypes.c_int, [_P, _VP, ctypes.c_double, _VP]),
    "prc_macros": (ctypes.c_int, [_P, _VP, _DP, _DP, _DP, _VP]),
    "prc_solve": (ctypes.c_int, [_P, _VP, _VP, _DP, _VP, ctypes.c_double, ctypes.c_int64,
                                 ctypes.c_int64, _I64P, ctypes.POINTER(ctypes.c_double),
                                 ctypes.c_int64, _I64P, _VP]),
    "prc_tune": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), _VP]),
    "prc_set_tile": (ctypes.c_int, [_P, ctypes.c_int32]),
    "prc_tile_info": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    "prc_release_graphs": (ctypes.c_int, []),
    "prc_release_resident": (ctypes.c_int, []),
    "prc_resident_status": (ctypes.c_int, []),
    "prc_set_streamed": (ctypes.c_int, [ctypes.c_int32]),
    "prc_set_resident_wait": (ctypes.c_int, [ctypes.c_int64]),
    "prc_last_error": (ctypes.c_char_p, []),
    "prc_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_VP)]),
    "prc_batch_destroy": (ctypes.c_int, [_VP]),
    "prc_batch_add": (ctypes.c_int, [_VP, _P, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_int32)]),
    "prc_batch_remove": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "prc_batch_count": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "prc_batch_step": (ctypes.c_int, [_VP, ctypes.c_int64, _VP]),
    "prc_batch_residual": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), _VP]),
    "prc_batch_solve": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int32), _I64P,
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_int64, _I64P,
                                       _VP]),
    "prc_batch_tune": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32), _VP]),
    "prc_batch_set_tile": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "prc_server_create": (ctypes.c_int, [ctypes.POINTER(prc_serve_config), _VP,
                                        ctypes.POINTER(_VP)]),
    "prc_server_submit": (ctypes.c_int, [_VP, _P, _VP, _VP, _I64P]),
    "prc_server_poll": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.POINTER(prc_server_result),
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "prc_server_status": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "prc_server_destroy": (ctypes.c_int, [_VP]),
    "prc_serve": (ctypes.c_int, [ctypes.POINTER(prc_serve_config), ctypes.POINTER(prc_request),
                                 ctypes.c_int32, ctypes.POINTER(prc_result), _VP]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load ``libprc.so`` (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return list(_PROTOS)


def last_error() -> str:
    return (lib().prc_last_error() or b"").decode()


def _check(fn: str, st: int, ok=(PRC_OK,)) -> int:
    if st not in ok:
        raise PrcError(fn, st, last_error())
    return st


# ---- same-named wrappers -------------------------------------------------

def prc_params_default() -> prc_params:
    p = prc_params()
    _check("prc_params_default", lib().prc_params_default(ctypes.byref(p)))
    return p


def prc_params_from_re(p: prc_params, re: float) -> prc_params:
    _check("prc_params_from_re", lib().prc_params_from_re(ctypes.byref(p), float(re)))
    return p


def prc_validate(p: prc_params) -> None:
    _check("prc_validate", lib().prc_validate(ctypes.byref(p)))


def prc_layout(p: prc_params):
    """(row_stride, plane_stride) in elements."""
    row, plane = ctypes.c_int64(), ctypes.c_int64()
    _check("prc_layout", lib().prc_layout(ctypes.byref(p), ctypes.byref(row),
                                          ctypes.byref(plane)))
    return row.value, plane.value


def prc_state_bytes(p: prc_params) -> int:
    n = lib().prc_state_bytes(ctypes.byref(p))
    if n == 0:
        raise PrcError("prc_state_bytes", PRC_EINVAL, last_error())
    return n


def prc_scratch_bytes(p: prc_params) -> int:
    n = lib().prc_scratch_bytes(ctypes.byref(p))
    if n == 0:
        raise PrcError("prc_scratch_bytes", PRC_EINVAL, last_error())
    return n


def prc_init(p: prc_params, f: int, stream: int = 0) -> None:
    _check("prc_init", lib().prc_init(ctypes.byref(p), f, stream))


def prc_step(p: prc_params, f_a: int, f_b: int, nsteps: int, stream: int = 0) -> None:
    _check("prc_step", lib().prc_step(ctypes.byref(p), f_a, f_b, int(nsteps), stream))


def prc_step_timed(p: prc_params, f_a: int, f_b: int, nsteps: int, start: int, stop: int,
                   kernel_only: bool = False, stream: int = 0) -> None:
    _check("prc_step_timed", lib().prc_step_timed(ctypes.byref(p), f_a, f_b, nsteps, start, stop,
                                                  int(bool(kernel_only)), stream))


def prc_residual(p: prc_params, f: int, u_prev: int, scratch: int, stream: int = 0):
    out = (ctypes.c_double * 4)()
    _check("prc_residual", lib().prc_residual(ctypes.byref(p), f, u_prev, scratch, out, stream))
    return list(out)


def prc_residual_noalloc(p: prc_params, f: int, u_prev: int, stream: int = 0):
    out = (ctypes.c_double * 4)()
    _check("prc_residual_noalloc",
           lib().prc_residual_noalloc(ctypes.byref(p), f, u_prev, out, stream))
    return list(out)


def prc_convert(p: prc_params, f: int, storage_to: int, f_to: int, stream: int = 0) -> None:
    _check("prc_convert", lib().prc_convert(ctypes.byref(p), f, int(storage_to), f_to, stream))


def prc_add_density(p: prc_params, f: int, drho: float, stream: int = 0) -> None:
    _check("prc_add_density", lib().prc_add_density(ctypes.byref(p), f, float(drho), stream))


def prc_macros(p: prc_params, f: int, rho: int | None, ux: int | None, uy: int | None,
               stream: int = 0) -> None:
    _check("prc_macros", lib().prc_macros(ctypes.byref(p), f, rho, ux, uy, stream))


def prc_solve(p: prc_params, f_a: int, f_b: int, u_prev: int, scratch: int, tol: float,
              check_every: int, max_steps: int, hist_cap: int = 4096, stream: int = 0):
    """Returns (status, steps, residual history); status is PRC_OK,
    PRC_NOT_CONVERGED or PRC_EDIVERGED (other statuses raise)."""
    steps, nh = ctypes.c_int64(), ctypes.c_int64()
    hist = (ctypes.c_double * max(1, hist_cap))()
    st = lib().prc_solve(ctypes.byref(p), f_a, f_b, u_prev, scratch, float(tol),
                         int(check_every), int(max_steps), ctypes.byref(steps), hist,
                         int(hist_cap), ctypes.byref(nh), stream)
    _check("prc_solve", st, ok=(PRC_OK, PRC_NOT_CONVERGED, PRC_EDIVERGED))
    return st, steps.value, list(hist[: min(nh.value, hist_cap)])


def prc_release_graphs() -> None:
    _check("prc_release_graphs", lib().prc_release_graphs())


def prc_release_resident() -> None:
    _check("prc_release_resident", lib().prc_release_resident())


def prc_resident_status() -> None:
    """Raises PrcError (PRC_EHIP) once for a resident launch that lost a wait."""
    _check("prc_resident_status", lib().prc_resident_status())


def prc_set_streamed(mode: int) -> None:
    _check("prc_set_streamed", lib().prc_set_streamed(int(mode)))


def prc_set_resident_wait(ticks: int) -> None:
    _check("prc_set_resident_wait", lib().prc_set_resident_wait(int(ticks)))


def prc_last_error() -> str:
    return last_error()


def prc_tune(p: prc_params, stream: int = 0) -> int:
    """Time the sweep's tile shapes for this problem; returns the chosen index."""
    t = ctypes.c_int32(-1)
    _check("prc_tune", lib().prc_tune(ctypes.byref(p), ctypes.byref(t), stream))
    return t.value


def prc_tile_info(tile: int):
    """(threads along x, threads along y, time steps per launch) of a tile index."""
    tx, ty, st = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check("prc_tile_info", lib().prc_tile_info(int(tile), ctypes.byref(tx), ctypes.byref(ty),
                                                ctypes.byref(st)))
    return tx.value, ty.value, st.value


def prc_set_tile(p: prc_params, tile: int) -> None:
    _check("prc_set_tile", lib().prc_set_tile(ctypes.byref(p), int(tile)))


# ---- batches ---------------------------------------------------------------

def prc_batch_create(storage: int, bc: int) -> int:
    """Returns the opaque batch handle (an integer)."""
    h = _VP()
    _check("prc_batch_create", lib().prc_batch_create(int(storage), int(bc), ctypes.byref(h)))
    return h.value


def prc_batch_destroy(b: int) -> None:
    _check("prc_batch_destroy", lib().prc_batch_destroy(b))


def prc_batch_add(b: int, p: prc_params, f_a: int, f_b: int, u_prev: int) -> int:
    i = ctypes.c_int32(-1)
    _check("prc_batch_add", lib().prc_batch_add(b, ctypes.byref(p), f_a, f_b, u_prev,
                                                ctypes.byref(i)))
    return i.value


def prc_batch_remove(b: int, member: int) -> None:
    _check("prc_batch_remove", lib().prc_batch_remove(b, int(member)))


def prc_batch_count(b: int):
    """(members added, members active)."""
    n, a = ctypes.c_int32(), ctypes.c_int32()
    _check("prc_batch_count", lib().prc_batch_count(b, ctypes.byref(n), ctypes.byref(a)))
    return n.value, a.value


def prc_batch_step(b: int, nsteps: int, stream: int = 0) -> None:
    _check("prc_batch_step", lib().prc_batch_step(b, int(nsteps), stream))


def prc_batch_residual(b: int, stream: int = 0):
    """{id: [N, D, mass, max |u|^2]} for the active members."""
    n, _ = prc_batch_count(b)
    out = (ctypes.c_double * max(1, 4 * n))(*([float("nan")] * max(1, 4 * n)))
    _check("prc_batch_residual", lib().prc_batch_residual(b, out, stream))
    return out


def prc_batch_solve(b: int, tol: float, check_every: int, max_steps: int, hist_cap: int = 0,
                    stream: int = 0):
    """Returns (status[id], steps[id], hist[id] lists) for every member added."""
    n, _ = prc_batch_count(b)
    m = max(1, n)
    status = (ctypes.c_int32 * m)()
    steps = (ctypes.c_int64 * m)()
    hl = (ctypes.c_int64 * m)()
    hist = (ctypes.c_double * max(1, m * hist_cap))() if hist_cap > 0 else None
    _check("prc_batch_solve", lib().prc_batch_solve(b, float(tol), int(check_every),
                                                    int(max_steps), status, steps, hist,
                                                    int(hist_cap), hl, stream))
    hists = [list(hist[i * hist_cap: i * hist_cap + min(hl[i], hist_cap)]) if hist else []
             for i in range(n)]
    return list(status[:n]), list(steps[:n]), hists


def prc_batch_tune(b: int, stream: int = 0) -> int:
    t = ctypes.c_int32(-1)
    _check("prc_batch_tune", lib().prc_batch_tune(b, ctypes.byref(t), stream))
    return t.value


def prc_batch_set_tile(b: int, tile: int) -> None:
    _check("prc_batch_set_tile", lib().prc_batch_set_tile(b, int(tile)))


# ---- serving -----------------------------------------------------------------

def prc_serve(cfg: prc_serve_config, reqs, stream: int = 0):
    """Serve a list of prc_request; returns the list of prc_result."""
    n = len(reqs)
    arr = (prc_request * max(1, n))(*reqs)
    res = (prc_result * max(1, n))()
    _check("prc_serve", lib().prc_serve(ctypes.byref(cfg), arr, n, res, stream))
    return [res[i] for i in range(n)]


def prc_server_create(cfg: prc_serve_config, stream: int = 0) -> int:
    h = _VP()
    _check("prc_server_create", lib().prc_server_create(ctypes.byref(cfg), stream, ctypes.byref(h)))
    return h.value


def prc_server_submit(srv: int, p: prc_params, ux: int | None = None, uy: int | None = None) -> int:
    t = ctypes.c_int64()
    _check("prc_server_submit", lib().prc_server_submit(srv, ctypes.byref(p), ux, uy,
                                                        ctypes.byref(t)))
    return t.value


def prc_server_poll(srv: int, wait_s: float = 0.0, cap: int = 256):
    out = (prc_server_result * max(1, cap))()
    n = ctypes.c_int32()
    _check("prc_server_poll", lib().prc_server_poll(srv, float(wait_s), out, int(cap),
                                                    ctypes.byref(n)))
    return [out[i] for i in range(n.value)]


def prc_server_status(srv: int):
    w, a, u = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check("prc_server_status", lib().prc_server_status(srv, ctypes.byref(w), ctypes.byref(a),
                                                        ctypes.byref(u)))
    return w.value, a.value, u.value


def prc_server_destroy(srv: int) -> None:
    _check("prc_server_destroy", lib().prc_server_destroy(srv))
