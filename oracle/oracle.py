"""Python access to the FP64 reference ("oracle") of the PRC-LBM.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  It wraps
``oracle/prc_oracle.c`` (plain C, double precision) through ctypes and shares
nothing with the GPU library.  Arrays are numpy float64, populations laid out
``[alpha][j][i]`` (``alpha`` in the velocity order of Sec. 2, eq. 3a/3b).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "prc_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

BC_CAVITY, BC_PERIODIC, BC_CHANNEL = 0, 1, 2
CORR_THETA, CORR_LAMBDA, CORR_K11, CORR_ALL = 1, 2, 4, 7
FRAME_CENTRAL, FRAME_RAW = 0, 1

# velocity set of Sec. 2 (e_y in units of r)
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liborc.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("r", ctypes.c_double), ("gamma", ctypes.c_double),
        ("omega_nu", ctypes.c_double), ("omega_xi", ctypes.c_double),
        ("omega_1", ctypes.c_double), ("omega_3", ctypes.c_double),
        ("omega_4", ctypes.c_double),
        ("u_lid", ctypes.c_double), ("fx", ctypes.c_double),
        ("fy", ctypes.c_double), ("rho0", ctypes.c_double),
        ("bc", ctypes.c_int32), ("corrections", ctypes.c_int32),
        ("frame", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Params)
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        L.orc_lattice.argtypes = [ctypes.c_double, dp, dp]
        L.orc_omega_nu_from_re.argtypes = [pp, ctypes.c_double]
        L.orc_omega_nu_from_re.restype = ctypes.c_double
        L.orc_rest_populations.argtypes = [pp, dp]
        L.orc_raw_moments_square.argtypes = [dp, dp]
        L.orc_scale_rect.argtypes = [ctypes.c_double, dp]
        L.orc_central_from_raw.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_raw_from_central.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_unscale_rect.argtypes = [ctypes.c_double, dp]
        L.orc_populations_from_square_raw.argtypes = [dp, dp]
        L.orc_collide_node.argtypes = [pp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_equilibrium_node.argtypes = [pp, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, dp]
        L.orc_stream.argtypes = [pp, dp, dp]
        L.orc_macros.argtypes = [pp, dp, dp, dp, dp]
        L.orc_grad_rho.argtypes = [pp, dp, dp, dp]
        L.orc_step.argtypes = [pp, dp, ctypes.c_int64]
        L.orc_step.restype = ctypes.c_int
        L.orc_velocity.argtypes = [pp, dp, dp, dp, dp]
        L.orc_velocity.restype = ctypes.c_int
        L.orc_residual.argtypes = [pp, dp, dp, dp, dp]
        L.orc_residual.restype = ctypes.c_int
        L.orc_solve.argtypes = [pp, dp, ctypes.c_double, ctypes.c_int64,
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), dp,
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.orc_solve.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params(nx, ny, r, gamma, omega_nu, *, omega_xi=1.0, omega_1=1.0, omega_3=1.0,
           omega_4=1.0, u_lid=0.0, fx=0.0, fy=0.0, rho0=1.0, bc=BC_CAVITY,
           corrections=CORR_ALL, frame=FRAME_CENTRAL) -> Params:
    return Params(int(nx), int(ny), float(r), float(gamma), float(omega_nu),
                  float(omega_xi), float(omega_1), float(omega_3), float(omega_4),
                  float(u_lid), float(fx), float(fy), float(rho0), int(bc),
                  int(corrections), int(frame))


def with_re(p: Params, re: float) -> Params:
    """Copy of p with omega_nu set from Re = U H / nu, H = ny r (Sec. 5.1)."""
    q = Params.from_buffer_copy(p)
    q.omega_nu = lib().orc_omega_nu_from_re(ctypes.byref(q), float(re))
    return q


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Use n threads in the oracle's parallel loops from now on."""
    lib().orc_set_threads(int(n))


def lattice(r: float):
    q = ctypes.c_double()
    c2 = ctypes.c_double()
    lib().orc_lattice(float(r), ctypes.byref(q), ctypes.byref(c2))
    return q.value, c2.value


def rest_populations(p: Params) -> np.ndarray:
    w = np.zeros(9)
    lib().orc_rest_populations(ctypes.byref(p), _ptr(w))
    return w


def rest_state(p: Params) -> np.ndarray:
    w = rest_populations(p)
    return np.ascontiguousarray(np.broadcast_to(w[:, None, None], (9, p.ny, p.nx)))


def _vec(fn, *args):
    out = np.zeros(9)
    fn(*args, _ptr(out))
    return out


def raw_moments_square(f):
    return _vec(lib().orc_raw_moments_square, _ptr(np.ascontiguousarray(f, np.float64)))


def scale_rect(r, m):
    m = np.array(m, dtype=np.float64)
    lib().orc_scale_rect(float(r), _ptr(m))
    return m


def unscale_rect(r, m):
    m = np.array(m, dtype=np.float64)
    lib().orc_unscale_rect(float(r), _ptr(m))
    return m


def central_from_raw(m, ux, uy):
    return _vec(lib().orc_central_from_raw, _ptr(np.ascontiguousarray(m, np.float64)),
                float(ux), float(uy))


def raw_from_central(k, ux, uy):
    return _vec(lib().orc_raw_from_central, _ptr(np.ascontiguousarray(k, np.float64)),
                float(ux), float(uy))


def populations_from_square_raw(m):
    return _vec(lib().orc_populations_from_square_raw,
                _ptr(np.ascontiguousarray(m, np.float64)))


def collide_node(p: Params, f, gx=0.0, gy=0.0):
    f = np.ascontiguousarray(f, np.float64)
    ft = np.zeros(9)
    diag = np.zeros(8)
    lib().orc_collide_node(ctypes.byref(p), _ptr(f), float(gx), float(gy), _ptr(ft),
                           _ptr(diag))
    return ft, dict(zip(["rho", "ux", "uy", "dxux", "dyuy", "R2s", "R2d", "det"], diag))


def equilibrium_node(p: Params, rho, ux, uy):
    out = np.zeros(9)
    lib().orc_equilibrium_node(ctypes.byref(p), float(rho), float(ux), float(uy),
                               _ptr(out))
    return out


def equilibrium_field(p: Params, rho, ux, uy) -> np.ndarray:
    rho = np.broadcast_to(np.asarray(rho, np.float64), (p.ny, p.nx))
    ux = np.broadcast_to(np.asarray(ux, np.float64), (p.ny, p.nx))
    uy = np.broadcast_to(np.asarray(uy, np.float64), (p.ny, p.nx))
    out = np.zeros((9, p.ny, p.nx))
    for j in range(p.ny):
        for i in range(p.nx):
            out[:, j, i] = equilibrium_node(p, rho[j, i], ux[j, i], uy[j, i])
    return out


def _field(p):
    return np.zeros((p.ny, p.nx))


def stream(p: Params, ft: np.ndarray) -> np.ndarray:
    ft = np.ascontiguousarray(ft, np.float64)
    f = np.zeros_like(ft)
    lib().orc_stream(ctypes.byref(p), _ptr(ft), _ptr(f))
    return f


def macros(p: Params, f: np.ndarray):
    f = np.ascontiguousarray(f, np.float64)
    rho, ux, uy = _field(p), _field(p), _field(p)
    lib().orc_macros(ctypes.byref(p), _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy))
    return rho, ux, uy


def grad_rho(p: Params, rho: np.ndarray):
    rho = np.ascontiguousarray(rho, np.float64)
    gx, gy = _field(p), _field(p)
    lib().orc_grad_rho(ctypes.byref(p), _ptr(rho), _ptr(gx), _ptr(gy))
    return gx, gy


def step(p: Params, ft: np.ndarray, nsteps: int) -> np.ndarray:
    """Advance in place; ``ft`` holds post-collision populations."""
    assert ft.shape == (9, p.ny, p.nx)
    rc = lib().orc_step(ctypes.byref(p), _ptr(ft), int(nsteps))
    if rc != 0:
        raise MemoryError("oracle step failed")
    return ft


def velocity(p: Params, ft: np.ndarray):
    ft = np.ascontiguousarray(ft, np.float64)
    rho, ux, uy = _field(p), _field(p), _field(p)
    lib().orc_velocity(ctypes.byref(p), _ptr(ft), _ptr(rho), _ptr(ux), _ptr(uy))
    return rho, ux, uy


def residual(p: Params, ft: np.ndarray, ux_prev: np.ndarray, uy_prev: np.ndarray):
    out = np.zeros(4)
    lib().orc_residual(ctypes.byref(p), _ptr(np.ascontiguousarray(ft)), _ptr(ux_prev),
                       _ptr(uy_prev), _ptr(out))
    return out


def solve(p: Params, ft: np.ndarray, tol: float, check_every: int, max_steps: int,
          hist_cap: int = 100000):
    """Run to a relative velocity residual below ``tol``.

    Returns (status, steps, residual history); status 0 converged, 1 step
    limit, -3 diverged."""
    steps = ctypes.c_int64()
    nh = ctypes.c_int64()
    hist = np.zeros(hist_cap)
    st = lib().orc_solve(ctypes.byref(p), _ptr(ft), float(tol), int(check_every),
                         int(max_steps), ctypes.byref(steps), _ptr(hist),
                         int(hist_cap), ctypes.byref(nh))
    return st, steps.value, hist[: min(nh.value, hist_cap)].copy()
