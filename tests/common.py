"""Shared helpers for the parity tests: one problem description turned into
the oracle's parameters and the library's parameters, each side computing its
own derived quantities (relaxation rate from Re, rest weights)."""
from __future__ import annotations

import numpy as np

STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
BC = {"cavity": 0, "periodic": 1, "channel": 2}


def spec(nx, ny, r=1.0, gamma=1.0, *, re=None, omega_nu=1.2, u_lid=0.0, fx=0.0, fy=0.0,
         bc="cavity", storage="f32", corrections=7, omega_xi=1.0, omega_1=1.0, omega_3=1.0,
         omega_4=1.0, rho0=1.0, frame=0):
    return dict(nx=nx, ny=ny, r=r, gamma=gamma, re=re, omega_nu=omega_nu, u_lid=u_lid, fx=fx,
                fy=fy, bc=bc, storage=storage, corrections=corrections, omega_xi=omega_xi,
                omega_1=omega_1, omega_3=omega_3, omega_4=omega_4, rho0=rho0, frame=frame)


def oracle_params(O, s):
    w = s["omega_nu"] if s["omega_nu"] is not None else 1.0   # replaced below when re is set
    p = O.params(s["nx"], s["ny"], s["r"], s["gamma"], w, omega_xi=s["omega_xi"],
                 omega_1=s["omega_1"], omega_3=s["omega_3"], omega_4=s["omega_4"],
                 u_lid=s["u_lid"], fx=s["fx"], fy=s["fy"], rho0=s["rho0"], bc=BC[s["bc"]],
                 corrections=s["corrections"], frame=s.get("frame", 0))
    if s["re"] is not None:
        p = O.with_re(p, s["re"])
    return p


def lib_params(s):
    from paper_2208_03562_amd import solver
    return solver.make_params(
        s["nx"], s["ny"], s["r"], s["gamma"], re=s["re"],
        omega_nu=None if s["re"] is not None else s["omega_nu"], u_lid=s["u_lid"], fx=s["fx"],
        fy=s["fy"], rho0=s["rho0"], bc=BC[s["bc"]], storage=STORAGE[s["storage"]],
        corrections=s["corrections"], omega_xi=s["omega_xi"], omega_1=s["omega_1"],
        omega_3=s["omega_3"], omega_4=s["omega_4"], frame=s.get("frame", 0))


def oracle_deviation(O, po, ft):
    """oracle populations minus the oracle's own rest state"""
    return ft - O.rest_populations(po)[:, None, None]


def max_rel_velocity_error(ux_a, uy_a, ux_b, uy_b, U):
    return float(max(np.abs(np.asarray(ux_a) - ux_b).max(),
                     np.abs(np.asarray(uy_a) - uy_b).max()) / U)
