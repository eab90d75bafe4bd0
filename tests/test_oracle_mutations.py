"""Mutation check of the oracle's pins for the density-gradient path.

Each case plants one plausible mistake in a copy of the oracle's C source
(a dropped term, a wrong sign, a wrong factor, an index slip in eq. 38-40,
43, 45 or in the gradient stencil), builds the copy on the CPU and runs the
pins of test_oracle_gradient against it: at least one pin must fail for
every mistake, and none may fail for the oracle as it is.  The mistakes are
planted on the CPU only, in a temporary folder; the GPU library is not
involved.
"""
from __future__ import annotations

import importlib.util
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from tests import test_oracle_gradient as G

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.join(os.path.dirname(HERE), "oracle")

# name -> list of (regex, replacement); each regex must match the source
MUTATIONS = {
    # every lambda coefficient of eq. 38-40 doubled
    "lambda_doubled": [(r"(const double l(?:bx|by|sx|sy|11x|11y) = )", r"\g<1>2.0 * ")],
    # e_b and e_s (eq. 43) left out of R2s and R2d (eq. 45)
    "e_terms_dropped": [(r"R2s = n2s \+ eb;", "R2s = n2s;"), (r"R2d = n2d \+ es;", "R2d = n2d;")],
    # the lambda~ terms of eq. 40 with the wrong sign
    "lambda_tilde_sign": [(r"const double l11x = -ig1", "const double l11x = ig1"),
                          (r"const double l11y = -ig1", "const double l11y = ig1")],
    # the y derivative of the density three times too large
    "grad_y_scaled": [(r"gy\[\(size_t\)j \* nx \+ i\] = sy / c2;",
                       "gy[(size_t)j * nx + i] = 3.0 * sy / c2;")],
    # eq. 39: lambda_4y with the sign of lambda_3y
    "lambda_sy_sign": [(r"const double lsy = \(Ug", "const double lsy = -(Ug")],
    # eq. 43: B with the x factor (U_gamma c2 - 1) instead of (U_gamma c2 - r^2)
    "B_index_slip": [(r"const double B = 0\.5 \* \(Ug \* c2 - r2\)", "const double B = 0.5 * (Ug * c2 - 1.0)")],
    # eq. 38: the bulk lambdas with the shear rate
    "lambda_b_rate": [(r"const double lbx = -\(Ug \* c2 - 1\.0\) \* hxi",
                       "const double lbx = -(Ug * c2 - 1.0) * hnu"),
                      (r"const double lby = -\(Ug \* c2 - r2\) \* hxi",
                       "const double lby = -(Ug * c2 - r2) * hnu")],
    # e_s with the sign of e_b
    "e_s_sign": [(r"const double es = -A \* drx \+ B \* dry;", "const double es = -A * drx - B * dry;")],
    # a five-point gradient (axis neighbours only), still exact on linear rho
    "five_point_gradient": [(r"for \(int a = 1; a < 9; \+\+a\) \{\n(\s+)int ni = i \+ EX\[a\]",
                             "for (int a = 1; a < 5; ++a) {\n\\1int ni = i + EX[a]"),
                            (r"gx\[\(size_t\)j \* nx \+ i\] = sx / c2;",
                             "gx[(size_t)j * nx + i] = sx / (2.0 * wx(1, c2) * wy(0, c2, p->r));"),
                            (r"gy\[\(size_t\)j \* nx \+ i\] = sy / c2;",
                             "gy[(size_t)j * nx + i] = sy / (2.0 * wx(0, c2) * wy(1, c2, p->r) * p->r * p->r);")],
}


def pin_failures(O) -> list[str]:
    """Names of the gradient-path pins that fail for oracle module O."""
    bad = []
    for r in (0.5, 1.0, 2.0):
        e = G.linear_gradient_errors(O, r)
        if max(e.values()) > 1e-11:
            bad.append(f"linear_gradient_r{r}")
    try:
        G.test_grad_rho_leading_error_isotropic_on_square_grid(O)
    except AssertionError:
        bad.append("isotropic_gradient")
    for case in G.ACOUSTIC + G.TRANSVERSE:
        errs = G.acoustic_errors(O, *case)
        if any(e["damping"] > G.TOL_DAMPING or e["frequency"] > G.TOL_FREQUENCY
               or e.get("transverse", 0.0) > G.TOL_TRANSVERSE or not np.isfinite(e["damping"])
               for e in errs):
            bad.append(f"acoustic_{case[0]}_{case[3]}_{case[5]}")
    for case in G.STRAIN:
        e = G.strain_rate_errors(O, *case)
        if not max(e.values()) < G.TOL_STRAIN:
            bad.append(f"strain_{case[0]}_{case[3]}")
    return bad


def _load(so_path: str, name: str):
    """A fresh copy of the oracle's Python wrapper bound to another build."""
    spec = importlib.util.spec_from_file_location(f"oracle_{name}",
                                                  os.path.join(ORACLE_DIR, "oracle.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.LIB = so_path
    mod._lib = None
    return mod


def _build_mutant(tmp, name):
    src = open(os.path.join(ORACLE_DIR, "prc_oracle.c")).read()
    for pat, rep in MUTATIONS[name]:
        src, n = re.subn(pat, rep, src)
        assert n > 0, f"mutation {name}: pattern {pat!r} no longer matches the oracle source"
    d = tmp / name
    d.mkdir()
    open(d / "prc_oracle.c", "w").write(src)
    shutil.copy(os.path.join(ORACLE_DIR, "prc_oracle.h"), d)
    so = str(d / "liborc.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", so,
                    str(d / "prc_oracle.c"), "-lm"], check=True)
    return _load(so, name)


def test_pins_hold_for_the_oracle(O):
    assert pin_failures(O) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_a_pin(tmp_path_factory, name):
    O = _build_mutant(tmp_path_factory.mktemp("mut"), name)
    with np.errstate(all="ignore"):
        bad = pin_failures(O)
    assert bad, f"no pin catches the planted mistake {name}"
