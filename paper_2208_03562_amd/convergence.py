"""Convergence acceleration by preconditioning: the cavity experiments of
Sec. 5.2 and Sec. 6 of arXiv 2208.03562, run as one batch on the GPU.

For each setup the steady state is computed with gamma = 1 (no
preconditioning) and with the paper's smaller gammas; the number of steps
until the relative velocity residual first falls below a threshold is
compared.  The paper's residual is the L2 norm of the change of u over 20
steps and its step counts are read off convergence-history figures, so only
the ratios are comparable, and only roughly; this run uses the library's
residual (both components, relative, over 1000 steps) in FP64.

    python -m paper_2208_03562_amd.convergence [--out FILE]

writes a Markdown table (and prints one JSON line).
"""
from __future__ import annotations

import argparse
import json
import math
import time
from dataclasses import dataclass

import numpy as np

from . import capi, solver


@dataclass(frozen=True)
class Setup:
    name: str
    nx: int
    ny: int
    r: float
    re: float
    ma: float
    gammas: tuple
    frame: int = capi.PRC_FRAME_CENTRAL
    paper: str = ""


# grid aspect ratio r = dy/dx, cavity L = nx, H = ny r (Sec. 5.2)
SETUPS = [
    Setup("shallow AR 0.25, Re 100, Ma 0.06", 100, 125, 0.2, 100.0, 0.06, (1.0, 0.5, 0.1, 0.08),
          paper="~610,000 steps at gamma 1, ~24,000 at gamma 0.08 (x25)"),
    Setup("shallow AR 0.25, Re 100, Ma 0.01", 100, 125, 0.2, 100.0, 0.01, (1.0, 0.5, 0.1, 0.05),
          paper="~5,000,000 steps at gamma 1, ~97,000 at gamma 0.05 (x51)"),
    Setup("deep AR 2, Re 100, Ma 0.06", 100, 125, 1.6, 100.0, 0.06, (1.0, 0.5, 0.1, 0.08),
          paper="x14 at gamma 0.08"),
    Setup("deep AR 2, Re 100, Ma 0.02", 100, 125, 1.6, 100.0, 0.02, (1.0, 0.5, 0.1, 0.05),
          paper="x23 at gamma 0.05 (at its stability limit)"),
    Setup("deep AR 2, Re 1000, Ma 0.06", 100, 150, 4.0 / 3.0, 1000.0, 0.06, (1.0, 0.1),
          paper="~11,154,000 steps at gamma 1, ~583,000 at gamma 0.1 (x19)"),
    Setup("shallow AR 0.25, r 0.5, Re 100, Ma 0.06, PRC", 100, 50, 0.5, 100.0, 0.06, (0.5, 0.1),
          paper="PRC and PRNR converge at the same rate"),
    Setup("shallow AR 0.25, r 0.5, Re 100, Ma 0.06, PRNR", 100, 50, 0.5, 100.0, 0.06, (0.5, 0.1),
          frame=capi.PRC_FRAME_RAW),
]

CHECK = 1000
THRESHOLDS = (1e-6, 1e-8, 1e-10, 1e-12)
TOL = 1e-12


def lid_speed(ma: float, r: float) -> float:
    """U = Ma c_s with c_s = q / sqrt(3), q = min(1, r) (eq. 2)."""
    return ma * min(1.0, r) / math.sqrt(3.0)


def first_below(hist, thr):
    for k, R in enumerate(hist):
        if R < thr:
            return (k + 1) * CHECK
    return None


def run(max_steps: int = 16_000_000, log=print):
    """One batch per setup (its gammas side by side); a line per setup as it
    finishes.  Returns the rows and the total wall time."""
    rows = []
    t_all = time.perf_counter()
    for s in SETUPS:
        U = lid_speed(s.ma, s.r)
        b = solver.Batch(storage=capi.PRC_F64)
        ids = []
        for g in s.gammas:
            p = solver.make_params(s.nx, s.ny, s.r, g, re=s.re, u_lid=U, storage=capi.PRC_F64,
                                   frame=s.frame)
            ids.append((g, b.add(p), p.omega_nu))
        t0 = time.perf_counter()
        status, steps, hists = b.solve(TOL, CHECK, max_steps, hist_cap=max_steps // CHECK)
        b.close()
        for g, i, w in ids:
            rows.append(dict(setup=s.name, gamma=g, omega_nu=w, status=status[i], steps=steps[i],
                             reach={f"{t:g}": first_below(hists[i], t) for t in THRESHOLDS}))
        log(f"[convergence] {s.name}: {time.perf_counter() - t0:.1f} s, steps "
            + ", ".join(f"gamma {g:g}: {steps[i]} ({status[i]})" for g, i, _ in ids))
    return rows, time.perf_counter() - t_all


def markdown(rows, wall, cmd):
    names = {0: "converged", 1: "step limit", -3: "diverged"}
    out = ["# Convergence acceleration by preconditioning (cavity setups of Sec. 5.2, 6)", "",
           "Steps until the relative velocity residual (both components, over 1000 steps, "
           "FP64) first falls below each threshold; ratio = steps at gamma 1 / steps at "
           "this gamma, at the deepest threshold reached by both.  The paper's counts come from its figures and use its own "
           "residual (change of u over 20 steps), so only the ratios compare, roughly.", "",
           f"Command: `{cmd}` (one batch per setup, {wall:.1f} s in all on one MI355X).", ""]
    setups = []
    for r in rows:
        if r["setup"] not in setups:
            setups.append(r["setup"])
    for name in setups:
        s = next(x for x in SETUPS if x.name == name)
        rs = [r for r in rows if r["setup"] == name]
        base = next((r for r in rs if r["gamma"] == 1.0), None)
        out += [f"## {name}", "",
                f"{s.nx} x {s.ny} nodes, r = {s.r:g}; paper: {s.paper}", "",
                "| gamma | omega_nu | outcome | " + " | ".join(f"steps to {t:g}" for t in THRESHOLDS)
                + " | ratio |", "|---|---|---|" + "---|" * (len(THRESHOLDS) + 1)]
        for r in rs:
            reach = [r["reach"][f"{t:g}"] for t in THRESHOLDS]
            ratio = ""
            if base:
                both = [t for t in THRESHOLDS
                        if base["reach"][f"{t:g}"] and r["reach"][f"{t:g}"]]
                if both:
                    t = f"{both[-1]:g}"
                    ratio = f"{base['reach'][t] / r['reach'][t]:.1f} (at {t})"
            out.append(f"| {r['gamma']:g} | {r['omega_nu']:.4f} | {names.get(r['status'], r['status'])} | "
                       + " | ".join(f"{x:,}" if x else "-" for x in reach) + f" | {ratio} |")
        out.append("")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="")
    ap.add_argument("--max-steps", type=int, default=16_000_000)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    rows, wall = run(args.max_steps, log=lambda m: print(m, flush=True))
    print(json.dumps({"wall_s": wall, "runs": rows}), flush=True)
    if args.out:
        cmd = "python -m paper_2208_03562_amd.convergence --out " + args.out
        with open(args.out, "w") as fh:
            fh.write(markdown(rows, wall, cmd))


if __name__ == "__main__":
    main()
