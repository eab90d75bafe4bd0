"""Write batch_steps_to_convergence.txt: steps to convergence of six
instances of the seeded uneven-instance workload (Nx, Ny log-uniform in
[64, 512], r in {0.5, 1, 2, 4}, gamma uniform in [0.05, 1], Re log-uniform in
[100, 5000], lid 0.05; numpy seed 0, 256 draws) in the FP64 oracle: relative
velocity residual over 500 steps below 1e-7 (the residual of Sec. 5.2 as
read in the oracle: both components, normalised by |u|), at most 100,000
steps.  The six are the smallest of the workload that converge within that
budget.  Also writes batch_residual_history.txt: the residual at every check
of those runs, from which the step of any larger tolerance follows.  Calls
only the oracle.

    python tests/golden/make_batch_steps.py
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

INDICES = (231, 185, 46, 13, 127, 146)
TOL, CHECK, MAX_STEPS = 1e-7, 500, 100_000


def solve(i):
    import workloads
    from oracle import oracle as O
    O.set_threads(1)
    it = workloads.batch_instances(256, seed=0)[i]
    p = O.with_re(O.params(it.nx, it.ny, it.r, it.gamma, 1.0, u_lid=it.u_lid), it.re)
    ft = O.rest_state(p)
    st, n, hist = O.solve(p, ft, TOL, CHECK, MAX_STEPS)
    before = hist[-2] if len(hist) > 1 else float("nan")
    return i, it, st, n, before, hist[-1], list(hist)


def main():
    with mp.Pool(len(INDICES)) as pool:
        rows = pool.map(solve, INDICES)
    out = os.path.join(HERE, "batch_steps_to_convergence.txt")
    with open(out, "w") as fh:
        fh.write("# Steps to convergence in the FP64 oracle (tests/golden/make_batch_steps.py):\n")
        fh.write(f"# tol {TOL:g} on the relative velocity residual, checked every {CHECK} steps,\n")
        fh.write("# from rest; residuals of the last two checks (before and at convergence).\n")
        fh.write("# index nx ny r gamma re u_lid status steps R_before R_at\n")
        for i, it, st, n, rb, ra, _ in rows:
            fh.write(f"{i} {it.nx} {it.ny} {it.r:.17g} {it.gamma:.17g} {it.re:.17g} "
                     f"{it.u_lid:.17g} {st} {n} {rb:.6e} {ra:.6e}\n")
    hist_out = os.path.join(HERE, "batch_residual_history.txt")
    with open(hist_out, "w") as fh:
        fh.write("# Relative velocity residual at every check (every 500 steps, the first\n")
        fh.write("# at step 500) of the runs in batch_steps_to_convergence.txt, FP64 oracle\n")
        fh.write("# (tests/golden/make_batch_steps.py).  index R_1 R_2 ...\n")
        for i, *_, hist in rows:
            fh.write(f"{i} " + " ".join(f"{R:.9e}" for R in hist) + "\n")
    print(open(out).read())


if __name__ == "__main__":
    main()
