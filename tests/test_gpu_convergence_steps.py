"""Steps to convergence on the GPU against the FP64 oracle, on six instances
of the seeded uneven-instance workload (relative velocity residual checked
every 500 steps, from rest).  The oracle's residual at every check is stored
in tests/golden/batch_residual_history.txt (and its steps to 1e-7 in
batch_steps_to_convergence.txt) by tests/golden/make_batch_steps.py, which
calls only the oracle; the oracle's step count for any tolerance is the
first check below it.

* FP64 storage: within 1 % of the oracle's steps at 1e-5, 1e-6 and 1e-7
  (round-off only, so the same check).
* FP32 storage: within 1 % at 1e-5 and 1e-6.  At 1e-7 the FP32 state's
  residual levels off between 0.7e-7 and 1.2e-7 (its rounding floor: the
  velocity of an FP32 state is known to about 1e-7 of itself), so FP32
  reaches 1e-7 later than FP64 or not at all; the test requires it never
  earlier, and for the instances whose FP64 residual drops clearly through
  1e-7 (by at least a factor 2 at that check) within 20 % of the oracle's
  steps (measured on MI355X: 3.5 % to 15 % later)."""
import os

import numpy as np
import pytest

from tests.common import lib_params, spec

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CHECK, MAX_STEPS = 500, 100_000


def _rows():
    out = []
    for line in open(os.path.join(HERE, "golden", "batch_steps_to_convergence.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        out.append(dict(index=int(f[0]), nx=int(f[1]), ny=int(f[2]), r=float(f[3]),
                        gamma=float(f[4]), re=float(f[5]), u_lid=float(f[6]), status=int(f[7]),
                        steps=int(f[8])))
    hist = {}
    for line in open(os.path.join(HERE, "golden", "batch_residual_history.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        hist[int(f[0])] = np.array([float(x) for x in f[1:]])
    for r in out:
        r["hist"] = hist[r["index"]]
    return out


ROWS = _rows()


def oracle_steps(row, tol):
    """First check below tol in the oracle's history, in steps."""
    h = row["hist"]
    below = np.nonzero(h < tol)[0]
    return (int(below[0]) + 1) * CHECK


def _spec(row, storage):
    return spec(row["nx"], row["ny"], row["r"], row["gamma"], re=row["re"], omega_nu=None,
                u_lid=row["u_lid"], storage=storage)


def gpu_history(row, storage):
    from paper_2208_03562_amd import solver
    sol = solver.Solver(lib_params(_spec(row, storage)))
    st, n, hist = sol.solve(0.0, CHECK, MAX_STEPS)  # tol 0: the whole residual history
    assert st == 1 and n == MAX_STEPS
    return np.asarray(hist)


def first_below(hist, tol):
    below = np.nonzero(hist < tol)[0]
    return (int(below[0]) + 1) * CHECK if below.size else None


def test_stored_counts_agree_with_stored_histories():
    for row in ROWS:
        assert row["status"] == 0 and oracle_steps(row, 1e-7) == row["steps"], row["index"]


@pytest.mark.parametrize("row", ROWS, ids=lambda r: f"i{r['index']}_{r['nx']}x{r['ny']}")
def test_fp64_steps_to_convergence_match_oracle(row):
    h = gpu_history(row, "f64")
    for tol in (1e-5, 1e-6, 1e-7):
        ref = oracle_steps(row, tol)
        got = first_below(h, tol)
        assert got is not None and abs(got - ref) <= 0.01 * ref, (tol, got, ref)


@pytest.mark.parametrize("row", ROWS, ids=lambda r: f"i{r['index']}_{r['nx']}x{r['ny']}")
def test_fp32_steps_to_convergence_match_oracle(row):
    h = gpu_history(row, "f32")
    for tol in (1e-5, 1e-6):
        ref = oracle_steps(row, tol)
        got = first_below(h, tol)
        assert got is not None and abs(got - ref) <= 0.01 * ref, (tol, got, ref)
    ref = oracle_steps(row, 1e-7)
    got = first_below(h, 1e-7)
    assert got is None or got >= ref, (got, ref)
    k = ref // CHECK - 1
    if row["hist"][k - 1] >= 2.0 * row["hist"][k]:
        assert got is not None and got <= 1.2 * ref, (got, ref)


def test_batched_members_take_the_solo_steps():
    """The six side by side in one FP32 batch at tol 1e-6: each converges at
    the oracle's step."""
    from paper_2208_03562_amd import capi, solver
    b = solver.Batch()
    for row in ROWS:
        b.add(lib_params(_spec(row, "f32")))
    status, steps, _ = b.solve(1e-6, CHECK, MAX_STEPS)
    for row, s, n in zip(ROWS, status, steps):
        assert s == capi.PRC_MEMBER_CONVERGED and n == oracle_steps(row, 1e-6), (row["index"], s, n)
    b.close()
