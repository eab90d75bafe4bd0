"""Batches (prc_batch_*): problems of different sizes and parameters swept
by shared launches must give, member by member, exactly the results of the
same problem run alone through prc_step / prc_residual / prc_solve -- the
same bits, the same residual history, the same steps and status -- and those
single-problem paths are in turn held to the oracle by test_gpu_parity.py.
One member is also compared with the oracle directly."""
import numpy as np
import pytest

import workloads
from tests.common import lib_params, max_rel_velocity_error, oracle_deviation, oracle_params, spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


# Mixed members, all lid-driven cavities: sizes from 3 x 3 to wider than a
# tile, every r of the batch workload, gamma from 0.05 to 1, a body force and
# a reduced correction mask (the general sweep variant), and one member that
# diverges at its first check (gamma = 0.05 at U = 0.05 on a coarse grid).
MIX = [
    spec(64, 32, 2.0, 1.0, re=100.0, omega_nu=None, u_lid=0.05),
    spec(37, 53, 1.0, 0.3, re=200.0, omega_nu=None, u_lid=0.03),
    spec(130, 20, 0.5, 0.5, re=150.0, omega_nu=None, u_lid=0.02),
    spec(3, 3, 1.0, 1.0, omega_nu=1.1, u_lid=0.01),
    spec(70, 9, 4.0, 0.2, re=80.0, omega_nu=None, u_lid=0.04),
    spec(48, 24, 2.0, 0.05, re=1000.0, omega_nu=None, u_lid=0.05),   # diverges
    spec(40, 40, 1.0, 0.6, omega_nu=1.3, u_lid=0.02, fx=1e-6, fy=-2e-6),  # general variant
    spec(33, 65, 2.0, 0.4, re=120.0, omega_nu=None, u_lid=0.03, corrections=3),
    spec(200, 130, 1.0, 0.8, re=300.0, omega_nu=None, u_lid=0.05),
]


def alone(s, tol, K, max_steps):
    from paper_2208_03562_amd import solver
    sol = solver.Solver(lib_params(s))
    st, n, hist = sol.solve(tol, K, max_steps)
    return sol, st, n, hist


@pytest.mark.parametrize("tile", [None, 1, 2, 5, 6, 7])
def test_batch_solve_is_bitwise_the_single_solve(torch_cuda, tile):
    from paper_2208_03562_amd import solver
    tol, K, max_steps = 1e-4, 100, 1600
    b = solver.Batch()
    if tile is not None:
        b.set_tile(tile)
    for s in MIX:
        b.add(lib_params(s))
    status, steps, hists = b.solve(tol, K, max_steps, hist_cap=max_steps // K)
    assert status[5] == -3, status
    assert any(st == 0 for st in status) and any(st == 1 for st in status), status
    for i, s in enumerate(MIX):
        sol, st, n, hist = alone(s, tol, K, max_steps)
        assert (status[i], steps[i]) == (st, n), (i, status[i], steps[i], st, n)
        assert hists[i] == hist or (np.isnan(hists[i]).any() and st == -3), i
        a = b.members[i].get_state()
        c = sol.get_state()
        assert bool(((a == c) | (a.isnan() & c.isnan())).all()), i
    b.close()


def test_batch_step_and_residual_are_bitwise_single(torch_cuda):
    from paper_2208_03562_amd import solver
    specs = [MIX[0], MIX[1], MIX[3], MIX[6], MIX[8]]
    b = solver.Batch()
    singles = []
    for s in specs:
        b.add(lib_params(s))
        singles.append(solver.Solver(lib_params(s)))
    b.residual()          # snapshot
    for sol in singles:
        sol.residual()
    for n in (2, 130, 300):
        b.step(n)
        out = b.residual()
        for i, sol in enumerate(singles):
            sol.step(n)
            assert out[i] == sol.residual(), (i, n)
            assert bool((b.members[i].get_state() == sol.get_state()).all()), (i, n)
    b.close()


def test_member_joining_later_and_removal(torch_cuda):
    """A member added after others have run, and one removed mid-run: the
    first is bitwise its own solve, the second's buffers are left alone."""
    from paper_2208_03562_amd import solver
    b = solver.Batch()
    b.add(lib_params(MIX[0]))
    b.add(lib_params(MIX[2]))
    b.step(200)
    late = b.add(lib_params(MIX[1]))
    b.remove(1)
    frozen = b.members[1].get_state().clone()
    status, steps, hists = b.solve(1e-4, 100, 1000, hist_cap=10)
    assert status[1] == -5 and steps[1] == 200
    assert bool((b.members[1].get_state() == frozen).all())
    sol, st, n, hist = alone(MIX[1], 1e-4, 100, 1000)
    assert (status[late], steps[late], hists[late]) == (st, n, hist)
    assert bool((b.members[late].get_state() == sol.get_state()).all())
    # the first member had 200 steps before the solve: its limit counts them
    assert steps[0] <= 1000 and steps[0] % 100 == 0
    b.close()


@pytest.mark.parametrize("storage,tile", [("f64", None), ("f16", None), ("bf16", None),
                                          ("f16", 5), ("bf16", 6), ("f64", 5), ("f64", 6),
                                          ("f16", 7), ("bf16", 7), ("f64", 7)])
def test_batch_other_storage_types(torch_cuda, storage, tile):
    from paper_2208_03562_amd import capi, solver
    specs = [dict(MIX[0], storage=storage), dict(MIX[1], storage=storage),
             dict(MIX[6], storage=storage)]
    b = solver.Batch(storage=getattr(capi, "PRC_" + storage.upper()))
    if tile is not None:
        b.set_tile(tile)
    for s in specs:
        b.add(lib_params(s))
    status, steps, hists = b.solve(1e-3, 50, 400, hist_cap=8)
    for i, s in enumerate(specs):
        sol, st, n, hist = alone(s, 1e-3, 50, 400)
        assert (status[i], steps[i], hists[i]) == (st, n, hist)
        assert bool((b.members[i].get_state() == sol.get_state()).all())
    b.close()


@pytest.mark.parametrize("tile", [6, 7])
def test_batch_streamed_from_hbm_gives_the_single_step_bits(torch_cuda, tile):
    """Three 2048 x 1024 FP32 members: together their states exceed the
    last-level cache, so the batch stores non-temporally (and the 64 x 16
    shape runs its instance for streamed states); ten steps give each
    member the bits of ten single steps of it alone."""
    from paper_2208_03562_amd import capi, solver
    specs = [spec(2048, 1024, r, g, omega_nu=w, u_lid=0.05, storage="f32")
             for r, g, w in ((2.0, 0.5, 1.3), (0.5, 0.2, 1.1), (1.0, 1.0, 1.7))]
    b = solver.Batch()
    b.set_tile(tile)
    for k, s in enumerate(specs):
        i = b.add(lib_params(s))
        b.members[i].set_state(workloads.deviation_noise(s["nx"], s["ny"], 40 + k, 1e-3))
    b.step(10)
    torch_cuda.cuda.synchronize()
    got = [m.get_state() for m in b.members]
    b.close()
    del b
    for k, s in enumerate(specs):
        p = lib_params(s)
        capi.prc_set_tile(p, 1)  # single steps
        sol = solver.Solver(p)
        sol.set_state(workloads.deviation_noise(s["nx"], s["ny"], 40 + k, 1e-3))
        sol.step(10)
        assert bool((sol.get_state() == got[k]).all()), k
        capi.prc_set_tile(p, -1)
        del sol
    capi.prc_release_graphs()


def test_batch_member_against_oracle(O, torch_cuda):
    """FP64 member in a mixed batch against the oracle: round-off only."""
    from paper_2208_03562_amd import capi, solver
    specs = [dict(MIX[i], storage="f64") for i in (0, 2, 4)]
    b = solver.Batch(storage=capi.PRC_F64)
    for s in specs:
        b.add(lib_params(s))
    b.step(300)
    for i, s in enumerate(specs):
        po = oracle_params(O, s)
        ft = O.rest_state(po)
        O.step(po, ft, 300)
        dev = oracle_deviation(O, po, ft)
        got = b.members[i].get_state().cpu().numpy()
        assert np.abs(got - dev).max() < 1e-12 * 300 * max(np.abs(dev).max(), 1e-30), i
        _, ux, uy = (a.cpu().numpy() for a in b.members[i].macros())
        _, oux, ouy = O.velocity(po, ft)
        assert max_rel_velocity_error(ux, uy, oux, ouy, s["u_lid"]) < 1e-11
    b.close()


def test_batch_tune_keeps_results(torch_cuda):
    from paper_2208_03562_amd import solver
    a = solver.Batch()
    c = solver.Batch()
    for s in MIX[:5]:
        a.add(lib_params(s))
        c.add(lib_params(s))
    a.step(20)
    t = a.tune()          # sweeps f_a into f_b only: the state is unchanged
    assert t in range(7)
    a.step(40)
    c.step(60)
    for i in range(5):
        assert bool((a.members[i].get_state() == c.members[i].get_state()).all()), i
    a.close()
    c.close()


def test_batch_of_workload_instances_small(torch_cuda):
    """The first 24 instances of the 256-instance batch workload (seed 0),
    200 steps: every member bitwise equal to its own prc_step run."""
    from paper_2208_03562_amd import solver
    insts = workloads.batch_instances(256, seed=0)[:24]
    b = solver.Batch()
    specs = [spec(it.nx, it.ny, it.r, it.gamma, re=it.re, omega_nu=None, u_lid=it.u_lid)
             for it in insts]
    for s in specs:
        b.add(lib_params(s))
    b.tune()
    b.step(200)
    for i, s in enumerate(specs):
        sol = solver.Solver(lib_params(s))
        sol.step(200)
        a, c = b.members[i].get_state(), sol.get_state()
        assert bool(((a == c) | (a.isnan() & c.isnan())).all()), i
    b.close()
