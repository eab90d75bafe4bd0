"""prc_residual_noalloc: the convergence check with its scratch in a static
device array instead of a caller's buffer, for callers that cannot allocate.
Two calls in a row -- a grid that uses the largest partition of the
reduction (1024 blocks), then a smaller one that uses 9 -- each against
prc_residual on the same state and snapshot, bit for bit, sums and updated
snapshot alike."""
import numpy as np
import pytest
import torch

import workloads
from tests.common import lib_params, spec

pytestmark = pytest.mark.gpu


def _state(s, nsteps):
    from paper_2208_03562_amd import solver
    sol = solver.Solver(lib_params(s))
    sol.set_state(workloads.deviation_noise(s["nx"], s["ny"], s["nx"] + s["ny"], 1e-3))
    sol.step(nsteps)
    torch.cuda.synchronize()
    return sol


def test_noalloc_residual_matches_prc_residual():
    from paper_2208_03562_amd import capi
    cases = [spec(1024, 512, 2.0, 0.1, omega_nu=1.2, u_lid=0.03, storage="f32"),
             spec(70, 30, 0.5, 0.5, omega_nu=1.4, u_lid=0.02, storage="f64")]
    for s in cases:
        sol = _state(s, 11)
        f = sol.current().data_ptr()
        prev = torch.from_numpy(np.random.default_rng(s["nx"]).uniform(
            -0.01, 0.01, (2, s["ny"], s["nx"]))).to("cuda")
        a, b = prev.clone(), prev.clone()
        for _ in range(2):  # the second round starts from the updated snapshots
            ref = capi.prc_residual(sol.p, f, a.data_ptr(), sol.scratch.data_ptr(), sol.s)
            got = capi.prc_residual_noalloc(sol.p, f, b.data_ptr(), sol.s)
            assert got == ref, (s["nx"], got, ref)
            assert bool((a == b).all())
        assert ref[1] > 0 and np.isfinite(ref).all()
