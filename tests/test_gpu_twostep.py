"""Two time steps per launch (tile shapes 5-8): every node passes through
exactly the single-step arithmetic, with the intermediate state rounded to
the storage type, so the results must be the single-step sweep's bits -- for
every boundary type, storage (FP64, FP32, FP16, BF16), sweep variant and frame, on
grids smaller than a tile and with ragged edges, over step counts that use
the two-step launches alone, with single steps around them, and through the
captured graphs."""
import pytest

import workloads
from tests.common import lib_params, spec

pytestmark = pytest.mark.gpu

TWO_STEP_TILES = [5, 6, 7, 8]

CASES = [
    ("cavity", 2.0, 0.5, dict(u_lid=0.05)),
    ("cavity", 0.5, 0.1, dict(u_lid=0.02, fx=1e-6)),
    ("periodic", 1.0, 0.3, dict(fx=1e-5, fy=-2e-5)),
    ("channel", 4.0, 1.0, dict(u_lid=0.03, frame=1)),
    ("cavity", 1.0, 0.7, dict(u_lid=0.04, corrections=3, omega_3=1.2)),
]
GRIDS = [(150, 37), (7, 5), (3, 70), (130, 260)]


def run(s, tile, nsteps, seed):
    from paper_2208_03562_amd import capi, solver
    sol = solver.Solver(lib_params(s))
    capi.prc_set_tile(sol.p, tile)
    sol.set_state(workloads.deviation_noise(s["nx"], s["ny"], seed, 1e-3))
    sol.step(nsteps)
    out = sol.get_state()
    capi.prc_set_tile(sol.p, -1)
    capi.prc_release_graphs()
    return out


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-r{c[1]}-g{c[2]}")
@pytest.mark.parametrize("nx,ny", GRIDS)
def test_two_step_launches_give_the_single_step_bits(storage, case, nx, ny):
    bc, r, gamma, extra = case
    s = spec(nx, ny, r, gamma, omega_nu=1.3, bc=bc, storage=storage, **extra)
    for nsteps in (4, 7):
        ref = run(s, 0, nsteps, seed=nx + ny)
        for tile in TWO_STEP_TILES:
            got = run(s, tile, nsteps, seed=nx + ny)
            assert bool((got == ref).all()), (tile, nsteps)


def test_two_step_graph_replays():
    """136 steps: two replays of the 64-step graph and 8 more steps."""
    s = spec(300, 140, 2.0, 0.2, re=500.0, omega_nu=None, u_lid=0.05, storage="f32")
    ref = run(s, 1, 136, seed=9)
    for tile in TWO_STEP_TILES:
        assert bool((run(s, tile, 136, seed=9) == ref).all()), tile


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("case", CASES[:3], ids=lambda c: f"{c[0]}-r{c[1]}-g{c[2]}")
def test_streamed_instance_gives_the_single_step_bits(storage, case):
    """The 1024-thread two-step tiles have an instance for states streamed
    from HBM (chosen by size); forced on small ragged grids it must give the
    single-step bits too."""
    from paper_2208_03562_amd import capi
    bc, r, gamma, extra = case
    for nx, ny in ((150, 37), (130, 260)):
        s = spec(nx, ny, r, gamma, omega_nu=1.3, bc=bc, storage=storage, **extra)
        ref = run(s, 0, 7, seed=nx + ny)
        capi.prc_set_streamed(1)
        try:
            for tile in (7, 8):
                got = run(s, tile, 7, seed=nx + ny)
                assert bool((got == ref).all()), (tile, nx, ny)
        finally:
            capi.prc_set_streamed(-1)
            capi.prc_release_graphs()
