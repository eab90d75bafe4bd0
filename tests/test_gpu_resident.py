"""The resident sweep (tile 9): many steps per launch with the state held in
LDS, subdomains exchanging their edges through memory.  Every node passes
through the single-step arithmetic with the state rounded to the storage type
between steps, so the results must be the single-step sweep's bits -- for
every boundary type, 32- and 16-bit storage, both sweep variants and frames,
grids smaller than a subdomain and with ragged edges, odd and even step
counts, long calls, replays of a graph the caller captured, and the
1024 x 512 cavity that takes one subdomain per compute unit."""
import pytest
import torch

import workloads
from tests.common import lib_params, spec

pytestmark = pytest.mark.gpu

RESIDENT = 9

CASES = [
    ("cavity", 2.0, 0.5, dict(u_lid=0.05), [(150, 37), (7, 5), (3, 70), (130, 260)]),
    ("cavity", 0.5, 0.1, dict(u_lid=0.02, fx=1e-6), [(150, 37), (64, 32)]),
    ("periodic", 1.0, 0.3, dict(fx=1e-5, fy=-2e-5), [(128, 64), (64, 96)]),
    ("channel", 4.0, 1.0, dict(u_lid=0.03, frame=1), [(128, 37), (64, 70)]),
    ("cavity", 1.0, 0.7, dict(u_lid=0.04, corrections=3, omega_3=1.2), [(200, 90)]),
]


def run(s, tile, nsteps, seed):
    from paper_2208_03562_amd import capi, solver
    sol = solver.Solver(lib_params(s))
    capi.prc_set_tile(sol.p, tile)
    sol.set_state(workloads.deviation_noise(s["nx"], s["ny"], seed, 1e-3))
    sol.step(nsteps)
    out = sol.get_state()
    sol.residual()  # reports a resident launch that lost a wait
    capi.prc_set_tile(sol.p, -1)
    capi.prc_release_graphs()
    return out


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-r{c[1]}-g{c[2]}")
def test_resident_sweep_gives_the_single_step_bits(storage, case):
    bc, r, gamma, extra, grids = case
    for nx, ny in grids:
        s = spec(nx, ny, r, gamma, omega_nu=1.3, bc=bc, storage=storage, **extra)
        for nsteps in (1, 2, 7):
            ref = run(s, 0, nsteps, seed=nx + ny)
            got = run(s, RESIDENT, nsteps, seed=nx + ny)
            assert bool((got == ref).all()), (nx, ny, nsteps)


def test_resident_long_call():
    """136 steps in one call: one resident launch (the resident sweep takes
    any number of steps per launch; no launch graph is cached for it)."""
    s = spec(300, 140, 2.0, 0.2, re=500.0, omega_nu=None, u_lid=0.05, storage="f32")
    ref = run(s, 1, 136, seed=9)
    assert bool((run(s, RESIDENT, 136, seed=9) == ref).all())


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_resident_1024x512_cavity(storage):
    """One 64 x 32 subdomain per compute unit; 300 steps against the
    single-step sweep, bit for bit, and a residual that reports no lost
    wait."""
    w = workloads.CAVITY_1024x512_F32_MA006
    s = spec(w.nx, w.ny, w.r, w.gamma, re=w.re, omega_nu=None, u_lid=w.u_lid, storage=storage)
    ref = run(s, 1, 300, seed=3)
    got = run(s, RESIDENT, 300, seed=3)
    assert bool(torch.isfinite(got.float()).all())
    assert bool((got == ref).all())


def test_resident_rejects_grids_beyond_the_lds():
    """A state too large for one subdomain per compute unit, FP64, and a
    periodic side that cuts a subdomain are refused."""
    from paper_2208_03562_amd import capi, solver
    for s in (spec(4096, 2048, 1.0, 1.0, u_lid=0.05, storage="f32"),
              spec(128, 64, 1.0, 1.0, u_lid=0.05, storage="f64"),
              spec(100, 64, 1.0, 1.0, bc="channel", u_lid=0.05, storage="f32")):
        p = lib_params(s)
        with pytest.raises(capi.PrcError):
            capi.prc_set_tile(p, RESIDENT)


@pytest.mark.parametrize("mode", ["plain", "timed", "kernel_only"])
def test_resident_steps_captured_by_the_caller(mode):
    """A caller captures prc_step (one resident launch of 64 steps) into a
    graph of its own and replays it three times, with eager work and host
    synchronisation between the replays: the base of the step tags lives on
    the device, so every replay continues the count, and after each replay
    the state equals that of 64 more single steps, bit for bit.  The same
    for prc_step_timed (its events become event-record nodes of the graph,
    and each replay's pair gives a positive elapsed time)."""
    from paper_2208_03562_amd import capi, solver
    nx, ny = 200, 90
    s = spec(nx, ny, 2.0, 0.5, omega_nu=1.3, u_lid=0.05, storage="f32")
    p = lib_params(s)
    noise = workloads.deviation_noise(nx, ny, 5, 1e-3)
    try:
        capi.prc_set_tile(p, 1)  # reference: single steps
        ref = solver.Solver(p)
        ref.set_state(noise)
        ref.step(2)
        want = []
        for _ in range(3):
            ref.step(64)
            want.append(ref.get_state())
        del ref

        capi.prc_set_tile(p, RESIDENT)
        stream = torch.cuda.Stream()
        sol = solver.Solver(p, stream=stream)
        sol.set_state(noise)
        sol.step(2)  # the first resident call sets up its counters, outside capture
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record(stream)
        ev[1].record(stream)
        stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            # 64 steps: the newest state is back in the same buffer
            if mode == "plain":
                sol.step(64)
            else:
                sol.step_timed(64, *ev, kernel_only=(mode == "kernel_only"))
        for k in range(3):
            g.replay()
            sol.residual()  # synchronises; reports a lost wait
            scratch = torch.ones(1 << 20, device="cuda:0").sum()  # eager work between replays
            torch.cuda.synchronize()
            assert float(scratch) == float(1 << 20)
            assert bool((sol.get_state() == want[k]).all()), k
            if mode != "plain":
                assert ev[0].elapsed_time(ev[1]) > 0.0
    finally:
        capi.prc_set_tile(p, -1)
        capi.prc_release_graphs()


@pytest.mark.parametrize("mode", ["plain", "timed", "kernel_only"])
def test_resident_calls_on_two_streams_give_the_single_step_bits(mode):
    """Two problems on two streams issue resident calls back to back with no
    synchronisation between them: the library orders resident launches on one
    device (a launch on another stream waits for the latest one), so each
    problem gets the single-step bits and no launch loses a wait.  Plain
    calls, timed calls (the caller's events around the call: the launch
    records its ordering event itself) and timed calls whose dispatch records
    the caller's events."""
    from paper_2208_03562_amd import capi, solver
    specs = [spec(200, 90, 2.0, 0.5, omega_nu=1.3, u_lid=0.05, storage="f32"),
             spec(256, 128, 0.5, 0.2, omega_nu=1.1, u_lid=0.02, storage="f32")]
    counts = [[3, 8, 1, 12], [5, 2, 9, 4]]
    ref = [run(s, 0, sum(c), seed=20 + k) for k, (s, c) in enumerate(zip(specs, counts))]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    sols = []
    for k, s in enumerate(specs):
        sol = solver.Solver(lib_params(s), stream=streams[k])
        capi.prc_set_tile(sol.p, RESIDENT)
        sol.set_state(workloads.deviation_noise(s["nx"], s["ny"], 20 + k, 1e-3))
        sols.append(sol)
    events = []
    for k in range(2):
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record(streams[k])
        ev[1].record(streams[k])
        events.append(ev)
    torch.cuda.synchronize()
    for i in range(4):
        for k in range(2):
            if mode == "plain":
                sols[k].step(counts[k][i])
            else:
                sols[k].step_timed(counts[k][i], *events[k], kernel_only=(mode == "kernel_only"))
    torch.cuda.synchronize()
    capi.prc_resident_status()  # raises if a launch lost a wait
    for k in range(2):
        assert bool((sols[k].get_state() == ref[k]).all()), k
        capi.prc_set_tile(sols[k].p, -1)


def test_lost_wait_is_reported_once_and_the_next_launch_is_clean():
    """A wait limit of zero ticks makes the first value that is not there yet
    end the launch (every workgroup still finishes normally).  The failure is
    reported once -- by prc_resident_status here -- and the next launch,
    with the default limit, gives the single-step bits again."""
    from paper_2208_03562_amd import capi, solver
    w = workloads.CAVITY_1024x512_F32
    s = spec(w.nx, w.ny, w.r, w.gamma, re=w.re, omega_nu=None, u_lid=w.u_lid, storage="f32")
    sol = solver.Solver(lib_params(s))
    capi.prc_set_tile(sol.p, RESIDENT)
    capi.prc_resident_status()  # nothing pending
    capi.prc_set_resident_wait(0)
    try:
        sol.step(2000)
        torch.cuda.synchronize()
    finally:
        capi.prc_set_resident_wait(-1)
    try:
        capi.prc_resident_status()
        lost = False
    except capi.PrcError as e:
        assert e.status == capi.PRC_EHIP
        lost = True
    capi.prc_resident_status()  # reported once, then clear
    if not lost:
        capi.prc_set_tile(sol.p, -1)
        pytest.skip("no value arrived late in 2000 steps: nothing to report")
    # a clean launch from a fresh state
    small = spec(200, 90, 2.0, 0.5, omega_nu=1.3, u_lid=0.05, storage="f32")
    ref = run(small, 0, 7, seed=31)
    assert bool((run(small, RESIDENT, 7, seed=31) == ref).all())
    capi.prc_set_tile(sol.p, -1)


@pytest.mark.parametrize("tile", [RESIDENT, 7, 0])
def test_timed_step_gives_the_same_bits_and_a_kernel_time(tile):
    """prc_step_timed: the same state as prc_step; its events (taken by the
    resident sweep's dispatch, around the call for other shapes) give a
    positive elapsed time."""
    from paper_2208_03562_amd import capi, solver
    s = spec(256, 128, 2.0, 0.5, omega_nu=1.3, u_lid=0.05, storage="f32")
    ref = run(s, tile, 37, seed=5)
    sol = solver.Solver(lib_params(s))
    capi.prc_set_tile(sol.p, tile)
    sol.set_state(workloads.deviation_noise(256, 128, 5, 1e-3))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(sol.stream)
    b.record(sol.stream)
    sol.step_timed(20, a, b)
    sol.step_timed(17, a, b, kernel_only=True)
    torch.cuda.synchronize()
    assert a.elapsed_time(b) > 0.0
    assert bool((sol.get_state() == ref).all())
    capi.prc_set_tile(sol.p, -1)
    capi.prc_release_graphs()


def draw_resident(seed):
    """A seeded random problem the resident sweep takes: up to 16 x 16
    subdomains (grids up to 1024 x 512, ragged on walled sides, whole
    subdomains on periodic ones), any boundary type, 32- or 16-bit storage,
    the method as published or a general setting, 1 to 29 steps."""
    import numpy as np
    rng = np.random.default_rng(5000 + seed)
    bc = ["cavity", "periodic", "channel"][rng.integers(3)]
    nx = int(rng.integers(3, 1025)) if bc == "cavity" else 64 * int(rng.integers(1, 17))
    ny = 32 * int(rng.integers(1, 17)) if bc == "periodic" else int(rng.integers(3, 513))
    r = float(rng.choice([0.5, 1.0, 2.0]))
    extra = dict(u_lid=0.0 if bc == "periodic" else float(rng.uniform(0.0, 0.05)))
    if rng.random() < 0.5:
        extra.update(corrections=int(rng.integers(0, 8)), frame=int(rng.integers(2)),
                     omega_xi=float(rng.uniform(0.8, 1.5)), omega_3=float(rng.uniform(0.8, 1.5)),
                     fx=float(rng.uniform(-1e-5, 1e-5)), fy=float(rng.uniform(-1e-5, 1e-5)))
    s = spec(nx, ny, r, float(rng.uniform(0.1, 1.0)), omega_nu=float(rng.uniform(0.6, 1.8)), bc=bc,
             storage=["f32", "f16", "bf16"][rng.integers(3)], **extra)
    return s, int(rng.integers(1, 30))


@pytest.mark.parametrize("seed", range(24))
def test_resident_random_problem_gives_the_single_step_bits(seed):
    s, nsteps = draw_resident(seed)
    ref = run(s, 0, nsteps, seed=seed)
    got = run(s, RESIDENT, nsteps, seed=seed)
    assert bool((got == ref).all()), (s, nsteps)
