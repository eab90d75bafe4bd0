"""Thin PyTorch-side convenience over the C ABI.

PyTorch only provides device memory and the stream here; all computation runs
in ``libprc.so``.  A :class:`Solver` owns the two population buffers, the
velocity snapshot and the scratch buffer of one problem, and tracks which
buffer holds the newest state (the ping-pong rule of ``prc_step``).
"""
from __future__ import annotations

import torch

from . import capi
from .capi import prc_params

TORCH_DTYPE = {capi.PRC_F64: torch.float64, capi.PRC_F32: torch.float32,
               capi.PRC_F16: torch.float16, capi.PRC_BF16: torch.bfloat16}


def make_params(nx, ny, r=1.0, gamma=1.0, *, re=None, omega_nu=None, u_lid=0.0, fx=0.0, fy=0.0,
                rho0=1.0, bc=capi.PRC_BC_CAVITY, storage=capi.PRC_F32,
                corrections=capi.PRC_CORR_ALL, omega_xi=1.0, omega_1=1.0, omega_3=1.0,
                omega_4=1.0, frame=capi.PRC_FRAME_CENTRAL) -> prc_params:
    p = capi.prc_params_default()
    p.nx, p.ny, p.r, p.gamma = int(nx), int(ny), float(r), float(gamma)
    p.u_lid, p.fx, p.fy, p.rho0 = float(u_lid), float(fx), float(fy), float(rho0)
    p.bc, p.storage, p.corrections, p.frame = int(bc), int(storage), int(corrections), int(frame)
    p.omega_xi, p.omega_1, p.omega_3, p.omega_4 = omega_xi, omega_1, omega_3, omega_4
    if re is not None:
        capi.prc_params_from_re(p, re)
    elif omega_nu is not None:
        p.omega_nu = float(omega_nu)
    capi.prc_validate(p)
    return p


class Solver:
    def __init__(self, p: prc_params, device="cuda:0", stream: torch.cuda.Stream | None = None):
        capi.prc_validate(p)
        self.p = p.copy()
        self.device = torch.device(device)
        self.row_stride, self.plane_stride = capi.prc_layout(self.p)
        dt = TORCH_DTYPE[self.p.storage]
        nbytes = capi.prc_state_bytes(self.p)
        esize = torch.tensor([], dtype=dt).element_size()
        assert nbytes % esize == 0
        self.fa = torch.empty(nbytes // esize, dtype=dt, device=self.device)
        self.fb = torch.empty(nbytes // esize, dtype=dt, device=self.device)
        self.u_prev = torch.zeros((2, self.p.ny, self.p.nx), dtype=torch.float64, device=self.device)
        self.scratch = torch.empty(capi.prc_scratch_bytes(self.p), dtype=torch.uint8,
                                   device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.steps = 0
        self.init()

    # -- buffers --------------------------------------------------------
    @property
    def s(self) -> int:
        return self.stream.cuda_stream

    def current(self) -> torch.Tensor:
        return self.fa if self.steps % 2 == 0 else self.fb

    def other(self) -> torch.Tensor:
        return self.fb if self.steps % 2 == 0 else self.fa

    def init(self):
        capi.prc_init(self.p, self.fa.data_ptr(), self.s)
        capi.prc_init(self.p, self.fb.data_ptr(), self.s)
        self.steps = 0

    def view(self, buf: torch.Tensor) -> torch.Tensor:
        """[9][ny][nx] view of a state buffer (the library's strides)."""
        return torch.as_strided(buf, (9, self.p.ny, self.p.nx), (self.plane_stride, self.row_stride, 1))

    def set_state(self, dev) -> None:
        """Load deviations f - rho0 w (array [9][ny][nx]) as the current state."""
        t = torch.as_tensor(dev).to(device=self.device, dtype=self.fa.dtype)
        assert t.shape == (9, self.p.ny, self.p.nx)
        with torch.cuda.stream(self.stream):
            self.view(self.current()).copy_(t)

    def get_state(self) -> torch.Tensor:
        with torch.cuda.stream(self.stream):
            out = self.view(self.current()).to(torch.float64)
        self.stream.synchronize()
        return out

    # -- method ---------------------------------------------------------
    def step(self, n: int) -> None:
        capi.prc_step(self.p, self.current().data_ptr(), self.other().data_ptr(), n, self.s)
        self.steps += int(n)

    def step_timed(self, n: int, start: torch.cuda.Event, stop: torch.cuda.Event,
                   kernel_only: bool = False) -> None:
        """step(n) with start/stop (timing events, recorded once already so
        that their HIP events exist) recorded by the library around the work,
        or with kernel_only by the resident sweep's dispatch itself."""
        capi.prc_step_timed(self.p, self.current().data_ptr(), self.other().data_ptr(), n,
                            start.cuda_event, stop.cuda_event, kernel_only, self.s)
        self.steps += int(n)

    def macros(self):
        ny, nx = self.p.ny, self.p.nx
        rho = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        ux = torch.empty_like(rho)
        uy = torch.empty_like(rho)
        capi.prc_macros(self.p, self.current().data_ptr(), rho.data_ptr(), ux.data_ptr(),
                        uy.data_ptr(), self.s)
        self.stream.synchronize()
        return rho, ux, uy

    def residual(self):
        return capi.prc_residual(self.p, self.current().data_ptr(), self.u_prev.data_ptr(),
                                 self.scratch.data_ptr(), self.s)

    def converted(self, storage: int) -> "Solver":
        """A new solver for the same problem in another storage type, holding
        this solver's current state (prc_convert) and velocity snapshot, on
        the same stream."""
        q = self.p.copy()
        q.storage = storage
        out = Solver(q, device=self.device, stream=self.stream)
        capi.prc_convert(self.p, self.current().data_ptr(), storage, out.fa.data_ptr(), self.s)
        with torch.cuda.stream(self.stream):
            out.u_prev.copy_(self.u_prev)
        return out

    def solve(self, tol: float, check_every: int, max_steps: int):
        """Run from the current state; returns (status, steps taken, history)."""
        fa, fb = self.current(), self.other()
        st, n, hist = capi.prc_solve(self.p, fa.data_ptr(), fb.data_ptr(), self.u_prev.data_ptr(),
                                     self.scratch.data_ptr(), tol, check_every, max_steps,
                                     hist_cap=max(1, max_steps // check_every + 1), stream=self.s)
        self.steps += n
        return st, n, hist


class Batch:
    """Many problems advanced side by side by shared launches (prc_batch_*).

    Each member is a :class:`Solver` (it owns the member's buffers); the
    batch holds the library's batch object.  All members share one storage
    type, one boundary type and the batch's stream."""

    def __init__(self, storage=capi.PRC_F32, bc=capi.PRC_BC_CAVITY, device="cuda:0",
                 stream: torch.cuda.Stream | None = None):
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = capi.prc_batch_create(storage, bc)
        self.members: list[Solver] = []
        self.active: list[bool] = []
        self._joined_at: list[int] = []

    @property
    def s(self) -> int:
        return self.stream.cuda_stream

    def add(self, p: prc_params) -> int:
        """Allocate a problem at rest and add it; returns its id."""
        return self.add_solver(Solver(p, device=self.device, stream=self.stream))

    def add_solver(self, sol: Solver) -> int:
        """Add an existing problem (its newest state must be in its first buffer)."""
        assert sol.steps % 2 == 0, "the newest state must be in f_a"
        i = capi.prc_batch_add(self.handle, sol.p, sol.fa.data_ptr(), sol.fb.data_ptr(),
                               sol.u_prev.data_ptr())
        assert i == len(self.members)
        self.members.append(sol)
        self.active.append(True)
        self._joined_at.append(sol.steps)
        return i

    def active_ids(self):
        return [i for i, a in enumerate(self.active) if a]

    def remove(self, i: int) -> None:
        capi.prc_batch_remove(self.handle, i)
        self.active[i] = False

    def step(self, n: int) -> None:
        capi.prc_batch_step(self.handle, n, self.s)
        for i in self.active_ids():
            self.members[i].steps += int(n)

    def residual(self):
        """{id: [N, D, mass, max |u|^2]} of the active members."""
        out = capi.prc_batch_residual(self.handle, self.s)
        return {i: list(out[4 * i: 4 * i + 4]) for i in self.active_ids()}

    def solve(self, tol: float, check_every: int, max_steps: int, hist_cap: int = 0):
        """prc_batch_solve; returns (status, steps since joining, histories) per id."""
        status, steps, hists = capi.prc_batch_solve(self.handle, tol, check_every, max_steps,
                                                    hist_cap=hist_cap, stream=self.s)
        for i, m in enumerate(self.members):
            if self.active[i]:
                m.steps = self._joined_at[i] + steps[i]  # even: newest state in f_a
                self.active[i] = status[i] == capi.PRC_MEMBER_ACTIVE
        return status, steps, hists

    def tune(self) -> int:
        return capi.prc_batch_tune(self.handle, self.s)

    def set_tile(self, tile: int) -> None:
        capi.prc_batch_set_tile(self.handle, tile)

    def close(self) -> None:
        if self.handle:
            capi.prc_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
