"""Host side of ``prc_serve`` and of the online server (``prc_server_*``):
building requests, keeping their result arrays alive, reading results.

Argument marshalling and bookkeeping only; the serving loop (admission,
batching, memory pool, worker thread) runs in the library."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import capi
from .capi import prc_params


@dataclass
class Served:
    status: int
    steps: int
    residual: float
    arrival_s: float
    admit_s: float
    done_s: float
    ux: np.ndarray | None = None
    uy: np.ndarray | None = None

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def serve(problems: list[prc_params], arrivals: list[float], *, storage=capi.PRC_F32,
          bc=capi.PRC_BC_CAVITY, tol=1e-7, check_every=500, max_steps=20000,
          hbm_budget=8 << 30, max_active=0, tile=-1, fields=False, stream: int = 0):
    """Run prc_serve on problems arriving at `arrivals` (seconds, sorted);
    returns one :class:`Served` per request, with the final velocity fields
    when ``fields`` is set."""
    assert len(problems) == len(arrivals)
    outs = []
    reqs = []
    for p, t in zip(problems, arrivals):
        if fields:
            ux = np.empty((p.ny, p.nx), dtype=np.float64)
            uy = np.empty((p.ny, p.nx), dtype=np.float64)
            outs.append((ux, uy))
            reqs.append(capi.prc_request(float(t), p, ux.ctypes.data_as(ctypes.c_void_p),
                                         uy.ctypes.data_as(ctypes.c_void_p)))
        else:
            outs.append((None, None))
            reqs.append(capi.prc_request(float(t), p, None, None))
    cfg = capi.prc_serve_config(storage=storage, bc=bc, tol=tol, check_every=check_every,
                                max_steps=max_steps, hbm_budget=int(hbm_budget),
                                max_active=max_active, tile=tile)
    res = capi.prc_serve(cfg, reqs, stream)
    return [Served(r.status, r.steps, r.residual, float(t), r.admit_s, r.done_s, ux, uy)
            for r, t, (ux, uy) in zip(res, arrivals, outs)]


@dataclass
class Finished:
    ticket: int
    status: int
    steps: int
    residual: float
    submit_s: float
    admit_s: float
    done_s: float
    ux: np.ndarray | None = None
    uy: np.ndarray | None = None

    @property
    def latency_s(self) -> float:
        return self.done_s - self.submit_s


class OnlineServer:
    """A running ``prc_server``: requests are submitted at any time and
    finished ones polled; the worker thread inside the library admits,
    batches and retires them."""

    def __init__(self, *, storage=capi.PRC_F32, bc=capi.PRC_BC_CAVITY, tol=1e-7,
                 check_every=500, max_steps=20000, hbm_budget=8 << 30, max_active=0, tile=-1,
                 stream: int = 0):
        cfg = capi.prc_serve_config(storage=storage, bc=bc, tol=tol, check_every=check_every,
                                    max_steps=max_steps, hbm_budget=int(hbm_budget),
                                    max_active=max_active, tile=tile)
        self.h = capi.prc_server_create(cfg, stream)
        self._fields = {}  # ticket -> (ux, uy) host arrays the library writes

    def submit(self, p: prc_params, fields: bool = False) -> int:
        ux = uy = None
        if fields:
            ux = np.empty((p.ny, p.nx), dtype=np.float64)
            uy = np.empty((p.ny, p.nx), dtype=np.float64)
        t = capi.prc_server_submit(self.h, p, ux.ctypes.data if fields else None,
                                   uy.ctypes.data if fields else None)
        self._fields[t] = (ux, uy)
        return t

    def poll(self, wait_s: float = 0.0) -> list[Finished]:
        out = []
        for r in capi.prc_server_poll(self.h, wait_s):
            ux, uy = self._fields.pop(r.ticket, (None, None))
            out.append(Finished(r.ticket, r.status, r.steps, r.residual, r.submit_s, r.admit_s,
                                r.done_s, ux, uy))
        return out

    def status(self):
        """(waiting, active, finished but not polled)"""
        return capi.prc_server_status(self.h)

    def close(self) -> None:
        if self.h:
            capi.prc_server_destroy(self.h)
            self.h = None
            self._fields.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_online(problems: list[prc_params], arrivals: list[float], **kw) -> list[Served]:
    """Replay a trace through an OnlineServer from Python: each problem is
    submitted at its arrival time (seconds after the server starts) while
    finished ones are polled.  Latency is measured from submission."""
    import time
    fields = kw.pop("fields", False)
    srv = OnlineServer(**kw)
    t0 = time.perf_counter()
    ticket_of = {}
    got = {}
    i = 0
    try:
        while len(got) < len(problems):
            now = time.perf_counter() - t0
            while i < len(problems) and arrivals[i] <= now:
                ticket_of[srv.submit(problems[i], fields)] = i
                i += 1
            wait = max(0.0, arrivals[i] - (time.perf_counter() - t0)) if i < len(problems) else 1.0
            for f in srv.poll(wait):
                got[ticket_of[f.ticket]] = f
    finally:
        srv.close()
    return [Served(got[k].status, got[k].steps, got[k].residual, got[k].submit_s,
                   got[k].admit_s, got[k].done_s, got[k].ux, got[k].uy)
            for k in range(len(problems))]


def footprint_bytes(p: prc_params) -> int:
    """Device bytes prc_serve sets aside for a request: two states and the
    velocity snapshot, each rounded up to 256 bytes."""
    rnd = lambda n: (n + 255) // 256 * 256  # noqa: E731
    return 2 * rnd(capi.prc_state_bytes(p)) + rnd(16 * p.nx * p.ny)


def summary(served: list[Served]) -> dict:
    """Throughput and latency percentiles over the requests that ran."""
    ran = [s for s in served if s.status != capi.PRC_EINVAL]
    lat = np.array([s.latency_s for s in ran])
    span = max(s.done_s for s in ran) - min(s.arrival_s for s in ran)
    by = {}
    for s in served:
        by[s.status] = by.get(s.status, 0) + 1
    names = {0: "converged", 1: "max_steps", -3: "diverged", -1: "rejected"}
    # last relative residual of the requests that ran to their step budget
    res = np.array([s.residual for s in served if s.status == 1 and np.isfinite(s.residual)])
    conv = np.array([s.latency_s for s in served if s.status == 0])
    steps = np.array([s.steps for s in served if s.status == 0])
    return {
        "requests": len(served),
        "outcomes": {names.get(k, str(k)): v for k, v in sorted(by.items())},
        "solves_per_s": len(ran) / span if span > 0 else None,
        "converged_per_s": by.get(0, 0) / span if span > 0 else None,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(lat.max()),
        # latency of the requests that reached the tolerance (arrival to result)
        "converged_latency_p50_s": float(np.percentile(conv, 50)) if conv.size else None,
        "converged_latency_p99_s": float(np.percentile(conv, 99)) if conv.size else None,
        "converged_steps_p50": int(np.median(steps)) if steps.size else None,
        "span_s": span,
        "budget_residual_p50": float(np.median(res)) if res.size else None,
    }
