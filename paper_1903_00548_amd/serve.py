"""Continuous-batching request loop for transport solves.

Each request is one device (leads, slab blocks, potential) with an energy
grid.  The loop keeps a set of active requests; every step it forms ONE
batched solve (qtx_solve_batch) from the next chunk of energies of every
active request, so requests that arrive while others are on the GPU join
the next launch and their work overlaps on the device.  Requests are
admitted in arrival order while the number of active slots and the HBM
footprint of the admitted requests stay within their limits; a finished
request frees its slot and its memory at once.

Every energy is solved by the same kernels whatever else is in the batch,
so a request's result does not depend on the mix (the GPU tests check this
bit for bit).  The scheduling itself is host logic over a backend with
open / solve / close; QtxBackend drives the HIP library.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, List, Optional

import numpy as np


def padded_block(m: int) -> int:
    """Block size the library pads m to (16, 32, 48, 64, 96, 128)."""
    return ((m + 15) // 16) * 16 if m <= 64 else (96 if m <= 96 else 128)


def request_footprint(N: int, m: int, nE: int, uniform: bool, energies_per_step: int) -> int:
    """HBM bytes held for one admitted request: its device and lead blocks,
    potential, result buffers, and its share of one step's self-energy and
    broadening buffers (4 M^2 complex doubles per energy)."""
    M = padded_block(m)
    blocks = 0 if uniform else (4 * N - 2) * M * M * 16
    leads = 2 * 4 * M * M * 16
    outputs = nE * (2 * N + 1) * 8
    step = min(nE, energies_per_step) * 4 * M * M * 16
    return blocks + leads + N * 8 + outputs + step


@dataclasses.dataclass
class Request:
    rid: int
    t_arrival: float
    device: object                    # workloads.Device
    E: np.ndarray
    T: Optional[np.ndarray] = None
    ldos: Optional[np.ndarray] = None
    next: int = 0                     # first energy not yet solved
    handle: object = None
    footprint: int = 0
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    status: int = 0

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.t_arrival


class QtxBackend:
    """The HIP library: one batch context; one problem context per request."""

    def __init__(self, device: int = 0, eta: float = 1e-6, precision: int = 0, want_ldos: bool = True):
        from . import _lib
        self._lib = _lib
        self.ctx = _lib.Context(device)
        self.eta = eta
        self.precision = precision
        self.want_ldos = want_ldos

    def open(self, dev):
        return self._lib.fill(self.ctx.problem(), dev)

    def solve(self, handles, grids):
        Ts, Ls, st = self._lib.solve_batch(self.ctx, handles, grids, self.eta, self.precision, self.want_ldos)
        return Ts, Ls, st

    def close(self, handle):
        handle.close()


class Server:
    def __init__(self, backend, hbm_budget: int = 64 << 30, max_active: int = 32,
                 energies_per_step: int = 512, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.backend = backend
        self.sleep = sleep
        self.hbm_budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.energies_per_step = int(energies_per_step)
        self.clock = clock
        self.pending: collections.deque = collections.deque()
        self.active: List[Request] = []
        self.done: List[Request] = []
        self.rejected: List[Request] = []
        self.used = 0
        self.steps = 0
        self.energies_solved = 0
        self.batch_sizes: List[int] = []
        self.solve_seconds = 0.0          # wall time inside backend.solve (the GPU's share of the loop)

    # ------------------------------------------------------------ intake
    def submit(self, req: Request):
        d = req.device
        req.footprint = request_footprint(d.N, d.m, len(req.E), d.uniform, self.energies_per_step)
        if req.footprint > self.hbm_budget:
            self.rejected.append(req)        # can never fit
            return
        self.pending.append(req)

    def _admit(self, now: float):
        while self.pending and self.pending[0].t_arrival <= now and len(self.active) < self.max_active \
                and self.used + self.pending[0].footprint <= self.hbm_budget:
            r = self.pending.popleft()
            r.handle = self.backend.open(r.device)
            r.T = np.empty(len(r.E))
            r.ldos = np.empty((len(r.E), 2, r.device.N))
            r.t_admit = now
            self.used += r.footprint
            self.active.append(r)

    # -------------------------------------------------------------- step
    def step(self) -> int:
        """One batched launch over the next chunk of every active request;
        returns the number of energies solved."""
        if not self.active:
            return 0
        chunks = []
        for r in self.active:
            a = r.next
            b = min(len(r.E), a + self.energies_per_step)
            chunks.append((r, a, b))
        t_call = self.clock()
        Ts, Ls, st = self.backend.solve([r.handle for r, _, _ in chunks], [r.E[a:b] for r, a, b in chunks])
        now = self.clock()
        self.solve_seconds += now - t_call
        n = 0
        still = []
        for (r, a, b), T, L in zip(chunks, Ts, Ls):
            r.T[a:b] = T
            if L is not None:
                r.ldos[a:b] = L
            r.status = max(r.status, int(st))
            r.next = b
            n += b - a
            if r.next >= len(r.E):
                r.t_done = now
                self.backend.close(r.handle)
                r.handle = None
                self.used -= r.footprint
                self.done.append(r)
            else:
                still.append(r)
        self.active = still
        self.steps += 1
        self.energies_solved += n
        self.batch_sizes.append(n)
        return n

    # --------------------------------------------------------------- run
    def run(self, requests: List[Request], time_limit: Optional[float] = None, realtime: bool = True):
        """Serve requests whose t_arrival are seconds after the start.  With
        realtime, arrivals follow the wall clock (the loop idles until the
        next arrival when nothing is active); without, every request is
        available at once.  Stops when all are done or after time_limit s."""
        t0 = self.clock()
        for r in sorted(requests, key=lambda x: x.t_arrival):
            if realtime:
                r.t_arrival = t0 + r.t_arrival
            else:
                r.t_arrival = t0
            self.submit(r)
        while self.pending or self.active:
            now = self.clock()
            if time_limit is not None and now - t0 > time_limit:
                break
            self._admit(now)
            if not self.active:
                if self.pending:
                    nxt = self.pending[0].t_arrival
                    if nxt > now:
                        self.sleep(min(nxt - now, 0.05))
                    continue
                break
            self.step()
        wall = self.clock() - t0
        self.close_all()
        return self.stats(wall)

    def close_all(self):
        """Release the problems of requests still active (after a time limit)."""
        for r in self.active:
            if r.handle is not None:
                self.backend.close(r.handle)
                r.handle = None
                self.used -= r.footprint

    def stats(self, wall: float) -> dict:
        lat = np.array([r.latency for r in self.done]) if self.done else np.zeros(0)
        return {
            "wall_s": wall,
            "completed": len(self.done),
            "unfinished": len(self.active) + len(self.pending),
            "rejected": len(self.rejected),
            "energies_solved": self.energies_solved,
            "energy_solves_per_s": self.energies_solved / wall if wall > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "steps": self.steps,
            "solve_fraction_of_wall": self.solve_seconds / wall if wall > 0 else 0.0,
            "mean_energies_per_step": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
        }
