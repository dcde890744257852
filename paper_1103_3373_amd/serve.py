"""Continuous-batching server for many independent simulations.

Requests (box size, scheme, Riemann solver, initial condition, number of
steps) arrive over time.  The server keeps every admitted simulation's state
resident in device memory, admits waiting requests in arrival order as soon
as their memory footprint fits under the cap, and advances *all* active
simulations by one step per tick: one batched launch of the fused solver per
(scheme, solver) specialization, each simulation a box-mode segment with its
own time step read from device memory, followed by that simulation's FP64
CFL time step.  The classes of a tick run on one stream per scheme, so their
launches overlap on the device, and their segment tables stay resident.  Requests that arrive while others are on the GPU join at the
next tick; finished ones retire and free their memory.  Host bookkeeping of
the next tick overlaps the device work of the current one.

Per-step latency is the completion time of step s minus the time the request
became eligible for it (its arrival for step 0, the completion of step s-1
afterwards); completion times come from device events.

The compute backend is pluggable: GpuBackend drives the HIP library; tests
of the admission/retirement/latency logic use a host-only backend.
"""
from __future__ import annotations

import dataclasses
import heapq
import time
from typing import Callable

import numpy as np

GROUP_BYTES_F32 = 5 * 4096 * 4


@dataclasses.dataclass
class Request:
    id: int
    arrival: float          # seconds since the start of the run
    n: int                  # box size (cells per side, multiple of 16)
    scheme: int
    riemann: int
    ic: str
    seed: int
    steps: int = 50


@dataclasses.dataclass
class Sim:
    req: Request
    footprint: int
    handle: object = None
    step: int = 0           # steps completed
    launched: int = 0       # steps launched (ticks run one ahead of completion)
    eligible: float = 0.0   # time at which the next step became eligible
    admitted: float = 0.0
    latencies: list = dataclasses.field(default_factory=list)
    finished: float = -1.0


def footprint_bytes(req: Request) -> int:
    """Device bytes held by a simulation: two state buffers, plus for VL its
    share of the library's half-step scratch.  Every simulation is a
    periodic-box segment, so that scratch holds the half step of the
    interiors only: one more state-sized buffer per VL simulation of the
    batched launch."""
    state = (req.n ** 3) * 20
    extra = state if req.scheme == 1 else 0
    return 2 * state + extra


class Server:
    def __init__(self, backend, mem_cap: float = 200e9, clock: Callable[[], float] | None = None):
        self.backend = backend
        self.mem_cap = mem_cap
        self.clock = clock or time.perf_counter
        self.pending: list = []        # heap of (arrival, id, Request)
        self.active: dict = {}         # id -> Sim
        self.done: dict = {}           # id -> Sim
        self.used = 0
        self.peak_used = 0
        self.t0 = None
        self.ticks = 0
        self.cell_updates = 0

    # -- request intake ---------------------------------------------------
    def submit(self, req: Request):
        if footprint_bytes(req) > self.mem_cap:
            raise ValueError(f"request {req.id} can never fit under the memory cap")
        heapq.heappush(self.pending, (req.arrival, req.id, req))

    def now(self) -> float:
        return self.clock() - self.t0

    # -- admission / retirement -------------------------------------------
    def _admit(self, now: float):
        admitted = []
        while self.pending and self.pending[0][0] <= now:
            req = self.pending[0][2]
            fp = footprint_bytes(req)
            if self.used + fp > self.mem_cap:
                break  # arrival order: later requests wait behind this one
            heapq.heappop(self.pending)
            sim = Sim(req, fp, eligible=req.arrival, admitted=now)
            sim.handle = self.backend.admit(req)
            self.used += fp
            self.peak_used = max(self.peak_used, self.used)
            self.active[req.id] = sim
            admitted.append(sim)
        return admitted

    def _retire(self, sim: Sim, t_done: float):
        sim.finished = t_done
        self.backend.retire(sim.handle)
        self.used -= sim.footprint
        del self.active[sim.req.id]
        self.done[sim.req.id] = sim

    # -- main loop ----------------------------------------------------------
    def run(self, until_empty: bool = True, max_ticks: int | None = None):
        self.t0 = self.clock()
        self.backend.start(self.clock, self.t0)
        inflight = None  # (tick token, sims stepped)
        while True:
            now = self.now()
            self._admit(now)
            if inflight is None and not any(s.launched < s.req.steps for s in self.active.values()):
                if self.active:  # nothing left to launch for the active ones (cannot happen)
                    raise RuntimeError("active simulations with no work and no tick in flight")
                if not self.pending:
                    break
                nxt = self.pending[0][0]
                self.backend.idle_until(self.t0 + nxt)
                continue
            token = None
            stepped = [s for s in self.active.values() if s.launched < s.req.steps]
            if stepped:
                token = self.backend.tick([s.handle for s in stepped])
                for s in stepped:
                    s.launched += 1
                self.ticks += 1
            # Complete the previous tick while the current one runs.
            if inflight is not None:
                self._complete(*inflight)
            inflight = (token, stepped) if token is not None else None
            if max_ticks is not None and self.ticks >= max_ticks:
                break
        if inflight is not None:
            self._complete(*inflight)
        self.backend.finish()

    def _complete(self, token, stepped):
        t_done = self.backend.wait(token)  # completion time (s since t0)
        for sim in stepped:
            if sim.req.id not in self.active:
                continue
            sim.latencies.append(t_done - sim.eligible)
            sim.eligible = t_done
            sim.step += 1
            self.cell_updates += sim.req.n ** 3
            if sim.step >= sim.req.steps:
                self._retire(sim, t_done)

    # -- report ---------------------------------------------------------------
    def report(self) -> dict:
        lat = np.array([x for s in self.done.values() for x in s.latencies]) * 1e3
        wall = max((s.finished for s in self.done.values()), default=0.0)
        waits = np.array([s.admitted - s.req.arrival for s in self.done.values()]) * 1e3
        return {
            "requests": len(self.done),
            "ticks": self.ticks,
            "cell_updates": int(self.cell_updates),
            "wall_s": wall,
            "cell_updates_per_s": self.cell_updates / wall if wall > 0 else 0.0,
            "p50_step_latency_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_step_latency_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_admission_wait_ms": float(waits.mean()) if waits.size else None,
            "peak_footprint_GB": self.peak_used / 1e9,
        }


class HostBackend:
    """Host-only backend for testing the server logic: a tick takes a fixed
    time per cell update and 'completes' on a simulated clock."""

    def __init__(self, s_per_cell=1e-10, s_fixed=1e-4):
        self.s_per_cell = s_per_cell
        self.s_fixed = s_fixed
        self.t = 0.0
        self.steps = {}

    def clock(self):
        return self.t

    def start(self, clock, t0):
        pass

    def admit(self, req):
        self.steps[req.id] = 0
        return req

    def retire(self, h):
        self.steps.pop(h.id)

    def idle_until(self, t):
        self.t = max(self.t, t)

    def tick(self, handles):
        cells = sum(h.n ** 3 for h in handles)
        self.t += self.s_fixed + self.s_per_cell * cells
        for h in handles:
            self.steps[h.id] += 1
        return self.t

    def wait(self, token):
        return token

    def finish(self):
        pass


class GpuBackend:
    """Backend on the HIP library: resident grouped boxes, batched box-mode
    launches per (scheme, solver) class, per-simulation FP64 dt, device
    events.

    overlap=True (default): every simulation lives on the stream of its
    scheme (three streams at the default priority, so the classes of one tick
    run concurrently on the device), and each class keeps its segment tables
    resident in device memory, one per parity of the tick (the two ping-pong
    buffers of each simulation swap roles every step); a class's tables are
    rebuilt only when its membership changes.  overlap=False: everything on
    the caller's stream with a table built and uploaded per class and tick
    (the former design, kept for comparison)."""

    def __init__(self, gamma=1.4, recon=None, char=True, limiter=None, cfl=None, ic_cache=None,
                 keep_results=False, overlap=True):
        import torch
        from . import hydro as H
        from . import workloads as W
        self.torch, self.H, self.W = torch, H, W
        self.gamma = gamma
        self.recon = H.PPM if recon is None else recon
        self.limiter = H.VANLEER if limiter is None else limiter
        self.char = char
        self.cfl = cfl or {H.MHM: 0.3, H.VL: 0.3, H.CTU: 0.5}
        self.dev = torch.device("cuda")
        self.stream = torch.cuda.current_stream()
        self.ic_cache = ic_cache if ic_cache is not None else {}
        self.keep_results = keep_results
        self.results = {}
        self.specs = {}
        self.overlap = overlap
        self.scheme_streams = {}
        self.classes = {}
        self.tick_no = 0
        self.table_builds = 0

    class Handle:
        __slots__ = ("req", "a", "b", "dt", "flip", "G", "stream")

    class Class:
        __slots__ = ("stream", "members", "tables", "total")

    def _ic(self, req):
        key = (req.ic, req.n, req.seed)
        if key not in self.ic_cache:
            box = self.W.initial_box(req.ic, req.n, self.gamma, req.seed)
            self.ic_cache[key] = self.torch.from_numpy(self.W.box_to_groups(box).astype(np.float32)).pin_memory()
        return self.ic_cache[key]

    def _stream_of(self, scheme):
        if not self.overlap:
            return self.stream
        if scheme not in self.scheme_streams:
            self.scheme_streams[scheme] = self.torch.cuda.Stream(device=self.dev)  # default priority
        return self.scheme_streams[scheme]

    def start(self, clock, t0):
        torch = self.torch
        self.t0_host = t0
        self.ev0 = torch.cuda.Event(enable_timing=True)
        self.ev0.record(self.stream)
        torch.cuda.synchronize()
        self.t0_gpu = clock() - t0  # host time of the reference event

    def admit(self, req):
        torch = self.torch
        h = GpuBackend.Handle()
        h.req = req
        host = self._ic(req)
        h.G = host.shape[0]
        h.stream = self._stream_of(req.scheme)
        # Buffers are allocated, filled and first used on the simulation's
        # stream, so the allocator orders their reuse after its work.
        with torch.cuda.stream(h.stream):
            h.a = torch.empty_like(host, device=self.dev)
            h.a.copy_(host, non_blocking=True)
            h.b = torch.empty_like(h.a)
            h.dt = torch.empty(1, dtype=torch.float64, device=self.dev)
            self.H.cfl_dt(h.a, 1.0 / req.n, self.gamma, self.cfl[req.scheme], dt_out=h.dt, stream=h.stream)
        h.flip = False
        return h

    def retire(self, h):
        if self.keep_results:
            with self.torch.cuda.stream(h.stream):
                src = h.b if h.flip else h.a
                self.results[h.req.id] = src.cpu()
        h.a = h.b = None

    def idle_until(self, t_abs):
        d = t_abs - time.perf_counter()
        if d > 0:
            time.sleep(d)

    def _spec(self, scheme, riemann):
        key = (scheme, riemann)
        if key not in self.specs:
            # Every simulation is a periodic box segment: VL computes its
            # half step once per cell.
            self.specs[key] = self.H.make_spec(scheme, self.recon, riemann, self.limiter, gamma=self.gamma,
                                               char=self.char, box_segs=True)
        return self.specs[key]

    def _table(self, hs, swapped):
        """Device segment table of a class: each simulation's step from its
        current buffer into the other (swapped: the step after)."""
        rows, first = [], 0
        for h in hs:
            src, dst = (h.b, h.a) if h.flip != swapped else (h.a, h.b)
            ng = h.req.n // 16
            rows.append((src, dst, None, h.dt, 1.0, 1.0 / h.req.n, first, h.G, (ng, ng, ng)))
            first += h.G
        self.table_builds += 1
        return self.H.seg_table(rows, self.dev), first

    def tick(self, handles):
        torch, H = self.torch, self.H
        by_spec = {}
        for h in handles:
            by_spec.setdefault((h.req.scheme, h.req.riemann), []).append(h)
        parity = self.tick_no & 1
        used = []
        for (scheme, riemann), hs in by_spec.items():
            cls = self.classes.get((scheme, riemann))
            if cls is None:
                cls = self.classes[(scheme, riemann)] = GpuBackend.Class()
                cls.stream, cls.members, cls.tables, cls.total = self._stream_of(scheme), None, [None, None], 0
            with torch.cuda.stream(cls.stream):
                ids = tuple(h.req.id for h in hs)
                if not self.overlap:
                    table, cls.total = self._table(hs, False)
                else:
                    if ids != cls.members:
                        # Every member steps every tick until its last step,
                        # so the two tables stay valid while the membership
                        # does: this tick's, and the next one's.
                        cls.members = ids
                        cls.tables[parity], cls.total = self._table(hs, False)
                        cls.tables[1 - parity], _ = self._table(hs, True)
                    table = cls.tables[parity]
                H.solve_batch(table, len(hs), cls.total, self._spec(scheme, riemann), stream=cls.stream)
                # the same table: each segment's new state (`out`) -> its dt
                H.cfl_dt_batch(table, len(hs), cls.total, gamma=self.gamma, cfl=self.cfl[scheme], stream=cls.stream)
            for h in hs:
                h.flip = not h.flip
            if cls.stream not in used:
                used.append(cls.stream)
        for st in used:
            if st is not self.stream:
                ev = torch.cuda.Event()
                ev.record(st)
                self.stream.wait_event(ev)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        self.tick_no += 1
        return ev

    def wait(self, ev):
        ev.synchronize()
        return self.t0_gpu + self.ev0.elapsed_time(ev) * 1e-3

    def finish(self):
        self.torch.cuda.synchronize()

    def final_state(self, req_id):
        return self.results.get(req_id)
