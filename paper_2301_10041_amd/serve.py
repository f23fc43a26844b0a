"""Request loop for independent FSI steps (continuous admission under an HBM budget).

Each request is one semi-implicit step (fsi_step) on its own fluid grid and solid mesh.
A slot is a resident libfsi context for one grid size n, with its own HIP stream; its
fluid blocks and multigrid hierarchy stay on the device and the solid is swapped per
request with fsi_set_solid (grow-only buffers, so a warm slot allocates nothing).
Requests are admitted in arrival order as soon as a slot of their size is idle, or a new
slot fits the HBM budget (idle slots of other sizes are evicted, least recently used
first, to make room); requests that do not fit yet wait while later ones that fit go
ahead.  Slots run concurrently (the ctypes calls release the GIL), so the work of
different requests overlaps on the device.  Results are independent of the mix: every
kernel is deterministic and slots share no device state.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import fsi


@dataclass
class Request:
    rid: int
    arrival: float               # seconds from the start of the trace
    workload: object             # inputs.Workload (one solid)
    u_seed: int = 0


@dataclass
class Result:
    rid: int
    n: int
    arrival: float
    start: float = 0.0
    done: float = 0.0
    stats: dict = field(default_factory=dict)
    state: np.ndarray | None = None
    slot: int = -1

    @property
    def latency(self):
        return self.done - self.arrival


class Slot:
    def __init__(self, sid, n, wl, stream):
        self.sid = sid
        self.n = n
        self.stream = stream
        xy, tri = wl.solid_mesh()
        self.ctx = fsi.Context(n, xy, tri, nu=wl.nu, rho=wl.rho, dt=wl.dt, kappa=wl.kappa, stream=stream)
        self.busy = False
        self.last_used = time.perf_counter()
        self.bytes = self.ctx.sizes["device_bytes"]

    def close(self):
        self.ctx.close()


class Server:
    def __init__(self, hbm_budget=None, max_slots=16, prec=fsi.FP32, pc=fsi.PC_TRI, rtol=1e-8,
                 keep_states=False):
        import torch
        self.torch = torch
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = max(free - (8 << 30), 1 << 30)
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.opts = fsi.Opts(restart=30, rtol=rtol, pc=pc, prec=prec)
        self.keep_states = keep_states
        self.slots: list[Slot] = []
        self.cv = threading.Condition()
        self.reserved = 0            # bytes of live slots (estimates until measured)
        self.max_inflight = 0
        self.evictions = 0
        self._next_sid = 0

    # -- admission ---------------------------------------------------------------
    def _bytes_needed(self, wl):
        xy, tri = wl.solid_mesh()
        need = fsi.footprint(wl.n, xy.shape[0], tri.shape[0], wl.nu, wl.rho, wl.dt)
        if need > self.budget:
            raise fsi.FsiError(fsi.FSI_E_NOMEM, f"request of {need} B can never fit the budget {self.budget} B")
        return need

    def prewarm(self, workloads):
        """Create idle slots ahead of the traffic (one per workload given, e.g. the largest
        solid of each grid size, so later requests of that size allocate nothing)."""
        torch = self.torch
        for wl in workloads:
            with self.cv:
                need = self._bytes_needed(wl)
                if self.reserved + need > self.budget:
                    continue
            slot = Slot(self._next_sid, wl.n, wl, torch.cuda.Stream())
            self._next_sid += 1
            with self.cv:
                self.slots.append(slot)
                self.reserved += slot.bytes

    def _try_admit(self, req):
        """Called with the lock held: an idle slot of the request's size, a new slot, or
        None.  May evict idle slots of other sizes to make room."""
        n = req.workload.n
        for s in self.slots:
            if not s.busy and s.n == n:
                return s, False
        busy = sum(1 for s in self.slots if s.busy)
        if busy >= self.max_slots:
            return None, False
        need = self._bytes_needed(req.workload)
        idle = sorted((s for s in self.slots if not s.busy), key=lambda s: s.last_used)
        while self.reserved + need > self.budget and idle:
            v = idle.pop(0)
            self.slots.remove(v)
            self.reserved -= v.bytes
            v.close()
            self.evictions += 1
        if self.reserved + need > self.budget:
            return None, False
        if len(self.slots) >= 2 * self.max_slots and idle:
            v = idle.pop(0)
            self.slots.remove(v)
            self.reserved -= v.bytes
            v.close()
            self.evictions += 1
        self.reserved += need
        return need, True

    # -- one request on one slot -----------------------------------------------------
    def _execute(self, slot, req, res, t0):
        torch = self.torch
        wl = req.workload
        xy, tri = wl.solid_mesh()
        with torch.cuda.stream(slot.stream):
            slot.ctx.set_solid(xy, tri, kappa=wl.kappa)
            N2 = slot.ctx.sizes["N2"]
            N = slot.ctx.sizes["N"]
            from . import inputs
            u = torch.from_numpy(inputs.uniform(2 * N2, req.u_seed)).to("cuda", non_blocking=False)
            X = torch.from_numpy(np.concatenate([xy[:, 0], xy[:, 1]])).to("cuda")
            state = torch.zeros(N, dtype=torch.float64, device="cuda")
            slot.stream.synchronize()
            res.stats = slot.ctx.step(u, X, state, self.opts)
            host = state.cpu()
        res.done = time.perf_counter() - t0
        if self.keep_states:
            res.state = host.numpy()

    def run(self, requests, realtime=True):
        """Serve the requests (sorted by arrival); returns the list of Results."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: r.arrival)
        results = {r.rid: Result(r.rid, r.workload.n, r.arrival) for r in reqs}
        pending: list[Request] = []
        state = {"next": 0, "done": 0, "inflight": 0, "error": None}
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        def release_arrivals():
            while state["next"] < len(reqs) and (not realtime or reqs[state["next"]].arrival <= now()):
                pending.append(reqs[state["next"]])
                state["next"] += 1

        def worker():
            try:
                serve_loop()
            except Exception as e:                  # surfaced to the caller after the loop
                with self.cv:
                    if state["error"] is None:
                        state["error"] = e
                    self.cv.notify_all()

        def serve_loop():
            while True:
                with self.cv:
                    while True:
                        if state["error"] is not None:
                            return
                        release_arrivals()
                        if state["done"] + state["inflight"] >= len(reqs) and not pending:
                            return
                        pick = None
                        for i, r in enumerate(pending):
                            got, new = self._try_admit(r)
                            if got is not None:
                                pick = (i, r, got, new)
                                break
                        if pick is not None:
                            break
                        wait = 0.05
                        if state["next"] < len(reqs) and realtime:
                            wait = max(0.0, min(wait, reqs[state["next"]].arrival - now()))
                        self.cv.wait(timeout=wait if wait > 0 else 0.001)
                    i, r, got, new = pick
                    pending.pop(i)
                    if new:
                        sid = self._next_sid
                        self._next_sid += 1
                        slot = None
                    else:
                        slot = got
                        slot.busy = True
                    state["inflight"] += 1
                    self.max_inflight = max(self.max_inflight, state["inflight"])
                res = results[r.rid]
                res.start = now()
                try:
                    if slot is None:
                        stream = torch.cuda.Stream()
                        slot = Slot(sid, r.workload.n, r.workload, stream)
                        # keep the estimate until the slot's Krylov space exists
                        slot.bytes = max(slot.bytes, got)
                        with self.cv:
                            self.reserved += slot.bytes - got
                            slot.busy = True
                            self.slots.append(slot)
                    res.slot = slot.sid
                    self._execute(slot, r, res, t0)
                    slot.bytes_now = slot.ctx.refresh_sizes()["device_bytes"]
                except Exception:
                    with self.cv:
                        state["inflight"] -= 1
                    raise
                with self.cv:
                    if slot.bytes_now > slot.bytes:
                        self.reserved += slot.bytes_now - slot.bytes
                        slot.bytes = slot.bytes_now
                    slot.busy = False
                    slot.last_used = time.perf_counter()
                    state["inflight"] -= 1
                    state["done"] += 1
                    self.cv.notify_all()

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.max_slots)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if state["error"] is not None:
            raise state["error"]
        return [results[r.rid] for r in reqs]

    def close(self):
        for s in self.slots:
            s.close()
        self.slots.clear()
        self.reserved = 0


def requests_from_trace(trace):
    """Requests from inputs.request_trace: (arrival, Workload) pairs; request i draws u^n
    from its workload's seed (1000 + i)."""
    return [Request(i, t, wl, u_seed=wl.seed) for i, (t, wl) in enumerate(trace)]


def summarize(results, wall=None):
    lat = np.array([r.latency for r in results])
    first = min(r.arrival for r in results)
    last = max(r.done for r in results)
    span = last - first if wall is None else wall
    by_n = {}
    for n in sorted({r.n for r in results}):
        svc = [r.done - r.start for r in results if r.n == n]
        by_n[n] = dict(count=len(svc), service_ms=float(np.mean(svc) * 1e3))
    return dict(requests=len(results), p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
                throughput_req_s=len(results) / span, span_s=span,
                its_mean=float(np.mean([r.stats.get("its", 0) for r in results])),
                converged=int(sum(1 for r in results if r.stats.get("converged"))), by_n=by_n)
