"""Request loop for independent FSI steps (continuous admission under an HBM budget).

Each request is one semi-implicit step on its own fluid grid and solid mesh.  A slot holds
resident libfsi contexts of one fluid grid (n, nu, rho, dt) on one HIP stream; their fluid
blocks and multigrid hierarchies stay on the device and the solid is swapped per request
with fsi_set_solid (grow-only buffers, so a warm slot allocates nothing).  Requests are
admitted in arrival order as soon as a slot of their grid is idle, or a new slot fits the
HBM budget (idle slots of other grids are evicted, least recently used first, to make
room); requests that do not fit yet wait while later ones that fit go ahead.  A job takes
the admitted request and up to lanes(n) - 1 more waiting requests of the same grid and runs
them as one lockstep batch (fsi_step_batch: one launch sequence for all, the inner solves
as lanes of the same kernels), so small systems cost about one step's launches per batch.
Slots run concurrently (the ctypes calls release the GIL), so the work of different jobs
overlaps on the device.  Results are independent of the mix and of the batching: every
kernel is deterministic, a batched system's result is bitwise its result alone, and slots
share no device state.
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
    """Resident contexts of one fluid grid on one stream (more are made as batches grow)."""

    def __init__(self, sid, wl, stream, lanes=1):
        self.sid = sid
        self.key = grid_key(wl)
        self.n = wl.n
        self.stream = stream
        self.lanes = lanes
        self.ctxs = [self._new_ctx(wl)]
        self.busy = False
        self.last_used = time.perf_counter()
        self.bytes = self.ctxs[0].sizes["device_bytes"]
        self.bytes_now = self.bytes

    def _new_ctx(self, wl):
        xy, tri = wl.solid_mesh()
        ctx = fsi.Context(wl.n, xy, tri, nu=wl.nu, rho=wl.rho, dt=wl.dt, kappa=wl.kappa, stream=self.stream)
        # jobs run concurrently: a step enqueued past convergence would take device time from
        # the other jobs, so the inner solves wait for each step's convergence check
        ctx.set_inner_check(fsi.CHECK_EVERY_STEP)
        return ctx

    @property
    def ctx(self):
        return self.ctxs[0]

    def ensure(self, k, wl):
        while len(self.ctxs) < k:
            self.ctxs.append(self._new_ctx(wl))

    def device_bytes(self):
        return sum(c.refresh_sizes()["device_bytes"] for c in self.ctxs)

    def close(self):
        for c in self.ctxs:
            c.close()


def grid_key(wl):
    return (wl.n, float(wl.nu), float(wl.rho), float(wl.dt))


def default_lanes(n):
    """Requests per lockstep batch: 16 for every grid size of the request trace (measured on
    the 512-request trace, 32^2 to 256^2, two slots per grid: 97.6 requests/s with 16 lanes
    everywhere, 94.8 with 8 at 256^2, 87.1 with 16/16/8/4, 71.8 with 8/8/4/2; 32 lanes
    measured no faster than 16)."""
    return 16


class Server:
    def __init__(self, hbm_budget=None, max_slots=16, prec=fsi.FP32, pc=fsi.PC_TRI, rtol=1e-8,
                 keep_states=False, lanes=default_lanes, slots_per_grid=None):
        import torch
        self.torch = torch
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = max(free - (8 << 30), 1 << 30)
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.opts = fsi.Opts(restart=30, rtol=rtol, pc=pc, prec=prec)
        self.keep_states = keep_states
        self.lanes = lanes if callable(lanes) else (lambda n, k=int(lanes): k)
        self.slots_per_grid = slots_per_grid   # None: as many as the budget allows
        self.batches = 0             # jobs run, and requests in them
        self.batched = 0
        self.slots: list[Slot] = []
        self.cv = threading.Condition()
        self.reserved = 0            # bytes of live slots (estimates until measured)
        self.max_inflight = 0
        self.evictions = 0
        self._next_sid = 0
        self._pending = {}           # grid key -> slots admitted but not yet built (outside the lock)

    # -- admission ---------------------------------------------------------------
    def _bytes_needed(self, wl):
        xy, tri = wl.solid_mesh()
        need = fsi.footprint(wl.n, xy.shape[0], tri.shape[0], wl.nu, wl.rho, wl.dt)
        if need > self.budget:
            raise fsi.FsiError(fsi.FSI_E_NOMEM, f"request of {need} B can never fit the budget {self.budget} B")
        return need

    def prewarm(self, workloads):
        """Create idle slots ahead of the traffic (one per workload given, e.g. the largest
        solid of each grid size, with a context for every lane of a batch of that size, so
        later requests of that size allocate nothing)."""
        torch = self.torch
        for wl in workloads:
            k = self.lanes(wl.n)
            with self.cv:
                need = self._bytes_needed(wl)
                if self.reserved + k * need > self.budget:
                    continue
            slot = Slot(self._next_sid, wl, torch.cuda.Stream(), k)
            slot.ensure(k, wl)
            slot.bytes = max(k * need, slot.device_bytes())
            self._next_sid += 1
            with self.cv:
                self.slots.append(slot)
                self.reserved += slot.bytes

    def _try_admit(self, req):
        """Called with the lock held: an idle slot of the request's size, a new slot, or
        None.  May evict idle slots of other sizes to make room."""
        key = grid_key(req.workload)
        for s in self.slots:
            if not s.busy and s.key == key:
                return s, False
        if self.slots_per_grid is not None and (sum(1 for s in self.slots if s.key == key) +
                                                self._pending.get(key, 0)) >= self.slots_per_grid:
            return None, False
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
        self._pending[key] = self._pending.get(key, 0) + 1   # until the new slot is registered
        return need, True

    # -- one job (a lockstep batch of requests of one grid) on one slot ----------------
    def _execute(self, slot, reqs, results, t0):
        torch = self.torch
        from . import inputs
        slot.ensure(len(reqs), reqs[0].workload)
        ctxs = slot.ctxs[:len(reqs)]
        us, Xs, states = [], [], []
        with torch.cuda.stream(slot.stream):
            for ctx, req in zip(ctxs, reqs):
                wl = req.workload
                xy, tri = wl.solid_mesh()
                ctx.set_solid(xy, tri, kappa=wl.kappa)
                us.append(torch.from_numpy(inputs.uniform(2 * ctx.sizes["N2"], req.u_seed)).to("cuda"))
                Xs.append(torch.from_numpy(np.concatenate([xy[:, 0], xy[:, 1]])).to("cuda"))
                states.append(torch.zeros(ctx.sizes["N"], dtype=torch.float64, device="cuda"))
            slot.stream.synchronize()
            if len(reqs) == 1:
                stats = [ctxs[0].step(us[0], Xs[0], states[0], self.opts)]
            else:
                stats, rcs = fsi.step_batch(ctxs, us, Xs, states, self.opts)
                bad = [(r.rid, rc) for r, rc in zip(reqs, rcs) if rc != fsi.FSI_OK]
                if bad:
                    raise fsi.FsiError(bad[0][1], f"request {bad[0][0]} did not converge in its batch")
            hosts = [st.cpu() for st in states]
        done = time.perf_counter() - t0
        for req, st, h in zip(reqs, stats, hosts):
            res = results[req.rid]
            res.stats = st
            res.done = done
            if self.keep_states:
                res.state = h.numpy()

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
                    # more waiting requests of the same grid join the job (arrival order), as
                    # far as the slot's contexts or new ones that fit the budget allow
                    key, cap = grid_key(r.workload), self.lanes(r.workload.n)
                    have = 1 if new else len(got.ctxs)
                    members, extra = [r], 0
                    j = 0
                    while len(members) < cap and j < len(pending):
                        q = pending[j]
                        if grid_key(q.workload) != key:
                            j += 1
                            continue
                        if len(members) >= have:
                            need_q = self._bytes_needed(q.workload)
                            if self.reserved + extra + need_q > self.budget:
                                break
                            extra += need_q
                        members.append(pending.pop(j))
                    self.reserved += extra
                    if new:
                        sid = self._next_sid
                        self._next_sid += 1
                        slot = None
                    else:
                        slot = got
                        slot.busy = True
                    state["inflight"] += len(members)
                    self.max_inflight = max(self.max_inflight, state["inflight"])
                    self.batches += 1
                    self.batched += len(members)
                t_start = now()
                for q in members:
                    results[q.rid].start = t_start
                try:
                    if slot is None:
                        try:
                            stream = torch.cuda.Stream()
                            slot = Slot(sid, r.workload, stream, self.lanes(r.workload.n))
                        except Exception:
                            with self.cv:
                                self._pending[key] -= 1
                                self.reserved -= got
                            raise
                        # keep the estimate until the slot's Krylov space exists
                        slot.bytes = max(slot.bytes, got)
                        with self.cv:
                            self.reserved += slot.bytes - got
                            slot.busy = True
                            self.slots.append(slot)
                            self._pending[key] -= 1
                    with self.cv:
                        slot.bytes += extra      # contexts the batch adds (reserved above)
                    for q in members:
                        results[q.rid].slot = slot.sid
                    self._execute(slot, members, results, t0)
                    slot.bytes_now = slot.device_bytes()
                except Exception:
                    with self.cv:
                        state["inflight"] -= len(members)
                    raise
                with self.cv:
                    if slot.bytes_now > slot.bytes:
                        self.reserved += slot.bytes_now - slot.bytes
                        slot.bytes = slot.bytes_now
                    slot.busy = False
                    slot.last_used = time.perf_counter()
                    state["inflight"] -= len(members)
                    state["done"] += len(members)
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
