"""Continuous batching of gasket life solves on one GPU.

Requests (a gasket level r, an initial state and a number of generations)
arrive over time.  The scheduler admits them first-come first-served while
their HBM footprint (two n x n uint8 buffers) fits under a cap, keeps their
state resident on the device, and in every iteration advances every admitted
request by up to `steps_per_pass` generations in ONE batched pass over the
lambda tiles of all of them.  A request that finishes is retired and its
memory released, so requests that arrived meanwhile join at the next
iteration: their work overlaps on the device with the requests already
running.

The scheduler only orders work; the executor owns the buffers and runs the
passes.  ``GpuExecutor`` runs them through libsg's batched pass; tests drive
the same scheduler with a CPU executor.
"""
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of serving
    r: int                  # level: n = 2^r
    steps: int              # life generations to run
    state: Optional[np.ndarray] = None   # uint8 n x n initial state (host)
    template: Optional[int] = None       # or: the level of a device-resident template state


@dataclass
class Result:
    rid: int
    r: int
    steps: int
    arrival: float
    admitted: float
    finished: float
    output: Optional[np.ndarray] = None
    rejected: bool = False

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def footprint(r: int) -> int:
    """HBM bytes a request holds while resident: two n x n uint8 buffers."""
    return 2 * (1 << r) * (1 << r)


@dataclass
class _Slot:
    req: Request
    handle: object
    remaining: int
    admitted: float


@dataclass
class ServeStats:
    results: List[Result] = field(default_factory=list)
    makespan: float = 0.0
    iterations: int = 0      # scheduling rounds (one device wait each)
    passes: int = 0          # batched passes
    max_resident_bytes: int = 0
    max_active: int = 0

    def summary(self) -> Dict[str, float]:
        done = [x for x in self.results if not x.rejected]
        lat = np.array([x.latency for x in done]) if done else np.zeros(1)
        cells = float(sum((3 ** x.r) * x.steps for x in done))
        return {"requests": len(done), "rejected": len(self.results) - len(done),
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3),
                "makespan_s": self.makespan, "cells_per_s": cells / max(self.makespan, 1e-12),
                "iterations": self.iterations, "passes": self.passes,
                "max_active": self.max_active,
                "max_resident_gb": self.max_resident_bytes / 1e9}


class ContinuousBatcher:
    """FIFO admission by HBM footprint, one batched pass per iteration."""

    def __init__(self, executor, cap_bytes: int, steps_per_pass: int,
                 keep_outputs: bool = False, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep,
                 max_cells_per_pass: Optional[int] = None,
                 horizon_cells: Optional[int] = None):
        """max_cells_per_pass: optional budget of cell updates per pass;
        resident requests join a pass in admission order until it is spent
        (at least one always runs), so earlier requests finish first while
        small ones still share passes.

        horizon_cells: passes are queued back to back, without waiting for
        the device, until a request finishes, a new request arrives, or this
        many cell updates are queued (None: one pass per iteration)."""
        self.ex = executor
        self.cap = cap_bytes
        self.T = steps_per_pass
        self.keep_outputs = keep_outputs
        self.clock = clock
        self.sleep = sleep
        self.budget = max_cells_per_pass
        self.horizon = horizon_cells

    def serve(self, requests: Sequence[Request]) -> ServeStats:
        """Serve `requests` (arrival times in seconds after the start)."""
        pending = sorted(requests, key=lambda q: (q.arrival, q.rid))
        queue: List[Request] = []
        active: List[_Slot] = []
        used = 0
        st = ServeStats()
        t0 = self.clock()
        now = 0.0
        i = 0
        while i < len(pending) or queue or active:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival <= now:
                queue.append(pending[i])
                i += 1
            # admission: first come first served while the footprint fits
            while queue:
                q = queue[0]
                fp = footprint(q.r)
                if fp > self.cap:  # can never fit
                    queue.pop(0)
                    st.results.append(Result(q.rid, q.r, q.steps, q.arrival, now, now, rejected=True))
                    continue
                if used + fp > self.cap:
                    break
                queue.pop(0)
                h = self.ex.admit(q)
                used += fp
                active.append(_Slot(q, h, q.steps, now))
            st.max_resident_bytes = max(st.max_resident_bytes, used)
            st.max_active = max(st.max_active, len(active))
            if not active:
                if i < len(pending):  # idle until the next arrival
                    wait = pending[i].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(min(wait, 0.001))
                continue
            # batched passes over the resident requests (in admission order,
            # within the optional budget), queued back to back up to the horizon
            queued = 0
            while True:
                work, spent = [], 0
                for s in active:
                    k = min(self.T, s.remaining)
                    cost = (3 ** s.req.r) * k
                    if work and self.budget is not None and spent + cost > self.budget:
                        k = 0
                    spent += cost if k else 0
                    work.append((s.handle, k))
                self.ex.run_pass(work)
                st.passes += 1
                finished = False
                for s, (_, k) in zip(active, work):
                    s.remaining -= k
                    finished |= s.remaining == 0
                queued += spent
                if finished or self.horizon is None or queued >= self.horizon:
                    break
                if i < len(pending) and pending[i].arrival <= self.clock() - t0:
                    break
            self.ex.sync()
            st.iterations += 1
            now = self.clock() - t0
            still = []
            for s in active:
                if s.remaining > 0:
                    still.append(s)
                    continue
                out = self.ex.download(s.handle) if self.keep_outputs else None
                self.ex.release(s.handle)
                used -= footprint(s.req.r)
                st.results.append(Result(s.req.rid, s.req.r, s.req.steps, s.req.arrival,
                                         s.admitted, now, out))
            active = still
        st.makespan = self.clock() - t0
        return st


class GpuExecutor:
    """Device-resident states and libsg's batched pass (one launch per
    iteration over all resident requests)."""

    def __init__(self, tune, capacity: int = 4096, templates: Optional[Dict[int, object]] = None,
                 cap_bytes: Optional[int] = None):
        """cap_bytes: the scheduler's footprint cap; the buffers the executor
        holds (pooled and resident) are kept under it by dropping idle pooled
        buffers of other levels before a new one would pass it."""
        import torch
        from .batch import PassContext
        self.torch = torch
        self.tune = tune
        self.ctx = PassContext(capacity)
        self.templates = templates or {}
        self.cap = cap_bytes
        self.allocated = 0       # bytes of the buffers held, pooled or resident
        self.max_allocated = 0
        # released buffers, by level: they hold 0 on every cell off the gasket
        # (passes never write there), which is all a destination needs
        self.pool: Dict[int, List[object]] = {}

    def _new(self, r: int):
        n = 1 << r
        t = self.torch.zeros((n, n), dtype=self.torch.uint8, device="cuda")
        self.allocated += n * n
        self.max_allocated = max(self.max_allocated, self.allocated)
        return t

    def reserve(self, levels: Sequence[int], cap_bytes: int) -> int:
        """Pre-allocate the buffer pool, as a server sizes its memory at start:
        two buffers per entry of `levels` (in order) while the bytes held stay
        under `cap_bytes`.  Returns the bytes held."""
        for r in levels:
            if self.allocated + footprint(r) > cap_bytes:
                break
            self.pool.setdefault(r, []).extend(self._new(r) for _ in range(2))
        return self.allocated

    def _buffer(self, r: int):
        free = self.pool.get(r)
        if free:
            return free.pop()
        need = (1 << r) * (1 << r)
        if self.cap is not None:
            # idle buffers of other levels go first (the scheduler's
            # admission test keeps resident footprints under the cap)
            for lv, bufs in self.pool.items():
                while lv != r and bufs and self.allocated + need > self.cap:
                    bufs.pop()
                    self.allocated -= (1 << lv) * (1 << lv)
        return self._new(r)

    def admit(self, q: Request):
        from .batch import checked_ptr
        cur = self._buffer(q.r)
        try:
            nxt = self._buffer(q.r)
        except Exception:
            self.pool.setdefault(q.r, []).append(cur)
            raise
        if q.template is not None:
            cur.copy_(self.templates[q.template])
        else:
            cur.copy_(self.torch.from_numpy(np.ascontiguousarray(q.state)))
        return {"r": q.r, "buf": [cur, nxt],
                "p": [checked_ptr(cur, q.r, "state"), checked_ptr(nxt, q.r, "state")]}

    def run_pass(self, work):
        from .batch import PASS_ITEM
        items = np.array([(h["p"][0], h["p"][1], h["r"], k) for h, k in work], dtype=PASS_ITEM)
        self.ctx.run_array(items, self.tune)
        for h, k in work:
            if k > 0:
                h["buf"].reverse()
                h["p"].reverse()

    def sync(self):
        self.torch.cuda.synchronize()

    def download(self, h):
        return h["buf"][0].cpu().numpy()

    def release(self, h):
        self.pool.setdefault(h["r"], []).extend(h["buf"])
        h["buf"] = None

    def close(self):
        self.ctx.close()


def sequential_baseline(service_times: Sequence[float], arrivals: Sequence[float]):
    """Latencies of a single-server FIFO queue that runs one request at a time
    with the given measured service times (same arrivals, same order)."""
    order = np.argsort(np.asarray(arrivals), kind="stable")
    finish = 0.0
    lat = np.zeros(len(arrivals))
    for j in order:
        start = max(arrivals[j], finish)
        finish = start + service_times[j]
        lat[j] = finish - arrivals[j]
    return lat, finish


class NativeServer:
    """The continuous-batching loop of libsg (sg_server_*): the same policy as
    ContinuousBatcher -- FIFO admission by footprint, batched passes over every
    resident request, oldest first within an optional budget, passes queued
    until a request finishes or a horizon of cell updates -- with the queue,
    the device buffer pool and the pass planning in native code."""

    def __init__(self, tune, cap_bytes: int, max_requests: int, horizon_cells: int = 0,
                 budget_cells: int = 0, stream=None):
        import ctypes

        import torch
        from . import sg
        self._sg = sg
        self._ct = ctypes
        self._u8 = torch.uint8
        self._h = None
        h = ctypes.c_void_p()
        sg._check(sg.load().sg_server_create(ctypes.byref(tune), int(cap_bytes), int(max_requests),
                                             int(horizon_cells), int(budget_cells),
                                             sg._stream(stream), ctypes.byref(h)),
                  "sg_server_create")
        self._h = h
        self._done = (sg.sg_server_done * max_requests)()
        self.max_requests = max_requests

    def reserve(self, levels: Sequence[int]):
        arr = (self._ct.c_int32 * max(1, len(levels)))(*levels)
        self._sg._check(self._sg.load().sg_server_reserve(self._h, arr, len(levels)),
                        "sg_server_reserve")

    def submit(self, r: int, steps: int, init, tag: int, out=None):
        """init (and out, if given): uint8 n x n CUDA tensors kept alive by the caller."""
        sg = self._sg
        pi = sg._dev(init, self._u8, (1 << r) * (1 << r), "init")
        po = sg._dev(out, self._u8, (1 << r) * (1 << r), "out") if out is not None else None
        sg._check(sg.load().sg_server_submit(self._h, r, steps, pi, po, tag), "sg_server_submit")

    def submit_host(self, r: int, steps: int, h_init, tag: int, h_out=None):
        """h_init (and h_out, if given): pinned uint8 n x n CPU tensors kept
        alive, and h_out unread, until the request is reported."""
        n2 = (1 << r) * (1 << r)
        for name, t in (("h_init", h_init), ("h_out", h_out)):
            if t is None:
                continue
            if t.is_cuda or not t.is_pinned() or t.dtype != self._u8 or t.numel() != n2 \
                    or not t.is_contiguous():
                raise ValueError(f"{name}: a pinned contiguous uint8 CPU tensor of {n2} bytes")
        self._sg._check(self._sg.load().sg_server_submit_host(
            self._h, r, steps, h_init.data_ptr(), h_out.data_ptr() if h_out is not None else None,
            tag), "sg_server_submit_host")

    def set_max_active(self, k: int):
        """At most k requests in flight (0: no limit; 1: one at a time)."""
        self._sg._check(self._sg.load().sg_server_set_max_active(self._h, int(k)),
                        "sg_server_set_max_active")

    def set_transfer_window(self, k: int):
        """At most k host requests uploading or reading back (0: no limit)."""
        self._sg._check(self._sg.load().sg_server_set_transfer_window(self._h, int(k)),
                        "sg_server_set_transfer_window")

    def replay(self, requests: Sequence[Request], inits: Dict[int, object],
               outs: Optional[Dict[int, object]] = None) -> "ServeStats":
        """Serves `requests` in native code (sg_server_replay): each is
        submitted at its arrival time and rounds run while any is open.
        inits[rid] / outs[rid]: CUDA tensors, or pinned CPU tensors for
        requests whose state is uploaded and read back by the server."""
        order = sorted(requests, key=lambda q: (q.arrival, q.rid))
        arr = (self._sg.sg_server_request * max(1, len(order)))()
        n2 = lambda r: (1 << r) * (1 << r)  # noqa: E731
        for i, q in enumerate(order):
            init = inits[q.rid]
            out = outs.get(q.rid) if outs else None
            host = not init.is_cuda
            if host:
                for t in (init, out):
                    if t is not None and (t.is_cuda or not t.is_pinned() or t.numel() != n2(q.r)):
                        raise ValueError("host requests need pinned CPU tensors of n x n bytes")
                pi, po = init.data_ptr(), (out.data_ptr() if out is not None else None)
            else:
                pi = self._sg._dev(init, self._u8, n2(q.r), "init").value
                po = (self._sg._dev(out, self._u8, n2(q.r), "out").value
                      if out is not None else None)
            arr[i].arrival_s, arr[i].r, arr[i].steps = float(q.arrival), q.r, q.steps
            arr[i].init, arr[i].out, arr[i].host = pi, po, int(host)
        fin = (self._ct.c_double * max(1, len(order)))()
        rej = (self._ct.c_int32 * max(1, len(order)))()
        s0 = self.stats()
        self._sg._check(self._sg.load().sg_server_replay(self._h, arr, len(order), fin, rej),
                        "sg_server_replay")
        s = self.stats()
        st = ServeStats()
        for i, q in enumerate(order):
            st.results.append(Result(q.rid, q.r, q.steps, q.arrival, fin[i], fin[i],
                                     rejected=bool(rej[i])))
        st.makespan = max((fin[i] for i in range(len(order))), default=0.0)
        st.iterations, st.passes = s["rounds"] - s0["rounds"], s["passes"] - s0["passes"]
        # the server's maxima cover its whole life, not this replay alone
        st.max_resident_bytes, st.max_active = s["max_resident_bytes"], s["max_active"]
        return st

    def step(self):
        """One scheduling round: [(tag, rejected), ...] of the requests it ended."""
        n = self._ct.c_int()
        self._sg._check(self._sg.load().sg_server_step(self._h, self._done, self.max_requests,
                                                       self._ct.byref(n)), "sg_server_step")
        return [(int(self._done[i].tag), bool(self._done[i].rejected)) for i in range(n.value)]

    def stats(self) -> Dict[str, int]:
        st = self._sg.sg_server_stats()
        self._sg._check(self._sg.load().sg_server_get_stats(self._h, self._ct.byref(st)),
                        "sg_server_get_stats")
        return st.as_dict()

    def close(self):
        if self._h:
            self._sg.load().sg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_native(server: NativeServer, requests: Sequence[Request], inits: Dict[int, object],
                 outs: Optional[Dict[int, object]] = None,
                 clock: Callable[[], float] = time.perf_counter) -> ServeStats:
    """Drives `server` with requests arriving in real time (arrival seconds
    after the start): each is submitted once its arrival time has passed, and
    the server runs a round whenever it has work.  inits[rid] (and outs[rid],
    if given) are the requests' device tensors."""
    pending = sorted(requests, key=lambda q: (q.arrival, q.rid))
    by_id = {q.rid: q for q in pending}
    st = ServeStats()
    s0 = server.stats()
    t0 = clock()
    i = 0
    open_ids = set()
    while i < len(pending) or open_ids:
        now = clock() - t0
        while i < len(pending) and pending[i].arrival <= now:
            q = pending[i]
            server.submit(q.r, q.steps, inits[q.rid], q.rid, outs.get(q.rid) if outs else None)
            open_ids.add(q.rid)
            i += 1
        if not open_ids:
            continue  # idle until the next arrival
        finished = server.step()
        now = clock() - t0
        for rid, rejected in finished:
            q = by_id[rid]
            open_ids.discard(rid)
            st.results.append(Result(rid, q.r, q.steps, q.arrival, now, now, rejected=rejected))
    st.makespan = clock() - t0
    s = server.stats()
    st.iterations, st.passes = s["rounds"] - s0["rounds"], s["passes"] - s0["passes"]
    st.max_resident_bytes, st.max_active = s["max_resident_bytes"], s["max_active"]
    return st
