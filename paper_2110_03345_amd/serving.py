"""Continuous-batching solve server on one GPU.

Requests (forward solves or shot gradients of 1-16 shots, each with its own
model and geometry) arrive over time.  Their shots are admitted into engine
slots as slots and HBM budget free up: one engine (and one HIP stream) per
padded grid, each advancing all its active shots one time step per tick in
shared batched launches replayed as hipGraph chunks (libstride_hip engine).
Models stay resident on the device for the life of a request; shot gradients
are summed on the device in shot order, so a request's result does not
depend on what else was in flight.

The paper dispatches all shots of an iteration at once and lets workers start
as soon as work arrives, keeping objects warm on their node or accelerator
(Sec. 2.5, Sec. 3.3); this server is that idea on one device.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _abi
from ._abi import STRIDE_MODE_FORWARD, STRIDE_MODE_GRADIENT, Plan


def _ws_bytes(grid, nrec: int, kind: str, grad_cap: int) -> int:
    """Workspace of one shot (no allocation): forward, or a gradient keeping
    every state when that fits grad_cap and checkpointing within it otherwise."""
    if kind == "forward":
        return _abi.stride_workspace_query(grid, 1, nrec, STRIDE_MODE_FORWARD)
    full = _abi.stride_workspace_query(grid, 1, nrec, STRIDE_MODE_GRADIENT)
    if full <= grad_cap:
        return full
    cap = grad_cap
    while True:   # below the checkpointing minimum: take the smallest workable size
        try:
            return _abi.stride_workspace_query(grid, 1, nrec, STRIDE_MODE_GRADIENT, cap)
        except _abi.StrideError as e:
            if e.code != _abi.STRIDE_E_WORKSPACE or cap >= full:
                raise
            cap = min(full, int(cap * 1.25) + (1 << 20))


class _Arena:
    """Device memory for shot workspaces: one allocation made up front and
    carved first-fit with coalescing, so admission never depends on the
    fragmentation of a general-purpose cache.  Offsets are 256-byte aligned."""

    ALIGN = 256

    def __init__(self, nbytes: int, device):
        nbytes -= nbytes % self.ALIGN
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.size = nbytes
        self.free = [(0, nbytes)]          # sorted (offset, size)
        self.used = 0
        self.peak = 0

    def alloc(self, n: int):
        n = -(-n // self.ALIGN) * self.ALIGN
        for i, (o, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, sz - n)
                self.used += n
                self.peak = max(self.peak, self.used)
                return o, self.buf[o:o + n]
        return None, None

    def release(self, off: int, n: int):
        n = -(-n // self.ALIGN) * self.ALIGN
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, sz in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + sz)
            else:
                merged.append((o, sz))
        self.free = merged


@dataclass
class _Shot:
    req: "_Req"
    index: int
    plan: Plan
    ws: torch.Tensor
    traces: Optional[torch.Tensor]
    misfit: Optional[torch.Tensor]
    dvp: Optional[torch.Tensor]
    observed: Optional[torch.Tensor]
    bytes: int
    ws_bytes: int = 0
    ws_off: int = -1
    slot: int = -1
    done: bool = False


@dataclass
class _Req:
    spec: object
    vp: Optional[torch.Tensor] = None
    wavelet: Optional[torch.Tensor] = None
    vp_max: float = 0.0
    next_shot: int = 0
    shots: List[_Shot] = field(default_factory=list)
    finished_shots: int = 0
    t_done: float = -1.0
    result: Optional[dict] = None
    bytes: int = 0
    grid: object = None


class _Bucket:
    """One engine and stream for requests of one padded grid."""

    def __init__(self, spec, max_slots: int, max_chunk: int, use_graphs: bool, max_receivers: int):
        self.grid = _abi.make_grid(**spec.grid_kwargs())
        self.max_slots = max_slots
        self.max_chunk = max_chunk
        self.handle = _abi.stride_engine_create(self.grid, max_slots, max_receivers, max_chunk,
                                                use_graphs)
        self.stream = torch.cuda.Stream()
        self.owner: Dict[int, _Shot] = {}     # engine slot -> attached shot
        self.inflight = collections.deque()   # (event, [shots whose outputs are complete at it])

    def free_slots(self):
        return self.max_slots - len(self.owner)

    def close(self):
        if self.handle is not None:
            _abi.stride_engine_destroy(self.handle)
            self.handle = None


class Server:
    """Admits shots by free HBM budget and slot availability, runs them in
    continuous batches, and records per-request latency."""

    def __init__(self, hbm_budget: Optional[int] = None, max_slots: int = 32, max_chunk: int = 64,
                 use_graphs: bool = True, grad_cap: int = 24 << 30, max_inflight: int = 3,
                 max_receivers: int = 1024, io_limit: Optional[int] = None, device=None):
        """hbm_budget: bytes of the workspace arena (default 80 % of free HBM).
        io_limit: bytes of the I/O buffers (models, wavelets, observed data,
        traces, gradients), which sit outside hbm_budget; default max(1 GiB,
        5 % of free HBM).  The limit is soft: when no shot runs anywhere, the
        oldest waiting request may take one shot beyond it."""
        self.device = torch.device(device or "cuda")
        free, _ = torch.cuda.mem_get_info(self.device)
        self.budget = int(hbm_budget if hbm_budget is not None else 0.80 * free)
        self.max_slots = max_slots
        self.max_chunk = max_chunk
        self.use_graphs = use_graphs
        # a gradient keeps every state when that fits its cap, else checkpoints
        # within it; the cap leaves room for other shots in the budget
        self.grad_cap = min(grad_cap, self.budget // 4)
        self.max_inflight = max_inflight
        self.max_receivers = max_receivers
        # workspaces come from the arena; models, traces and gradients (small
        # next to the workspaces) are ordinary tensors counted in io_used
        self.arena = _Arena(self.budget, self.device)
        self.io_limit = int(io_limit) if io_limit is not None else max(1 << 30, int(0.05 * free))
        self.io_used = 0
        self.io_peak = 0
        self.peak_used = 0
        self.max_attached = 0
        self.buckets: Dict[tuple, _Bucket] = {}
        self.upload = torch.cuda.Stream()

    # ------------------------------------------------------------ internals
    def _bucket(self, spec) -> _Bucket:
        b = self.buckets.get(spec.key)
        if b is None:
            b = _Bucket(spec, self.max_slots, self.max_chunk, self.use_graphs, self.max_receivers)
            self.buckets[spec.key] = b
        return b

    def _stage(self, req: _Req):
        """Models and wavelets resident on the device for the request's life."""
        s = req.spec
        with torch.cuda.stream(self.upload):
            req.vp = torch.from_numpy(s.vp).pin_memory().to(self.device, non_blocking=True)
            req.wavelet = torch.from_numpy(s.wavelet).pin_memory().to(self.device, non_blocking=True)
        req.vp_max = float(s.vp.max())
        req.bytes = req.vp.numel() * 4 + req.wavelet.numel() * 4
        self.io_used += req.bytes

    def _try_admit(self, req: _Req, bucket: _Bucket, force_io: bool = False) -> bool:
        """Attach the request's next shot if a slot and the budget allow
        (force_io: the I/O limit may be exceeded by this shot)."""
        s = req.spec
        i = req.next_shot
        if bucket.free_slots() == 0:
            return False
        nrec = s.rec_xyz.shape[0]
        if req.grid is None:
            req.grid = _abi.make_grid(**s.grid_kwargs())
        nb = _ws_bytes(req.grid, nrec, s.kind, self.grad_cap)
        io = nrec * s.nt * 4 * (2 if s.kind == "gradient" else 1) + \
            (req.vp.numel() * 4 if s.kind == "gradient" else 0)
        if self.io_used + io > self.io_limit and not force_io:
            return False
        ws_off, ws = self.arena.alloc(nb)
        if ws is None:
            return False
        plan = Plan(s.shape, s.spacing, s.space_order, s.nb, s.vref, s.dt, s.nt,
                    s.src_xyz[i:i + 1], s.rec_xyz)
        dev = self.device
        with torch.cuda.stream(self.upload):
            traces = torch.empty((plan.nrec, s.nt), dtype=torch.float32, device=dev)
            misfit = dvp = obs = None
            if s.kind == "gradient":
                misfit = torch.zeros(1, dtype=torch.float64, device=dev)
                dvp = torch.empty(s.shape, dtype=torch.float32, device=dev)
                obs = torch.from_numpy(s.observed[i]).pin_memory().to(dev, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(self.upload)
        bucket.stream.wait_event(ev)
        mode = STRIDE_MODE_GRADIENT if s.kind == "gradient" else STRIDE_MODE_FORWARD
        shot = _Shot(req, i, plan, ws, traces, misfit, dvp, obs, nb + io, nb, ws_off)
        shot.slot = _abi.stride_engine_attach(bucket.handle, plan.handle, mode, req.vp, req.vp_max,
                                              req.wavelet, obs, traces, misfit, dvp, ws,
                                              bucket.stream)
        # keep the allocations alive until the work that uses them is done
        traces.record_stream(bucket.stream)
        for t in (misfit, dvp, obs):
            if t is not None:
                t.record_stream(bucket.stream)
        bucket.owner[shot.slot] = shot
        req.shots.append(shot)
        req.next_shot += 1
        self.io_used += io
        self.io_peak = max(self.io_peak, self.io_used)
        self.peak_used = max(self.peak_used, self.arena.used + self.io_used)
        self.max_attached = max(self.max_attached, sum(len(b.owner) for b in self.buckets.values()))
        return True

    def _shot_done(self, sh: _Shot):
        """The shot's outputs are complete: release its workspace."""
        sh.done = True
        sh.ws = None
        self.arena.release(sh.ws_off, sh.ws_bytes)

    def _finalize(self, req: _Req, bucket: _Bucket):
        """Enqueue the request's reduction (shot gradients summed in shot
        order on the device) and return an event that marks completion."""
        s = req.spec
        if s.kind == "gradient":
            with torch.cuda.stream(bucket.stream):
                total = torch.zeros(s.shape, dtype=torch.float32, device=self.device)
                for sh in req.shots:
                    _abi.stride_accumulate(total, sh.dvp, bucket.stream)
            req.result = {"dvp": total}
        ev = torch.cuda.Event()
        ev.record(bucket.stream)
        return ev

    def _complete(self, req: _Req, now: float):
        s = req.spec
        res = req.result or {}
        res.update({"rid": s.rid, "kind": s.kind, "traces": [sh.traces for sh in req.shots]})
        if s.kind == "gradient":
            res["misfit"] = float(sum(float(sh.misfit.item()) for sh in req.shots))
            for sh in req.shots:
                sh.dvp = None
        req.result = res
        req.t_done = now
        self.io_used -= req.bytes + sum(sh.bytes - sh.ws_bytes for sh in req.shots)

    # ------------------------------------------------------------ main loop
    def run(self, specs, realtime: bool = True, progress=None) -> dict:
        """Serve the request stream (arrival times honoured when realtime,
        else every request is present at t = 0); returns results and timing.
        progress(done, total), if given, is called after every 25th completed
        request and after the last."""
        order = sorted(specs, key=lambda r: r.arrival)
        arrival = {r.rid: (r.arrival if realtime else 0.0) for r in order}
        pending = collections.deque(order)
        waiting: collections.deque = collections.deque()
        finals: List[tuple] = []          # (event, request) awaiting the reduction
        reqs: List[_Req] = []
        t0 = time.perf_counter()
        shots_total = sum(r.nshots for r in specs)
        ticks = 0
        n_done = 0
        while n_done < len(order):
            now = time.perf_counter() - t0
            while pending and arrival[pending[0].rid] <= now:
                r = _Req(pending.popleft())
                reqs.append(r)
                waiting.append(r)
            # admission: first come, first served within each grid.  The I/O
            # limit is soft: finished shots keep their outputs counted until
            # their request completes, and staged requests their inputs, which
            # can fill it while no shot runs; then the oldest waiting request
            # that fits the arena takes one shot beyond it, so the stream
            # always moves.
            idle = not any(b.owner for b in self.buckets.values())
            blocked = set()
            for r in list(waiting):
                b = self._bucket(r.spec)
                if id(b) in blocked:
                    continue
                if r.vp is None:
                    self._stage(r)
                while r.next_shot < r.spec.nshots and self._try_admit(r, b, force_io=idle):
                    idle = False
                if r.next_shot < r.spec.nshots:
                    blocked.add(id(b))
                else:
                    waiting.remove(r)
            # one chunk per bucket with attached shots, at most max_inflight ahead
            progressed = False
            for b in self.buckets.values():
                if not b.owner or len(b.inflight) >= self.max_inflight:
                    continue
                n, fin = _abi.stride_engine_run(b.handle, self.max_chunk, self.max_slots, b.stream)
                if n == 0 and not fin:
                    continue
                ticks += n
                ev = torch.cuda.Event()
                ev.record(b.stream)
                shots = [b.owner.pop(j) for j in fin]
                for j in fin:
                    _abi.stride_engine_detach(b.handle, j)
                b.inflight.append((ev, shots))
                progressed = True
            # completions
            for b in self.buckets.values():
                while b.inflight and b.inflight[0][0].query():
                    _, shots = b.inflight.popleft()
                    for sh in shots:
                        self._shot_done(sh)
                        r = sh.req
                        r.finished_shots += 1
                        if r.finished_shots == r.spec.nshots:
                            finals.append((self._finalize(r, b), r))
            now = time.perf_counter() - t0
            still = []
            for ev, r in finals:
                if ev.query():
                    self._complete(r, now)
                    n_done += 1
                    if progress and (n_done % 25 == 0 or n_done == len(order)):
                        progress(n_done, len(order))
                else:
                    still.append((ev, r))
            finals = still
            if not progressed:
                # every engine has its queue full (or is idle): poll, so that
                # no engine waits on another one's chunk
                if any(b.inflight for b in self.buckets.values()) or finals:
                    time.sleep(50e-6)
                elif pending:
                    time.sleep(max(0.0, min(0.002, arrival[pending[0].rid] - now)))
                elif waiting and not any(b.owner for b in self.buckets.values()):
                    r = waiting[0]
                    nb = _ws_bytes(r.grid or _abi.make_grid(**r.spec.grid_kwargs()),
                                   r.spec.rec_xyz.shape[0], r.spec.kind, self.grad_cap)
                    raise RuntimeError(
                        f"request {r.spec.rid} ({r.spec.kind}, {r.spec.ndim}D n={r.spec.n}, "
                        f"nt={r.spec.nt}, shot {r.next_shot} of {r.spec.nshots}) does not fit the "
                        f"HBM budget: workspace {nb} B, arena {self.arena.size} B with "
                        f"{self.arena.used} B in use (largest free "
                        f"{max((sz for _, sz in self.arena.free), default=0)} B), I/O "
                        f"{self.io_used} of {self.io_limit} B")
        t_end = time.perf_counter() - t0
        lat = np.array([r.t_done - arrival[r.spec.rid] for r in reqs])
        return {
            "requests": reqs,
            "makespan_s": t_end,
            "shot_solves": shots_total,
            "solves_per_s": shots_total / t_end,
            "requests_per_s": len(reqs) / t_end,
            "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)),
            "ticks": ticks,
            "peak_hbm_gb": self.peak_used / 2**30,
            "io_peak_bytes": self.io_peak,
            "max_attached_shots": self.max_attached,
            "workspace_peak_bytes": self.arena.peak,
            "workspace_budget_bytes": self.arena.size,
        }

    def close(self):
        for b in self.buckets.values():
            b.close()
        self.buckets.clear()
        self.arena = None


def solve_one(spec, device=None, grad_cap: int = 24 << 30, stream=None):
    """Plain one-shot-at-a-time solve of a request with the single-shot entry
    points (no batching, no graphs).  Returns the same result layout."""
    dev = torch.device(device or "cuda")
    vp = torch.from_numpy(spec.vp).to(dev)
    wav = torch.from_numpy(spec.wavelet).to(dev)
    res = {"rid": spec.rid, "kind": spec.kind, "traces": []}
    total = torch.zeros(spec.shape, dtype=torch.float32, device=dev) if spec.kind == "gradient" else None
    misfit = 0.0
    for i in range(spec.nshots):
        plan = Plan(spec.shape, spec.spacing, spec.space_order, spec.nb, spec.vref, spec.dt, spec.nt,
                    spec.src_xyz[i:i + 1], spec.rec_xyz)
        if spec.kind == "forward":
            res["traces"].append(plan.forward(vp, wav, stream=stream))
        else:
            nbytes = _ws_bytes(plan.grid, plan.nrec, "gradient", grad_cap)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            obs = torch.from_numpy(spec.observed[i]).to(dev)
            tr = torch.empty((plan.nrec, spec.nt), dtype=torch.float32, device=dev)
            m, d = plan.gradient(vp, wav, obs, ws=ws, traces=tr, stream=stream)
            _abi.stride_accumulate(total, d, stream)
            misfit += float(m.item())
            res["traces"].append(tr)
    if spec.kind == "gradient":
        res["dvp"] = total
        res["misfit"] = misfit
    torch.cuda.synchronize()
    return res


def serve_one_at_a_time(specs, realtime: bool = True, device=None, grad_cap: int = 24 << 30,
                        progress=None) -> dict:
    """FIFO baseline: each request in arrival order, its shots one after the
    other through the plain entry points (progress as in Server.run)."""
    order = sorted(specs, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    lat = []
    results = []
    for spec in order:
        arr = spec.arrival if realtime else 0.0
        wait = arr - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        results.append(solve_one(spec, device, grad_cap))
        lat.append(time.perf_counter() - t0 - arr)
        if progress and (len(lat) % 25 == 0 or len(lat) == len(order)):
            progress(len(lat), len(order))
    t_end = time.perf_counter() - t0
    shots = sum(r.nshots for r in specs)
    lat = np.array(lat)
    return {
        "results": results,
        "makespan_s": t_end,
        "shot_solves": shots,
        "solves_per_s": shots / t_end,
        "requests_per_s": len(specs) / t_end,
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
    }
