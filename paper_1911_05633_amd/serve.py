"""Serving loop: many independent P + Sigma evaluations on one GPU.

A request names a cell (kind), its number of imaginary-time points and an arrival
time.  The server keeps a persistent loop that

  * moves requests whose arrival time has passed into a FIFO queue;
  * admits queued requests while a slot (a HIP stream) is free and the request's
    device buffers (G(k), G(R), W, P, Sigma, electron count) can be carved out of
    one pre-allocated HBM pool: admission is by footprint, never by count alone.  A
    request that does not fit now is deferred; smaller requests behind it may be
    admitted meanwhile (backfill) until the head has been passed `max_bypass` times;
    a request larger than the whole pool is rejected with an error, never launched;
  * enqueues the admitted request's work on its slot's stream (input
    materialisation, then the whole path: k -> R, P, Sigma, R -> k + tau -> omega of
    both, electron count), so the work of different requests overlaps on the device;
  * polls completion events, returns the buffers to the pool and admits more.

Latency is completion - arrival.  The host-side logic (`Pool`, `Server`) does not
touch the GPU and is exercised on the CPU with a simulated executor; `GWExecutor`
is the device executor over the library's entry points.
"""
from __future__ import annotations

import bisect
import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

ALIGN = 256


def _align(n: int) -> int:
    return (int(n) + ALIGN - 1) // ALIGN * ALIGN


class Pool:
    """Offset allocator over [0, capacity): best fit, 256-byte alignment, coalescing frees.

    `fail_next` makes the next k calls of alloc() fail as an allocator error would
    (used to check that such a failure ends only the request that hit it)."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity) // ALIGN * ALIGN
        self._free: List[Tuple[int, int]] = [(0, self.capacity)] if self.capacity > 0 else []  # (offset, size)
        self._live: Dict[int, int] = {}
        self.used = 0
        self.peak = 0
        self.fail_next = 0

    def alloc(self, nbytes: int) -> Optional[int]:
        if self.fail_next > 0:
            self.fail_next -= 1
            raise MemoryError("injected allocation failure")
        size = _align(max(int(nbytes), 1))
        best = -1
        for i, (off, sz) in enumerate(self._free):
            if sz >= size and (best < 0 or sz < self._free[best][1]):
                best = i
        if best < 0:
            return None
        off, sz = self._free[best]
        if sz == size:
            del self._free[best]
        else:
            self._free[best] = (off + size, sz - size)
        self._live[off] = size
        self.used += size
        self.peak = max(self.peak, self.used)
        return off

    def free(self, off: int) -> None:
        size = self._live.pop(off)
        self.used -= size
        i = bisect.bisect_left(self._free, (off, 0))
        self._free.insert(i, (off, size))
        # merge with the right and then the left neighbour
        if i + 1 < len(self._free) and off + size == self._free[i + 1][0]:
            self._free[i] = (off, size + self._free[i + 1][1])
            del self._free[i + 1]
        if i > 0 and self._free[i - 1][0] + self._free[i - 1][1] == off:
            self._free[i - 1] = (self._free[i - 1][0], self._free[i - 1][1] + self._free[i][1])
            del self._free[i]

    def alloc_all(self, sizes: Sequence[int]) -> Optional[List[int]]:
        """All of `sizes` or nothing (None if they do not fit now)."""
        got: List[int] = []
        try:
            for s in sizes:
                off = self.alloc(s)
                if off is None:
                    for o in got:
                        self.free(o)
                    return None
                got.append(off)
        except MemoryError:
            for o in got:
                self.free(o)
            raise
        return got

    @property
    def largest_free(self) -> int:
        return max((s for _, s in self._free), default=0)


@dataclass
class Record:
    request_id: int
    kind: str
    n_tau: int
    arrival: float
    nbytes: int = 0
    admitted: Optional[float] = None
    done: Optional[float] = None
    status: str = "queued"  # queued | running | done | rejected | failed | cancelled
    error: Optional[str] = None
    result: Dict = field(default_factory=dict)
    bypassed: int = 0

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


def percentile(values: Sequence[float], p: float) -> float:
    """Nearest-rank percentile."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, math.ceil(p / 100.0 * len(v)))
    return v[k - 1]


class Server:
    """Continuous-batching loop over an executor.

    The executor provides
      sizes(req) -> list of buffer sizes in bytes (the footprint),
      launch(req, slot, offsets) -> handle    (enqueue all work; may raise),
      poll(handle) -> bool,  completion(handle) -> seconds since start() or None,
      finish(handle, rec) -> None  (fill rec.result; buffers still valid),
      start() -> None  (called once when the clock starts), wait(seconds) -> None.
    """

    def __init__(self, executor, capacity: int, slots: int = 4, backfill: bool = True, max_bypass: int = 8,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.pool = Pool(capacity)
        self.slots = int(slots)
        self.backfill = backfill
        self.max_bypass = int(max_bypass)
        self.clock = clock
        self._cancel: set = set()

    def cancel(self, request_id: int) -> None:
        """Cancel a request: dropped if still queued; if running, its result is discarded."""
        self._cancel.add(request_id)

    def run(self, requests, on_done: Optional[Callable] = None) -> List[Record]:
        recs = {r.request_id: Record(r.request_id, r.kind, r.n_tau, float(r.arrival)) for r in requests}
        order = sorted(requests, key=lambda r: (r.arrival, r.request_id))
        queue: deque = deque()
        running: Dict[int, Tuple[Record, object, object, List[int]]] = {}
        self.ex.start()
        t0 = self.clock()
        i = 0
        while i < len(order) or queue or running:
            now = self.clock() - t0
            while i < len(order) and order[i].arrival <= now:
                queue.append(order[i])
                i += 1
            progressed = False
            # completions
            for slot in list(running):
                rec, req, h, offs = running[slot]
                if self.ex.poll(h):
                    tc = self.ex.completion(h)
                    rec.done = tc if tc is not None else self.clock() - t0
                    if rec.request_id in self._cancel:
                        rec.status = "cancelled"
                    else:
                        rec.status = "done"
                        self.ex.finish(h, rec)
                        if on_done is not None:
                            on_done(rec, h)
                    self.ex.release(h)
                    for o in offs:
                        self.pool.free(o)
                    del running[slot]
                    progressed = True
            # cancellations of queued requests
            if self._cancel and queue:
                for req in list(queue):
                    if req.request_id in self._cancel:
                        queue.remove(req)
                        recs[req.request_id].status = "cancelled"
            # admission
            j = 0
            while j < len(queue) and len(running) < self.slots:
                req = queue[j]
                rec = recs[req.request_id]
                sizes = self.ex.sizes(req)
                rec.nbytes = sum(_align(s) for s in sizes)
                if rec.nbytes > self.pool.capacity:
                    rec.status, rec.error = "rejected", f"footprint {rec.nbytes} B exceeds the pool ({self.pool.capacity} B)"
                    del queue[j]
                    progressed = True
                    continue
                try:
                    offs = self.pool.alloc_all(sizes)
                except MemoryError as e:
                    rec.status, rec.error = "failed", str(e)
                    del queue[j]
                    progressed = True
                    continue
                if offs is None:
                    # defer; look further down the queue unless the head has waited long enough
                    if not self.backfill or recs[queue[0].request_id].bypassed >= self.max_bypass:
                        break
                    j += 1
                    continue
                slot = next(s for s in range(self.slots) if s not in running)
                rec.admitted = self.clock() - t0
                try:
                    h = self.ex.launch(req, slot, offs)
                except Exception as e:  # the request fails alone; its buffers go back
                    for o in offs:
                        self.pool.free(o)
                    rec.status, rec.error = "failed", f"{type(e).__name__}: {e}"
                    del queue[j]
                    progressed = True
                    continue
                rec.status = "running"
                running[slot] = (rec, req, h, offs)
                for k in range(j):  # everything ahead of it was passed over once more
                    recs[queue[k].request_id].bypassed += 1
                del queue[j]
                progressed = True
            if not progressed:
                nxt = order[i].arrival - (self.clock() - t0) if i < len(order) else None
                self.ex.wait(nxt)
        return [recs[r.request_id] for r in requests]


def summarize(recs: Sequence[Record], makespan: Optional[float] = None) -> Dict:
    done = [r for r in recs if r.status == "done"]
    lat = [r.latency for r in done]
    if makespan is None:
        makespan = max((r.done for r in done), default=0.0) - min((r.arrival for r in recs), default=0.0)
    out = {"requests": len(recs), "done": len(done),
           "rejected": sum(r.status == "rejected" for r in recs),
           "failed": sum(r.status == "failed" for r in recs),
           "cancelled": sum(r.status == "cancelled" for r in recs),
           "makespan_s": makespan,
           "throughput_req_per_s": len(done) / makespan if makespan > 0 else float("nan"),
           "p50_ms": percentile(lat, 50) * 1e3, "p99_ms": percentile(lat, 99) * 1e3,
           "mean_ms": (sum(lat) / len(lat) * 1e3) if lat else float("nan")}
    return out


# ---------------------------------------------------------------------------
# device executor
# ---------------------------------------------------------------------------
class GWExecutor:
    """Runs each request's whole path on its slot's stream, with buffers carved from one HBM pool.

    Per request (prec "bf16x3" or "fp32" = mixed: complex64 G(R), W, P; BF16 split or FP32
    matrix cores; FP64 transforms, Sigma sums and electron count; "fp64" = plain FP64):
      the inputs G(k, tau) and W(R, tau), materialised on the slot's stream by the caller's
      input provider (`inputs.materialize`), then
      gw_fourier_k2r, gw_polarizability, gw_self_energy, gw_drain (P, bosonic),
      gw_drain (Sigma, fermionic), gw_density.
    The input provider also describes the cells: `inputs.spec(kind, n_tau)` (a description with
    species, n_orb, n_pb, mesh, n_tau, beta, tau, spin, N_R, N_orb, N_pb), `inputs.kind_data(kind,
    dtype)` (its "C" entry holds the product-basis coefficients) and `inputs.cell_data(spec,
    dtype)`.  Cells and T matrices (per kind and n_tau) and the provider's data are prepared
    once and kept; only the pool's views change between requests.
    """

    def __init__(self, inputs, prec: str = "bf16x3", capacity: Optional[int] = None, headroom: int = 12 << 30,
                 slots: int = 4, keep: Sequence[str] = ()):
        import torch
        from . import Cell, gw_tau2omega_matrix, matsubara
        self.torch, self.inputs = torch, inputs
        self._Cell, self._T, self._mats = Cell, gw_tau2omega_matrix, matsubara
        if prec not in ("fp64", "fp32", "bf16x3"):
            raise ValueError(f"unknown precision {prec}")
        self.prec = prec
        self.keep = tuple(keep)
        if capacity is None:
            free, _ = torch.cuda.mem_get_info()
            capacity = free - headroom
        self.capacity = int(capacity) // ALIGN * ALIGN
        self.buf = torch.empty(self.capacity, dtype=torch.uint8, device="cuda")
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.host_n = [torch.empty(1, dtype=torch.float64, pin_memory=True) for _ in range(slots)]
        self._kind: Dict[str, Dict] = {}
        self._cell: Dict[Tuple[str, int], Tuple] = {}
        self._t0 = None

    def _cdt(self):
        return self.torch.complex128 if self.prec == "fp64" else self.torch.complex64

    # -- preparation (host work done once per kind / per (kind, n_tau)) --
    def prepare_kind(self, kind: str):
        if kind not in self._kind:
            self._kind[kind] = self.inputs.kind_data(kind, self._cdt())
            self.torch.cuda.synchronize()  # the slots' streams read these without further ordering
        return self._kind[kind]

    def prepare(self, req):
        key = (req.kind, req.n_tau)
        if key in self._cell:
            return self._cell[key]
        torch = self.torch
        k = self.prepare_kind(req.kind)
        spec = self.inputs.spec(req.kind, req.n_tau)
        cell = self._Cell.from_spec(spec, k["C"])
        tau = spec.tau
        TP = torch.from_numpy(self._T(tau, self._mats(spec.n_tau, spec.beta, "bosonic"))).cuda()
        TS = torch.from_numpy(self._T(tau, self._mats(spec.n_tau, spec.beta, "fermionic"))).cuda()
        cd = self.inputs.cell_data(spec, self._cdt())
        torch.cuda.synchronize()
        self._cell[key] = (spec, cell, TP, TS, cd)
        return self._cell[key]

    def _layout(self, spec) -> List[Tuple[str, Tuple[int, ...], object]]:
        torch = self.torch
        cdt = torch.complex128 if self.prec == "fp64" else torch.complex64
        nt, NR, No, Np = spec.n_tau, spec.N_R, spec.N_orb, spec.N_pb
        return [("Gk", (nt, NR, No, No), torch.complex128), ("GR", (nt, NR, No, No), cdt),
                ("W", (nt, NR, Np, Np), cdt), ("P", (nt, NR, Np, Np), cdt),
                ("S", (nt, NR, No, No), torch.complex128), ("n", (1,), torch.float64)]

    @staticmethod
    def _nbytes(shape, dtype_size):
        n = 1
        for s in shape:
            n *= s
        return n * dtype_size

    def sizes(self, req) -> List[int]:
        spec = self.prepare(req)[0]
        return [self._nbytes(s, d.itemsize) for _, s, d in self._layout(spec)]

    # -- the loop's hooks --
    def start(self):
        torch = self.torch
        torch.cuda.synchronize()
        self._t0 = torch.cuda.Event(enable_timing=True)
        self._t0.record()
        torch.cuda.synchronize()

    def wait(self, seconds):
        time.sleep(min(seconds, 2e-4) if seconds is not None and seconds > 0 else 5e-5)

    def launch(self, req, slot, offs):
        from . import gw_fourier_k2r, gw_polarizability, gw_self_energy, gw_drain, gw_density
        torch = self.torch
        spec, cell, TP, TS, cd = self.prepare(req)
        k = self._kind[req.kind]
        t = {}
        for (name, shape, dt), off in zip(self._layout(spec), offs):
            nb = self._nbytes(shape, dt.itemsize)
            t[name] = self.buf[off:off + nb].view(dt).view(shape)
        s = self.streams[slot]
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        host_n = self.host_n[slot]  # read in finish(), before the slot takes another request
        with torch.cuda.stream(s):
            ev0.record()
            self.inputs.materialize(k, cd, spec, t["Gk"], t["W"])
            # the path
            gw_fourier_k2r(cell, t["Gk"], t["GR"], basis=0)
            gw_polarizability(cell, t["GR"], t["P"], spec.spin, prec=self.prec)
            gw_self_energy(cell, t["GR"], t["W"], t["S"], prec=self.prec)
            gw_drain(cell, TP, t["P"], t["P"], basis=1, parity=1)
            gw_drain(cell, TS, t["S"], t["S"], basis=0, parity=-1)
            if self.prec == "fp64":
                gw_density(cell, t["GR"], spec.spin, t["n"], space=0)
            else:
                gw_density(cell, t["Gk"], spec.spin, t["n"], space=1)
            host_n.copy_(t["n"], non_blocking=True)
            ev1.record()
        return {"req": req, "spec": spec, "t": t, "ev0": ev0, "ev1": ev1, "n": host_n, "stream": s}

    def poll(self, h) -> bool:
        return h["ev1"].query()

    def completion(self, h) -> float:
        return self._t0.elapsed_time(h["ev1"]) * 1e-3

    def finish(self, h, rec):
        spec = h["spec"]
        rec.result["n"] = float(h["n"][0])
        rec.result["n_expected"] = spec.spin * spec.N_orb / 2.0
        rec.result["gpu_ms"] = h["ev0"].elapsed_time(h["ev1"])
        rec.result["t_start"] = self._t0.elapsed_time(h["ev0"]) * 1e-3
        rec.result["t_end"] = self._t0.elapsed_time(h["ev1"]) * 1e-3
        for name in self.keep:
            rec.result[name] = h["t"][name].cpu()

    def release(self, h):
        h["t"].clear()
