"""Continuous-batching request loop for SPME solves of differing sizes.

Requests (a system of the pool and an arrival time) are served from
resident slots of one device arena (BatchPool over the C batch API,
pme_batch_*): a slot holds a system's plan workspace and its input/output
buffers, admitted by footprint (PME_EBUSY when the arena has no free
range), kept after its request completes and reused by the next request for
the same system; idle slots of other systems are retired, least recently
used first, when a new system needs room.  Slots for the pool are admitted
before the clock starts where the arena holds them (resident grids).  Each
tick launches every request whose input has reached the device as one
batched step of their slots on the compute stream (pme_batch_launch: one
launch per kernel and grid group, the groups on forked streams), while
copies run on a separate stream and earlier ticks may still be executing:
requests that arrive while others are on the GPU join the next tick.
Latency is the host time from a request's scheduled arrival to the moment
its forces and energy are in host memory.
"""
from dataclasses import dataclass, field
import ctypes
import gc
import time

import numpy as np
import torch

from . import _lib
from .plan import BatchPool

# Request copies go straight to the HIP runtime the step library is linked
# against (the process's one): a non-blocking torch copy of pinned memory
# also records an event in torch's host allocator, which these copies, into
# buffers that live as long as the server, do not need.
_H2D, _D2H = 1, 2  # hipMemcpyKind


def _hip():
    lib = _lib.load()
    f = lib.hipMemcpyAsync
    if f.argtypes is None:
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    return f


def _copy(dst, src, kind, stream):
    """Asynchronous copy of src's bytes into dst (same size, contiguous) on
    stream, through the HIP runtime."""
    n = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == n and dst.is_contiguous() and src.is_contiguous()
    rc = _hip()(dst.data_ptr(), src.data_ptr(), n, kind, stream.cuda_stream)
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({rc})")


@dataclass
class PoolSystem:
    """One system a request may ask for: host positions/charges and box."""
    pos: np.ndarray
    q: np.ndarray
    box: np.ndarray
    K: int
    order: int = 4
    beta: float = 0.34


class Slot:
    """A resident system: its batch slot, device buffers and pinned host
    buffers for the results (taken from the server's per-system cache:
    page-locking host memory takes milliseconds, so it never happens inside
    the request loop once a system has been seen)."""

    def __init__(self, system_id, slot, pool, sysd, footprint, host_bufs):
        self.system_id = system_id
        self.slot = slot
        self.pos, self.q, self.forces, self.ev = pool.io(slot)
        self.q.copy_(torch.from_numpy(np.ascontiguousarray(sysd.q)), non_blocking=False)
        # results: forces and E/virial in one copy when the arena holds them
        # back to back (host_raw is then the pinned bytes both are views of)
        self.host_raw, self.host_f, self.host_ev = host_bufs
        sp = pool.results_span(slot)
        self.span = sp[0] if sp is not None and self.host_raw is not None \
            and sp[0].numel() == self.host_raw.numel() else None
        self.footprint = footprint
        self.busy = False
        self.last_used = 0.0


@dataclass
class Request:
    rid: int
    system_id: int
    arrival: float
    slot: Slot = None
    h2d: object = None
    d2h: object = None
    admitted: float = None
    done: float = None
    energy: float = None
    forces: np.ndarray = None
    copied: int = 0  # atoms of forces copied out of the slot's host buffer so far


@dataclass
class ServeStats:
    completed: int = 0
    wall_s: float = 0.0
    latencies_s: list = field(default_factory=list)
    batch_sizes: list = field(default_factory=list)
    peak_resident_bytes: int = 0
    peak_inflight: int = 0
    slots_created: int = 0
    slots_prewarmed: int = 0
    longest_turn_s: float = 0.0  # longest single pass of the request loop (host stalls)
    longest_turn_at_s: float = 0.0
    worst_request: dict = field(default_factory=dict)
    rejected_for_budget: int = 0
    evictions: int = 0

    def summary(self):
        lat = np.array(self.latencies_s) * 1e6
        return {
            "completed": self.completed,
            "throughput_per_s": self.completed / self.wall_s if self.wall_s > 0 else 0.0,
            "latency_us": {"p50": float(np.percentile(lat, 50)) if len(lat) else None,
                           "p99": float(np.percentile(lat, 99)) if len(lat) else None,
                           "mean": float(lat.mean()) if len(lat) else None,
                           "max": float(lat.max()) if len(lat) else None},
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "max_batch": int(max(self.batch_sizes)) if self.batch_sizes else 0,
            "ticks": len(self.batch_sizes),
            "peak_resident_bytes": int(self.peak_resident_bytes),
            "peak_inflight": int(self.peak_inflight),
            "slots_prewarmed": int(self.slots_prewarmed),
            "slots_created_while_serving": int(self.slots_created),
            "waits_for_budget": int(self.rejected_for_budget),
            "evictions": int(self.evictions),
            "longest_loop_turn_us": float(self.longest_turn_s * 1e6),
            "longest_loop_turn_at_s": float(self.longest_turn_at_s),
            "worst_request": self.worst_request,
        }


class Server:
    """Open-loop serving of SPME solves with admission by device footprint."""

    def __init__(self, pool, hbm_budget_bytes, precision="fp32_fixed", max_batch=64,
                 slots_per_system=2, device=None, keep_forces=None, prewarm=True):
        self.pool = list(pool)
        self.budget = int(hbm_budget_bytes)
        self.precision = precision
        self.max_batch = int(max_batch)
        self.slots_per_system = int(slots_per_system)
        self.device = torch.device(device if device is not None else "cuda")
        # keep_forces: None (keep none), True (keep all) or a predicate on the
        # request id
        self.keep_forces = keep_forces
        # three streams: inputs in, the batched steps, results out.  Inputs
        # of new requests are copied while earlier batches compute and copy
        # their results back (one stream for both directions would queue an
        # input copy behind the previous batch's result copy, and so behind
        # its compute)
        self.compute = torch.cuda.Stream(device=self.device)
        self.h2d = torch.cuda.Stream(device=self.device)
        self.d2h = torch.cuda.Stream(device=self.device)
        self.batch = BatchPool(self.budget, max_systems=max(64, 2 * len(self.pool)),
                               device=self.device, stream=self.compute)
        self.fp = [self.batch.footprint(p.K, p.order, len(p.q), precision) for p in self.pool]
        for i, f in enumerate(self.fp):
            if f == 0 or f > self.budget:
                raise ValueError(f"pool system {i} needs more device memory than the budget")
        self.slots = {i: [] for i in range(len(self.pool))}
        # request payloads: the inputs a client hands over, in pinned host memory
        self.inputs = [torch.from_numpy(np.ascontiguousarray(p.pos)).pin_memory() for p in self.pool]
        self.resident = 0
        self.stats = ServeStats()
        # completion events, recycled: creating one inside the loop can stall
        # the host for milliseconds when the runtime grows its signal pool
        self._events = [torch.cuda.Event() for _ in range(256)]
        self.host_cache = {}
        if prewarm:
            # resident slots for the pool while the arena holds them (one per
            # system, then a second, ...), each run once with its inputs in
            # place so that no kernel is loaded and no host memory is pinned
            # for the first time inside the timed loop
            full = False
            for k in range(self.slots_per_system):
                for i in range(len(self.pool)):
                    sl = self._new_slot(i, evict=False)
                    if sl is None:
                        full = True
                        break
                    with torch.cuda.stream(self.compute):
                        sl.pos.copy_(self.inputs[i])
                    self.stats.slots_prewarmed += 1
                if full:
                    break
            resident = [sl.slot for lst in self.slots.values() for sl in lst]
            if resident:
                self.batch.launch(resident)
            torch.cuda.synchronize(self.device)
            self.stats.slots_created = 0

    # -- admission ------------------------------------------------------------
    def _new_slot(self, system_id, evict=True):
        sysd = self.pool[system_id]
        with torch.cuda.stream(self.compute):
            slot = self.batch.admit(sysd.K, sysd.order, sysd.beta, sysd.box, len(sysd.q),
                                    precision=self.precision)
            while slot is None and evict:
                # retire idle slots of other systems, least recently used first
                idle = [s for lst in self.slots.values() for s in lst
                        if not s.busy and s.system_id != system_id]
                if not idle:
                    break
                victim = min(idle, key=lambda s: s.last_used)
                self.slots[victim.system_id].remove(victim)
                self.batch.retire(victim.slot)
                self.resident -= victim.footprint
                self.stats.evictions += 1
                slot = self.batch.admit(sysd.K, sysd.order, sysd.beta, sysd.box, len(sysd.q),
                                        precision=self.precision)
            if slot is None:
                return None
            s = Slot(system_id, slot, self.batch, sysd, self.fp[system_id],
                     self._host_bufs(system_id))
        self.slots[system_id].append(s)
        self.resident += s.footprint
        self.stats.slots_created += 1
        self.stats.peak_resident_bytes = max(self.stats.peak_resident_bytes, self.resident)
        return s

    def _host_bufs(self, system_id):
        """Pinned result buffers (bytes, forces view, E/virial view) for a new
        slot of this system: a cached set that no live slot holds, else a new
        one."""
        cache = self.host_cache.setdefault(system_id, [])
        held = {id(sl.host_raw) for sl in self.slots[system_id]}
        for pair in cache:
            if id(pair[0]) not in held:
                return pair
        n = len(self.pool[system_id].q)
        # pinned bytes laid out as the arena carves forces and E/virial:
        # [n][3] doubles, padding to 256 bytes, 7 doubles
        fb = (n * 24 + 255) // 256 * 256
        raw = torch.empty(fb + 56, dtype=torch.uint8, pin_memory=True)
        pair = (raw, raw[:n * 24].view(torch.float64).view(n, 3),
                raw[fb:fb + 56].view(torch.float64))
        cache.append(pair)
        return pair

    def _free_slot(self, system_id):
        for s in self.slots[system_id]:
            if not s.busy:
                return s
        if len(self.slots[system_id]) >= self.slots_per_system:
            return None
        s = self._new_slot(system_id)
        if s is None:
            self.stats.rejected_for_budget += 1
        return s

    def _admit(self, req, now):
        s = self._free_slot(req.system_id)
        if s is None:
            return False
        s.busy = True
        s.last_used = now
        req.slot = s
        req.admitted = now
        _copy(s.pos, self.inputs[req.system_id], _H2D, self.h2d)
        req.h2d = self._event()
        req.h2d.record(self.h2d)
        return True

    def _event(self):
        return self._events.pop() if self._events else torch.cuda.Event()

    def _keep(self, rid):
        k = self.keep_forces
        return bool(k(rid)) if callable(k) else bool(k)

    # -- the loop -------------------------------------------------------------
    def run(self, arrivals, system_ids, stall_s=30.0):
        """Serve requests with scheduled arrival times (seconds from start).
        Raises if no request completes for stall_s seconds."""
        reqs = [Request(i, int(k), float(t)) for i, (t, k) in enumerate(zip(arrivals, system_ids))]
        waiting, staged, running, done = [], [], [], []
        # no garbage-collector pauses inside the loop (its objects are
        # few and acyclic); restored on exit
        gc_was = gc.isenabled()
        gc.disable()
        try:
            return self._loop(reqs, waiting, staged, running, done, stall_s)
        finally:
            if gc_was:
                gc.enable()

    # atoms of kept forces copied out of a slot's host buffer per loop turn,
    # so that keeping a large system's forces never stalls the loop for long
    COPY_CHUNK = 16384

    def _copy_kept(self, pending):
        """One chunk of the oldest pending copy of kept forces; the slot is
        released once its forces are out."""
        r = pending[0]
        n = r.forces.shape[0]
        e = min(n, r.copied + self.COPY_CHUNK)
        r.forces[r.copied:e] = r.slot.host_f.numpy()[r.copied:e]
        r.copied = e
        if e == n:
            r.slot.busy = False
            pending.pop(0)

    def _loop(self, reqs, waiting, staged, running, done, stall_s):
        nxt = 0
        t0 = time.perf_counter()
        last_progress = 0.0
        pending = []  # completed requests whose kept forces are still being copied
        prev = 0.0
        while len(done) < len(reqs) or pending:
            now = time.perf_counter() - t0
            if now - prev > self.stats.longest_turn_s:
                self.stats.longest_turn_s, self.stats.longest_turn_at_s = now - prev, prev
            prev = now
            if now - last_progress > stall_s and now > (reqs[-1].arrival if reqs else 0.0):
                raise RuntimeError(f"serving stalled: {len(done)} of {len(reqs)} requests done")
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            # admit in arrival order; a request whose system has no free slot
            # waits without blocking requests for other systems
            still = []
            for r in waiting:
                if not self._admit(r, now):
                    still.append(r)
                else:
                    staged.append(r)
            waiting = still
            # one tick: the staged requests in one launch, ordered after their
            # input copies on the device (no host round trip in between)
            ready = staged[: self.max_batch]
            if ready:
                staged = staged[len(ready):]
                for r in ready:
                    self.compute.wait_event(r.h2d)
                    self._events.insert(0, r.h2d)  # the wait is enqueued: reusable later
                    r.h2d = None
                self.batch.launch([r.slot.slot for r in ready])
                ev = self._event()
                ev.record(self.compute)
                self.d2h.wait_event(ev)
                self._events.insert(0, ev)  # reused only after later events
                for r in ready:
                    if r.slot.span is not None:
                        _copy(r.slot.host_raw, r.slot.span, _D2H, self.d2h)
                    else:
                        _copy(r.slot.host_f, r.slot.forces, _D2H, self.d2h)
                        _copy(r.slot.host_ev, r.slot.ev, _D2H, self.d2h)
                    r.d2h = self._event()
                    r.d2h.record(self.d2h)
                running.extend(ready)
                self.stats.batch_sizes.append(len(ready))
            self.stats.peak_inflight = max(self.stats.peak_inflight, len(running) + len(staged))
            # completions
            still = []
            for r in running:
                if r.d2h.query():
                    r.done = time.perf_counter() - t0
                    self._events.append(r.d2h)
                    r.d2h = None
                    r.energy = float(r.slot.host_ev[0])
                    r.slot.last_used = r.done
                    if self._keep(r.rid):
                        # copied out in chunks over the next loop turns; the
                        # slot stays busy until then
                        r.forces = np.empty(tuple(r.slot.host_f.shape), dtype=np.float64)
                        pending.append(r)
                    else:
                        r.slot.busy = False
                    done.append(r)
                    last_progress = r.done
                    self.stats.latencies_s.append(r.done - r.arrival)
                else:
                    still.append(r)
            running = still
            if pending:
                self._copy_kept(pending)
            if not ready and not running and not staged and nxt < len(reqs) and not waiting:
                # idle until the next arrival: sleep only while it is far off
                # (a sleep overshoots by tens of microseconds), then spin
                dt = reqs[nxt].arrival - (time.perf_counter() - t0)
                if dt > 3e-4:
                    time.sleep(min(dt - 2e-4, 5e-4))
        self.stats.wall_s = time.perf_counter() - t0
        self.stats.completed = len(done)
        if done:
            w = max(done, key=lambda r: r.done - r.arrival)
            self.stats.worst_request = {"rid": w.rid, "system": w.system_id,
                                        "atoms": int(w.slot.host_f.shape[0]),
                                        "arrival_s": w.arrival, "admitted_s": w.admitted,
                                        "done_s": w.done}
        return done

    def close(self):
        self.batch.close()
