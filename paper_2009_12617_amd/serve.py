"""Continuous-batching request loop for SPME solves of differing sizes.

Requests (a system of the pool and an arrival time) are admitted into
resident slots -- a plan with its workspace and device buffers -- while the
device memory they hold stays within an HBM budget; a slot is kept after its
request completes and reused by the next request for the same system.  Each
tick launches every staged request (inputs already copied to the device) as
one batched run (pme_batch_run) on the compute stream, while copies run on a
separate stream and earlier ticks may still be executing: requests that
arrive while others are on the GPU join the next tick.  Latency is the host
time from a request's scheduled arrival to the moment its forces and energy
are in host memory.
"""
from dataclasses import dataclass, field
import time

import numpy as np
import torch

from .plan import Batch, Plan


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
    """A resident solver for one pool system."""

    def __init__(self, system_id, sysd, precision, device):
        n = len(sysd.q)
        self.system_id = system_id
        self.plan = Plan(sysd.K, sysd.order, sysd.beta, max_atoms=n, precision=precision,
                         device=device)
        self.pos = torch.empty((n, 3), dtype=torch.float64, device=device)
        self.q = torch.from_numpy(np.ascontiguousarray(sysd.q)).to(device)
        self.forces, self.ev = self.plan.bind(self.pos, self.q, sysd.box)
        self.host_f = torch.empty((n, 3), dtype=torch.float64, pin_memory=True)
        self.host_ev = torch.empty(7, dtype=torch.float64, pin_memory=True)
        self.footprint = slot_footprint(sysd, precision)
        self.busy = False
        self.last_used = 0.0

    def release(self):
        self.plan.close()
        self.plan = self.pos = self.q = self.forces = self.ev = None


def slot_footprint(sysd, precision):
    """Device bytes one resident slot holds: plan workspace and buffers."""
    n = len(sysd.q)
    return (Plan.workspace_bytes_for(sysd.K, sysd.order, n, precision) + 256
            + n * 3 * 8 * 2 + n * 8 + 7 * 8)


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


@dataclass
class ServeStats:
    completed: int = 0
    wall_s: float = 0.0
    latencies_s: list = field(default_factory=list)
    batch_sizes: list = field(default_factory=list)
    peak_resident_bytes: int = 0
    peak_inflight: int = 0
    slots_created: int = 0
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
            "slots_created": int(self.slots_created),
            "waits_for_budget": int(self.rejected_for_budget),
            "evictions": int(self.evictions),
        }


class Server:
    """Open-loop serving of SPME solves with admission by HBM footprint."""

    def __init__(self, pool, hbm_budget_bytes, precision="fp32_fixed", max_batch=64,
                 slots_per_system=2, device=None, keep_forces=False):
        self.pool = list(pool)
        self.budget = int(hbm_budget_bytes)
        self.precision = precision
        self.max_batch = int(max_batch)
        self.slots_per_system = int(slots_per_system)
        self.device = torch.device(device if device is not None else "cuda")
        self.keep_forces = keep_forces
        for i, p in enumerate(self.pool):
            if slot_footprint(p, precision) > self.budget:
                raise ValueError(f"pool system {i} needs more device memory than the budget")
        self.slots = {i: [] for i in range(len(self.pool))}
        # request payloads: the inputs a client hands over, in pinned host memory
        self.inputs = [torch.from_numpy(np.ascontiguousarray(p.pos)).pin_memory() for p in self.pool]
        self.resident = 0
        self.compute = torch.cuda.Stream(device=self.device)
        self.copy = torch.cuda.Stream(device=self.device)
        self.stats = ServeStats()

    # -- admission ------------------------------------------------------------
    def _free_slot(self, system_id, now):
        for s in self.slots[system_id]:
            if not s.busy:
                return s
        if len(self.slots[system_id]) >= self.slots_per_system:
            return None
        need = slot_footprint(self.pool[system_id], self.precision)
        if self.resident + need > self.budget:
            # evict idle slots of other systems, least recently used first
            idle = [s for lst in self.slots.values() for s in lst if not s.busy]
            idle.sort(key=lambda s: s.last_used)
            for s in idle:
                if self.resident + need <= self.budget:
                    break
                self.slots[s.system_id].remove(s)
                self.resident -= s.footprint
                s.release()
                self.stats.evictions += 1
        if self.resident + need > self.budget:
            self.stats.rejected_for_budget += 1
            return None
        s = Slot(system_id, self.pool[system_id], self.precision, self.device)
        self.slots[system_id].append(s)
        self.resident += s.footprint
        self.stats.slots_created += 1
        self.stats.peak_resident_bytes = max(self.stats.peak_resident_bytes, self.resident)
        return s

    def _admit(self, req, now):
        s = self._free_slot(req.system_id, now)
        if s is None:
            return False
        s.busy = True
        s.last_used = now
        req.slot = s
        req.admitted = now
        with torch.cuda.stream(self.copy):
            s.pos.copy_(self.inputs[req.system_id], non_blocking=True)
            req.h2d = torch.cuda.Event()
            req.h2d.record(self.copy)
        return True

    # -- the loop -------------------------------------------------------------
    def run(self, arrivals, system_ids, stall_s=30.0):
        """Serve requests with scheduled arrival times (seconds from start).
        Raises if no request completes for stall_s seconds."""
        reqs = [Request(i, int(k), float(t)) for i, (t, k) in enumerate(zip(arrivals, system_ids))]
        waiting, staged, running, done = [], [], [], []
        nxt = 0
        t0 = time.perf_counter()
        last_progress = 0.0
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
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
            # one tick: every staged request whose input is on the device
            ready = [r for r in staged if r.h2d.query()][: self.max_batch]
            if ready:
                ids = {id(r) for r in ready}
                staged = [r for r in staged if id(r) not in ids]
                Batch([r.slot.plan for r in ready]).run(self.compute)
                ev = torch.cuda.Event()
                ev.record(self.compute)
                self.copy.wait_event(ev)
                with torch.cuda.stream(self.copy):
                    for r in ready:
                        r.slot.host_f.copy_(r.slot.forces, non_blocking=True)
                        r.slot.host_ev.copy_(r.slot.ev, non_blocking=True)
                        r.d2h = torch.cuda.Event()
                        r.d2h.record(self.copy)
                running.extend(ready)
                self.stats.batch_sizes.append(len(ready))
            self.stats.peak_inflight = max(self.stats.peak_inflight, len(running) + len(staged))
            # completions
            still = []
            for r in running:
                if r.d2h.query():
                    r.done = time.perf_counter() - t0
                    r.energy = float(r.slot.host_ev[0])
                    if self.keep_forces:
                        r.forces = r.slot.host_f.numpy().copy()
                    r.slot.busy = False
                    r.slot.last_used = r.done
                    done.append(r)
                    last_progress = r.done
                    self.stats.latencies_s.append(r.done - r.arrival)
                else:
                    still.append(r)
            running = still
            if not ready and not running and not staged and nxt < len(reqs) and not waiting:
                # idle until the next arrival
                dt = reqs[nxt].arrival - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(min(dt, 0.0005))
        self.stats.wall_s = time.perf_counter() - t0
        self.stats.completed = len(done)
        return done
