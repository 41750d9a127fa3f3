#!/usr/bin/env python3
"""Benchmark of the SPME reciprocal-space step on one MI355X.

Workload: 21,845 TIP3P-like waters (65,535 atoms) in an 86.8 A cubic box, 64^3
grid, B-spline order 4, beta = 0.34 1/A; a random walk of N(0, 0.01 A) per
coordinate per frame gives the frame sequence, staged in HBM before timing.
A step is one full pme_step (bin, spread + x FFT, y/z FFTs + influence
function + energy/virial + inverse z/y FFTs, inverse x FFT + force
interpolation: four launches) on the next frame, stream-ordered after the
previous one; the timed region replays one HIP graph of all timed steps.

Prints one JSON line.  Beside the headline: per-kernel times inside graph
replay, by difference against steps that launch one kernel twice (the
roofline entry is the dominant kernel's; `--profile` runs only those graph
replays, for rocprofv3), the autotuner's table for the workload, the plain FP64
path and the binary16/bfloat16 spectra on the same frames, per-step latency,
the real-space term, the 64x64x128 and 128^3 workloads, the 64-system batch
(batch admission API, grid groups on forked streams), serving at the
configured request rate and at a saturating one, and -- in the oracle leg
only -- parity of sampled frames, batch members and served requests against
the CPU oracle, and the oracle's own time on a bounded sample (one core).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
KERNELS = ("bin", "spread_x", "convolve_yz", "interpolate")


def algorithmic_bytes(N, K, kernel, fp64=False):
    """Algorithmic HBM bytes one launch of `kernel` moves:
    atoms 32 B read by spreading, 32 B read + 24 B written by interpolation;
    the charge grid (8 B/point) written and read; the half spectrum
    (8 or 16 B/point) across the two corner turns (written by the forward
    slab pass, read and written by the pencil pass, read by the inverse slab
    pass); the potential written and read.  Each term is charged to the
    kernel that performs that step.  K: an int (cubic grid) or (K1, K2, K3)."""
    K1, K2, K3 = (K, K, K) if np.ndim(K) == 0 else tuple(K)
    pts = K1 * K2 * K3                 # grid points
    half = K2 * K3 * (K1 // 2 + 1)     # half-spectrum points
    cs = 16 if fp64 else 8       # complex bytes
    rs = 8 if fp64 else 4        # potential bytes
    return {
        "bin": 32 * N,
        "spread_x": 16 * pts + cs * half,
        "convolve_yz": 2 * cs * half,
        "interpolate": cs * half + 2 * rs * pts + 56 * N,
    }[kernel]


def step_bytes(N, K, fp64=False):
    return sum(algorithmic_bytes(N, K, k, fp64) for k in KERNELS)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def source_digest():
    """Digest of the kernel sources (the counter profiles are tied to it)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2009_12617_amd", "csrc")
    for f in ("spme_kernels.h", "spme_kernels.hip", "spme_device.h", "spme_internal.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload="water_65535_k64"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    for line in lines:
        if line.startswith("BENCH_TRAFFIC_JSON "):
            d = json.loads(line.split(" ", 1)[1])
            if d.get("source_digest") != source_digest():
                return None
            k = d.get("kernels", {}).get(kernel)
            return None if k is None else k.get("bytes_per_launch")
    return None


def rel_rms(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------
class Frames:
    """The headline frame sequence, staged on the device."""

    def __init__(self, torch, dev, I, n_frames):
        w = I.HEADLINE_64
        pos0, self.q, self.box = w.make()
        self.w, self.N, self.K = w, len(self.q), w.K
        self.F = n_frames
        self.host = I.jitter_stream(pos0, self.F, I.HEADLINE_JITTER_SIGMA, I.HEADLINE_JITTER_SEED)
        self.dev_pos = torch.from_numpy(self.host).to(dev)
        self.dev_q = torch.from_numpy(self.q).to(dev)

    def pos(self, t):
        return self.dev_pos[t % self.F]


def curtain(torch, dev):
    """Untimed device work enqueued right before a timed graph replay: a
    one-wavefront spin of about 0.1 ms that touches no memory, so that the
    GPU is still busy while the host submits the graph and the caches are
    left as the previous steps left them: the timed region then holds the
    replayed steps back to back, not the submission latency in front of
    them."""
    torch.cuda._sleep(250000)


def capture(torch, dev, plan, fr, first, steps, forces, ev):
    """One HIP graph holding `steps` consecutive steps (frames first, first+1, ...)."""
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream(device=dev)
    with torch.cuda.graph(g, stream=cs):
        plan.set_stream(torch.cuda.current_stream(dev))
        for t in range(steps):
            plan.step(fr.pos(first + t), fr.dev_q, fr.box, forces=forces, ev=ev)
    plan.set_stream(torch.cuda.current_stream(dev))
    return g


def run_graph(torch, dev, plan, fr, steps, warmup, exact=True):
    """The timed region replays one captured graph of `steps` stream-ordered
    steps; the replay's last step is then checked against a host-launched
    step on the same frame, twice with eager work between (bit for bit on the
    fixed-point path; the FP64 path accumulates its grid with FP64 atomics,
    whose order, and so last-bit rounding, varies run to run)."""
    forces = torch.empty((fr.N, 3), dtype=torch.float64, device=dev)
    ev = torch.empty(7, dtype=torch.float64, device=dev)
    for t in range(warmup):
        plan.step(fr.pos(t), fr.dev_q, fr.box, forces=forces, ev=ev)
    torch.cuda.synchronize()
    g = capture(torch, dev, plan, fr, warmup, steps, forces, ev)
    g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    curtain(torch, dev)
    t0 = time.perf_counter()
    start.record(stream)
    g.replay()
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / steps
    last = warmup + steps - 1
    ok = True
    for _ in range(2):
        fg, eg = forces.clone(), ev.clone()
        fe, ee = plan.step(fr.pos(last), fr.dev_q, fr.box)
        torch.cuda.synchronize()
        if exact:
            ok &= bool(torch.equal(fg, fe)) and bool(torch.equal(eg, ee))
        else:
            ok &= bool(torch.allclose(fg, fe, rtol=1e-11, atol=1e-14))
            ok &= bool(torch.allclose(eg, ee, rtol=1e-11, atol=1e-14))
        g.replay()
        torch.cuda.synchronize()
    del g
    return ms, wall / steps * 1e3, ok


def graph_us(torch, dev, plan, fr, steps, repeat, first=0, reps=3):
    """Microseconds per step of one replayed graph of `steps` probe steps
    (pme_step_probe with kernel `repeat` launched twice; 0: plain steps),
    best of `reps` replays."""
    forces = torch.empty((fr.N, 3), dtype=torch.float64, device=dev)
    ev = torch.empty(7, dtype=torch.float64, device=dev)
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream(device=dev)
    with torch.cuda.graph(g, stream=cs):
        plan.set_stream(torch.cuda.current_stream(dev))
        for t in range(steps):
            plan.step_probe(fr.pos(first + t), fr.dev_q, fr.box, forces, ev, repeat)
    plan.set_stream(torch.cuda.current_stream(dev))
    g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        curtain(torch, dev)
        a.record(stream)
        g.replay()
        b.record(stream)
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) * 1e3 / steps)
    del g
    return best


def kernel_times(torch, dev, plan, fr, steps):
    """Per-kernel time inside graph-replayed steps, by difference: replays of
    steps that launch one kernel a second time (pme_step_probe; the results
    are unchanged) against replays of plain steps, timed with events around
    each replay.  Binning is repeated together with a one-workgroup clearing
    launch, which is timed alone and subtracted.  Microseconds per launch."""
    from paper_2009_12617_amd.plan import PROBE
    base = graph_us(torch, dev, plan, fr, steps, PROBE["none"])
    t = {k: graph_us(torch, dev, plan, fr, steps, PROBE[k]) - base
         for k in ("spread_x", "convolve_yz", "interpolate", "bin", "clear")}
    out = {"bin": t["bin"] - t["clear"], "spread_x": t["spread_x"], "convolve_yz": t["convolve_yz"],
           "interpolate": t["interpolate"]}
    # leave the plan with a whole step done
    plan.step(fr.pos(0), fr.dev_q, fr.box)
    torch.cuda.synchronize()
    return out, base


def profiled_kernel_us(workload="water_65535_k64"):
    """Per-kernel average durations (us per launch slot) from the committed
    rocprofv3 summary of this workload, or None when it is missing or was
    taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"kernels_{workload}.txt")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    for line in lines:
        if line.startswith("BENCH_KERNELS_JSON "):
            d = json.loads(line.split(" ", 1)[1])
            if d.get("source_digest") != source_digest():
                return None
            return d.get("kernels_us")
    return None


def roofline_entry(N, K, live_us, traffic_fn=None, profiled=None):
    """The dominant kernel's achieved algorithmic bandwidth.  Its duration is
    the rocprofv3 average of the committed profile when that profile was
    taken on the current kernel sources, else the live graph-replay time;
    both are reported."""
    kus = profiled if profiled else live_us
    dom = max(kus, key=kus.get)
    b = algorithmic_bytes(N, K, dom)
    achieved = b / (kus[dom] * 1e-6) / 1e9
    out = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "traffic": traffic_fn(dom) if traffic_fn else None,
           "algorithmic_bytes_per_launch": b, "kernel_us": kus[dom],
           "duration_source": ("rocprofv3 kernel statistics of the committed profile "
                               "(same kernel sources)" if profiled else
                               "live: graph-replayed steps repeating the kernel minus plain steps"),
           "live_kernel_us": live_us,
           "live_frac": {k: algorithmic_bytes(N, K, k) / (v * 1e-6) / 1e9 / HBM_PEAK_GBS
                         for k, v in live_us.items()}}
    if profiled:
        out["profiled_kernel_us"] = profiled
    return out


def graph_latency(torch, dev, plan, fr, steps):
    """Per-step latency of single-step graph launches (one frame each)."""
    forces = torch.empty((fr.N, 3), dtype=torch.float64, device=dev)
    ev = torch.empty(7, dtype=torch.float64, device=dev)
    gs = [capture(torch, dev, plan, fr, t, 1, forces, ev) for t in range(min(steps, fr.F, 200))]
    stream = torch.cuda.current_stream(dev)
    for g in gs[:5]:
        g.replay()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for t in range(steps):
        gs[t % len(gs)].replay()
        evs[t + 1].record(stream)
    torch.cuda.synchronize()
    return np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]) * 1e3


def bench_system(torch, dev, Plan, I, pos, q, box, K, order, beta, steps, warmup, name,
                 jitter_seed):
    """One more single-system workload, FP32/fixed path: one graph of `steps`
    steps over 16 jittered frames, per-kernel times by difference of
    graph-replayed probe steps, each kernel's algorithmic GB/s against
    8 TB/s; returns the last frame's forces for the oracle leg."""
    class F:
        pass
    fr = F()
    fr.N, fr.F, fr.box, fr.q = len(q), 16, box, q
    fr.host = I.jitter_stream(pos, fr.F, I.HEADLINE_JITTER_SIGMA, jitter_seed)
    fr.dev_pos = torch.from_numpy(fr.host).to(dev)
    fr.dev_q = torch.from_numpy(q).to(dev)
    fr.pos = lambda t: fr.dev_pos[t % fr.F]
    plan = Plan(K, order, beta, max_atoms=fr.N, device=dev)
    ms, _, same = run_graph(torch, dev, plan, fr, steps, warmup)
    kus, _ = kernel_times(torch, dev, plan, fr, min(steps, 100))
    kfrac = {k: algorithmic_bytes(fr.N, K, k) / (kus[k] * 1e-6) / 1e9 / HBM_PEAK_GBS for k in kus}
    last = (warmup + steps - 1) % fr.F
    fe, ee = plan.step(fr.pos(last), fr.dev_q, box)
    torch.cuda.synchronize()
    K3 = list(K) if np.ndim(K) else [int(K)] * 3
    out = {"workload": name, "atoms": fr.N, "grid": K3, "order": order, "beta": beta,
           "box_A": [float(box[i, i]) for i in range(3)], "us_per_step": ms * 1e3,
           "tuning": plan.tuning, "kernels_us": kus, "kernels_roofline_frac": kfrac,
           "step_algorithmic_bytes": int(step_bytes(fr.N, K)),
           "step_roofline_frac": step_bytes(fr.N, K) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "replay_same_as_eager": same}
    check = {"pos": fr.host[last], "q": q, "box": box, "K": K, "order": order, "beta": beta,
             "forces": fe.cpu().numpy(), "E": float(ee[0].item())}
    return out, check


def stacked_water(I):
    """The headline density on an elongated cell: two independent 86.8 A water
    boxes stacked along z (131,070 atoms, 86.8 x 86.8 x 173.6 A)."""
    L = 86.8
    a = I.water_box(21845, L, 2101)
    b = I.water_box(21845, L, 2102)
    pos = np.concatenate([a[0], b[0] + np.array([0.0, 0.0, L])])
    q = np.concatenate([a[1], b[1]])
    return pos, q, np.diag([L, L, 2 * L])


def bench_batched(torch, dev, Plan, BatchPool, Batch, I, reps=100):
    """64 independent water boxes of uneven size (3k..65k atoms, grids 32/48/64
    by ~1 A spacing) admitted into one arena (pme_batch_admit), kernel
    variants per grid group autotuned on the batch, one step of all of them
    per launch (pme_batch_launch: grid groups on forked streams), timed as
    graph replays; each system's result (from a replay into poisoned
    outputs) is checked against its own single step.  The same systems through pme_batch_run (one stream) for
    comparison."""
    mix = I.batch_mix()
    stream = torch.cuda.Stream(device=dev)
    pool = BatchPool(8 << 30, max_systems=128, device=dev, stream=stream)
    members = []
    with torch.cuda.stream(stream):
        for m in mix:
            pos, q, box = m.make()
            s = pool.admit(m.K, 4, 0.34, box, len(q))
            io = pool.io(s)
            io[0].copy_(torch.from_numpy(pos))
            io[1].copy_(torch.from_numpy(q))
            members.append((m, s, pos, q, box))
    stream.synchronize()
    # variants per grid group measured on the whole batch
    tuned = pool.autotune()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        pool.launch()
    # replays and their events on one stream (a replay runs on the current one)
    with torch.cuda.stream(stream):
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        curtain(torch, dev)
        evs[0].record(stream)
        for r in range(reps):
            g.replay()
            evs[r + 1].record(stream)
        torch.cuda.synchronize()
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(reps)]) * 1e3
    # steady state: every timed launch in one graph, replayed once (the way
    # the single-step value is timed), so no graph submission sits between
    # batches
    gs = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gs, stream=stream):
        for _ in range(reps):
            pool.launch()
    with torch.cuda.stream(stream):
        gs.replay()
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        curtain(torch, dev)
        s0.record(stream)
        gs.replay()
        s1.record(stream)
        torch.cuda.synchronize()
    steady = s0.elapsed_time(s1) * 1e3 / reps
    del gs
    # every system once more from poisoned outputs: the replay itself computes them
    for m, s, pos, q, box in members:
        pool.io(s)[2].fill_(float("nan"))
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        g.replay()
    torch.cuda.synchronize()
    same = True
    checks = []
    for k, (m, s, pos, q, box) in enumerate(members):
        plan = Plan(m.K, 4, 0.34, max_atoms=len(q), device=dev)
        plan.set_tuning(**pool.tuning_of(s))
        fa, ea = plan.step(torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev), box)
        fb, eb = pool.io(s)[2], pool.io(s)[3]
        same &= bool(torch.equal(fa, fb)) and bool(torch.equal(ea, eb))
        if k % 16 == 0:
            checks.append({"pos": pos, "q": q, "box": box, "K": m.K, "order": 4, "beta": 0.34,
                           "forces": fb.cpu().numpy(), "E": float(eb[0].item())})
    del g
    # the same systems through pme_batch_run on one stream (same variants)
    plans, keep = [], []
    for m, s, pos, q, box in members:
        p = Plan(m.K, 4, 0.34, max_atoms=len(q), device=dev)
        p.set_tuning(**pool.tuning_of(s))
        dp, dq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
        p.bind(dp, dq, box)
        plans.append(p)
        keep.append((dp, dq))
    b = Batch(plans)
    g2 = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream(device=dev)
    with torch.cuda.graph(g2, stream=cs):
        for _ in range(20):
            b.run(torch.cuda.current_stream(dev))
    g2.replay()
    torch.cuda.synchronize()
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    curtain(torch, dev)
    a0.record()
    g2.replay()
    a1.record()
    torch.cuda.synchronize()
    one_stream = a0.elapsed_time(a1) / 20 * 1e3
    del g2
    pool.close()
    atoms = sum(len(x[3]) for x in members)
    grids = {}
    for m in mix:
        grids[str(m.K)] = grids.get(str(m.K), 0) + 1
    nbytes = sum(step_bytes(len(x[3]), x[0].K) for x in members)
    out = {
        "workload": "64 water boxes, atoms log-uniform in [3000, 65000], grid by ~1 A spacing, p=4, beta=0.34",
        "systems": len(members), "atoms": int(atoms), "grids": grids,
        "us_per_batch": steady,
        "us_per_batch_what": f"one HIP graph of {reps} launches replayed once, as the single-step value",
        "latency_us": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                       "mean": float(per.mean()), "replays": reps,
                       "what": "one graph replay of one launch per batch, back to back"},
        "atoms_per_s": atoms / (steady * 1e-6),
        "step_algorithmic_bytes": int(nbytes),
        "roofline_frac": nbytes / (steady * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "same_as_single_steps": bool(same),
        "launch": "pme_batch_launch in one HIP graph: binning, spreading, convolution and "
                  "interpolation per grid group, the groups on three forked streams",
        "one_stream_pme_batch_run_us": one_stream,
        "one_stream_what": "pme_batch_run of the same plans, 20 runs in one graph replayed once",
        "autotune": tuned,
    }
    return out, checks


def bench_serving(torch, dev, I, n_requests, rate, budget_gib, keep_every, label):
    """Open-loop Poisson arrivals over the batch mix plus four 128^3 boxes;
    every request's energy against its system's own single step; the forces
    of every keep_every-th request are kept for the oracle leg."""
    from paper_2009_12617_amd.serve import PoolSystem, Server
    from paper_2009_12617_amd import Plan
    members = I.serving_pool()
    pool = []
    for m in members:
        pos, q, box = m.make()
        pool.append(PoolSystem(pos, q, box, m.K))
    arrivals, ids = I.poisson_requests(n_requests=n_requests, rate=rate)
    srv = Server(pool, hbm_budget_bytes=int(budget_gib * (1 << 30)), max_batch=64, device=dev,
                 keep_forces=lambda rid: rid % keep_every == 0)
    done = srv.run(arrivals, ids)
    st = srv.stats.summary()
    srv.close()
    ref_e = {}
    same = True
    for r in done:
        if r.system_id not in ref_e:
            s = pool[r.system_id]
            plan = Plan(s.K, 4, 0.34, max_atoms=len(s.q), device=dev)
            _, e = plan.step(torch.from_numpy(s.pos).to(dev), torch.from_numpy(s.q).to(dev), s.box)
            ref_e[r.system_id] = e[0].item()
        same &= (r.energy == ref_e[r.system_id])
    kept = [(r.system_id, r.forces) for r in done if r.forces is not None]
    st.update({
        "workload": f"{n_requests} requests, Poisson {rate:g}/s; 90% from the 64-box mix, "
                    "10% 128^3 / 209,715-atom boxes",
        "leg": label,
        "hbm_budget_gib": budget_gib,
        "energies_same_as_single_steps": bool(same),
        "latency_definition": "host: scheduled arrival to forces and energy in host memory",
    })
    return st, kept, pool


# ---------------------------------------------------------------------------
# The oracle leg: everything that runs the CPU oracle
# ---------------------------------------------------------------------------
def oracle_leg(args, fr, got_frames, reduced_got, more_checks, batch_checks, real_check,
               serving_kept, serving_pool):
    """Parity of sampled GPU results against the FP64 CPU oracle, and the
    oracle's own time on a bounded sample pinned to one core."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle._load()
    w = fr.w
    out = {}
    workers = min(16, os.cpu_count() or 1)

    def spme_ref(c):
        return oracle.spme(c["pos"], c["q"], c["box"], c["K"], c["order"], c["beta"])

    def per_atom(f, ref):
        # largest per-atom force error over the RMS force magnitude
        rms = np.sqrt(np.mean(np.sum(ref ** 2, axis=1)))
        return float(np.max(np.linalg.norm(f - ref, axis=1)) / rms)

    if got_frames:
        def check(item):
            t, f, e = item
            ref = oracle.spme(fr.host[t], fr.q, fr.box, fr.K, w.order, w.beta)
            return (rel_rms(f, ref["forces"]), abs(e - ref["E"]) / abs(ref["E"]),
                    per_atom(f, ref["forces"]))
        with ThreadPoolExecutor(max_workers=workers) as ex:
            errs = list(ex.map(check, got_frames))
        out["parity"] = {"frames": len(errs), "every": args.parity_every,
                         "force_rel_rms_max": max(x[0] for x in errs),
                         "energy_rel_max": max(x[1] for x in errs),
                         "force_max_atom_over_rms_max": max(x[2] for x in errs),
                         "within_bar": bool(all(x[0] <= 1e-5 and x[1] <= 1e-6 for x in errs)),
                         "reference": "FP64 CPU oracle"}
        t0 = got_frames[0][0]
        if reduced_got:
            ref = oracle.spme(fr.host[t0], fr.q, fr.box, fr.K, w.order, w.beta)
            for prec, (f, e) in reduced_got.items():
                out[prec] = {"force_rel_rms": rel_rms(f, ref["forces"]),
                             "energy_rel": abs(e - ref["E"]) / abs(ref["E"]), "parity_frame": t0}
    if more_checks:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            refs = list(ex.map(spme_ref, [c for _, c in more_checks]))
        out["more_workloads"] = {name: {"force_rel_rms": rel_rms(c["forces"], r["forces"]),
                                        "energy_rel": abs(c["E"] - r["E"]) / abs(r["E"]),
                                        "force_max_atom_over_rms": per_atom(c["forces"], r["forces"])}
                                 for (name, c), r in zip(more_checks, refs)}
    if batch_checks:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            refs = list(ex.map(spme_ref, batch_checks))
        out["batched"] = {"members_checked": len(refs),
                          "force_rel_rms_max": max(rel_rms(c["forces"], r["forces"])
                                                   for c, r in zip(batch_checks, refs)),
                          "energy_rel_max": max(abs(c["E"] - r["E"]) / abs(r["E"])
                                                for c, r in zip(batch_checks, refs))}
    if real_check is not None:
        c = real_check
        want = oracle.ewald_real_atoms(np.mod(c["pos"], c["box"][0, 0]), c["q"], c["box"],
                                       c["beta"], c["atoms"], nimg=1, rcut=c["rcut"])
        ex_all = oracle.ewald_excl(c["pos"], c["q"], c["box"], c["beta"], c["off"], c["idx"],
                                   rcut=c["rcut"])
        want = want + ex_all["forces"][c["atoms"]]
        out["real_space"] = {"atoms_checked": len(c["atoms"]),
                             "force_rel_rms": rel_rms(c["forces"], want),
                             "reference": "oracle real-space rows of the sampled atoms + exclusions"}
    if serving_kept:
        # every leg draws from the same pool: one oracle run per system used
        pool = next(iter(serving_pool.values()))
        need = sorted({sid for kept in serving_kept.values() for sid, _ in kept})

        def ref_of(sid):
            s = pool[sid]
            return sid, oracle.spme(s.pos, s.q, s.box, s.K, 4, 0.34)["forces"]
        with ThreadPoolExecutor(max_workers=workers) as ex:
            refs = dict(ex.map(ref_of, need))
        for label, kept in serving_kept.items():
            errs = [rel_rms(f, refs[sid]) for sid, f in kept]
            out["serving_" + label] = {"requests_checked": len(errs),
                                       "systems": len({sid for sid, _ in kept}),
                                       "force_rel_rms_max": max(errs),
                                       "fraction_within_1e-5": float(np.mean(np.array(errs) <= 1e-5))}
    cpu = None
    if not args.no_cpu_baseline:
        # one core: the oracle is single-threaded C; the calling thread is
        # pinned to one CPU for the sample
        try:
            old_aff = os.sched_getaffinity(0)
            core = min(old_aff)
            os.sched_setaffinity(0, {core})
        except (AttributeError, OSError):
            old_aff, core = None, None
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds or n == 0:
            oracle.spme(fr.host[n % fr.F], fr.q, fr.box, fr.K, w.order, w.beta)
            n += 1
        dt = time.perf_counter() - t0
        frames_used = min(n, fr.F)
        cpu = {"value": dt / n * 1e6, "unit": "us/step", "cores": 1, "kind": "oracle",
               "sample": f"{n} full oracle steps (single-threaded FP64 C) of the same workload, "
                         f"cycling over its first {frames_used} jittered frames",
               "pinned_core": core, "host": cpu_model(), "nproc": os.cpu_count()}

        def phases(pos_, q_, box_, K_, p_, b_, reps):
            runs = [oracle.spme(pos_, q_, box_, K_, p_, b_, want_times=True)["times"] for _ in range(reps)]
            tot = [sum(r.values()) for r in runs]
            mid = runs[int(np.argsort(tot)[len(tot) // 2])]
            return {"s_per_step": float(np.median(tot)), **{k: float(v) for k, v in mid.items()}}
        from paper_2009_12617_amd import inputs as I
        cpu["median_of_5"] = phases(fr.host[0], fr.q, fr.box, fr.K, w.order, w.beta, 5)
        ps, qs, bs = I.SMALL_32.make()
        cpu["water_4095_k32_median_of_5"] = phases(ps, qs, bs, I.SMALL_32.K, I.SMALL_32.order,
                                                   I.SMALL_32.beta, 5)
        if not args.no_large:
            for wl in (I.LARGE_128_P4, I.LARGE_128_P6):
                pl, ql, bl = wl.make()
                cpu[wl.name] = phases(pl, ql, bl, wl.K, wl.order, wl.beta, 1)
        if old_aff is not None:
            os.sched_setaffinity(0, old_aff)
    return out, cpu


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 path timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--parity-frames", type=int, default=1000,
                    help="at most this many frames checked against the oracle (0: no oracle leg checks)")
    ap.add_argument("--parity-every", type=int, default=10,
                    help="check every n-th frame of the timed run")
    ap.add_argument("--no-half", action="store_true", help="skip the binary16- and bfloat16-spectrum variants")
    ap.add_argument("--no-real", action="store_true", help="skip the real-space term")
    ap.add_argument("--profile", action="store_true",
                    help="for a profiler: only the headline's graph replays of plain and probe steps")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-system batched run")
    ap.add_argument("--no-noncubic", action="store_true", help="skip the 64 x 64 x 128 grid run")
    ap.add_argument("--no-large", action="store_true", help="skip the 128^3 (209,715-atom) runs")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner table")
    ap.add_argument("--profile-leg", default="",
                    help="for profilers: only `steps` host-launched evaluations of one leg "
                         "(real, batched, or a workload name such as water_209715_k128_p4; "
                         "a name ending in _fp64 runs that workload's plain FP64 path)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving runs")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--saturate-requests", type=int, default=4000)
    ap.add_argument("--saturate-rate", type=float, default=8000.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="with --profile: also run one plain device copy of this many MiB "
                         "(calibrates hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this SPME step runs on one GPU; --gpus {args.gpus} is not supported "
              "(one system is not sharded across GPUs here)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_12617_amd import Plan, Batch, BatchPool
    from paper_2009_12617_amd import inputs as I

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.profile_leg:
        profile_leg(torch, dev, Plan, BatchPool, I, args.profile_leg, args.steps)
        return
    F = max(1, min(args.frames, args.steps + args.warmup))
    fr = Frames(torch, dev, I, F)
    w, N, K = fr.w, fr.N, fr.K
    print(f"# staged {F} frames of {N} atoms ({fr.dev_pos.numel() * 8 / 1e9:.2f} GB) on "
          f"{torch.cuda.get_device_name(0)}", file=sys.stderr, flush=True)

    plan = Plan(K, w.order, w.beta, max_atoms=N, precision="fp32_fixed", device=dev)
    if args.profile:
        # for a profiler: the headline's graph replays (plain steps and the
        # probe steps of the per-kernel times) and nothing else
        for t in range(args.warmup):
            plan.step(fr.pos(t), fr.dev_q, fr.box)
        torch.cuda.synchronize()
        kus, base = kernel_times(torch, dev, plan, fr, args.steps)
        if args.copy_mib > 0:
            n = args.copy_mib * (1 << 20) // 8
            src = torch.ones(n, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            print(f"# calibration copy: {args.copy_mib} MiB read + {args.copy_mib} MiB written",
                  file=sys.stderr, flush=True)
        print(json.dumps({"mode": "profile", "steps": args.steps, "us_per_step": base,
                          "kernels_us": kus, "tuning": plan.tuning, "source_digest": source_digest()}))
        return
    ms_step, wall_ms, graph_ok = run_graph(torch, dev, plan, fr, args.steps, args.warmup)
    print(f"# fp32_fixed graph replay: {ms_step * 1e3:.2f} us/step, replay == eager: {graph_ok}",
          file=sys.stderr, flush=True)
    if not graph_ok:
        print("bench.py: graph replay differs from host-launched steps", file=sys.stderr)
        sys.exit(1)
    kus, _ = kernel_times(torch, dev, plan, fr, 100)
    print("# per-kernel us (graph replay, by difference): " + ", ".join(f"{k}={v:.2f}" for k, v in kus.items()),
          file=sys.stderr, flush=True)
    prof = profiled_kernel_us()
    roof = roofline_entry(N, K, kus, measured_traffic, prof)
    kfrac = {k: algorithmic_bytes(N, K, k) / (v * 1e-6) / 1e9 / HBM_PEAK_GBS
             for k, v in (prof or kus).items()}
    lat = graph_latency(torch, dev, plan, fr, min(args.steps, 1000))
    tuned = None
    if not args.no_autotune:
        # the autotuner's table for this workload (a second plan, so the
        # headline keeps the built-in choice it was timed with)
        tp = Plan(K, w.order, w.beta, max_atoms=N, device=dev)
        default = tp.tuning
        r = tp.autotune(fr.pos(0), fr.dev_q, fr.box, reps=20)
        tuned = {"default": default, "best": r["best"], "best_us": r["us"],
                 "candidates_us": {f"conv{c['conv']}/interp{c['interp']}/chunk{c['bin_chunk']}": t
                                   for c, t in r["candidates"] if t is not None},
                 "what": "pme_autotune: host-launched steps per variant, best of 3 sweeps"}
        print(f"# autotune: default {default}, best {r['best']} at {r['us']:.2f} us (host-launched)",
              file=sys.stderr, flush=True)
        del tp

    fp64 = None
    if not args.no_fp64:
        plan64 = Plan(K, w.order, w.beta, max_atoms=N, precision="fp64", device=dev)
        ms64, _, ok64 = run_graph(torch, dev, plan64, fr, args.steps, args.warmup, exact=False)
        if not ok64:
            print("bench.py: FP64 graph replay differs from host-launched steps", file=sys.stderr)
            sys.exit(1)
        fp64 = {"us_per_step": ms64 * 1e3, "speedup_fp32_fixed": ms64 / ms_step,
                "tuning": plan64.tuning,
                "step_roofline_frac": step_bytes(N, K, True) / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS}
        print(f"# fp64: {ms64 * 1e3:.2f} us/step", file=sys.stderr, flush=True)
        del plan64

    reduced, reduced_got = {}, {}
    if not args.no_half:
        for prec in ("fp32_fixed_half", "fp32_fixed_bf16"):
            plan16 = Plan(K, w.order, w.beta, max_atoms=N, precision=prec, device=dev)
            ms16, _, ok16 = run_graph(torch, dev, plan16, fr, args.steps, args.warmup)
            if not ok16:
                print(f"bench.py: {prec} graph replay differs from host-launched steps", file=sys.stderr)
                sys.exit(1)
            kh = K // 2 + 1
            reduced[prec] = {"us_per_step": ms16 * 1e3, "speedup_vs_fp32_fixed": ms_step / ms16,
                             "tuning": plan16.tuning,
                             "step_algorithmic_bytes": step_bytes(N, K) - 16 * K * K * kh}
            f, e = plan16.step(fr.pos(0), fr.dev_q, fr.box)
            reduced_got[prec] = (f.cpu().numpy(), float(e[0].item()))
            print(f"# {prec}: {ms16 * 1e3:.2f} us/step", file=sys.stderr, flush=True)
            del plan16

    real, real_check = None, None
    if not args.no_real:
        # the real-space term beside the step, same frames: erfc pair sum
        # (rcut 9 A, beta 0.34: erfc(beta rcut) ~ 1e-5), self term and the
        # intramolecular exclusions of every water
        from paper_2009_12617_amd import RealSpace
        rcut = 9.0
        rs = RealSpace(N, device=dev)
        off, idx = I.water_exclusions(N)
        excl = (torch.from_numpy(off).to(dev), torch.from_numpy(idx).to(dev))
        fr_out = torch.empty((N, 3), dtype=torch.float64, device=dev)
        for t in range(5):
            rs(fr.pos(t), fr.dev_q, fr.box, w.beta, rcut, exclusions=excl, forces=fr_out)
        torch.cuda.synchronize()
        nrep = 50
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        for t in range(nrep):
            rs(fr.pos(t), fr.dev_q, fr.box, w.beta, rcut, exclusions=excl, forces=fr_out)
        stop.record()
        torch.cuda.synchronize()
        ms_rs = start.elapsed_time(stop) / nrep
        nc = int(np.floor(fr.box[0, 0] / rcut))
        real = {"us_per_eval": ms_rs * 1e3, "rcut_A": rcut, "beta": w.beta, "cells": [nc] * 3,
                "launches": 6, "what": "pme_real: FP64 erfc pair sum, self term, water exclusions"}
        last = (nrep - 1) % F
        atoms = np.random.default_rng(7).choice(N, size=64, replace=False)
        real_check = {"pos": fr.host[last], "q": fr.q, "box": fr.box, "beta": w.beta, "rcut": rcut,
                      "atoms": atoms, "off": off, "idx": idx,
                      "forces": fr_out.cpu().numpy()[atoms]}
        print(f"# real space: {ms_rs * 1e3:.1f} us per evaluation", file=sys.stderr, flush=True)

    more, more_checks = {}, []
    legs = []
    if not args.no_noncubic:
        pos2, q2, box2 = stacked_water(I)
        legs.append(("water_131070_k64x64x128", pos2, q2, box2, (64, 64, 128), 4, 0.34, 2103))
    if not args.no_large:
        for wl in (I.LARGE_128_P4, I.LARGE_128_P6):
            pos2, q2, box2 = wl.make()
            legs.append((wl.name, pos2, q2, box2, wl.K, wl.order, wl.beta, 2104))
    for name, pos2, q2, box2, K2, p2, b2, js in legs:
        more[name], chk = bench_system(torch, dev, Plan, I, pos2, q2, box2, K2, p2, b2,
                                       min(args.steps, 200), min(args.warmup, 20), name, js)
        more_checks.append((name, chk))
        r = more[name]
        print(f"# {name}: {r['us_per_step']:.2f} us/step, step at {100 * r['step_roofline_frac']:.1f}% "
              f"of HBM roofline; per kernel " +
              ", ".join(f"{k}={v:.1f} us ({100 * r['kernels_roofline_frac'][k]:.0f}%)"
                        for k, v in r["kernels_us"].items()), file=sys.stderr, flush=True)

    batched, batch_checks = None, []
    if not args.no_batched:
        batched, batch_checks = bench_batched(torch, dev, Plan, BatchPool, Batch, I)
        print(f"# batched: {batched['us_per_batch']:.1f} us per 64-system batch "
              f"(one-launch replays p50 {batched['latency_us']['p50']:.1f}, "
              f"p99 {batched['latency_us']['p99']:.1f}; one stream "
              f"{batched['one_stream_pme_batch_run_us']:.1f}), same as single: "
              f"{batched['same_as_single_steps']}", file=sys.stderr, flush=True)

    serving, serving_kept, serving_pool = None, {}, {}
    if not args.no_serving:
        serving = {}
        for label, nreq, rate, every in (("nominal", args.serve_requests, args.serve_rate, 100),
                                         ("saturating", args.saturate_requests, args.saturate_rate, 40)):
            if nreq <= 0:
                continue
            st, kept, pool = bench_serving(torch, dev, I, nreq, rate, args.serve_budget_gib, every, label)
            serving[label] = st
            serving_kept[label] = kept
            serving_pool[label] = pool
            print(f"# serving ({label}): {st['throughput_per_s']:.0f} req/s, p50 {st['latency_us']['p50']:.0f} us, "
                  f"p99 {st['latency_us']['p99']:.0f} us, max {st['latency_us']['max']:.0f} us, "
                  f"mean batch {st['mean_batch']:.2f}; longest loop turn {st['longest_loop_turn_us']:.0f} us "
                  f"at {st['longest_loop_turn_at_s']:.4f} s; worst request {st['worst_request']}",
                  file=sys.stderr, flush=True)

    # sampled frames of the headline for the oracle leg (host-launched steps)
    got_frames = []
    if args.parity_frames > 0:
        pick = list(range(0, F, max(1, args.parity_every)))[:max(args.parity_frames, 1)]
        for t in pick:
            f, e = plan.step(fr.pos(t), fr.dev_q, fr.box)
            got_frames.append((t, f.cpu().numpy(), float(e[0].item())))
    else:
        more_checks, batch_checks, real_check, serving_kept, reduced_got = [], [], None, {}, {}
    checks, cpu = oracle_leg(args, fr, got_frames, reduced_got, more_checks, batch_checks,
                             real_check, serving_kept, serving_pool)
    if "parity" in checks:
        p = checks["parity"]
        print(f"# parity on {p['frames']} frames: force rel RMS max {p['force_rel_rms_max']:.2e}, "
              f"energy rel max {p['energy_rel_max']:.2e}, worst atom {p['force_max_atom_over_rms_max']:.2e} "
              "of the RMS force", file=sys.stderr, flush=True)
    for prec, d in reduced.items():
        d.update(checks.get(prec, {}))
    for name, d in more.items():
        d.update(checks.get("more_workloads", {}).get(name, {}))
    if batched is not None and "batched" in checks:
        batched["oracle"] = checks["batched"]
    if real is not None and "real_space" in checks:
        real["parity"] = checks["real_space"]
    if serving:
        for label in serving:
            if "serving_" + label in checks:
                serving[label].update(checks["serving_" + label])
    if cpu is not None:
        print(f"# oracle: {cpu['value'] / 1e3:.1f} ms/step on one core ({cpu['host']})",
              file=sys.stderr, flush=True)

    us = ms_step * 1e3
    out = {
        "metric": "us/PME step (65,535 atoms, 64^3), FP32/fixed-point path",
        "value": us,
        "unit": "us/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": us / 206.0,
        "baseline_note": "paper: 206 us/step, 65,536 atoms, 64^3, 4 Stratix 10 FPGAs (context; other hardware)",
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "atoms": N, "grid": K, "order": w.order, "beta": w.beta,
                   "box_A": float(fr.box[0, 0]), "frames": F, "jitter_A": I.HEADLINE_JITTER_SIGMA,
                   "tuning": plan.tuning,
                   "precision": "fp32 splines/FFT/convolution, int64 fixed-point charge grid, fp64 energy/virial"},
        "latency_us": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean()), "steps": int(len(lat)),
                       "what": "one step per single-step graph launch, stream-ordered"},
        "host_wall_us_per_step": wall_ms * 1e3,
        "timed_region": "one HIP graph replay of all timed steps (captured pme_step calls), enqueued "
                    "behind untimed device work so that graph submission is not timed",
        "kernels_us": kus,
        "kernels_us_what": "live: graph-replayed steps repeating the kernel minus plain steps",
        "kernels_us_profiled": prof,
        "kernels_roofline_frac": kfrac,
        "roofline": roof,
        "step_roofline_frac": step_bytes(N, K) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "step_algorithmic_bytes": step_bytes(N, K),
        "source_digest": source_digest(),
        "autotune": tuned,
        "fp64_path": fp64,
        "half_spectrum_path": reduced.get("fp32_fixed_half"),
        "bf16_spectrum_path": reduced.get("fp32_fixed_bf16"),
        "real_space": real,
        "more_workloads": more,
        "batched": batched,
        "serving": serving,
        "parity": checks.get("parity"),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def profile_leg(torch, dev, Plan, BatchPool, I, leg, steps):
    """Host-launched evaluations of one leg and nothing else, so that a
    profiler's statistics cover that leg only."""
    if leg == "real":
        from paper_2009_12617_amd import RealSpace
        w = I.HEADLINE_64
        pos, q, box = w.make()
        rs = RealSpace(len(q), device=dev)
        off, idx = I.water_exclusions(len(q))
        excl = (torch.from_numpy(off).to(dev), torch.from_numpy(idx).to(dev))
        dp, dq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
        fr = torch.empty((len(q), 3), dtype=torch.float64, device=dev)
        run = lambda: rs(dp, dq, box, w.beta, 9.0, exclusions=excl, forces=fr)  # noqa: E731
    elif leg == "batched":
        stream = torch.cuda.current_stream(dev)
        pool = BatchPool(8 << 30, max_systems=128, device=dev, stream=stream)
        for m in I.batch_mix():
            pos, q, box = m.make()
            s = pool.admit(m.K, 4, 0.34, box, len(q))
            pool.io(s)[0].copy_(torch.from_numpy(pos))
            pool.io(s)[1].copy_(torch.from_numpy(q))
        run = pool.launch
    else:
        named = {wl.name: wl for wl in (I.SMALL_32, I.HEADLINE_64, I.LARGE_128_P4, I.LARGE_128_P6)}
        precision = "fp32_fixed"
        if leg.endswith("_fp64"):  # a workload name with "_fp64": its plain FP64 path
            leg, precision = leg[: -len("_fp64")], "fp64"
        if leg == "water_131070_k64x64x128":
            pos, q, box = stacked_water(I)
            K, order, beta = (64, 64, 128), 4, 0.34
        elif leg in named:
            wl = named[leg]
            pos, q, box = wl.make()
            K, order, beta = wl.K, wl.order, wl.beta
        else:
            raise SystemExit(f"bench.py: unknown leg {leg!r}")
        plan = Plan(K, order, beta, max_atoms=len(q), precision=precision, device=dev)
        dp, dq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
        run = lambda: plan.step(dp, dq, box)  # noqa: E731
    for _ in range(3):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    print(json.dumps({"leg": leg, "precision": precision if leg not in ("real", "batched") else None,
                      "evaluations": steps,
                      "us_per_evaluation": (time.perf_counter() - t0) / steps * 1e6, "mode": "profile"}))


if __name__ == "__main__":
    main()
