#!/usr/bin/env python3
"""Benchmark of the SPME reciprocal-space step on one MI355X.

Workload: 21,845 TIP3P-like waters (65,535 atoms) in an 86.8 A cubic box, 64^3
grid, B-spline order 4, beta = 0.34 1/A; a random walk of N(0, 0.01 A) per
coordinate per frame gives the frame sequence, staged in HBM before timing.
A step is one full pme_step (bin, spread + x FFT, y/z FFTs + influence
function + energy/virial + inverse z/y FFTs, inverse x FFT + force
interpolation: four launches) on the next frame, stream-ordered after the
previous one.

Prints one JSON line (rank 0).  Extra fields: the plain FP64 path's time on
the same frames, per-step p50/p99 latency, per-kernel times, the roofline of
the dominant kernel, parity against the CPU oracle on sampled frames, and the
oracle's own CPU time on a bounded sample.
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
    return sum(algorithmic_bytes(N, K, k, fp64) for k in
               ("bin", "spread_x", "convolve_yz", "interpolate"))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def source_digest():
    h = hashlib.sha256()
    for f in ("spme_kernels.hip", "spme_device.h", "spme_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2009_12617_amd", "csrc", f), "rb").read())
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


def bench_batched(torch, dev, Plan, Batch, I, reps=200):
    """64 independent water boxes of uneven size (3k..65k atoms, grids 32/48/64
    by ~1 A spacing), one step of all of them per batched run, timed as graph
    replays; each system's result is checked against its own single step."""
    mix = I.batch_mix()
    systems = []
    for m in mix:
        pos, q, box = m.make()
        plan = Plan(m.K, 4, 0.34, max_atoms=len(q), device=dev)
        dp = torch.from_numpy(pos).to(dev)
        dq = torch.from_numpy(q).to(dev)
        f, e = plan.bind(dp, dq, box)
        systems.append((m, plan, dp, dq, box, f, e))
    batch = Batch([s[1] for s in systems])
    for _ in range(3):
        batch.run()
    torch.cuda.synchronize()
    got = [(s[5].clone(), s[6].clone()) for s in systems]
    same = True
    for s, (fb, eb) in zip(systems, got):
        fa, ea = s[1].step(s[2], s[3], s[4])
        same &= bool(torch.equal(fa, fb)) and bool(torch.equal(ea, eb))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream(device=dev)
    with torch.cuda.graph(g, stream=cs):
        batch.run(torch.cuda.current_stream(dev))
    g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    evs[0].record(stream)
    for r in range(reps):
        g.replay()
        evs[r + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(reps)]) * 1e3
    replay_same = all(bool(torch.equal(s[5], fb)) and bool(torch.equal(s[6], eb))
                      for s, (fb, eb) in zip(systems, got))
    atoms = sum(len(s[3]) for s in systems)
    grids = {}
    for m in mix:
        grids[str(m.K)] = grids.get(str(m.K), 0) + 1
    nbytes = sum(step_bytes(len(s[3]), s[0].K) for s in systems)
    return {
        "workload": "64 water boxes, atoms log-uniform in [3000, 65000], grid by ~1 A spacing, p=4, beta=0.34",
        "systems": len(systems), "atoms": int(atoms), "grids": grids,
        "us_per_batch": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                         "mean": float(per.mean()), "replays": reps},
        "atoms_per_s": atoms / (per.mean() * 1e-6),
        "step_algorithmic_bytes": int(nbytes),
        "roofline_frac": nbytes / (per.mean() * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "same_as_single_steps": bool(same and replay_same),
        "launch": "one HIP graph: 4 kernels x 3 grid groups, each launch over all systems of its group",
    }


def bench_system(torch, dev, Plan, I, pos, q, box, K, order, beta, steps, warmup, parity, name,
                 jitter_seed):
    """One more single-system workload, FP32/fixed path: the replay of one graph
    of `steps` steps over 16 jittered frames, per-kernel times from events on
    the dispatches (host-launched steps), each kernel's algorithmic GB/s
    against 8 TB/s, and the oracle's verdict on one frame."""
    N = len(q)
    F = 16
    frames = I.jitter_stream(pos, F, I.HEADLINE_JITTER_SIGMA, jitter_seed)
    d_frames = torch.from_numpy(frames).to(dev)
    d_q = torch.from_numpy(q).to(dev)
    plan = Plan(K, order, beta, max_atoms=N, device=dev)
    forces = torch.empty((N, 3), dtype=torch.float64, device=dev)
    ev = torch.empty(7, dtype=torch.float64, device=dev)
    for t in range(warmup):
        plan.step(d_frames[t % F], d_q, box, forces=forces, ev=ev)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream(device=dev)
    with torch.cuda.graph(g, stream=cs):
        plan.set_stream(torch.cuda.current_stream(dev))
        for t in range(steps):
            plan.step(d_frames[t % F], d_q, box, forces=forces, ev=ev)
    plan.set_stream(torch.cuda.current_stream(dev))
    g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    g.replay()
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    last = (steps - 1) % F
    fg, eg = forces.clone(), ev.clone()
    fe, ee = plan.step(d_frames[last], d_q, box)
    torch.cuda.synchronize()
    same = bool(torch.equal(fg, fe)) and bool(torch.equal(eg, ee))
    del g
    plan.kernel_timing(True)
    for t in range(steps):
        plan.step(d_frames[t % F], d_q, box, forces=forces, ev=ev)
    kms, ksteps = plan.kernel_times()
    plan.kernel_timing(False)
    kus = {k: v / max(ksteps, 1) * 1e3 for k, v in kms.items()}
    kfrac = {k: algorithmic_bytes(N, K, k) / (kus[k] * 1e-6) / 1e9 / HBM_PEAK_GBS for k in kus}
    K3 = list(K) if np.ndim(K) else [int(K)] * 3
    out = {"workload": name, "atoms": N, "grid": K3, "order": order, "beta": beta,
           "box_A": [float(box[i, i]) for i in range(3)], "us_per_step": ms * 1e3,
           "kernels_us": kus, "kernels_roofline_frac": kfrac,
           "step_algorithmic_bytes": int(step_bytes(N, K)),
           "step_roofline_frac": step_bytes(N, K) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "replay_same_as_eager": same}
    if parity:
        import oracle
        ref = oracle.spme(frames[last], q, box, K, order, beta)
        out["force_rel_rms"] = float(np.linalg.norm(fe.cpu().numpy() - ref["forces"]) /
                                     np.linalg.norm(ref["forces"]))
        out["energy_rel"] = float(abs(ee[0].item() - ref["E"]) / abs(ref["E"]))
    return out


def stacked_water(I):
    """The headline density on an elongated cell: two independent 86.8 A water
    boxes stacked along z (131,070 atoms, 86.8 x 86.8 x 173.6 A)."""
    L = 86.8
    a = I.water_box(21845, L, 2101)
    b = I.water_box(21845, L, 2102)
    pos = np.concatenate([a[0], b[0] + np.array([0.0, 0.0, L])])
    q = np.concatenate([a[1], b[1]])
    return pos, q, np.diag([L, L, 2 * L])


def profile_leg(torch, dev, Plan, I, leg, steps):
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
    else:
        named = {wl.name: wl for wl in (I.SMALL_32, I.HEADLINE_64, I.LARGE_128_P4, I.LARGE_128_P6)}
        if leg == "water_131070_k64x64x128":
            pos, q, box = stacked_water(I)
            K, order, beta = (64, 64, 128), 4, 0.34
        elif leg in named:
            wl = named[leg]
            pos, q, box = wl.make()
            K, order, beta = wl.K, wl.order, wl.beta
        else:
            raise SystemExit(f"bench.py: unknown leg {leg!r}")
        plan = Plan(K, order, beta, max_atoms=len(q), device=dev)
        dp, dq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
        run = lambda: plan.step(dp, dq, box)  # noqa: E731
    for _ in range(3):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    print(json.dumps({"leg": leg, "evaluations": steps,
                      "us_per_evaluation": (time.perf_counter() - t0) / steps * 1e6, "mode": "profile"}))


def bench_serving(torch, dev, I, n_requests, rate, budget_gib):
    """Open-loop Poisson arrivals over the batch mix plus four 128^3 boxes."""
    from paper_2009_12617_amd.serve import PoolSystem, Server
    from paper_2009_12617_amd import Plan
    members = I.serving_pool()
    pool = []
    for m in members:
        pos, q, box = m.make()
        pool.append(PoolSystem(pos, q, box, m.K))
    arrivals, ids = I.poisson_requests(n_requests=n_requests, rate=rate)
    srv = Server(pool, hbm_budget_bytes=int(budget_gib * (1 << 30)), max_batch=64, device=dev)
    done = srv.run(arrivals, ids)
    st = srv.stats.summary()
    # every request's energy against its system's own single step
    ref_e = {}
    same = True
    for r in done:
        if r.system_id not in ref_e:
            s = pool[r.system_id]
            plan = Plan(s.K, 4, 0.34, max_atoms=len(s.q), device=dev)
            _, e = plan.step(torch.from_numpy(s.pos).to(dev), torch.from_numpy(s.q).to(dev), s.box)
            ref_e[r.system_id] = e[0].item()
        same &= (r.energy == ref_e[r.system_id])
    st.update({
        "workload": f"{n_requests} requests, Poisson {rate:g}/s; 90% from the 64-box mix, 10% 128^3 / 209,715-atom boxes",
        "hbm_budget_gib": budget_gib,
        "energies_same_as_single_steps": bool(same),
        "latency_definition": "host: scheduled arrival to forces and energy in host memory",
    })
    return st


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
                    help="at most this many frames checked against the oracle (0: none)")
    ap.add_argument("--parity-every", type=int, default=10,
                    help="check every n-th frame of the timed run")
    ap.add_argument("--no-half", action="store_true", help="skip the binary16- and bfloat16-spectrum variants")
    ap.add_argument("--no-real", action="store_true", help="skip the real-space term")
    ap.add_argument("--profile", action="store_true",
                    help="short run for a profiler: fixed steps, no oracle legs")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-system batched run")
    ap.add_argument("--no-noncubic", action="store_true", help="skip the 64 x 64 x 128 grid run")
    ap.add_argument("--no-large", action="store_true", help="skip the 128^3 (209,715-atom) runs")
    ap.add_argument("--profile-leg", default="",
                    help="for profilers: only `steps` host-launched evaluations of one leg "
                         "(real, or a workload name such as water_209715_k128_p4)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="with --profile: also run one plain device copy of this many MiB "
                         "(calibrates hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this SPME step runs on one GPU; --gpus {args.gpus} is not supported "
              "(one system is not sharded across GPUs here)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_12617_amd import Plan, KERNEL_NAMES
    from paper_2009_12617_amd import inputs as I

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.profile_leg:
        profile_leg(torch, dev, Plan, I, args.profile_leg, args.steps)
        return
    w = I.HEADLINE_64
    pos0, q, box = w.make()
    N, K = len(q), w.K
    F = max(1, min(args.frames, args.steps + args.warmup))
    frames = I.jitter_stream(pos0, F, I.HEADLINE_JITTER_SIGMA, I.HEADLINE_JITTER_SEED)
    d_frames = torch.from_numpy(frames).to(dev)
    d_q = torch.from_numpy(q).to(dev)
    print(f"# staged {F} frames of {N} atoms ({d_frames.numel() * 8 / 1e9:.2f} GB) on {torch.cuda.get_device_name(0)}",
          file=sys.stderr, flush=True)

    def run(plan, steps, warmup, per_step=False):
        """Host-launched steps; device time per step from events around them."""
        forces = torch.empty((N, 3), dtype=torch.float64, device=dev)
        ev = torch.empty(7, dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream(dev)
        for t in range(warmup):
            plan.step(d_frames[t % F], d_q, box, forces=forces, ev=ev)
        torch.cuda.synchronize()
        if per_step:
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
            evs[0].record(stream)
            for t in range(steps):
                plan.step(d_frames[(warmup + t) % F], d_q, box, forces=forces, ev=ev)
                evs[t + 1].record(stream)
            torch.cuda.synchronize()
            return np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record(stream)
        for t in range(steps):
            plan.step(d_frames[(warmup + t) % F], d_q, box, forces=forces, ev=ev)
        stop.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return start.elapsed_time(stop) / steps, wall / steps * 1e3

    def capture(plan, first, steps, forces, ev):
        """One HIP graph holding `steps` consecutive steps (frames first, first+1, ...)."""
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream(device=dev)
        with torch.cuda.graph(g, stream=cs):
            plan.set_stream(torch.cuda.current_stream(dev))
            for t in range(steps):
                plan.step(d_frames[(first + t) % F], d_q, box, forces=forces, ev=ev)
        plan.set_stream(torch.cuda.current_stream(dev))
        return g

    def run_graph(plan, steps, warmup, exact=True):
        """The timed region replays one captured graph of `steps` stream-ordered
        steps; replays are checked against host-launched steps (bit for bit on
        the fixed-point path; the FP64 path accumulates its grid with FP64
        atomics, whose order, and so last-bit rounding, varies run to run)."""
        forces = torch.empty((N, 3), dtype=torch.float64, device=dev)
        ev = torch.empty(7, dtype=torch.float64, device=dev)
        for t in range(warmup):
            plan.step(d_frames[t % F], d_q, box, forces=forces, ev=ev)
        torch.cuda.synchronize()
        g = capture(plan, warmup, steps, forces, ev)
        g.replay()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream(dev)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record(stream)
        g.replay()
        stop.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = start.elapsed_time(stop) / steps
        # the replay's last step against a host-launched step on the same frame,
        # twice, with eager work in between
        last = (warmup + steps - 1) % F
        ok = True
        for _ in range(2):
            fg, eg = forces.clone(), ev.clone()
            fe, ee = plan.step(d_frames[last], d_q, box)
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

    def graph_latency(plan, steps):
        """Per-step latency of single-step graph launches (one frame each)."""
        forces = torch.empty((N, 3), dtype=torch.float64, device=dev)
        ev = torch.empty(7, dtype=torch.float64, device=dev)
        gs = [capture(plan, t, 1, forces, ev) for t in range(min(steps, F, 200))]
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
        return np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])

    plan = Plan(K, w.order, w.beta, max_atoms=N, precision="fp32_fixed", device=dev)
    ms_eager, wall_eager = run(plan, args.steps, args.warmup)
    print(f"# fp32_fixed host-launched: {ms_eager * 1e3:.2f} us/step (device events), "
          f"{wall_eager * 1e3:.2f} us/step (host wall)", file=sys.stderr, flush=True)
    ms_step, wall_ms, graph_ok = run_graph(plan, args.steps, args.warmup)
    print(f"# fp32_fixed graph replay: {ms_step * 1e3:.2f} us/step, replay == eager: {graph_ok}",
          file=sys.stderr, flush=True)
    if not graph_ok:
        print("bench.py: graph replay differs from host-launched steps", file=sys.stderr)
        sys.exit(1)
    if args.profile:
        if args.copy_mib > 0:
            n = args.copy_mib * (1 << 20) // 8
            src = torch.ones(n, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            print(f"# calibration copy: {args.copy_mib} MiB read + {args.copy_mib} MiB written",
                  file=sys.stderr, flush=True)
        print(json.dumps({"metric": "us/PME step (65,535 atoms, 64^3)", "value": ms_step * 1e3,
                          "unit": "us/step", "mode": "profile",
                          "host_launched_us_per_step": ms_eager * 1e3}))
        return

    lat = graph_latency(plan, min(args.steps, 1000)) * 1e3
    lat_eager = run(plan, min(args.steps, 1000), 5, per_step=True) * 1e3
    plan.kernel_timing(True)
    run(plan, min(args.steps, 500), 0)
    kms, ksteps = plan.kernel_times()
    plan.kernel_timing(False)
    kavg_us = {k: v / max(ksteps, 1) * 1e3 for k, v in kms.items()}
    print("# per-kernel us: " + ", ".join(f"{k}={v:.2f}" for k, v in kavg_us.items()),
          file=sys.stderr, flush=True)
    dom = max(kavg_us, key=kavg_us.get)
    dom_bytes = algorithmic_bytes(N, K, dom)
    achieved = dom_bytes / (kavg_us[dom] * 1e-6) / 1e9
    traffic = measured_traffic(dom)

    fp64 = None
    if not args.no_fp64:
        plan64 = Plan(K, w.order, w.beta, max_atoms=N, precision="fp64", device=dev)
        ms64, _, ok64 = run_graph(plan64, args.steps, args.warmup, exact=False)
        if not ok64:
            print("bench.py: FP64 graph replay differs from host-launched steps", file=sys.stderr)
            sys.exit(1)
        fp64 = {"us_per_step": ms64 * 1e3, "speedup_fp32_fixed": ms64 / ms_step,
                "step_roofline_frac": step_bytes(N, K, True) / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS}
        print(f"# fp64: {ms64 * 1e3:.2f} us/step", file=sys.stderr, flush=True)

    reduced = {}  # precision -> (plan, result dict)
    if not args.no_half:
        # the reduced-precision variants: the half spectrum in binary16 or
        # bfloat16 between launches (bytes of both corner turns halved);
        # accuracy below
        for prec in ("fp32_fixed_half", "fp32_fixed_bf16"):
            plan16 = Plan(K, w.order, w.beta, max_atoms=N, precision=prec, device=dev)
            ms16, _, ok16 = run_graph(plan16, args.steps, args.warmup)
            if not ok16:
                print(f"bench.py: {prec} graph replay differs from host-launched steps", file=sys.stderr)
                sys.exit(1)
            kh = K // 2 + 1
            reduced[prec] = (plan16, {"us_per_step": ms16 * 1e3, "speedup_vs_fp32_fixed": ms_step / ms16,
                                      "step_algorithmic_bytes": step_bytes(N, K) - 16 * K * K * kh})
            print(f"# {prec}: {ms16 * 1e3:.2f} us/step", file=sys.stderr, flush=True)

    real = None
    if not args.no_real:
        # the real-space term beside the step, same frames: erfc pair sum
        # (rcut 9 A, beta 0.34: erfc(beta rcut) ~ 1e-5), self term and the
        # intramolecular exclusions of every water
        from paper_2009_12617_amd import RealSpace
        rcut = 9.0
        rs = RealSpace(N, device=dev)
        off, idx = I.water_exclusions(N)
        excl = (torch.from_numpy(off).to(dev), torch.from_numpy(idx).to(dev))
        fr = torch.empty((N, 3), dtype=torch.float64, device=dev)
        for t in range(5):
            rs(d_frames[t % F], d_q, box, w.beta, rcut, exclusions=excl, forces=fr)
        torch.cuda.synchronize()
        nrep = 50
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        for t in range(nrep):
            rs(d_frames[t % F], d_q, box, w.beta, rcut, exclusions=excl, forces=fr)
        stop.record()
        torch.cuda.synchronize()
        ms_rs = start.elapsed_time(stop) / nrep
        nc = int(np.floor(box[0, 0] / rcut))
        real = {"us_per_eval": ms_rs * 1e3, "rcut_A": rcut, "beta": w.beta, "cells": [nc] * 3,
                "launches": 6, "what": "pme_real: FP64 erfc pair sum, self term, water exclusions"}
        print(f"# real space: {ms_rs * 1e3:.1f} us per evaluation", file=sys.stderr, flush=True)

    more = {}
    legs = []
    if not args.no_noncubic:
        # 64 x 64 x 128 grid (the headline's 1.36 A spacing) on the stacked cell
        pos2, q2, box2 = stacked_water(I)
        legs.append(("water_131070_k64x64x128", pos2, q2, box2, (64, 64, 128), 4, 0.34, 2103))
    if not args.no_large:
        for wl in (I.LARGE_128_P4, I.LARGE_128_P6):
            pos2, q2, box2 = wl.make()
            legs.append((wl.name, pos2, q2, box2, wl.K, wl.order, wl.beta, 2104))
    for name, pos2, q2, box2, K2, p2, b2, js in legs:
        more[name] = bench_system(torch, dev, Plan, I, pos2, q2, box2, K2, p2, b2,
                                  min(args.steps, 200), min(args.warmup, 20),
                                  args.parity_frames > 0, name, js)
        r = more[name]
        print(f"# {name}: {r['us_per_step']:.2f} us/step, step at {100 * r['step_roofline_frac']:.1f}% "
              f"of HBM roofline; per kernel " +
              ", ".join(f"{k}={v:.1f} us ({100 * r['kernels_roofline_frac'][k]:.0f}%)"
                        for k, v in r["kernels_us"].items()), file=sys.stderr, flush=True)

    batched = None
    if not args.no_batched:
        from paper_2009_12617_amd import Batch
        batched = bench_batched(torch, dev, Plan, Batch, I)
        print(f"# batched: {batched['us_per_batch']['mean']:.1f} us per 64-system batch "
              f"(p99 {batched['us_per_batch']['p99']:.1f}), same as single: {batched['same_as_single_steps']}",
              file=sys.stderr, flush=True)
    serving = None
    if not args.no_serving:
        serving = bench_serving(torch, dev, I, args.serve_requests, args.serve_rate,
                                args.serve_budget_gib)
        print(f"# serving: {serving['throughput_per_s']:.0f} req/s, p50 {serving['latency_us']['p50']:.0f} us, "
              f"p99 {serving['latency_us']['p99']:.0f} us", file=sys.stderr, flush=True)

    parity = None
    cpu = None
    if args.parity_frames > 0 or not args.no_cpu_baseline:
        import oracle
        oracle._load()
    if args.parity_frames > 0:
        # every args.parity_every-th frame of the timed run, one host-launched
        # step each, against the oracle (oracle calls run in threads: the C
        # library releases the GIL)
        from concurrent.futures import ThreadPoolExecutor
        pick = list(range(0, F, max(1, args.parity_every)))[:max(args.parity_frames, 1)]
        got = []
        for t in pick:
            f, e = plan.step(d_frames[t], d_q, box)
            got.append((f.cpu().numpy(), float(e[0].item())))

        def check(i):
            ref = oracle.spme(frames[pick[i]], q, box, K, w.order, w.beta)
            fr = float(np.linalg.norm(got[i][0] - ref["forces"]) / np.linalg.norm(ref["forces"]))
            return fr, float(abs(got[i][1] - ref["E"]) / abs(ref["E"]))

        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            errs = list(ex.map(check, range(len(pick))))
        parity = {"frames": len(pick), "every": args.parity_every,
                  "force_rel_rms_max": max(x[0] for x in errs),
                  "energy_rel_max": max(x[1] for x in errs),
                  "within_bar": bool(all(x[0] <= 1e-5 and x[1] <= 1e-6 for x in errs)),
                  "reference": "FP64 CPU oracle"}
        print(f"# parity on {len(pick)} frames: force rel RMS max {parity['force_rel_rms_max']:.2e}, "
              f"energy rel max {parity['energy_rel_max']:.2e}", file=sys.stderr, flush=True)
        if reduced:
            ref = oracle.spme(frames[pick[0]], q, box, K, w.order, w.beta)
            for plan16, half in reduced.values():
                f, e = plan16.step(d_frames[pick[0]], d_q, box)
                half["force_rel_rms"] = float(np.linalg.norm(f.cpu().numpy() - ref["forces"]) /
                                              np.linalg.norm(ref["forces"]))
                half["energy_rel"] = float(abs(e[0].item() - ref["E"]) / abs(ref["E"]))
                half["parity_frame"] = pick[0]
    if not args.no_cpu_baseline:
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds or n == 0:
            oracle.spme(frames[n % F], q, box, K, w.order, w.beta)
            n += 1
        dt = time.perf_counter() - t0
        cpu = {"value": dt / n * 1e6, "unit": "us/step", "cores": 1, "kind": "oracle",
               "sample": f"{n} full oracle steps (single-threaded FP64 C) on frames 0..{n - 1} of the same workload",
               "host": cpu_model(), "nproc": os.cpu_count()}
        # median of 5 steps with the oracle's own phase split, and the small
        # and large workloads for context
        def phases(pos_, q_, box_, K_, p_, b_, reps):
            runs = [oracle.spme(pos_, q_, box_, K_, p_, b_, want_times=True)["times"] for _ in range(reps)]
            tot = [sum(r.values()) for r in runs]
            mid = runs[int(np.argsort(tot)[len(tot) // 2])]
            return {"s_per_step": float(np.median(tot)), **{k: float(v) for k, v in mid.items()}}
        cpu["median_of_5"] = phases(frames[0], q, box, K, w.order, w.beta, 5)
        small = I.SMALL_32
        ps, qs, bs = small.make()
        cpu["water_4095_k32_median_of_5"] = phases(ps, qs, bs, small.K, small.order, small.beta, 5)
        if not args.no_large:
            for wl in (I.LARGE_128_P4, I.LARGE_128_P6):
                pl, ql, bl = wl.make()
                cpu[wl.name] = phases(pl, ql, bl, wl.K, wl.order, wl.beta, 1)
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
                   "box_A": float(box[0, 0]), "frames": F, "jitter_A": I.HEADLINE_JITTER_SIGMA,
                   "precision": "fp32 splines/FFT/convolution, int64 fixed-point charge grid, fp64 energy/virial"},
        "latency_us": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean()), "steps": int(len(lat)),
                       "what": "one step per single-step graph launch, stream-ordered"},
        "host_launched": {"us_per_step": ms_eager * 1e3, "host_wall_us_per_step": wall_eager * 1e3,
                          "latency_p50_us": float(np.percentile(lat_eager, 50)),
                          "latency_p99_us": float(np.percentile(lat_eager, 99))},
        "timed_region": "one HIP graph replay of all timed steps (captured pme_step calls)",
        "kernels_us": kavg_us,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": dom_bytes},
        "step_roofline_frac": step_bytes(N, K) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "step_algorithmic_bytes": step_bytes(N, K),
        "fp64_path": fp64,
        "half_spectrum_path": reduced.get("fp32_fixed_half", (None, None))[1],
        "bf16_spectrum_path": reduced.get("fp32_fixed_bf16", (None, None))[1],
        "real_space": real,
        "more_workloads": more,
        "batched": batched,
        "serving": serving,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
