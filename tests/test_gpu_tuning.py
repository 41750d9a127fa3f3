"""Kernel variants and autotuning (pme_set_tuning, pme_autotune).

Every variant computes the same step and matches the FP64 oracle at the
FP32 bars.  The fused and split convolutions, both interpolations and every
binning chunk perform the same per-element arithmetic, so their forces are
bit-identical and their energy/virial agree to summation order
(bit-identical within one convolution variant); the register-resident
convolution factors its transforms differently (radix 8 x 8 with its own
twiddle order), so it agrees with them to the rounding of the precision.  The autotuner's choice is
re-timed against the built-in default on the full-size workloads."""
import ctypes
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2009_12617_amd import inputs as I

pytestmark = pytest.mark.gpu

F32_FORCE, F32_ENERGY = 1e-5, 1e-6


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2009_12617_amd as pkg
    return pkg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def variants(plan):
    v = plan.variants()
    convs = [c for c, bit in ((0, 1), (1, 2), (2, 16)) if v & bit]
    interps = [i for i, bit in ((0, 4), (1, 8)) if v & bit]
    return [(c, i, b) for c in convs for i in interps for b in (256, 512, 1024)]


CASES = [  # name, waters, edge, grid, order, beta, precision
    ("k32_p4", 1365, 32.0, 32, 4, 0.35, "fp32_fixed"),
    ("k48_p6", 2000, 40.0, 48, 6, 0.34, "fp32_fixed"),
    ("k64_p4", 3000, 50.0, 64, 4, 0.34, "fp32_fixed"),
    ("k64x64x128_p4", 2500, (40.0, 40.0, 80.0), (64, 64, 128), 4, 0.34, "fp32_fixed"),
    ("k128_p6", 1500, 50.0, 128, 6, 0.34, "fp32_fixed"),
    ("k64_p6_fp64", 1500, 40.0, 64, 6, 0.34, "fp64"),
]


def make(case):
    name, nw, L, K, p, beta, prec = case
    if np.ndim(L) == 0:
        pos, q, box = I.water_box(nw, L, 300 + sum(map(ord, name)))
    else:
        pos, q, _ = I.water_box(nw, L[0], 300 + sum(map(ord, name)))
        pos[:, 2] *= L[2] / L[0]
        box = np.diag(L)
    return pos, q, box


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_every_variant_same_step(P, case):
    name, nw, L, K, p, beta, prec = case
    pos, q, box = make(case)
    plan = P.Plan(K, p, beta, max_atoms=len(q), precision=prec)
    ref = oracle.spme(pos, q, box, K, p, beta)
    dp, dq = dev(pos), dev(q)
    base = None
    fixed = prec != "fp64"
    for c, i, b in variants(plan):
        plan.set_tuning(conv=c, interp=i, bin_chunk=b)
        assert plan.tuning == {"conv": c, "interp": i, "bin_chunk": b}
        f, e = plan.step(dp, dq, box)
        fc, ec = f.cpu().numpy(), e.cpu().numpy()
        fr = np.linalg.norm(fc - ref["forces"]) / np.linalg.norm(ref["forces"])
        er = abs(ec[0] - ref["E"]) / abs(ref["E"])
        print(f"{name} conv={c} interp={i} chunk={b}: force {fr:.2e} energy {er:.2e}", flush=True)
        assert fr <= (F32_FORCE if fixed else 1e-10)
        assert er <= (F32_ENERGY if fixed else 1e-11)
        if base is None:
            base = (c, fc, ec)
            continue
        if c == 2:
            # another factorisation of the FFTs: FP32 rounding apart
            assert np.linalg.norm(fc - base[1]) <= 2e-6 * np.linalg.norm(base[1])
            assert abs(ec[0] - base[2][0]) <= 1e-6 * abs(base[2][0])
            continue
        if fixed:
            assert np.array_equal(fc, base[1]), (c, i, b)
        else:  # FP64 grid accumulation order varies run to run
            assert np.allclose(fc, base[1], rtol=1e-12, atol=1e-15)
        if c == base[0] and fixed:
            assert np.array_equal(ec, base[2])
        else:
            assert np.allclose(ec, base[2], rtol=1e-12, atol=1e-13 * abs(ec[0]))


def test_set_tuning_rejects_and_orders(P):
    pos, q, box = I.water_box(300, 16.0, 5)
    plan = P.Plan(16, 4, 0.4, max_atoms=len(q))
    with pytest.raises(RuntimeError):
        plan.set_tuning(conv=1)  # 16^3 has no split column passes
    with pytest.raises(RuntimeError):
        plan.set_tuning(bin_chunk=300)
    plan.spread(dev(pos), dev(q), box)
    with pytest.raises(RuntimeError):
        plan.set_tuning(interp=1)  # between spread and solve
    plan.solve()
    plan.set_tuning(interp=1)
    plan.gather()
    torch.cuda.synchronize()


def graph_us(P, plan, dp, dq, box, steps=100):
    """Mean microseconds per step of one graph replay of `steps` steps."""
    f = torch.empty((dp.shape[0], 3), dtype=torch.float64, device="cuda")
    ev = torch.empty(7, dtype=torch.float64, device="cuda")
    for _ in range(5):
        plan.step(dp, dq, box, forces=f, ev=ev)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=torch.cuda.Stream()):
        plan.set_stream(torch.cuda.current_stream())
        for _ in range(steps):
            plan.step(dp, dq, box, forces=f, ev=ev)
    plan.set_stream(torch.cuda.current_stream())
    g.replay()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) * 1e3 / steps)
    return best


@pytest.mark.parametrize("wl", ["water_65535_k64", "water_209715_k128_p4", "water_209715_k128_p6"])
def test_autotuned_never_slower_than_default(P, wl, tmp_path):
    from paper_2009_12617_amd import tuning
    w = {x.name: x for x in (I.HEADLINE_64, I.LARGE_128_P4, I.LARGE_128_P6)}[wl]
    pos, q, box = w.make()
    dp, dq = dev(pos), dev(q)
    plan = P.Plan(w.K, w.order, w.beta, max_atoms=len(q))
    default = plan.tuning
    t_default = graph_us(P, plan, dp, dq, box)
    path = str(tmp_path / "autotune.json")
    e = tuning.tune(plan, dp, dq, box, reps=10, path=path)
    assert plan.tuning == e["best"]
    assert e["default"] == default
    t_tuned = graph_us(P, plan, dp, dq, box)
    print(f"{wl}: default {default} {t_default:.2f} us, tuned {e['best']} {t_tuned:.2f} us; "
          f"candidates {e['candidates']}", flush=True)
    assert t_tuned <= 1.05 * t_default
    # parity unchanged under the tuned variants
    f, ev = plan.step(dp, dq, box)
    ref = oracle.spme(pos, q, box, w.K, w.order, w.beta)
    fr = np.linalg.norm(f.cpu().numpy() - ref["forces"]) / np.linalg.norm(ref["forces"])
    assert fr <= F32_FORCE
    assert abs(ev[0].item() - ref["E"]) / abs(ref["E"]) <= F32_ENERGY
    # the cache answers the next plan of this shape without measuring
    saved = json.load(open(path))
    assert len(saved) == 1
    plan2 = P.Plan(w.K, w.order, w.beta, max_atoms=len(q))
    plan2.autotune = None  # would raise if called
    e2 = tuning.tune(plan2, dp, dq, box, path=path)
    assert e2["best"] == e["best"] and plan2.tuning == e["best"]
    assert tuning.lookup(plan2, len(q), path=path) == e["best"]
