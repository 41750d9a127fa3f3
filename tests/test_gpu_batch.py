"""Batched runs (pme_bind + pme_batch_run): many independent systems of
uneven size and grid share each kernel launch.  Every system's result must be
the same as its own pme_step -- bit for bit on the fixed-point path (whose
grid is order-free), to 1e-11 on the FP64 path (FP64 grid accumulation order
varies) -- alone, in a mix, and under HIP graph replay."""
import numpy as np
import pytest
import torch

import oracle
from paper_2009_12617_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2009_12617_amd as pkg
    return pkg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def make_systems(P, members, precision="fp32_fixed", order=4, beta=0.34):
    out = []
    for m in members:
        pos, q, box = m.make()
        plan = P.Plan(m.K, order, beta, max_atoms=len(q), precision=precision)
        dp, dq = dev(pos), dev(q)
        f, e = plan.bind(dp, dq, box)
        out.append(dict(m=m, pos=pos, q=q, box=box, plan=plan, dp=dp, dq=dq, f=f, e=e))
    return out


def small_mix(n=12, seed=41):
    # a scaled-down version of the uneven batch (atoms 600..9000, grids 32/48/64)
    mix = I.batch_mix(n_systems=n, seed=seed, lo=600, hi=9000)
    return mix


@pytest.mark.parametrize("precision", ["fp32_fixed", "fp64", "fp32_fixed_half", "fp32_fixed_bf16"])
def test_batch_matches_single_steps(P, precision):
    mix = small_mix()
    assert len({m.K for m in mix}) >= 2
    sys = make_systems(P, mix, precision)
    batch = P.Batch([s["plan"] for s in sys])
    batch.run()
    torch.cuda.synchronize()
    got = [(s["f"].clone(), s["e"].clone()) for s in sys]
    for s, (fb, eb) in zip(sys, got):
        fa, ea = s["plan"].step(s["dp"], s["dq"], s["box"])
        if precision != "fp64":
            assert torch.equal(fa, fb) and torch.equal(ea, eb), s["m"].index
        else:
            assert torch.allclose(fa, fb, rtol=1e-11, atol=1e-15)
            assert torch.allclose(ea, eb, rtol=1e-11, atol=1e-15)
    # and against the oracle for a few members
    for s, (fb, eb) in list(zip(sys, got))[:3]:
        ref = oracle.spme(s["pos"], s["q"], s["box"], s["m"].K, 4, 0.34)
        fr = np.linalg.norm(fb.cpu().numpy() - ref["forces"]) / np.linalg.norm(ref["forces"])
        er = abs(eb[0].item() - ref["E"]) / abs(ref["E"])
        ftol, etol = {"fp32_fixed": (1e-5, 1e-6), "fp64": (1e-10, 1e-11),
                      "fp32_fixed_half": (1e-3, 2e-4), "fp32_fixed_bf16": (8e-3, 4e-3)}[precision]
        assert fr <= ftol and er <= etol


def test_result_same_alone_and_in_mix(P):
    mix = small_mix(n=9, seed=7)
    sys = make_systems(P, mix)
    alone = []
    for s in sys:
        P.Batch([s["plan"]]).run()
        torch.cuda.synchronize()
        alone.append((s["f"].clone(), s["e"].clone()))
    # the same systems in one mixed batch, in a different order, twice
    order = list(reversed(range(len(sys))))
    batch = P.Batch([sys[i]["plan"] for i in order])
    for _ in range(2):
        batch.run()
        torch.cuda.synchronize()
        for s, (fa, ea) in zip(sys, alone):
            assert torch.equal(s["f"], fa) and torch.equal(s["e"], ea)


def test_batch_graph_replay(P):
    mix = small_mix(n=6, seed=3)
    sys = make_systems(P, mix)
    batch = P.Batch([s["plan"] for s in sys])
    batch.run()
    torch.cuda.synchronize()
    ref = [(s["f"].clone(), s["e"].clone()) for s in sys]
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=cs):
        batch.run(torch.cuda.current_stream())
    for _ in range(3):
        for s in sys:
            s["f"].zero_()
            s["e"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for s, (fr, er) in zip(sys, ref):
            assert torch.equal(s["f"], fr) and torch.equal(s["e"], er)
        # eager work between replays
        sys[0]["plan"].step(sys[0]["dp"], sys[0]["dq"], sys[0]["box"])
        torch.cuda.synchronize()


def test_batch_edge_cases(P):
    from paper_2009_12617_amd._lib import SpmeError
    box = np.diag([20.0] * 3)
    empty = P.Plan(32, 4, 0.35, max_atoms=10)
    fe, ee = empty.bind(dev(np.zeros((0, 3))), dev(np.zeros(0)), box)
    pos, q, _ = I.random_neutral(1500, 20.0, 2)
    one = P.Plan(32, 4, 0.35, max_atoms=1500)
    f1, e1 = one.bind(dev(pos), dev(q), box)
    P.Batch([empty, one]).run()
    torch.cuda.synchronize()
    assert torch.count_nonzero(ee) == 0
    fa, ea = one.step(dev(pos), dev(q), box)
    assert torch.equal(fa, f1) and torch.equal(ea, e1)
    unbound = P.Plan(32, 4, 0.35, max_atoms=10)
    with pytest.raises(RuntimeError):
        P.Batch([unbound])


def test_batch_with_general_cells(P):
    # sheared copies of mix members run in the same launches as the cubic
    # ones; each result equals its own step and the oracle's
    mix = small_mix(n=6, seed=43)
    sys = make_systems(P, mix)
    sheared = []
    for m in mix[:3]:
        pos, q, box = m.make()
        L = box[0, 0]
        cell = np.array([[L, 0.0, 0.0], [0.2 * L, L, 0.0], [-0.1 * L, 0.15 * L, L]])
        plan = P.Plan(m.K, 4, 0.34, max_atoms=len(q))
        dp, dq = dev(pos), dev(q)
        f, e = plan.bind(dp, dq, cell)
        sheared.append(dict(m=m, pos=pos, q=q, box=cell, plan=plan, dp=dp, dq=dq, f=f, e=e))
    allsys = sys + sheared
    P.Batch([s["plan"] for s in allsys]).run()
    torch.cuda.synchronize()
    got = [(s["f"].clone(), s["e"].clone()) for s in allsys]
    for s, (fb, eb) in zip(allsys, got):
        fa, ea = s["plan"].step(s["dp"], s["dq"], s["box"])
        assert torch.equal(fa, fb) and torch.equal(ea, eb)
    for s, (fb, eb) in zip(sheared, got[len(sys):]):
        ref = oracle.spme(s["pos"], s["q"], s["box"], s["m"].K, 4, 0.34)
        fr = np.linalg.norm(fb.cpu().numpy() - ref["forces"]) / np.linalg.norm(ref["forces"])
        er = abs(eb[0].item() - ref["E"]) / abs(ref["E"])
        assert fr <= 1e-5 and er <= 1e-6


@pytest.mark.parametrize("precision", ["fp32_fixed", "fp64"])
def test_batch_large_grids_p6(P, precision):
    # 128^3 at p = 6 takes the split convolution and the once-per-plane
    # inverse x transform with the gather kernel; batched with a 64^3 plan,
    # each result equals its own single step
    specs = [(128, 900, 60.0, 51), (64, 700, 40.0, 52), (128, 600, 50.0, 53)]
    sys = []
    for K, nw, L, seed in specs:
        pos, q, box = I.water_box(nw, L, seed)
        plan = P.Plan(K, 6, 0.34, max_atoms=len(q), precision=precision)
        dp, dq = dev(pos), dev(q)
        f, e = plan.bind(dp, dq, box)
        sys.append(dict(plan=plan, dp=dp, dq=dq, pos=pos, q=q, box=box, K=K, f=f, e=e))
    P.Batch([s["plan"] for s in sys]).run()
    torch.cuda.synchronize()
    got = [(s["f"].clone(), s["e"].clone()) for s in sys]
    for s, (fb, eb) in zip(sys, got):
        fa, ea = s["plan"].step(s["dp"], s["dq"], s["box"])
        if precision == "fp32_fixed":
            assert torch.equal(fa, fb) and torch.equal(ea, eb)
        else:
            assert torch.allclose(fa, fb, rtol=1e-11, atol=1e-15)
            assert torch.allclose(ea, eb, rtol=1e-11, atol=1e-15)
    s = sys[0]
    ref = oracle.spme(s["pos"], s["q"], s["box"], s["K"], 6, 0.34)
    fr = np.linalg.norm(got[0][0].cpu().numpy() - ref["forces"]) / np.linalg.norm(ref["forces"])
    er = abs(got[0][1][0].item() - ref["E"]) / abs(ref["E"])
    assert fr <= (1e-5 if precision == "fp32_fixed" else 1e-10)
    assert er <= (1e-6 if precision == "fp32_fixed" else 1e-11)
