"""Batch admission through the C ABI (pme_batch_*): systems admitted into one
arena by footprint, their buffers carved from it, one launch over any set of
slots with grid groups on forked streams; every result bit-identical to the
system's own single step, under graph replay too; retire and re-admit reuse
arena ranges; a full arena answers PME_EBUSY; admission takes the split
interpolation on grids without register x transforms.  Also: pme_bind is
stream-ordered (a rebind does not disturb a batched run enqueued before
it)."""
import numpy as np
import pytest
import torch

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


def single(P, m, pos, q, box, tuning=None):
    plan = P.Plan(m.K, 4, 0.34, max_atoms=len(q))
    if tuning is not None:
        plan.set_tuning(**tuning)
    f, e = plan.step(dev(pos), dev(q), box)
    torch.cuda.synchronize()
    return f.clone(), e.clone()


def admit_all(P, pool, mix):
    slots = []
    for m in mix:
        pos, q, box = m.make()
        s = pool.admit(m.K, 4, 0.34, box, len(q))
        assert s is not None
        p, qq, f, e = pool.io(s)
        p.copy_(dev(pos))
        qq.copy_(dev(q))
        slots.append((s, m, pos, q, box))
    return slots


def test_pool_matches_single_steps_and_graph(P):
    mix = I.batch_mix(n_systems=10, seed=41, lo=600, hi=20000)
    assert len({m.K for m in mix}) == 3  # three grid groups on the fork streams
    stream = torch.cuda.Stream()
    pool = P.BatchPool(1 << 30, max_systems=16, stream=stream)
    with torch.cuda.stream(stream):
        slots = admit_all(P, pool, mix)
    st = pool.stats()
    assert st["admitted"] == len(mix) and st["bytes_used"] == sum(
        P.BatchPool.footprint(m.K, 4, len(q)) for _, m, _, q, _ in slots)
    # admission's variants: the single plan's, with the split interpolation
    # where the x rows have no register transform
    for s, m, *_ in slots:
        t = pool.tuning_of(s)
        assert t["interp"] == (0 if m.K == 64 else 1), (m.K, t)
    refs = [single(P, m, pos, q, box, pool.tuning_of(s)) for s, m, pos, q, box in slots]
    pool.launch()
    stream.synchronize()
    for (s, m, *_), (fr, er) in zip(slots, refs):
        _, _, f, e = pool.io(s)
        assert torch.equal(f, fr) and torch.equal(e, er), m.index
    # a subset of the slots, in another order
    sub = [slots[k][0] for k in (7, 2, 5)]
    for s in sub:
        pool.io(s)[2].zero_()
    torch.cuda.synchronize()
    pool.launch(sub)
    stream.synchronize()
    for k in (7, 2, 5):
        assert torch.equal(pool.io(slots[k][0])[2], refs[k][0])
    # graph capture of a launch (fork/join over the grid groups), replayed
    # with eager work in between; every replay equals the single steps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        pool.launch()
    for rep in range(3):
        for s, *_ in slots:
            pool.io(s)[2].fill_(float(rep))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (s, m, *_), (fr, er) in zip(slots, refs):
            _, _, f, e = pool.io(s)
            assert torch.equal(f, fr) and torch.equal(e, er), (rep, m.index)
    with pytest.raises(RuntimeError):
        pool.launch([slots[0][0], slots[0][0]])  # a slot twice
    pool.close()


def test_pool_busy_retire_readmit(P):
    mix = I.batch_mix(n_systems=6, seed=5, lo=800, hi=5000)  # six 32^3 systems
    fps = [P.BatchPool.footprint(m.K, 4, m.n_waters * 3) for m in mix]
    arena = sum(fps[:3]) + 512
    stream = torch.cuda.Stream()
    pool = P.BatchPool(arena, max_systems=8, stream=stream)
    with torch.cuda.stream(stream):
        first = admit_all(P, pool, mix[:3])
        m = mix[3]
        pos, q, box = m.make()
        if fps[3] > pool.stats()["largest_free"]:
            assert pool.admit(m.K, 4, 0.34, box, len(q)) is None   # PME_EBUSY
        # retire the middle system; an equal-sized one fits its range again
        s_mid, m_mid, pos_mid, q_mid, box_mid = first[1]
        pool.retire(s_mid)
        assert pool.stats()["admitted"] == 2
        s_new = pool.admit(m_mid.K, 4, 0.34, box_mid, len(q_mid))
        assert s_new is not None
        p, qq, _, _ = pool.io(s_new)
        p.copy_(dev(pos_mid))
        qq.copy_(dev(q_mid))
        pool.launch()
    stream.synchronize()
    fr, er = single(P, m_mid, pos_mid, q_mid, box_mid, pool.tuning_of(s_new))
    assert torch.equal(pool.io(s_new)[2], fr) and torch.equal(pool.io(s_new)[3], er)
    for s, mm, pos_, q_, box_ in (first[0], first[2]):
        f2, e2 = single(P, mm, pos_, q_, box_, pool.tuning_of(s))
        assert torch.equal(pool.io(s)[2], f2) and torch.equal(pool.io(s)[3], e2)
    # update: fewer atoms and a new box through the carved buffers
    s0, m0, pos0, q0, box0 = first[0]
    n = len(q0) - 3
    with torch.cuda.stream(stream):
        pool.update(s0, n, box0 * 1.01)
        pool.launch([s0])
    stream.synchronize()
    f3, e3 = single(P, m0, pos0[:n], q0[:n], box0 * 1.01, pool.tuning_of(s0))
    assert torch.equal(pool.io(s0)[2][:n], f3) and torch.equal(pool.io(s0)[3], e3)
    assert pool.check(s0) == 0
    pool.close()


def test_bind_is_stream_ordered(P):
    """Two bindings of one plan enqueued back to back on its stream, each
    followed by a batched run: each run sees its own binding."""
    m = I.batch_mix(n_systems=1, seed=3, lo=2000, hi=2001)[0]
    pos, q, box = m.make()
    pos2 = pos + 0.37
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(m.K, 4, 0.34, max_atoms=len(q), stream=stream)
        dp, dp2, dq = dev(pos), dev(pos2), dev(q)
        fa = torch.empty((len(q), 3), dtype=torch.float64, device="cuda")
        fb = torch.empty_like(fa)
        plan.bind(dp, dq, box, forces=fa)
        P.Batch([plan]).run(stream)
        plan.bind(dp2, dq, box, forces=fb)
        P.Batch([plan]).run(stream)
    stream.synchronize()
    ra, _ = single(P, m, pos, q, box)
    rb, _ = single(P, m, pos2, q, box)
    assert torch.equal(fa, ra) and torch.equal(fb, rb)


def test_pool_autotune_keeps_results(P):
    # variants per grid group chosen on the batch: never slower than where it
    # started (within timing noise), results still equal single steps run
    # with the chosen variants
    mix = I.batch_mix(n_systems=10, seed=41, lo=600, hi=20000)
    stream = torch.cuda.Stream()
    pool = P.BatchPool(1 << 30, max_systems=16, stream=stream)
    with torch.cuda.stream(stream):
        slots = admit_all(P, pool, mix)
    stream.synchronize()
    r = pool.autotune(launches=3)
    print(r, flush=True)
    assert r["us"] <= r["default_us"] * 1.05
    assert set(r["groups"]) == {f"{m.K}x{m.K}x{m.K}" for m in mix}
    for s, *_ in slots:
        pool.io(s)[2].fill_(float("nan"))
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        pool.launch()
    stream.synchronize()
    for s, m, pos, q, box in slots:
        plan = P.Plan(m.K, 4, 0.34, max_atoms=len(q))
        plan.set_tuning(**pool.tuning_of(s))
        f, e = plan.step(dev(pos), dev(q), box)
        torch.cuda.synchronize()
        assert torch.equal(pool.io(s)[2], f) and torch.equal(pool.io(s)[3], e), m.index
    pool.close()


def test_pool_mixed_binning_chunks_in_one_grid(P):
    # systems of one grid shape with different binning chunks form separate
    # groups (each group bins with one chunk size on its fork stream); every
    # result equals the system's own single step with that chunk
    mix = [m for m in I.batch_mix(n_systems=12, seed=41, lo=600, hi=20000) if m.K == 32][:4]
    assert len(mix) >= 3
    stream = torch.cuda.Stream()
    pool = P.BatchPool(1 << 30, max_systems=8, stream=stream)
    with torch.cuda.stream(stream):
        slots = admit_all(P, pool, mix)
    chunks = [256, 1024, 512, 1024][: len(slots)]
    refs = []
    for (s, m, pos, q, box), c in zip(slots, chunks):
        pool.set_tuning(s, bin_chunk=c)
        plan = P.Plan(m.K, 4, 0.34, max_atoms=len(q))
        plan.set_tuning(**pool.tuning_of(s))
        f, e = plan.step(dev(pos), dev(q), box)
        torch.cuda.synchronize()
        refs.append((f.clone(), e.clone()))
    pool.launch()
    stream.synchronize()
    for (s, m, *_), (fr, er) in zip(slots, refs):
        _, _, f, e = pool.io(s)
        assert torch.equal(f, fr) and torch.equal(e, er), m.index
    pool.close()


def test_pool_admission_variants_match_the_oracle(P):
    # one system of each grid group, in the variants admission picked (the
    # split interpolation on 32^3 and 48^3), against the FP64 oracle at the
    # FP32/fixed bars: force relative RMS, the worst component (extreme-value
    # factor of 3N independent errors), energy and virial
    import oracle
    mix = I.batch_mix(n_systems=12, seed=41, lo=600, hi=20000)
    pick = {}
    for m in mix:
        pick.setdefault(m.K, m)
    assert set(pick) == {32, 48, 64}
    stream = torch.cuda.Stream()
    pool = P.BatchPool(1 << 30, max_systems=4, stream=stream)
    with torch.cuda.stream(stream):
        slots = admit_all(P, pool, [pick[k] for k in (32, 48, 64)])
    pool.launch()
    stream.synchronize()
    for s, m, pos, q, box in slots:
        assert pool.tuning_of(s)["interp"] == (0 if m.K == 64 else 1)
        ref = oracle.spme(pos, q, box, m.K, 4, 0.34)
        _, _, f, e = pool.io(s)
        f, e = f.cpu().numpy(), e.cpu().numpy()
        rms = np.sqrt(np.mean(ref["forces"] ** 2))
        fr = np.linalg.norm(f - ref["forces"]) / np.linalg.norm(ref["forces"])
        worst = np.abs(f - ref["forces"]).max() / rms
        er = abs(e[0] - ref["E"]) / abs(ref["E"])
        vr = np.abs(e[1:] - ref["virial"]).max() / abs(ref["E"])
        print(f"K={m.K} atoms={len(q)} force {fr:.2e} worst {worst:.2e} energy {er:.2e} "
              f"virial {vr:.2e}", flush=True)
        assert fr <= 1e-5
        assert worst <= 1e-5 * np.sqrt(2.0 * np.log(3.0 * len(q)))
        assert er <= 1e-6 and vr <= 2e-6
    pool.close()
