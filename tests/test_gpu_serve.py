"""Continuous-batching serving loop: admission by HBM footprint, resident
slots reused, requests overlapping on the device, and every result the same
as the system's own single step (bit for bit on the fixed-point path)."""
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


def pool(n=6, seed=9):
    from paper_2009_12617_amd.serve import PoolSystem
    out = []
    for m in I.batch_mix(n_systems=n, seed=seed, lo=600, hi=6000):
        pos, q, box = m.make()
        out.append(PoolSystem(pos, q, box, m.K))
    return out


def reference(P, sysd):
    plan = P.Plan(sysd.K, sysd.order, sysd.beta, max_atoms=len(sysd.q))
    f, e = plan.step(torch.from_numpy(sysd.pos).cuda(), torch.from_numpy(sysd.q).cuda(), sysd.box)
    return f.cpu().numpy(), e[0].item()


def test_serving_results_admission_and_overlap(P):
    from paper_2009_12617_amd.serve import Server
    systems = pool()
    refs = [reference(P, s) for s in systems]
    rng = np.random.default_rng(0)
    n = 120
    arrivals = np.cumsum(rng.exponential(1.0 / 4000.0, size=n))
    ids = rng.integers(0, len(systems), size=n)
    # a budget for only a few resident slots forces requests to wait and reuse slots
    one = max(P.BatchPool.footprint(s.K, s.order, len(s.q)) for s in systems)
    srv = Server(systems, hbm_budget_bytes=3 * one, max_batch=8, keep_forces=True)
    done = srv.run(arrivals, ids, stall_s=20.0)
    st = srv.stats.summary()
    assert st["completed"] == n
    assert srv.stats.peak_resident_bytes <= 3 * one
    assert st["evictions"] > 0 and st["waits_for_budget"] > 0
    assert st["peak_inflight"] >= 2  # requests overlapped on the device
    for r in done:
        f, e = refs[r.system_id]
        assert r.energy == e
        assert np.array_equal(r.forces, f)
        assert r.done >= r.arrival


def test_serving_mixed_batches(P):
    from paper_2009_12617_amd.serve import Server
    systems = pool(n=5, seed=21)
    refs = [reference(P, s) for s in systems]
    # a burst: everything arrives at once, so ticks hold several systems
    n = 40
    arrivals = np.zeros(n)
    ids = np.arange(n) % len(systems)
    srv = Server(systems, hbm_budget_bytes=1 << 34, max_batch=16, slots_per_system=4,
                 keep_forces=True)
    done = srv.run(arrivals, ids, stall_s=20.0)
    assert srv.stats.summary()["max_batch"] > 1
    for r in done:
        f, e = refs[r.system_id]
        assert r.energy == e and np.array_equal(r.forces, f)
