"""pme_step_probe (steps that launch one kernel a second time, for timing by
difference) leaves the step's forces, energy and virial bit-identical to
pme_step, and the step after it is unaffected -- also under graph replay."""
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


@pytest.mark.parametrize("K,n", [(32, 1365), (64, 6000)])
def test_probe_steps_leave_results_unchanged(P, K, n):
    from paper_2009_12617_amd.plan import PROBE
    pos, q, box = I.water_box(n, 0.8 * K, 90 + K)
    dp = torch.from_numpy(pos).cuda()
    dp2 = torch.from_numpy(pos + 0.05).cuda()
    dq = torch.from_numpy(q).cuda()
    plan = P.Plan(K, 4, 0.34, max_atoms=len(q))
    f0, e0 = (t.clone() for t in plan.step(dp, dq, box))
    f1, e1 = (t.clone() for t in plan.step(dp2, dq, box))
    f = torch.empty_like(f0)
    e = torch.empty_like(e0)
    for name, code in PROBE.items():
        plan.step_probe(dp, dq, box, f, e, code)
        torch.cuda.synchronize()
        assert torch.equal(f, f0) and torch.equal(e, e0), name
        ff, ee = plan.step(dp2, dq, box)  # the next step is unaffected
        assert torch.equal(ff, f1) and torch.equal(ee, e1), name
    # graph replay of alternating probe steps
    g = torch.cuda.CUDAGraph()
    fa, ea = torch.empty_like(f0), torch.empty_like(e0)
    fb, eb = torch.empty_like(f0), torch.empty_like(e0)
    with torch.cuda.graph(g, stream=torch.cuda.Stream()):
        plan.set_stream(torch.cuda.current_stream())
        for code in PROBE.values():
            plan.step_probe(dp, dq, box, fa, ea, code)
            plan.step_probe(dp2, dq, box, fb, eb, code)
    plan.set_stream(torch.cuda.current_stream())
    for _ in range(2):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(fa, f0) and torch.equal(ea, e0)
        assert torch.equal(fb, f1) and torch.equal(eb, e1)
    assert plan.check() == 0
