"""Every supported grid shape x spline order x precision against the oracle.

The supported shapes are found through the library's own host-side
workspace query (no device needed to enumerate them), so a shape added to
the library is covered here without editing the test.  Each case is a small
water box whose edges give about 0.8 A grid spacing; the bars are those of
the other parity tests (FP32/fixed: bit-exact charge grid, force relative
RMS 1e-5, energy 1e-6; FP64: 1e-10 / 1e-11; binary16 spectrum: 1e-3 /
2e-4; bfloat16 spectrum: 8e-3 / 4e-3), and the FP32/fixed virial
components within 2e-6 |E|: twice the energy bar, because each component
sums the same per-mode energy terms with weights (delta_ab - 2 u m_a m_b)
whose energy-weighted mean magnitude is at most 2.
"""
import functools

import numpy as np
import pytest
import torch

import oracle
from paper_2009_12617_amd import _lib
from paper_2009_12617_amd import inputs as I

pytestmark = pytest.mark.gpu

CANDIDATES = [(k, k, k) for k in (8, 12, 16, 18, 20, 24, 27, 30, 32, 36, 40, 48, 54, 60, 64, 72,
                                  80, 96, 100, 108, 120, 128, 144)]
CANDIDATES += [(32, 32, 64), (64, 64, 128), (48, 32, 64), (64, 64, 32), (64, 32, 64),
               (128, 128, 64), (32, 48, 64)]


DOCUMENTED = [(k, k, k) for k in (16, 24, 32, 36, 48, 64, 72, 96, 128)] + [
    (32, 32, 64), (64, 64, 128), (48, 32, 64)]


def supported_shapes():
    try:
        lib = _lib.load()
    except Exception:  # collected without the built library: the documented list
        return DOCUMENTED
    return [g for g in CANDIDATES if lib.pme_workspace_bytes(*g, 4, 1000, 1) > 0]


SHAPES = supported_shapes()
# (force relative RMS, energy relative error, virial components / |E|)
BARS = {"fp32_fixed": (1e-5, 1e-6, 2e-6), "fp64": (1e-10, 1e-11, 1e-11),
        "fp32_fixed_half": (1e-3, 2e-4, 2e-4), "fp32_fixed_bf16": (8e-3, 4e-3, 4e-3)}


def test_shape_list_matches_the_documented_set():
    assert sorted(SHAPES) == sorted(DOCUMENTED)


@functools.lru_cache(maxsize=None)
def case(shape, p):
    edges = tuple(0.8 * k for k in shape)
    L0 = edges[0]
    nw = max(60, int(0.0334 * np.prod(edges) / 3 / 4))  # a quarter of water density
    pos, q, _ = I.water_box(nw, L0, 7000 + sum(shape) + p)
    pos = pos * (np.asarray(edges) / L0)
    box = np.diag(edges)
    beta = 3.2 / (0.8 * 12)  # erfc(beta * 12 * spacing) ~ 1e-5 at every shape
    ref = oracle.spme(pos, q, box, shape, p, beta)
    grid = oracle.mirror_grid(pos, q, box, shape, p)[0]
    return pos, q, box, beta, ref, grid


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2009_12617_amd as pkg
    return pkg


@pytest.mark.parametrize("precision", sorted(BARS))
@pytest.mark.parametrize("p", [4, 6])
@pytest.mark.parametrize("shape", SHAPES, ids=["x".join(map(str, g)) for g in SHAPES])
def test_every_shape_order_precision(P, shape, p, precision):
    pos, q, box, beta, ref, grid = case(shape, p)
    plan = P.Plan(shape, p, beta, max_atoms=len(q), precision=precision)
    plan.set_debug(True)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")  # noqa: E731
    f, e = plan.step(dev(pos), dev(q), box)
    if precision != "fp64":
        assert np.array_equal(plan.debug_grid(0).cpu().numpy(), grid)
    f = f.cpu().numpy()
    e = e.cpu().numpy()
    ftol, etol, vtol = BARS[precision]
    fr = float(np.linalg.norm(f - ref["forces"]) / np.linalg.norm(ref["forces"]))
    er = abs(e[0] - ref["E"]) / abs(ref["E"])
    vr = float(np.abs(e[1:] - ref["virial"]).max() / abs(ref["E"]))
    worst = float(np.abs(f - ref["forces"]).max() / np.sqrt(np.mean(ref["forces"] ** 2)))
    wbar = ftol * np.sqrt(2.0 * np.log(3.0 * len(q)))  # extreme-value bound of 3N errors
    print(f"{shape} p={p} {precision}: force {fr:.1e} worst {worst:.1e} energy {er:.1e} "
          f"virial {vr:.1e}", flush=True)
    assert fr <= ftol and er <= etol and vr <= vtol
    # the worst component, within the extreme-value factor of the RMS bar;
    # not for the 16-bit spectra, whose error is one shared rounding of the
    # spectrum rather than independent per-operation rounding
    if precision in ("fp32_fixed", "fp64"):
        assert worst <= wbar
