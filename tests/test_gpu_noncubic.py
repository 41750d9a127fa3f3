"""GPU parity on non-cubic grids (K1, K2, K3 unequal) against the CPU oracle.

Same bars as the cubic cases: the 64-bit fixed-point charge grid is
bit-identical to the oracle's quantised mirror; FP32/fixed forces within
1e-5 relative RMS, energy 1e-6, virial 1e-6 |E|; FP64 1e-10 / 1e-11.  The
cells are orthorhombic with unequal edges (grid spacing near 0.75 A), plus
one sheared cell; 48 x 32 x 64 has three different axis lengths, so an axis
mixed up anywhere in the path shows.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2009_12617_amd import inputs as I

pytestmark = pytest.mark.gpu

F32_FORCE, F32_ENERGY, F32_VIRIAL = 1e-5, 1e-6, 1e-6
F64_FORCE, F64_ENERGY = 1e-10, 1e-11

# (name, grid (K1, K2, K3), order, edges, waters, beta)
CASES = [
    ("g32x32x64_p4", (32, 32, 64), 4, (24.0, 24.0, 48.0), 700, 0.36),
    ("g32x32x64_p6", (32, 32, 64), 6, (24.0, 24.0, 48.0), 700, 0.36),
    ("g48x32x64_p4", (48, 32, 64), 4, (36.0, 24.0, 48.0), 1100, 0.36),
    ("g48x32x64_p6", (48, 32, 64), 6, (36.0, 24.0, 48.0), 1100, 0.36),
    ("g64x64x128_p4", (64, 64, 128), 4, (44.0, 44.0, 88.0), 4000, 0.34),
    ("g64x64x128_p6", (64, 64, 128), 6, (44.0, 44.0, 88.0), 4000, 0.34),
]
IDS = [c[0] for c in CASES]


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2009_12617_amd as pkg
    return pkg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def rel_rms(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def system(name, edges, nw, seed=23):
    # a cubic water box stretched along y and z to the cell's edges
    L0 = float(edges[0])
    pos, q, _ = I.water_box(nw, L0, seed + sum(map(ord, name)))
    return pos * (np.asarray(edges) / L0), q, np.diag(edges)


def compare(res, ref, ftol, etol, vtol):
    forces, ev = res
    f = forces.cpu().numpy()
    e = ev.cpu().numpy()
    fr = rel_rms(f, ref["forces"])
    er = abs(e[0] - ref["E"]) / abs(ref["E"])
    vr = float(np.abs(e[1:] - ref["virial"]).max() / abs(ref["E"]))
    print(f"force_rel_rms={fr:.3e} energy_rel={er:.3e} virial_rel={vr:.3e}", flush=True)
    assert fr <= ftol
    assert er <= etol
    assert vr <= vtol


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_grid_bit_exact_and_step_fp32_fixed(P, case):
    name, K, p, edges, nw, beta = case
    pos, q, box = system(name, edges, nw)
    pos[::5] += np.asarray(edges) * np.array([-1.0, 2.0, 1.0])  # wrapped atoms
    plan = P.Plan(K, p, beta, max_atoms=len(q))
    plan.set_debug(True)
    res = plan.step(dev(pos), dev(q), box)
    got = plan.debug_grid(0).cpu().numpy()
    ref_grid, ref32 = oracle.mirror_grid(pos, q, box, K, p)
    assert got.shape == (K[2], K[1], K[0])
    assert np.array_equal(got, ref_grid), f"{int((got != ref_grid).sum())} grid points differ"
    ref = oracle.spme(pos, q, box, K, p, beta, want_grids=True)
    compare(res, ref, F32_FORCE, F32_ENERGY, F32_VIRIAL)
    phi = plan.debug_grid(2).cpu().numpy()
    assert rel_rms(phi, ref["phi"]) <= 1e-5


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_step_fp64(P, case):
    name, K, p, edges, nw, beta = case
    pos, q, box = system(name, edges, nw)
    plan = P.Plan(K, p, beta, max_atoms=len(q), precision="fp64")
    plan.set_debug(True)
    res = plan.step(dev(pos), dev(q), box)
    ref = oracle.spme(pos, q, box, K, p, beta, want_grids=True)
    compare(res, ref, F64_FORCE, F64_ENERGY, 1e-11)
    assert np.abs(plan.debug_grid(0).cpu().numpy() - ref["Q"]).max() < 1e-13


def test_x_pass_spectrum_layout(P):
    name, K, p, edges, nw, beta = CASES[2]
    pos, q, box = system(name, edges, nw)
    plan = P.Plan(K, p, beta, max_atoms=len(q))
    plan.spread(dev(pos), dev(q), box)
    _, ref32 = oracle.mirror_grid(pos, q, box, K, p)
    spec = plan.debug_grid(1).cpu().numpy().astype(np.complex128)
    want = np.fft.rfft(ref32.astype(np.float64), axis=2).transpose(2, 0, 1)  # [x', z, y]
    assert spec.shape == want.shape == (K[0] // 2 + 1, K[2], K[1])
    assert np.abs(spec - want).max() / np.abs(want).max() < 2e-6


@pytest.mark.parametrize("precision,bars", [("fp32_fixed_half", (1e-3, 2e-4, 2e-4)),
                                            ("fp32_fixed_bf16", (8e-3, 4e-3, 4e-3))])
def test_half_spectrum(P, precision, bars):
    # 64 x 64 x 128 splits the convolution over three launches (full-precision
    # intermediate between them); bfloat16 rounds at 2^-8, eight times binary16
    name, K, p, edges, nw, beta = CASES[4]
    pos, q, box = system(name, edges, nw)
    plan = P.Plan(K, p, beta, max_atoms=len(q), precision=precision)
    res = plan.step(dev(pos), dev(q), box)
    compare(res, oracle.spme(pos, q, box, K, p, beta), *bars)


@pytest.mark.parametrize("precision", ["fp32_fixed", "fp64"])
def test_sheared_cell_non_cubic_grid(P, precision):
    cell = np.array([[36.0, 0.0, 0.0], [5.0, 24.0, 0.0], [-6.0, 4.0, 48.0]])
    pos, q, _ = I.water_box(1100, 36.0, 71)
    pos = (pos / 36.0) @ cell  # the cube's fractional coordinates in the sheared cell
    K, p, beta = (48, 32, 64), 6, 0.36
    plan = P.Plan(K, p, beta, max_atoms=len(q), precision=precision)
    plan.set_debug(True)
    res = plan.step(dev(pos), dev(q), cell)
    ref = oracle.spme(pos, q, cell, K, p, beta)
    if precision == "fp32_fixed":
        assert np.array_equal(plan.debug_grid(0).cpu().numpy(),
                              oracle.mirror_grid(pos, q, cell, K, p)[0])
        compare(res, ref, F32_FORCE, F32_ENERGY, F32_VIRIAL)
    else:
        compare(res, ref, F64_FORCE, F64_ENERGY, F64_ENERGY)


def test_batch_mixes_grid_shapes(P):
    # one batch with cubic and non-cubic plans: grouped by shape, each
    # system's result equals its own single-plan step
    # (64 x 64 x 128 takes the three-launch convolution)
    shapes = [(CASES[0], 32), (CASES[2], None), (CASES[4], None), (CASES[0], None),
              (CASES[2], 48), (CASES[4], None)]
    plans, inputs_, outs = [], [], []
    for i, (case, cubic) in enumerate(shapes):
        name, K, p, edges, nw, beta = case
        if cubic is not None:
            K, edges = cubic, (cubic * 0.75,) * 3
        pos, q, box = system(f"{name}{i}", edges, nw // 2)
        plan = P.Plan(K, 4, beta, max_atoms=len(q))
        f = torch.empty((len(q), 3), dtype=torch.float64, device="cuda")
        ev = torch.empty(7, dtype=torch.float64, device="cuda")
        plan.bind(dev(pos), dev(q), box, forces=f, ev=ev)
        plans.append(plan)
        inputs_.append((pos, q, box, K, beta))
        outs.append((f, ev))
    P.Batch(plans).run()
    torch.cuda.synchronize()
    for (pos, q, box, K, beta), (f, ev) in zip(inputs_, outs):
        compare((f, ev), oracle.spme(pos, q, box, K, 4, beta), F32_FORCE, F32_ENERGY, F32_VIRIAL)
