"""GPU real-space Ewald term (pme_real) against the CPU oracle's brute-force
real-space sum, self term and exclusion correction, and the full Ewald
energy of a rock-salt lattice on the GPU against the Madelung constant."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2009_12617_amd import inputs as I

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "constants.json")))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2009_12617_amd as P
    from paper_2009_12617_amd import _lib
    _lib.load()
    return P


def dev(a, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda")


def rel_rms(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("max_cells", [1 << 15, 27])
@pytest.mark.parametrize("with_excl", [False, True])
def test_real_space_matches_brute_force(P, with_excl, max_cells):
    # 400 waters in a 24 A box, rcut 7.9 A (three cells per axis, or the
    # coarsest grid when max_cells = 27), beta 0.35
    pos, q, box = I.water_box(400, 24.0, 31)
    pos[::5] += np.array([24.0, -48.0, 72.0])  # other images
    beta, rcut, c = 0.35, 7.9, 332.0637
    rs = P.RealSpace(len(q), max_cells=max_cells)
    excl = None
    if with_excl:
        off, idx = I.water_exclusions(len(q))
        excl = (dev(off, np.int32), dev(idx, np.int32))
    f, e = rs(dev(pos), dev(q), box, beta, rcut, exclusions=excl, coulomb=c)
    f, e = f.cpu().numpy(), e.cpu().numpy()
    # the brute-force sum reaches images |n| <= 1 only, so it is given the
    # positions wrapped into the cell (the sum is periodic in each position)
    wrapped = np.mod(pos, 24.0)
    ref = oracle.ewald_real(wrapped, q, box, beta, nimg=1, rcut=rcut, coulomb=c)
    want_f = ref["forces"].copy()
    want_excl = 0.0
    if with_excl:
        ex = oracle.ewald_excl(pos, q, box, beta, off, idx, rcut=rcut, coulomb=c)
        want_f += ex["forces"]
        want_excl = ex["E_excl"]
    print(f"force_rel_rms={rel_rms(f, want_f):.2e} E_real={e[0]:.10f} ref={ref['E_real']:.10f}", flush=True)
    assert rel_rms(f, want_f) <= 1e-11
    assert e[0] == pytest.approx(ref["E_real"], rel=1e-12)
    assert e[1] == pytest.approx(ref["E_self"], rel=1e-13)
    assert e[2] == pytest.approx(want_excl, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("edge,rcut", [(36.0, 6.0), (45.0, 7.5)])
def test_real_space_dense_cells(P, edge, rcut):
    # water density in a box whose 27-cell limit coarsens the cell grid to
    # 3 x 3 x 3 cells of 12 A (about 170 atoms per cell: the 2-lane split of
    # a home atom's candidates) and of 15 A (about 340 atoms per cell: more
    # than 64 home atoms per pair workgroup, so its multi-pass loop runs),
    # with the water exclusions, against the brute-force oracle
    nw = int(round(edge ** 3 * I.WATER_DENSITY))
    pos, q, box = I.water_box(nw, edge, 36)
    beta = 0.34
    rs = P.RealSpace(len(q), max_cells=27)
    off, idx = I.water_exclusions(len(q))
    f, e = rs(dev(pos), dev(q), box, beta, rcut, exclusions=(dev(off, np.int32), dev(idx, np.int32)))
    f, e = f.cpu().numpy(), e.cpu().numpy()
    w = np.mod(pos, edge)
    ref = oracle.ewald_real(w, q, box, beta, nimg=1, rcut=rcut)
    ex = oracle.ewald_excl(pos, q, box, beta, off, idx, rcut=rcut)
    want = ref["forces"] + ex["forces"]
    print(f"{len(q)} atoms, {len(q) / 27:.0f} per cell: force_rel_rms={rel_rms(f, want):.2e}", flush=True)
    assert rel_rms(f, want) <= 1e-11
    assert e[0] == pytest.approx(ref["E_real"], rel=1e-12)
    assert e[2] == pytest.approx(ex["E_excl"], rel=1e-12)


def test_real_space_rejects_bad_buffers(P):
    pos, q, box = I.water_box(50, 12.0, 37)
    rs = P.RealSpace(len(q))
    dp, dq = dev(pos), dev(q)
    with pytest.raises(TypeError):
        rs(torch.from_numpy(pos), dq, box, 0.4, 3.9)                   # host tensor
    with pytest.raises(ValueError):
        rs(dp[:-1], dq, box, 0.4, 3.9)                                 # short positions
    with pytest.raises(TypeError):
        rs(dp, dq, box, 0.4, 3.9, forces=torch.zeros((len(q), 3), device="cuda"))  # float32
    with pytest.raises(ValueError):
        rs(dp, dq, box, 0.4, 3.9, forces=torch.zeros((len(q) - 1, 3), dtype=torch.float64,
                                                      device="cuda"))
    off, idx = I.water_exclusions(len(q))
    with pytest.raises(TypeError):
        rs(dp, dq, box, 0.4, 3.9, exclusions=(dev(off, np.int64), dev(idx, np.int32)))
    with pytest.raises(ValueError):
        rs(dp, dq, box, 0.4, 3.9, exclusions=(dev(off, np.int32), dev(idx[:-2], np.int32)))
    big = P.RealSpace(10)
    with pytest.raises(ValueError):
        big(dp, dq, box, 0.4, 3.9)


@pytest.mark.parametrize("beta", [0.05, 0.755])
def test_real_space_screening_range(P, beta):
    # the erfc inside the cutoff comes from a Chebyshev series on
    # [0, beta rcut]: the two ends of the supported range of beta rcut
    # (0.4 and 5.96) against the oracle's brute-force sum; just past the
    # range (6.04) the call is refused
    from paper_2009_12617_amd._lib import SpmeError
    pos, q, box = I.water_box(400, 24.0, 34)
    rcut = 7.9
    rs = P.RealSpace(len(q))
    f, e = rs(dev(pos), dev(q), box, beta, rcut)
    f, e = f.cpu().numpy(), e.cpu().numpy()
    ref = oracle.ewald_real(np.mod(pos, 24.0), q, box, beta, nimg=1, rcut=rcut)
    print(f"beta*rcut={beta * rcut:.3f} force_rel_rms={rel_rms(f, ref['forces']):.2e} "
          f"E_real={e[0]:.12e} ref={ref['E_real']:.12e}", flush=True)
    assert rel_rms(f, ref["forces"]) <= 1e-11
    assert e[0] == pytest.approx(ref["E_real"], rel=1e-12)
    with pytest.raises(SpmeError) as ei:
        rs(dev(pos), dev(q), box, 6.04 / rcut, rcut)
    assert ei.value.code == 2


def test_coincident_atoms_are_not_paired(P):
    # atom B placed exactly on atom A (another water's oxygen): the pair
    # (A, B) is skipped, every other pair counts.  The oracle cannot take
    # the system whole (its A-B term is infinite), so the expected values
    # are combined from three systems it can take: without B, without A,
    # and without both (each pair term appears in exactly one of them with
    # the right sign)
    pos, q, box = I.water_box(300, 22.0, 35)
    A, B = 0, 3 * 150
    pos = pos.copy()
    pos[B] = pos[A]
    beta, rcut = 0.4, 7.0
    rs = P.RealSpace(len(q))
    f, e = rs(dev(pos), dev(q), box, beta, rcut)
    f, e = f.cpu().numpy(), e.cpu().numpy()
    keep = np.ones(len(q), bool)
    w = np.mod(pos, 22.0)

    def part(drop):
        m = keep.copy()
        m[list(drop)] = False
        r = oracle.ewald_real(w[m], q[m], box, beta, nimg=1, rcut=rcut)
        full = np.zeros_like(pos)
        full[m] = r["forces"]
        return full, r["E_real"]
    f_nb, e_nb = part([B])
    f_na, e_na = part([A])
    f_no, e_no = part([A, B])
    want_f = f_nb + f_na - f_no
    want_e = e_nb + e_na - e_no
    print(f"force_rel_rms={rel_rms(f, want_f):.2e} E_real={e[0]:.10f} ref={want_e:.10f}", flush=True)
    assert np.all(np.isfinite(f)) and np.isfinite(e[0])
    assert rel_rms(f, want_f) <= 1e-11
    assert e[0] == pytest.approx(want_e, rel=1e-11)


def test_real_space_accumulates_and_rejects_bad_geometry(P):
    from paper_2009_12617_amd._lib import SpmeError
    pos, q, box = I.water_box(100, 16.0, 32)
    rs = P.RealSpace(len(q))
    f0, _ = rs(dev(pos), dev(q), box, 0.4, 5.0)
    f1 = torch.ones_like(f0)
    rs(dev(pos), dev(q), box, 0.4, 5.0, forces=f1, accumulate=True)
    assert torch.allclose(f1, f0 + 1.0, rtol=0, atol=1e-12)
    with pytest.raises(SpmeError) as ei:
        rs(dev(pos), dev(q), box, 0.4, 6.0)  # rcut > L/3
    assert ei.value.code == 2
    sheared = box.copy()
    sheared[1, 0] = 1.0
    with pytest.raises(SpmeError) as ei:
        rs(dev(pos), dev(q), sheared, 0.4, 5.0)
    assert ei.value.code == 2


@pytest.mark.parametrize("offset", [(0.0, 0.0, 0.0), (0.37, 1.13, 2.71)])
def test_madelung_constant_on_gpu(P, offset):
    # full Ewald energy of a 4^3-ion rock-salt lattice with all
    # three terms on the GPU: reciprocal (FP64 SPME, K = 64, p = 6), real
    # space (rcut 3.7 A, beta 1.0), self
    M, r0, beta = 4, 2.8, 1.0
    pos, q, box = I.rock_salt(M, r0, offset)
    plan = P.Plan(64, 6, beta, max_atoms=len(q), precision="fp64")
    _, ev = plan.step(dev(pos), dev(q), box)
    rs = P.RealSpace(len(q))
    _, e = rs(dev(pos), dev(q), box, beta, 3.7)
    E = ev[0].item() + e[0].item() + e[1].item()
    madelung = -2.0 * E * r0 / len(q)
    g = GOLD["madelung_nacl"]
    print(f"madelung={madelung:.9f}", flush=True)
    assert abs(madelung - g["value"]) <= g["tolerance"]


def test_full_ewald_forces_with_exclusions(P):
    # complete electrostatics of 40 waters on the GPU -- reciprocal (FP64 SPME)
    # plus real space and exclusions accumulated into the same forces --
    # against the brute-force Ewald sums of the oracle (reciprocal to
    # |m| <= 14, real space with the same cutoff, exclusions)
    pos, q, box = I.water_box(40, 12.0, 33)
    off, idx = I.water_exclusions(len(q))
    beta, rcut = 0.8, 3.9
    plan = P.Plan(64, 6, beta, max_atoms=len(q), precision="fp64")
    f, ev = plan.step(dev(pos), dev(q), box)
    rs = P.RealSpace(len(q))
    _, e = rs(dev(pos), dev(q), box, beta, rcut, exclusions=(dev(off, np.int32), dev(idx, np.int32)),
              forces=f, accumulate=True)
    f = f.cpu().numpy()
    E = ev[0].item() + float(e.sum().item())
    wrapped = np.mod(pos, 12.0)
    rec = oracle.ewald_recip(pos, q, box, beta, 14)
    real = oracle.ewald_real(wrapped, q, box, beta, nimg=1, rcut=rcut)
    ex = oracle.ewald_excl(pos, q, box, beta, off, idx, rcut=rcut)
    want_f = rec["forces"] + real["forces"] + ex["forces"]
    want_E = rec["E"] + real["E_real"] + real["E_self"] + ex["E_excl"]
    print(f"force_rel_rms={rel_rms(f, want_f):.2e} E={E:.10f} ref={want_E:.10f}", flush=True)
    # the SPME approximation (K = 64, p = 6, beta 0.8 on 12 A: 1.2e-6 of the
    # reciprocal forces, 3.4e-7 of its energy in the oracle) sets the bound
    assert rel_rms(f, want_f) <= 1e-5
    # the total is a small difference of large terms: bound it by their size
    scale = abs(rec["E"]) + abs(real["E_real"]) + abs(real["E_self"]) + abs(ex["E_excl"])
    assert abs(E - want_E) <= 1e-6 * scale
