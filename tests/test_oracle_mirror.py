"""Pins for the oracle's quantised mirror of the 64-bit fixed-point charge grid.

The fixed-point grid is an implementation choice (order-free, hence
deterministic, accumulation); the mirror restates its arithmetic recipe in
plain C.  Its exact rounding sequence is a contract shared with the GPU path,
so it is pinned here against the FP64 method within the rounding it is
allowed, and by invariants that hold bit for bit.
"""
import numpy as np
import pytest

from paper_2009_12617_amd import inputs


@pytest.mark.parametrize("p", [4, 6])
def test_single_precision_recursion_tracks_fp64_splines(orc, p):
    rng = np.random.default_rng(p)
    ws = np.concatenate([[0.0, 0.5, 1.0 - 2 ** -24, 1.0], rng.uniform(0, 1, 200)])
    for w in ws:
        w32 = np.float32(w)
        th, dth = orc.mirror_spline(p, w32)
        th64, dth64 = orc.bspline(p, float(w32))
        np.testing.assert_allclose(th, th64, atol=4e-7)
        np.testing.assert_allclose(dth, dth64, atol=8e-7)
        assert abs(float(th.astype(np.float64).sum()) - 1.0) < 6e-7


def test_mirror_grid_tracks_fp64_grid_and_charge_sum(orc):
    pos, q, box = inputs.water_box(200, 14.0, 7)
    for K, p in [(16, 4), (24, 6), (32, 4)]:
        Qi, Qf = orc.mirror_grid(pos, q, box, K, p)
        Q64 = orc.spme(pos, q, box, K, p, 0.35, want_grids=True)["Q"]
        np.testing.assert_allclose(Qf, Q64, atol=2e-6)
        # sum of the fixed-point grid = sum of the quantised contributions,
        # each within 2^-33 of q*theta*theta*theta (FP32 rounding aside)
        tot = int(Qi.sum()) * 2.0 ** -32
        assert tot == pytest.approx(q.sum(), abs=len(q) * p ** 3 * 1e-7)
        np.testing.assert_array_equal(Qf, (Qi.astype(np.float64) * 2.0 ** -32).astype(np.float32))


def test_mirror_grid_general_cell(orc):
    # a sheared cell: the mirror's fractional coordinates come from the same
    # reciprocal vectors as the FP64 step, so its grid tracks the FP64 grid
    pos, q, box = inputs.water_box(200, 14.0, 9)
    box = np.array([[14.0, 0.0, 0.0], [3.5, 13.0, 0.0], [-2.0, 4.0, 12.5]])
    for K, p in [(16, 4), (32, 6)]:
        Qi, Qf = orc.mirror_grid(pos, q, box, K, p)
        Q64 = orc.spme(pos, q, box, K, p, 0.35, want_grids=True)["Q"]
        np.testing.assert_allclose(Qf, Q64, atol=2e-6)
        tot = int(Qi.sum()) * 2.0 ** -32
        assert tot == pytest.approx(q.sum(), abs=len(q) * p ** 3 * 1e-7)
    # a diagonal box written as a general cell with one tiny shear moves the
    # grid by no more than the shear does
    box2 = np.diag([14.0, 14.0, 14.0])
    a, _ = orc.mirror_grid(pos, q, box2, 16, 4)
    box3 = box2.copy()
    box3[1, 0] = 1e-12
    b, _ = orc.mirror_grid(pos, q, box3, 16, 4)
    assert np.abs(a - b).max() * 2.0 ** -32 < 1e-6


def test_mirror_grid_is_order_free(orc):
    pos, q, box = inputs.water_box(300, 15.0, 8)
    perm = np.random.default_rng(1).permutation(len(q))
    a, _ = orc.mirror_grid(pos, q, box, 16, 4)
    b, _ = orc.mirror_grid(pos[perm], q[perm], box, 16, 4)
    np.testing.assert_array_equal(a, b)


def test_mirror_wrap_edges(orc):
    box = np.diag([16.0, 16.0, 16.0])
    q = np.array([1.0])
    # a tiny negative coordinate wraps to s = 1.0, i.e. exactly grid point 0
    a, _ = orc.mirror_grid(np.array([[-1e-300, 3.0, 5.0]]), q, box, 16, 4)
    b, _ = orc.mirror_grid(np.array([[0.0, 3.0, 5.0]]), q, box, 16, 4)
    np.testing.assert_array_equal(a, b)
    # a fraction that rounds to 1.0f in single precision still spreads unit charge
    x = 3.0 + (1.0 - 1e-9)
    Qi, _ = orc.mirror_grid(np.array([[x, 3.25, 5.5]]), q, box, 16, 4)
    assert abs(int(Qi.sum()) * 2.0 ** -32 - 1.0) < 64 * 2.0 ** -32 + 2e-7


def test_mirror_frac_bits_and_nonfinite(orc):
    pos, q, box = inputs.water_box(50, 10.0, 9)
    Qa, _ = orc.mirror_grid(pos, q, box, 16, 4, frac_bits=32)
    Qb, _ = orc.mirror_grid(pos, q, box, 16, 4, frac_bits=20)
    np.testing.assert_allclose(Qb * 2.0 ** -20, Qa * 2.0 ** -32, atol=64 * 2.0 ** -20)
    bad = pos.copy()
    bad[4, 1] = np.nan
    with pytest.raises(ValueError):
        orc.mirror_grid(bad, q, box, 16, 4)
    Qn, _ = orc.mirror_grid(bad, q, box, 16, 4, allow_nonfinite=True)
    keep = np.ones(len(q), bool)
    keep[4] = False
    Qk, _ = orc.mirror_grid(pos[keep], q[keep], box, 16, 4)
    np.testing.assert_array_equal(Qn, Qk)
