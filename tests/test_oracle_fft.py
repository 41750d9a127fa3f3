"""Pins for the oracle's own DFT (O5/O9): the naive sum, numpy.fft, Parseval,
and inverse-of-forward.  The paper builds the 3D transform as a sequence of
1D transforms along each axis (section III.B), as the oracle does."""
import numpy as np
import pytest


def naive_dft(x, sign):
    n = len(x)
    j = np.arange(n)
    W = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
    return W @ x


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8, 12, 16, 24, 32, 48, 64, 96, 128])
@pytest.mark.parametrize("sign", [1, -1])
def test_fft1d_matches_naive_sum(orc, n, sign):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = naive_dft(x, sign)
    got = orc.fft1d(x, sign)
    np.testing.assert_allclose(got, ref, atol=1e-11 * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 16, 8), (16, 12, 24), (32, 32, 32)])
def test_fft3d_matches_numpy(orc, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    n = x.size
    fwd = orc.fft3d(x, -1)
    np.testing.assert_allclose(fwd, np.fft.fftn(x), atol=1e-10 * np.sqrt(n))
    inv = orc.fft3d(x, +1)
    np.testing.assert_allclose(inv, np.fft.ifftn(x) * n, atol=1e-10 * np.sqrt(n))
    # Parseval and inverse(forward(x)) = n x
    assert np.sum(np.abs(fwd) ** 2) == pytest.approx(n * np.sum(np.abs(x) ** 2), rel=1e-12)
    back = orc.fft3d(fwd, +1)
    np.testing.assert_allclose(back, n * x, atol=1e-9 * np.sqrt(n))
