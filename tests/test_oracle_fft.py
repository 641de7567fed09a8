"""Pins of the oracle's FFT against brute-force DFTs and a library FFT."""
import numpy as np
import pytest

pytestmark = []


def brute_dft_1d(x, sign):
    n = x.size
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n) @ x


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_matches_brute_force(orc, n, sign):
    rng = np.random.default_rng(n * 7 + sign)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = brute_dft_1d(x, sign)
    got = orc.fft1d(x, sign)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [128, 256, 512, 1024])
def test_fft1d_matches_library_fft(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert np.max(np.abs(orc.fft1d(x, -1) - np.fft.fft(x))) <= 1e-13 * np.sqrt(n) * np.max(np.abs(x)) * 4
    assert np.max(np.abs(orc.fft1d(x, 1) - n * np.fft.ifft(x))) <= 1e-13 * np.sqrt(n) * np.max(np.abs(x)) * 4


def test_fft3d_matches_brute_force_8cubed(orc):
    n = 8
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    idx = np.indices((n, n, n)).reshape(3, -1)          # (z, y, x) of every point
    phase = idx.T @ idx                                 # k . r for every (k, r) pair
    for sign in (-1, 1):
        ref = (np.exp(sign * 2j * np.pi * phase / n) @ x.reshape(-1)).reshape(n, n, n)
        got = orc.fft3d(x, sign)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_fft3d_roundtrip_and_parseval(orc):
    n = 16
    rng = np.random.default_rng(11)
    x = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    X = orc.fft3d(x, -1)
    assert abs(np.sum(np.abs(X) ** 2) / n ** 3 - np.sum(np.abs(x) ** 2)) <= 1e-12 * np.sum(np.abs(x) ** 2)
    back = orc.fft3d(X, 1) / n ** 3
    assert np.max(np.abs(back - x)) <= 1e-14 * 16


def test_fft3d_single_mode_is_a_delta(orc):
    n = 16
    z, y, x = np.indices((n, n, n))
    f = np.exp(2j * np.pi * (3 * x + 5 * y - 2 * z) / n)
    X = orc.fft3d(f, -1)
    expect = np.zeros_like(X)
    expect[(-2) % n, 5, 3] = n ** 3
    assert np.max(np.abs(X - expect)) <= 1e-11
