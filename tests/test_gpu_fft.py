"""Parity of the batched pencil FFT (the engine of every y/z pass) with a
brute-force DFT and a library FFT, on ragged line counts."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("lines", [1, 37, 1000])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pencils_match_library_fft(n, lines, prec):
    import torch
    import paper_2506_23712_amd as ens
    rng = np.random.default_rng(n * 1000 + lines)
    x = rng.standard_normal((n, lines)) + 1j * rng.standard_normal((n, lines))
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    xd = torch.from_numpy(x).to(dtype=dt, device="cuda")
    for sign in (-1, 1):
        got = ens.fft_pencils(xd, sign).cpu().numpy().astype(np.complex128)
        ref = np.fft.fft(x, axis=0) if sign < 0 else n * np.fft.ifft(x, axis=0)
        if prec == "fp32":
            ref32 = np.fft.fft(x.astype(np.complex64).astype(np.complex128), axis=0) if sign < 0 else \
                n * np.fft.ifft(x.astype(np.complex64).astype(np.complex128), axis=0)
            err = np.max(np.abs(got - ref32)) / np.max(np.abs(ref32))
            assert err < 2e-6 * np.log2(n), err
        else:
            err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            assert err < 4e-16 * np.log2(n) * 4, err


def test_pencils_brute_force_small_and_in_place():
    import torch
    import paper_2506_23712_amd as ens
    n, lines = 16, 5
    rng = np.random.default_rng(1)
    x = rng.standard_normal((n, lines)) + 1j * rng.standard_normal((n, lines))
    j = np.arange(n)
    ref = np.exp(-2j * np.pi * np.outer(j, j) / n) @ x
    xd = torch.from_numpy(x).cuda()
    got = ens.fft_pencils(xd, -1).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))
