"""Pins of the oracle's spectral diagnostics: the shell energy spectrum (the
paper's energy-spectra figure) and spectral refinement onto a finer grid (the
section on extrapolating to the frontier, where the most intense members are
rerun at twice the resolution).  Each check is fixed by the mathematics, not
by the oracle: hand-counted shells, brute-force enumeration of the initial
field's closed-form mode energies, Parseval, and point values of the
refined field in physical space (numpy's FFT, not the oracle's)."""
import math

import numpy as np
import pytest


def field(orc, n, seed):
    return orc.init_field(n, seed, k_peak=2.0, e0=0.5)


def test_shell_boundaries_by_hand(orc):
    # |m| = 1.414 -> shell 1; 1.732 -> 2; 2.449 -> 2; 2.646 -> 3; 0 -> 0; 5 -> 5
    assert list(orc.shell_index([0, 1, 2, 3, 6, 7, 25, 30, 31])) == [0, 1, 1, 2, 2, 3, 5, 5, 6]


@pytest.mark.parametrize("mode,shell", [((0, 0, 0), 0), ((3, 4, 0), 5), ((0, -1, 1), 1), ((1, 1, 1), 2),
                                        ((-2, 1, 2), 3), ((0, 5, 0), 5)])
def test_single_mode_lands_in_its_shell(orc, mode, shell):
    n = 16
    u = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    mz, my, mx = mode
    u[1, mz % n, my % n, mx] = 2.0 - 1.0j                     # |u|^2 = 5
    e = orc.spectrum(u, 8)
    want = np.zeros(8)
    want[shell] = 5.0 * (1.0 if mx > 0 else 0.5)              # half of |u|^2, twice for the mirror mode
    assert np.array_equal(e, want)


@pytest.mark.parametrize("n", [16, 32])
def test_parseval(orc, n):
    u = field(orc, n, 5)
    K = n // 3
    e = orc.spectrum(u, int(math.isqrt(3 * K * K)) + 2)
    assert abs(e.sum() - 0.5) <= 1e-14
    assert abs(e.sum() - orc.energy(u)) <= 1e-14
    assert e[0] == 0.0                                        # the mean flow is not set
    # truncating the shell list drops exactly the outer shells
    e5 = orc.spectrum(u, 5)
    assert np.allclose(e5, e[:5], rtol=0, atol=1e-16)


def test_initial_field_spectrum_closed_form(orc):
    """Every retained mode of the initial field holds |u_m|^2 = c^2 E(|k|) / (4 pi |k|^2)
    with E(k) = k^4 exp(-2 (k/k_p)^2) and c fixed by the total energy, so each shell's
    energy follows from counting integer vectors: brute force over the cube."""
    n, kp = 16, 2.0
    K = n // 3
    u = field(orc, n, 11)
    f = {}
    for mz in range(-K, K + 1):
        for my in range(-K, K + 1):
            for mx in range(-K, K + 1):
                m2 = mx * mx + my * my + mz * mz
                if m2 == 0:
                    continue
                k = math.sqrt(m2)
                s = int(math.floor(k + 0.5))
                f[s] = f.get(s, 0.0) + 0.5 * k ** 4 * math.exp(-2 * (k / kp) ** 2) / (4 * math.pi * m2)
    total = sum(f.values())
    ns = max(f) + 1
    want = np.array([0.5 * f.get(s, 0.0) / total for s in range(ns)])
    got = orc.spectrum(u, ns)
    assert np.max(np.abs(got - want)) <= 1e-14


def test_refine_is_spectral_interpolation(orc):
    """The refined field takes the coarse field's values at the coarse grid points
    (physical space through numpy's inverse FFT, unnormalised as the solver's)."""
    n = 16
    u = field(orc, n, 3)
    for nb in (16, 32, 64):
        r = orc.refine(u, nb)
        assert r.shape == (3, nb, nb, nb // 2 + 1)
        x = np.fft.irfftn(u, s=(n, n, n), axes=(1, 2, 3), norm="forward")
        y = np.fft.irfftn(r, s=(nb, nb, nb), axes=(1, 2, 3), norm="forward")
        st = nb // n
        assert np.max(np.abs(y[:, ::st, ::st, ::st] - x)) <= 1e-14 * np.max(np.abs(x))


def test_refine_keeps_energy_spectrum_and_divergence(orc):
    n, nb = 16, 32
    u = field(orc, n, 8)
    r = orc.refine(u, nb)
    K = n // 3
    ns = int(math.isqrt(3 * K * K)) + 2
    assert np.array_equal(orc.spectrum(r, ns), orc.spectrum(u, ns))
    assert orc.spectrum(r, 2 * ns)[ns:].sum() == 0.0
    assert abs(orc.dissipation(r, 0.01) - orc.dissipation(u, 0.01)) <= 1e-15 * orc.dissipation(u, 0.01)
    assert orc.divergence_ratio(r) <= 1e-14
    # identity at the same grid; a coarser target is refused
    assert np.array_equal(orc.refine(u, n), u)
    with pytest.raises(ValueError):
        orc.refine(u, 8)


def test_integral_scales_of_single_modes(orc):
    """One mode of wavenumber k: E = e, u'^2 = 2e/3 and L = 3 pi / (4 k) whatever the
    amplitude; two modes add their e/k; a box twice as large halves k."""
    n = 16
    u = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    u[0, 0, 3, 4] = 1.5 + 0.5j                                # m = (m_z, m_y, m_x) = (0, 3, 4), |m| = 5
    E, up, L, T = orc.integral_scales(u)
    e = 2.5                                                   # (1/2)|u|^2 = 1.25, twice for the mirror mode
    assert abs(E - e) <= 1e-15 and abs(up - math.sqrt(2 * e / 3)) <= 1e-15
    assert abs(L - 3 * math.pi / 20) <= 1e-15 and abs(T - L / up) <= 1e-15
    _, _, L4, _ = orc.integral_scales(u, box=4 * math.pi)
    assert abs(L4 - 2 * L) <= 1e-15
    u[2, 1, 0, 0] = 2.0                                       # m = (1, 0, 0) on the m_x = 0 plane ...
    u[2, n - 1, 0, 0] = 2.0                                   # ... and its mirror (-1, 0, 0): e = (4 + 4) / 2
    E2, _, L2, _ = orc.integral_scales(u)
    assert abs(E2 - (e + 4.0)) <= 1e-15
    assert abs(L2 - 3 * math.pi / (4 * E2) * (e / 5 + 4.0 / 1)) <= 1e-15
    assert orc.integral_scales(np.zeros_like(u)) == (0.0, 0.0, 0.0, 0.0)


def test_integral_scales_of_the_initial_field_closed_form(orc):
    """Brute force over the retained cube with the initial field's mode energies."""
    n, kp = 16, 2.0
    K = n // 3
    u = field(orc, n, 21)
    f, fk = 0.0, 0.0
    for mz in range(-K, K + 1):
        for my in range(-K, K + 1):
            for mx in range(-K, K + 1):
                m2 = mx * mx + my * my + mz * mz
                if m2:
                    k = math.sqrt(m2)
                    v = k ** 4 * math.exp(-2 * (k / kp) ** 2) / (4 * math.pi * m2)
                    f += v
                    fk += v / k
    E, up, L, T = orc.integral_scales(u)
    assert abs(E - 0.5) <= 1e-14
    want_L = math.pi / (2 * (2 * 0.5 / 3)) * 0.5 * fk / f
    assert abs(L - want_L) <= 1e-14 * want_L
    assert abs(T - want_L / math.sqrt(1 / 3)) <= 1e-13 * T
