"""Pins of the oracle's solver (initial field, right-hand side, time stepper)
against closed forms, invariants and a library FFT -- never against itself."""
import math

import numpy as np
import pytest


def to_canonical(u_phys):
    """Real (3, n, n, n) [c][z][y][x] field -> canonical spectral layout (library FFT)."""
    n = u_phys.shape[1]
    return np.stack([np.fft.rfftn(u_phys[c], axes=(0, 1, 2)) / n ** 3 for c in range(3)])


def to_physical(uhat):
    n = uhat.shape[1]
    return np.stack([np.fft.irfftn(uhat[c] * n ** 3, s=(n, n, n), axes=(0, 1, 2)) for c in range(3)])


def grid(n, box=2 * np.pi):
    x = np.arange(n) * box / n
    return np.meshgrid(x, x, x, indexing="ij")      # returns Z, Y, X


def taylor_green(n):
    Z, Y, X = grid(n)
    return np.stack([np.sin(X) * np.cos(Y) * np.cos(Z), -np.cos(X) * np.sin(Y) * np.cos(Z), 0 * X])


# ------------------------------------------------------------------ initial field
def test_splitmix64_published_vector(orc):
    # First outputs of splitmix64 seeded with 1234567, as published with the generator.
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    assert [orc.splitmix64(1234567, c) for c in range(5)] == expect


@pytest.mark.parametrize("n", [16, 32])
def test_init_field_properties(orc, n):
    u = orc.init_field(n, seed=23712 + n, k_peak=2.0, e0=0.5)
    assert abs(orc.energy(u) - 0.5) <= 1e-14
    assert orc.divergence_ratio(u) <= 1e-14
    mask = orc.retained_mask(n)
    assert np.all(u[:, ~mask] == 0)
    assert np.all(u[:, 0, 0, 0] == 0)
    # independent real and imaginary deviates: the phases of a mode's components
    # are spread (one deviate used twice would put each at 45 or 225 degrees)
    keep = mask & (np.sum(np.abs(u) ** 2, axis=0) > 0)
    same = np.all(np.abs(u.real - u.imag) <= 1e-9 * np.abs(u), axis=0)
    assert np.mean(same[keep]) < 0.01
    # Hermitian on the m_x = 0 plane: u(0, -m_y, -m_z) = conj(u(0, m_y, m_z))
    p = u[:, :, :, 0]
    mirrored = np.conj(p[:, (-np.arange(n)) % n][:, :, (-np.arange(n)) % n])
    assert np.max(np.abs(p - mirrored)) == 0
    # physical field is real: the library inverse transform of the Hermitian
    # extension agrees with the half-spectrum transform
    full = np.zeros((3, n, n, n), complex)
    full[..., : n // 2 + 1] = u
    for x in range(n // 2 + 1, n):
        full[..., x] = np.conj(u[:, (-np.arange(n)) % n][:, :, (-np.arange(n)) % n][..., n - x])
    phys = np.fft.ifftn(full * n ** 3, axes=(1, 2, 3))
    assert np.max(np.abs(phys.imag)) <= 1e-13 * np.max(np.abs(phys.real))


def test_init_field_spectrum_shape(orc):
    """Every retained mode carries |u_hat|^2 proportional to E(|k|)/(4 pi |k|^2) with
    E(k) = k^4 exp(-2 (k/k_peak)^2): only directions and phases are random."""
    n = 32
    u = orc.init_field(n, seed=7, k_peak=2.0, e0=0.5)
    mz, my, mx = orc.modes(n)
    k2 = (mz * mz + my * my + mx * mx).astype(float)
    mask = orc.retained_mask(n) & (k2 > 0)
    k = np.sqrt(k2[mask])
    model = k ** 4 * np.exp(-2 * (k / 2.0) ** 2) / (4 * np.pi * k * k)
    ratio = np.sum(np.abs(u) ** 2, axis=0)[mask] / model
    assert np.max(np.abs(ratio / ratio[0] - 1)) <= 1e-12


# ---------------------------------------------------------------- right-hand side
def test_taylor_green_nonlinear_and_viscous_closed_form(orc):
    n, nu = 16, 0.013
    u = to_canonical(taylor_green(n))
    m = orc.Member(n=n, nu=nu, eps=0.0, kf_lo=0, kf_hi=0)
    g, info = orc.rhs(m, u, terms=orc.T_NONLINEAR | orc.T_VISCOUS)
    Z, Y, X = grid(n)
    N0 = np.stack([-np.sin(2 * X) * np.cos(2 * Z) / 8, -np.sin(2 * Y) * np.cos(2 * Z) / 8,
                   (np.cos(2 * X) + np.cos(2 * Y)) * np.sin(2 * Z) / 8])
    expect = N0 - 3 * nu * taylor_green(n)
    got = to_physical(g)
    assert np.max(np.abs(got - expect)) <= 1e-14
    assert abs(np.mean(np.sum(to_physical(orc.rhs(m, u, terms=orc.T_NONLINEAR)[0]) ** 2, axis=0)) - 1 / 64) <= 1e-15
    assert info[3] <= 1e-14     # inverse transforms of a Hermitian field are real


def _random_field(orc, n, seed):
    return orc.init_field(n, seed=seed, k_peak=3.0, e0=0.5)


def _full_sum(a, b):
    w = np.ones(a.shape[-1]); w[1:] = 2
    return float(np.sum(np.real(np.conj(a) * b) * w))


@pytest.mark.parametrize("n", [16, 32])
def test_galerkin_nonlinear_term_conserves_energy_and_helicity(orc, n):
    u = _random_field(orc, n, 100 + n)
    m = orc.Member(n=n, nu=0.0, eps=0.0)
    N, _ = orc.rhs(m, u, terms=orc.T_NONLINEAR)
    mz, my, mx = orc.modes(n)
    k = [mx, my, mz]
    w = np.stack([1j * (k[1] * u[2] - k[2] * u[1]), 1j * (k[2] * u[0] - k[0] * u[2]),
                  1j * (k[0] * u[1] - k[1] * u[0])])
    scale = np.sqrt(_full_sum(u, u) * _full_sum(N, N)) * (n // 3) * np.sqrt(3)
    assert abs(_full_sum(u, N)) <= 1e-13 * scale
    assert abs(_full_sum(w, N)) <= 1e-13 * scale * (n // 3) * np.sqrt(3)
    assert orc.divergence_ratio(N) <= 1e-13
    assert np.all(N[:, ~orc.retained_mask(n)] == 0)


def test_single_fourier_mode_has_no_nonlinear_term(orc):
    n = 16
    Z, Y, X = grid(n)
    kv = np.array([2, -1, 3])                       # (k_x, k_y, k_z)
    a = np.array([1.0, 2.0, 0.0]); a -= kv * (kv @ a) / (kv @ kv)   # a perpendicular to k
    s = np.sin(kv[0] * X + kv[1] * Y + kv[2] * Z)
    u = to_canonical(np.stack([a[0] * s, a[1] * s, a[2] * s]))
    N, _ = orc.rhs(orc.Member(n=n, nu=0.0, eps=0.0), u, terms=orc.T_NONLINEAR)
    # u x omega is a pure gradient here; what is left is rounding of |a|^2 |k|
    assert np.max(np.abs(N)) <= 1e-15 * (a @ a) * np.sqrt(kv @ kv)


@pytest.mark.parametrize("band", [(0.0, 2.0, 32), (0.0, 2.5, 80), (1.4, 2.3, 50), (1.0, 2.0, 32), (1.0, 1.0, 6)])
def test_forcing_injects_exactly_eps(orc, band):
    lo, hi, count = band
    n = 16
    u = _random_field(orc, n, 3)
    m = orc.Member(n=n, nu=0.0, eps=0.37, kf_lo=lo, kf_hi=hi)
    g, info = orc.rhs(m, u, terms=orc.T_FORCING)
    assert abs(info[1] - 0.37) <= 1e-14
    assert abs(_full_sum(u, g) - 0.37) <= 1e-14
    # the band has the stated number of modes over the full spectrum
    mz, my, mx = orc.modes(n)
    m2 = mz * mz + my * my + mx * mx
    inband = (m2 > 0) & (m2 >= lo * lo) & (m2 <= hi * hi)
    w = np.ones(n // 2 + 1); w[1:] = 2
    assert int(np.sum(inband * w)) == count
    # f = eps / (2 E_f) u on the band, zero elsewhere
    Ef = 0.5 * float(np.sum(np.sum(np.abs(u) ** 2, axis=0) * inband * w))
    assert abs(info[0] - Ef) <= 1e-15
    assert np.max(np.abs(g - (0.37 / (2 * Ef)) * u * inband)) <= 1e-15


def test_forcing_is_projected_like_the_nonlinear_term(orc):
    """A solenoidal field plus a gradient field: the forcing acts on the
    solenoidal part only (the pressure takes the divergent part), with E_f of
    the whole field; a divergent part in the band is not amplified."""
    n = 16
    us = _random_field(orc, n, 5)
    mz, my, mx = orc.modes(n)
    rng = np.random.default_rng(6)
    phi = rng.standard_normal(mx.shape) + 1j * rng.standard_normal(mx.shape)
    m2 = mz * mz + my * my + mx * mx
    inband = (m2 > 0) & (m2 <= 4)
    phi = phi * inband * 0.1
    phi[:, :, 0] = 0                                  # keep it away from the self-conjugate plane
    ug = np.stack([1j * mx * phi, 1j * my * phi, 1j * mz * phi])
    m = orc.Member(n=n, nu=0.0, eps=0.5, kf_lo=0.0, kf_hi=2.0)
    g, info = orc.rhs(m, us + ug, terms=orc.T_FORCING)
    w = np.ones(n // 2 + 1); w[1:] = 2
    Ef = 0.5 * float(np.sum(np.sum(np.abs(us + ug) ** 2, axis=0) * inband * w))
    assert abs(info[0] - Ef) <= 1e-14 * Ef
    assert np.max(np.abs(g - (0.5 / (2 * Ef)) * us * inband)) <= 1e-15
    assert orc.divergence_ratio(g) <= 1e-15
    g0, _ = orc.rhs(m, ug, terms=orc.T_FORCING)
    assert np.max(np.abs(g0)) <= 1e-15 * np.max(np.abs(ug))


def test_forcing_acts_on_the_hermitian_part_of_the_m_x_0_plane(orc):
    """The velocity is real: u(0, -m_y, -m_z) = conj u(0, m_y, m_z) on the
    m_x = 0 plane of the half spectrum.  A part breaking that (here i r added
    at both modes of a pair) is invisible in physical space; the forcing and
    E_f ignore it, so it is not amplified."""
    n = 16
    u = _random_field(orc, n, 8)
    m = orc.Member(n=n, nu=0.0, eps=0.5, kf_lo=1.4, kf_hi=2.3)
    g, info = orc.rhs(m, u, terms=orc.T_FORCING)
    v = u.copy()
    for (my, mz), r in (((1, 1), (0.3, -0.2, 0.1)), ((2, 0), (0.0, 0.25, -0.4)), ((-1, 2), (0.1, 0.1, 0.2))):
        for c in range(3):
            v[c, mz % n, my % n, 0] += 1j * r[c]
            v[c, (-mz) % n, (-my) % n, 0] += 1j * r[c]
    gv, iv = orc.rhs(m, v, terms=orc.T_FORCING)
    assert abs(iv[0] - info[0]) <= 1e-15 * info[0]
    assert np.max(np.abs(gv - g)) <= 1e-15
    # the injection rate stays eps exactly
    assert abs(iv[1] - 0.5) <= 1e-14


def test_band_excludes_the_mean_mode(orc):
    """A band starting at 0 holds the modes 0 < |m| <= k_f,hi: a uniform flow
    (the m = 0 mode) is neither counted in E_f nor forced."""
    n = 16
    u = _random_field(orc, n, 12)
    m = orc.Member(n=n, nu=0.0, eps=0.4, kf_lo=0.0, kf_hi=2.0)
    g, info = orc.rhs(m, u, terms=orc.T_FORCING)
    v = u.copy()
    v[:, 0, 0, 0] = (0.3, -0.2, 0.45)
    gv, iv = orc.rhs(m, v, terms=orc.T_FORCING)
    assert abs(iv[0] - info[0]) <= 1e-15 * info[0]
    assert np.all(gv[:, 0, 0, 0] == 0)
    assert np.max(np.abs(gv - g)) <= 1e-15


def test_forcing_with_empty_band_energy_is_zero(orc):
    n = 16
    u = np.zeros((3, n, n, n // 2 + 1), complex)
    u[1, 0, 0, 5] = -0.5j                            # v = sin(5x): only |k| = 5, outside the band
    g, info = orc.rhs(orc.Member(n=n, nu=0.0, eps=1.0, kf_hi=2.0), u, terms=orc.T_FORCING)
    assert info[0] == 0 and np.all(g == 0)


@pytest.mark.parametrize("frac, forced", [(1e-12, False), (1e-11, False), (1e-9, True), (1e-6, True)])
def test_band_below_the_empty_threshold_is_not_forced(orc, frac, forced):
    """The linear forcing eps/(2 E_f) u is singular as E_f -> 0; a band holding
    at most 1e-10 of the field's energy counts as empty (no forcing, no
    injection), above it the injection is eps exactly."""
    n = 16
    u = np.zeros((3, n, n, n // 2 + 1), complex)
    u[1, 0, 0, 5] = -0.5j                            # energy 1/4 off the band
    E_off = orc.energy(u)
    a, _ = _single_mode(n, (1, 1, 0), amp=1.0)        # one band mode pair, |m|^2 = 2
    a *= math.sqrt(frac * E_off / orc.energy(a))
    v = u + a
    Ef = orc.energy(a)
    assert abs(Ef / orc.energy(v) - frac / (1 + frac)) <= 1e-15
    g, info = orc.rhs(orc.Member(n=n, nu=0.0, eps=0.7, kf_hi=2.0), v, terms=orc.T_FORCING)
    assert abs(info[0] - Ef) <= 1e-14 * Ef
    if forced:
        assert abs(info[1] - 0.7) <= 1e-14
        assert np.max(np.abs(g - (0.7 / (2 * Ef)) * a)) <= 1e-14 * 0.7 / (2 * Ef) * np.max(np.abs(a))
    else:
        assert info[1] == 0 and np.all(g == 0)


def test_single_off_band_mode_with_injection_decays_viscously(orc):
    """A single Fourier mode outside the band, eps > 0: the band stays empty,
    nothing is forced, and the mode decays exactly as exp(-nu k^2 t) (its own
    nonlinear term vanishes)."""
    n, nu = 16, 0.05
    u0, k2 = _single_mode(n, (3, 1, 0))
    m = orc.Member(n=n, nu=nu, eps=1.0, kf_lo=0, kf_hi=2.0, dt=0.05)
    u, diag = orc.run(m, u0, 20)
    assert np.max(np.abs(u - u0 * math.exp(-nu * k2 * 20 * 0.05))) <= 1e-14 * np.max(np.abs(u0))
    assert np.all(diag[:, 4] == 0)                    # no injection at any step


# ----------------------------------------------------------------- time stepping
def _single_mode(n, kv, amp=0.3):
    """u = a cos(k.x) with a perpendicular to k, written directly in spectral space."""
    kv = np.asarray(kv)
    assert kv[0] > 0
    a = np.array([1.0, -1.0, 0.5]); a -= kv * (kv @ a) / (kv @ kv); a *= amp
    u = np.zeros((3, n, n, n // 2 + 1), complex)
    u[:, kv[2] % n, kv[1] % n, kv[0]] = a / 2
    return u, float(kv @ kv)


@pytest.mark.parametrize("dt", [0.01, 0.3, 2.0])
def test_integrating_factor_decay_is_exact(orc, dt):
    n, nu = 16, 0.05
    u0, k2 = _single_mode(n, (3, 1, 0))
    m = orc.Member(n=n, nu=nu, eps=0.0, kf_lo=0, kf_hi=0, dt=dt)
    u, diag = orc.run(m, u0, 4)
    assert np.max(np.abs(u - u0 * math.exp(-nu * k2 * 4 * dt))) <= 1e-14 * np.max(np.abs(u0))
    assert abs(diag[-1, 0] - 4 * dt) <= 1e-15


@pytest.mark.parametrize("dt", [0.01, 0.2])
def test_explicit_variant_follows_rk3_stability_polynomial(orc, dt):
    n, nu = 16, 0.05
    u0, k2 = _single_mode(n, (3, 1, 0))
    m = orc.Member(n=n, nu=nu, eps=0.0, kf_lo=0, kf_hi=0, dt=dt, visc_mode=1)
    u, _ = orc.run(m, u0, 5)
    z = -nu * k2 * dt
    R = 1 + z + z * z / 2 + z ** 3 / 6
    assert np.max(np.abs(u - u0 * R ** 5)) <= 1e-14 * np.max(np.abs(u0))


def test_third_order_convergence(orc):
    n = 16
    u0 = to_canonical(taylor_green(n))
    T = 0.6
    finals = {}
    for dt in (0.1, 0.05, 0.025, 0.00625):
        m = orc.Member(n=n, nu=0.05, eps=0.0, kf_lo=0, kf_hi=0, dt=dt)
        finals[dt], _ = orc.run(m, u0, int(round(T / dt)))
    ref = finals[0.00625]
    e = [np.sqrt(np.sum(np.abs(finals[d] - ref) ** 2)) for d in (0.1, 0.05, 0.025)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 7.0 < r1 < 9.0 and 7.3 < r2 < 8.7, (r1, r2)


def test_taylor_green_early_time(orc):
    """E(t) = 1/8 - (3/4) nu t + (9/4) nu^2 t^2 + O(t^3); |k|^2 = 8 shell energy t^2/128 + O(t^3)."""
    n, nu = 16, 0.1
    u0 = to_canonical(taylor_green(n))
    mz, my, mx = orc.modes(n)
    m2 = mz * mz + my * my + mx * mx
    w = np.ones(n // 2 + 1); w[1:] = 2
    res_e, res_s = [], []
    for t in (0.04, 0.02, 0.01):
        m = orc.Member(n=n, nu=nu, eps=0.0, kf_lo=0, kf_hi=0, dt=t / 8)
        u, diag = orc.run(m, u0, 8)
        E = diag[-1, 2]
        res_e.append(abs(E - (1 / 8 - 0.75 * nu * t + 2.25 * nu * nu * t * t)) / t ** 3)
        e8 = 0.5 * float(np.sum(np.sum(np.abs(u) ** 2, axis=0) * (m2 == 8) * w))
        res_s.append(abs(e8 - t * t / 128) / t ** 3)
    # residuals over t^3 stay bounded (approach a constant) as t -> 0
    assert max(res_e) < 0.1 and res_e[-1] <= 1.2 * res_e[0] + 1e-6
    assert max(res_s) < 0.1 and res_s[-1] <= 1.2 * res_s[0] + 1e-6


def test_inviscid_energy_drift_is_third_order(orc):
    n = 16
    u0 = _random_field(orc, n, 77)
    drift = []
    for dt in (0.04, 0.02):
        m = orc.Member(n=n, nu=0.0, eps=0.0, kf_lo=0, kf_hi=0, dt=dt)
        u, diag = orc.run(m, u0, int(round(0.8 / dt)))
        drift.append(abs(diag[-1, 2] - 0.5) / 0.5)
    slope = math.log2(drift[0] / drift[1])
    assert 2.7 < slope < 3.3, (drift, slope)


def test_steps_stay_solenoidal_and_truncated(orc):
    n = 32
    u0 = orc.init_field(n, seed=23712)
    m = orc.Member(n=n, nu=0.02, eps=0.1, kf_hi=2.0, dt=0.01)
    u, diag = orc.run(m, u0, 10)
    assert orc.divergence_ratio(u) <= 1e-14
    assert np.all(u[:, ~orc.retained_mask(n)] == 0)
    assert np.allclose(diag[:, 4], 0.1, rtol=0, atol=1e-14)      # injection = eps at stage 1
    # energy budget over one step: dE ~ dt (eps - D) to O(dt^2)
    E0 = orc.energy(u0)
    D0 = orc.dissipation(u0, 0.02)
    assert abs((diag[0, 2] - E0) / 0.01 - (0.1 - D0)) < 0.02
    assert abs(diag[-1, 3] - orc.dissipation(u, 0.02)) <= 1e-14 * diag[-1, 3]


def test_energy_budget_with_the_reported_dissipation(orc):
    """dE/dt = eps - D (the nonlinear term conserves energy, the forcing injects
    eps): over every step the reported energies and dissipations satisfy
    E_n - E_(n-1) = dt (eps - (D_(n-1) + D_n) / 2) up to the trapezoid and
    RK3 errors, O(dt^3) per step."""
    n, nu, eps, dt = 16, 0.02, 0.1, 2e-3
    u0 = _random_field(orc, n, 31)
    m = orc.Member(n=n, nu=nu, eps=eps, kf_hi=2.0, dt=dt)
    _, diag = orc.run(m, u0, 8)
    E = np.concatenate([[orc.energy(u0)], diag[:, 2]])
    D = np.concatenate([[orc.dissipation(u0, nu)], diag[:, 3]])
    resid = (E[1:] - E[:-1]) / dt - (eps - 0.5 * (D[1:] + D[:-1]))
    assert np.max(np.abs(resid)) <= 1e-4 * np.max(D), (resid, D)


def test_cfl_time_step(orc):
    n = 32
    u0 = orc.init_field(n, seed=5)
    m = orc.Member(n=n, nu=0.02, eps=0.1, kf_hi=2.0, dt=0.0, cfl=0.5)
    _, diag = orc.run(m, u0, 3)
    dx = 2 * np.pi / n
    assert np.allclose(diag[:, 1] * diag[:, 6] / dx, 0.5, rtol=1e-14)
    # stage-1 velocity maximum of the initial field, from the library inverse transform
    up = to_physical(u0)
    assert abs(diag[0, 6] - np.max(np.sum(np.abs(up), axis=0))) <= 1e-13
