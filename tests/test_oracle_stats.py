"""Pins of the oracle's gradient statistics: invariants of band-limited fields,
Parseval identities, and brute-force binning of an analytic gradient field."""
import numpy as np
import pytest


def full_sum(a):
    w = np.ones(a.shape[-1]); w[1:] = 2
    return float(np.sum(a * w))


def taylor_green_spectral(n):
    x = np.arange(n) * 2 * np.pi / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.stack([np.sin(X) * np.cos(Y) * np.cos(Z), -np.cos(X) * np.sin(Y) * np.cos(Z), 0 * X])
    return np.stack([np.fft.rfftn(u[c]) / n ** 3 for c in range(3)]), (X, Y, Z)


def bin_rule(x, lo, hi, nb):
    """The documented bin rule, restated: -1 under, -2 over, -3 nan, else floor((x-lo)*nb/(hi-lo))."""
    x = np.asarray(x, float)
    b = np.floor((x - lo) * (nb / (hi - lo)))
    out = np.where(np.isnan(x), -3, np.where(x < lo, -1, np.where(b >= nb, -2, b)))
    return out.astype(np.int64)


# ranges offset so that no Taylor-Green grid value sits on a bin edge
H = dict(qr_bins=16, q_lo=-3.0123, q_hi=2.9431, r_lo=-3.0311, r_hi=2.9717, log_bins=32,
         log10_lo=-4.0137, log10_hi=2.0251, a_bins=40, a_lo=-2.0173, a_hi=1.9913,
         eps_ref=0.2, nu_ref=0.05)


def test_taylor_green_histograms_match_brute_force(orc):
    """Analytic A_ij of the Taylor-Green field, invariants by matrix products,
    binned with the documented rule, must give the oracle's counts exactly."""
    n, nu = 16, 0.05
    uh, (X, Y, Z) = taylor_green_spectral(n)
    h = orc.Hist(**H)
    counts, mom, near, trmax = orc.stats(orc.Member(n=n, nu=nu, eps=0.2), h, uh)
    sx, cx, sy, cy, sz, cz = np.sin(X), np.cos(X), np.sin(Y), np.cos(Y), np.sin(Z), np.cos(Z)
    A = np.zeros((n, n, n, 3, 3))
    A[..., 0, 0] = cx * cy * cz;  A[..., 0, 1] = -sx * sy * cz; A[..., 0, 2] = -sx * cy * sz
    A[..., 1, 0] = sx * sy * cz;  A[..., 1, 1] = -cx * cy * cz; A[..., 1, 2] = cx * sy * sz
    A2 = A @ A
    Q = -0.5 * np.trace(A2, axis1=-2, axis2=-1)
    R = -np.trace(A2 @ A, axis1=-2, axis2=-1) / 3
    S = 0.5 * (A + np.swapaxes(A, -1, -2))
    eps = 2 * nu * np.sum(S * S, axis=(-2, -1))
    om = np.stack([A[..., 2, 1] - A[..., 1, 2], A[..., 0, 2] - A[..., 2, 0], A[..., 1, 0] - A[..., 0, 1]], -1)
    ens = np.sum(om * om, -1)
    tau = np.sqrt(h.nu_ref / h.eps_ref)
    trs = h.eps_ref / (2 * h.nu_ref)
    got = h.split(counts)
    assert np.all(near[[0, 3, 4]] == 0)     # the comparisons below are all exercised
    # QR
    bq = bin_rule(Q / trs, h.q_lo, h.q_hi, h.qr_bins).ravel()
    br = bin_rule(R / trs ** 1.5, h.r_lo, h.r_hi, h.qr_bins).ravel()
    inside = (bq >= 0) & (br >= 0)
    ref_qr = np.bincount(bq[inside] * h.qr_bins + br[inside], minlength=h.qr_bins ** 2)
    if near[0] == 0:
        assert np.array_equal(got["qr"].ravel(), ref_qr)
        assert got["qr_special"][0] == np.sum(~inside)
    # log histograms (eps <= 0 -> underflow)
    for name, val, k in (("log_eps", eps / h.eps_ref, 1), ("log_ens", ens * h.nu_ref / h.eps_ref, 2)):
        v = val.ravel()
        b = np.where(v > 0, bin_rule(np.log10(np.where(v > 0, v, 1)), h.log10_lo, h.log10_hi, h.log_bins), -1)
        ref = np.bincount(b[b >= 0], minlength=h.log_bins)
        if near[k] == 0:
            assert np.array_equal(got[name], ref), name
            assert got[name + "_special"][0] == np.sum(b == -1)
            assert got[name + "_special"][1] == np.sum(b == -2)
    # pooled gradient components
    diag = np.stack([A[..., i, i] for i in range(3)]).ravel() * tau
    off = np.stack([A[..., i, j] for i in range(3) for j in range(3) if i != j]).ravel() * tau
    for name, v, k in (("a_long", diag, 3), ("a_trans", off, 4)):
        b = bin_rule(v, h.a_lo, h.a_hi, h.a_bins)
        if near[k] == 0:
            assert np.array_equal(got[name], np.bincount(b[b >= 0], minlength=h.a_bins)), name
    # moments
    for p in range(1, 7):
        assert np.isclose(mom[p - 1], np.sum(diag ** p), rtol=1e-12, atol=1e-12 * n ** 3)
        assert np.isclose(mom[5 + p], np.sum(off ** p), rtol=1e-12, atol=1e-12 * n ** 3)
    for p in range(1, 5):
        assert np.isclose(mom[11 + p], np.sum((eps / h.eps_ref) ** p), rtol=1e-12)
        assert np.isclose(mom[15 + p], np.sum((ens * h.nu_ref / h.eps_ref) ** p), rtol=1e-12)
    assert np.isclose(mom[24], np.sum((Q / trs) ** 2), rtol=1e-12)
    assert np.isclose(mom[25], np.sum((R / trs ** 1.5) ** 2), rtol=1e-12, atol=1e-20)
    assert trmax <= 1e-14


@pytest.mark.parametrize("n", [16, 32])
def test_band_limited_invariants(orc, n):
    """Tr A = 0 pointwise; grid <Q> = <R> = 0 exactly (no alias reaches k = 0 for
    |m_i| <= N/3); nu <omega^2> = <eps> = D; counts sum to the number of samples."""
    nu = 0.02
    u = orc.init_field(n, seed=42 + n, k_peak=3.0, e0=0.5)
    h = orc.Hist(qr_bins=32, eps_ref=0.1, nu_ref=nu)
    counts, mom, near, trmax = orc.stats(orc.Member(n=n, nu=nu, eps=0.1), h, u)
    npts = n ** 3
    tau = np.sqrt(h.nu_ref / h.eps_ref)
    trs_mean = mom[22] / npts                         # <S*_ij S*_ij>
    assert trmax * tau <= 1e-13 * np.sqrt(trs_mean)
    assert abs(mom[20] / npts) <= 1e-13 * trs_mean * 2
    assert abs(mom[21] / npts) <= 1e-13 * (2 * trs_mean) ** 1.5
    D = orc.dissipation(u, nu)
    assert np.isclose(mom[12] / npts * h.eps_ref, D, rtol=1e-12)        # <eps> = D
    assert np.isclose(mom[16] / npts * h.eps_ref, D, rtol=1e-12)        # nu <omega^2> = D
    # Parseval: sum_x A_ij^2 = N^3 sum_k |k_j u_i|^2 over the full spectrum
    mz, my, mx = orc.modes(n)
    k = [mx, my, mz]
    longi = sum(full_sum(np.abs(k[i] * u[i]) ** 2) for i in range(3))
    trans = sum(full_sum(np.abs(k[j] * u[i]) ** 2) for i in range(3) for j in range(3) if i != j)
    assert np.isclose(mom[1], npts * longi * tau ** 2, rtol=1e-12)
    assert np.isclose(mom[7], npts * trans * tau ** 2, rtol=1e-12)
    got = h.split(counts)
    for name, mult in (("qr", 1), ("log_eps", 1), ("log_ens", 1), ("a_long", 3), ("a_trans", 6)):
        assert int(got[name].sum() + got[name + "_special"].sum()) == mult * npts


def test_zero_field_fills_one_bin(orc):
    n = 16
    u = np.zeros((3, n, n, n // 2 + 1), complex)
    h = orc.Hist(qr_bins=8, q_lo=-1, q_hi=1, r_lo=-1, r_hi=1, log_bins=8, a_bins=8, a_lo=-1, a_hi=1)
    counts, mom, near, _ = orc.stats(orc.Member(n=n, nu=0.01, eps=1.0), h, u)
    got = h.split(counts)
    assert got["qr"][4, 4] == n ** 3 and got["qr"].sum() == n ** 3
    assert got["log_eps_special"][0] == n ** 3            # eps = 0 -> underflow
    assert got["a_long"][4] == 3 * n ** 3
    assert np.all(mom == 0)


def test_gradient_tolerance_bounds_the_bin_changes_of_a_perturbed_field(orc):
    """The near-edge allowance with grad_tol covers every bin change that a
    gradient perturbation of at most grad_tol * max|A_ij| can cause: the field
    u + s u + w (w random, its largest possible gradient t max|A| by the
    triangle inequality over its modes) bins like u except for at most the
    samples the oracle marks as near an edge; the plain rounding allowance
    does not cover it."""
    n, nu = 32, 0.02
    u = orc.init_field(n, seed=77, k_peak=3.0, e0=0.5)
    h = orc.Hist(qr_bins=64, log_bins=256, a_bins=256, a_lo=-20, a_hi=20, eps_ref=0.1, nu_ref=nu)
    m = orc.Member(n=n, nu=nu, eps=0.1)
    c0, _, near0, _ = orc.stats(m, h, u)
    # max |A_ij| of u from its physical gradients
    mz, my, mx = orc.modes(n)
    kk = [mx, my, mz]
    amax = 0.0
    for i in range(3):
        for j in range(3):
            g = np.fft.irfftn(1j * kk[j] * u[i], s=(n, n, n), axes=(0, 1, 2)) * n ** 3
            amax = max(amax, float(np.max(np.abs(g))))
    rng = np.random.default_rng(5)
    w = (rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)) * orc.retained_mask(n)
    wt = np.ones(n // 2 + 1); wt[1:] = 2.0
    wbound = max(float(np.sum(np.abs(kk[j] * w[i]) * wt)) for i in range(3) for j in range(3))
    s, t = 3e-5, 2e-5
    v = u * (1 + s) + w * (t * amax / wbound)
    c1, _, _, _ = orc.stats(m, h, v)
    _, _, near, _ = orc.stats(m, h, u, grad_tol=s + t)
    a, b = h.split(c0), h.split(c1)
    moved = 0
    for k, name in enumerate(("qr", "log_eps", "log_ens", "a_long", "a_trans")):
        diff = int(np.abs(np.concatenate([a[name].ravel(), a[name + "_special"]]).astype(np.int64)
                          - np.concatenate([b[name].ravel(), b[name + "_special"]]).astype(np.int64)).sum())
        assert diff <= 2 * int(near[k]), (name, diff, int(near[k]))
        assert int(near[k]) >= int(near0[k])
        moved += diff > 2 * int(near0[k])
    assert moved >= 3                                     # the perturbation does move samples across edges


def aliased_field(n, seed):
    """A solenoidal field with every mode |m_i| < n/2 (no 2/3 truncation, Nyquist
    planes zero), from a random real field by the library FFT: no symmetry of
    the Taylor-Green kind, and its grid sum of R is not zero (triple products
    of modes alias onto m = 0)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3, n, n, n))
    uh = np.stack([np.fft.rfftn(v[c]) / n ** 3 for c in range(3)])
    m = np.fft.fftfreq(n, 1.0 / n)
    mz, my, mx = m[:, None, None], m[None, :, None], np.arange(n // 2 + 1)[None, None, :]
    k2 = mz * mz + my * my + mx * mx
    kd = mx * uh[0] + my * uh[1] + mz * uh[2]
    k = (mx, my, mz)
    uh = np.stack([uh[c] - k[c] * kd / np.where(k2 > 0, k2, 1) for c in range(3)])
    uh[:, 0, 0, 0] = 0
    uh[:, n // 2], uh[:, :, n // 2], uh[..., n // 2] = 0, 0, 0
    # physical gradients by the library inverse FFT: A[..., i, j] = d_j u_i
    A = np.zeros((n, n, n, 3, 3))
    for i in range(3):
        for j in range(3):
            A[..., i, j] = np.fft.irfftn(1j * k[j] * uh[i], s=(n, n, n), axes=(0, 1, 2)) * n ** 3
    return uh, A


def test_aliased_field_statistics_from_matrix_invariants(orc):
    """Q and R as the coefficients of the characteristic polynomial of A
    (eigenvalues, determinant; lambda^3 + Q lambda + R = 0 for Tr A = 0), and
    eps = nu (|A|^2 - 2Q), omega^2 = |A|^2 + 2Q from A = S + W: the oracle's
    counts (bins and under/overflow slots) and moment sums must agree.  The
    field breaks every symmetry that would hide a wrong sign, a transposed
    index or a swapped strain/rotation part."""
    n, nu = 16, 0.05
    uh, A = aliased_field(n, 11)
    ev = np.linalg.eigvals(A)
    Q = np.real(ev[..., 0] * ev[..., 1] + ev[..., 1] * ev[..., 2] + ev[..., 2] * ev[..., 0])
    R = -np.linalg.det(A)
    F2 = np.sum(A * A, axis=(-2, -1))
    eps = nu * (F2 - 2 * Q)
    ens = F2 + 2 * Q
    eps_ref, nu_ref = 0.7, nu
    tau, trs = np.sqrt(nu_ref / eps_ref), eps_ref / (2 * nu_ref)
    qs, rs = (Q / trs).ravel(), (R / trs ** 1.5).ravel()
    es, ws = (eps / eps_ref).ravel(), (ens * nu_ref / eps_ref).ravel()
    diag = np.stack([A[..., i, i] for i in range(3)]).ravel() * tau
    off = np.stack([A[..., i, j] for i in range(3) for j in range(3) if i != j]).ravel() * tau
    # (sum Q vanishes on the grid for any solenoidal field with |m_i| < n/2; sum R does not)
    assert abs(np.sum(rs)) > 1e-2 * np.sum(np.abs(rs))

    def rng_of(v, lo_q, hi_q, nb):        # a range inside the data, off the grid of bin edges
        lo, hi = np.quantile(v, [lo_q, hi_q])
        return float(lo) - 0.123e-3 * (hi - lo), float(hi) + 0.0371e-3 * (hi - lo)

    q_lo, q_hi = rng_of(qs, 0.08, 0.93, 12)
    r_lo, r_hi = rng_of(rs, 0.06, 0.91, 12)
    lg = np.log10(np.concatenate([es, ws]))
    l_lo, l_hi = rng_of(lg, 0.05, 0.95, 40)
    a_lo, a_hi = rng_of(np.concatenate([diag, off]), 0.04, 0.97, 30)
    h = orc.Hist(qr_bins=12, q_lo=q_lo, q_hi=q_hi, r_lo=r_lo, r_hi=r_hi, log_bins=40, log10_lo=l_lo,
                 log10_hi=l_hi, a_bins=30, a_lo=a_lo, a_hi=a_hi, eps_ref=eps_ref, nu_ref=nu_ref)
    counts, mom, near, trmax = orc.stats(orc.Member(n=n, nu=nu, eps=0.1), h, uh)
    assert np.all(near == 0)
    got = h.split(counts)
    # QR joint histogram and its outside slot
    bq, br = bin_rule(qs, q_lo, q_hi, 12), bin_rule(rs, r_lo, r_hi, 12)
    inside = (bq >= 0) & (br >= 0)
    assert np.array_equal(got["qr"].ravel(), np.bincount(bq[inside] * 12 + br[inside], minlength=144))
    assert got["qr_special"][0] == np.sum(~inside) > 0
    # log histograms, under- and overflow
    for name, v in (("log_eps", es), ("log_ens", ws)):
        b = bin_rule(np.log10(v), l_lo, l_hi, 40)
        assert np.array_equal(got[name], np.bincount(b[b >= 0], minlength=40)), name
        assert got[name + "_special"][0] == np.sum(b == -1) > 0, name
        assert got[name + "_special"][1] == np.sum(b == -2) > 0, name
    # pooled components, under- and overflow
    for name, v in (("a_long", diag), ("a_trans", off)):
        b = bin_rule(v, a_lo, a_hi, 30)
        assert np.array_equal(got[name], np.bincount(b[b >= 0], minlength=30)), name
        assert got[name + "_special"][0] == np.sum(b == -1) > 0, name
        assert got[name + "_special"][1] == np.sum(b == -2) > 0, name
    # moment sums
    close = lambda a, b, scale: abs(a - b) <= 1e-11 * scale
    for p in range(1, 7):
        assert close(mom[p - 1], np.sum(diag ** p), np.sum(np.abs(diag) ** p)), p
        assert close(mom[5 + p], np.sum(off ** p), np.sum(np.abs(off) ** p)), p
    for p in range(1, 5):
        assert close(mom[11 + p], np.sum(es ** p), np.sum(es ** p)), p
        assert close(mom[15 + p], np.sum(ws ** p), np.sum(ws ** p)), p
    assert close(mom[20], np.sum(qs), np.sum(np.abs(qs)))
    assert close(mom[21], np.sum(rs), np.sum(np.abs(rs)))
    assert close(mom[22], np.sum(eps) / (2 * nu) * tau ** 2, np.sum(eps) / (2 * nu) * tau ** 2)
    assert close(mom[24], np.sum(qs ** 2), np.sum(qs ** 2))
    assert close(mom[25], np.sum(rs ** 2), np.sum(rs ** 2))
    assert mom[23] <= 1e-24 * np.sum(F2) * tau ** 2 and trmax <= 1e-12 * np.sqrt(np.max(F2))


def test_zero_gradient_sits_in_the_first_bin_of_a_range_starting_at_zero(orc):
    """The bin rule takes x = lo into bin 0 (x < lo is underflow)."""
    n = 16
    u = np.zeros((3, n, n, n // 2 + 1), complex)
    h = orc.Hist(qr_bins=8, q_lo=0.0, q_hi=1, r_lo=0.0, r_hi=1, log_bins=8, a_bins=8, a_lo=0.0, a_hi=1)
    counts, _, _, _ = orc.stats(orc.Member(n=n, nu=0.01, eps=1.0), h, u)
    got = h.split(counts)
    assert got["qr"][0, 0] == n ** 3 and got["qr_special"][0] == 0
    assert got["a_long"][0] == 3 * n ** 3 and got["a_long_special"][0] == 0
    assert got["a_trans"][0] == 6 * n ** 3 and got["a_trans_special"][0] == 0
