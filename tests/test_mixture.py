"""Pins of the oracle's ensemble-mixture arithmetic against the paper's printed
numbers (tests/golden/paper_values.json), closed forms and quadrature."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import mixture as mx

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
C = GOLD["c_quadratic"]["value"]


def paper_lambda_grid():
    """Reading of the ens256 lambda grid: lambda_i = i ln2/3, i = -22..25."""
    return [i * math.log(2) / 3 for i in range(-22, 26)]


def test_lambda_grid_reading_matches_printed_description():
    lam = paper_lambda_grid()
    assert len(lam) == GOLD["ens256_members"]["value"]
    lo, hi = GOLD["ens256_lambda_range"]["value"]
    assert round(min(lam), 1) == lo and round(max(lam), 1) == hi
    assert round(lam[1] - lam[0], 2) == GOLD["ens256_dlambda"]["value"]
    assert any(round(l, 2) == GOLD["tail_member_lambda"]["value"] for l in lam)
    # k_M eta scales as eps^(-1/4) = exp(-lambda/4) at fixed nu
    k0 = GOLD["ens256_kmeta_central"]["value"]
    kmin, kmax = GOLD["ens256_kmeta_range"]["value"]
    assert abs(k0 * math.exp(-max(lam) / 4) - kmin) / kmin < 0.02
    assert abs(k0 * math.exp(-min(lam) / 4) - kmax) / kmax < 0.01


@pytest.mark.parametrize("Z", [math.log(2), math.log(4), math.log(8), 3.0])
def test_gaussian_satisfies_mean_injection_constraint(Z):
    """int P(lambda; Z) dlambda = 1 and int P(lambda; Z) e^lambda dlambda = 1."""
    norm, _ = integrate.quad(lambda l: mx.lambda_pdf(l, C, Z), -40, 40, limit=200)
    inj, _ = integrate.quad(lambda l: mx.lambda_pdf(l, C, Z) * math.exp(l), -40, 40, limit=200)
    assert abs(norm - 1) < 1e-12 and abs(inj - 1) < 1e-10


def test_gaussian_convolution_property():
    """P(.; 2Z) = P(.; Z) * P(.; Z) (numerical convolution)."""
    Z = 1.3
    x = np.linspace(-12, 12, 4801)
    h = x[1] - x[0]
    p = np.array([mx.lambda_pdf(v, C, Z) for v in x])
    conv = np.convolve(p, p, mode="same") * h
    ref = np.array([mx.lambda_pdf(v, C, 2 * Z) for v in x])
    assert np.max(np.abs(conv - ref)) < 1e-6 * ref.max()


def test_moment_generating_function_is_the_quadratic_cumulant():
    """log int P e^(t lambda) = 9c(t^2 - t)Z/2 for the quadratic exponents."""
    Z = 2.0
    for t in (0.5, 1.0, 2.0, 3.0):
        m, _ = integrate.quad(lambda l: mx.lambda_pdf(l, C, Z) * math.exp(t * l), -60, 60, limit=400)
        assert abs(math.log(m) - 9 * C * (t * t - t) * Z / 2) < 1e-9


def test_weights_sum_to_one_and_delta_limit():
    lam = paper_lambda_grid()
    w = mx.weights(lam, C, math.log(8))
    assert abs(sum(w) - 1) < 1e-14
    w0 = mx.weights(lam, C, 0.0)
    assert w0[lam.index(0.0)] == 1 and sum(w0) == 1
    wsmall = mx.weights(lam, C, 1e-6)
    assert wsmall[lam.index(0.0)] > 1 - 1e-12


def test_delta_limit_on_a_bin_edge_goes_to_the_upper_bin():
    """P(lambda; 0) is a point mass at lambda = 0 and the bins are half-open,
    [a, b): with 0 on the edge between two members the whole weight goes to
    the member above the edge."""
    for mode in (0, 1):
        assert mx.weights([-1.0, 1.0], C, 0.0, mode=mode) == [0.0, 1.0]
        assert mx.weights([1.0, -1.0, 3.0], C, 0.0, mode=mode) == [1.0, 0.0, 0.0]


def test_tail_member_bin_mass_matches_paper():
    """Bin mass of the lambda = 3.93 member at R_lambda = 1300, c = 0.023.  Z from
    R_lambda ~ exp(2Z/3) through the 2048^3 reference (R = 261 at Z = log 8)."""
    g = GOLD["tail_member_bin_mass"]
    lam = paper_lambda_grid()
    Z = mx.z_from_rlambda(g["rlambda"], 261.0, math.log(8))
    w = mx.weights(lam, g["c"], Z)
    i = min(range(len(lam)), key=lambda j: abs(lam[j] - 3.93))
    assert float(f"{w[i]:.1e}") == g["value"]


def test_erfc_tails_keep_digits_far_out():
    lam = [0.0, 10.0, 11.0]
    w = mx.weights(lam, C, 1.0)
    mu, sig = mx.gaussian_params(C, 1.0)
    exact = 0.5 * math.erfc((10.5 - mu) / (sig * math.sqrt(2)))
    assert w[2] == pytest.approx(exact, rel=1e-13) and w[2] > 0


def test_closed_end_bins_renormalise():
    lam = [-1.0, 0.0, 1.0]
    w = mx.weights(lam, C, 2.0, mode=1)
    assert abs(sum(w) - 1) < 1e-15
    e = mx.cell_edges(lam, mode=1)
    assert e[0] == (-1.5, -0.5) and e[2] == (0.5, 1.5)


def test_importance_weights_estimate_the_injection_constraint():
    rng = np.random.default_rng(3)
    lam = list(rng.normal(0, math.sqrt(2), 20000))
    w = mx.weights(lam, C, math.log(8), mode=2, q_sigma=math.sqrt(2))
    est = sum(wi * math.exp(l) for wi, l in zip(w, lam))
    assert abs(est - 1) < 0.03


def test_mixture_of_identical_members_is_that_member():
    pdf = [0.1, 0.5, 0.3, 0.1]
    lam = paper_lambda_grid()
    w = mx.weights(lam, C, math.log(4))
    out = mx.mix(w, [pdf] * len(lam))
    assert np.allclose(out, pdf, rtol=0, atol=1e-15)
    # skewness from mixed moments of identical members is the member's
    m2, m3 = mx.mix(w, [[2.0, -1.0]] * len(lam))
    assert abs(mx.skewness(m2, m3) - (-1.0 / 2.0 ** 1.5)) < 1e-15


# Skewness, flatness and hyper-flatness (section "Modeling choices",
# eq. def_skewness_flatness) of zero-mean variables whose moments are fixed by
# mathematics.  The moments come from scipy's distributions (not from the ratio
# formulas under test); scales other than 1 make a wrong power of m2 visible.
@pytest.mark.parametrize("dist, S, F, H", [
    (stats.norm(scale=1.7), 0.0, 3.0, 15.0),                  # Gaussian: 3 = 3!!, 15 = 5!!
    (stats.expon(loc=-0.6, scale=0.6), 2.0, 9.0, 265.0),      # centred exponential: subfactorials !3, !4, !6
    (stats.laplace(scale=2.3), 0.0, 6.0, 90.0),               # 4!/2^2, 6!/2^3
    (stats.uniform(loc=-1.9, scale=3.8), 0.0, 9.0 / 5.0, 27.0 / 7.0),
])
def test_moment_ratios_of_known_distributions(dist, S, F, H):
    assert abs(dist.mean()) < 1e-14
    m2, m3, m4, m6 = (float(dist.moment(p)) for p in (2, 3, 4, 6))
    assert abs(mx.skewness(m2, m3) - S) <= 1e-12
    assert abs(mx.flatness(m2, m4) - F) <= 1e-12 * F
    assert abs(mx.hyperflatness(m2, m6) - H) <= 1e-8 * H      # scipy's 6th moment of the shifted exponential: 3e-9
    sk, ek = dist.stats(moments="sk")
    assert abs(mx.skewness(m2, m3) - float(sk)) <= 1e-12
    assert abs(mx.flatness(m2, m4) - (3.0 + float(ek))) <= 1e-12 * F


def test_moment_ratios_match_sample_statistics():
    """On a skewed sample (centred), the ratios of its central moments equal
    scipy's sample skewness and (Pearson) kurtosis."""
    rng = np.random.default_rng(11)
    x = rng.gamma(2.0, 1.5, 200000)
    x = x - x.mean()
    m2, m3, m4 = (float(np.mean(x ** p)) for p in (2, 3, 4))
    assert abs(mx.skewness(m2, m3) - float(stats.skew(x))) <= 1e-12
    assert abs(mx.flatness(m2, m4) - float(stats.kurtosis(x, fisher=True) + 3.0)) <= 1e-10


def test_cost_saving_matches_paper():
    g = GOLD["cost_saving"]
    r = mx.cost_ratio(g["rlambda_ref"], g["rlambda_ens"], g["n"])
    assert float(f"{r:.1e}") == g["value"]


# ---------------------------------------------------------------- truncated Gaussian (appendix)
@pytest.mark.parametrize("Z", [0.05, math.log(2), math.log(8), 3.0, 6.0])
def test_truncated_gaussian_is_normalised_and_conserves_injection(Z):
    """eq. (truncated_gaussian): int P = 1 and int P e^lambda = 1 (quadrature of the
    density itself, independent of the closed-form root condition)."""
    mu, sig = mx.truncated_params(C, Z)
    assert abs(sig * sig - 9 * C * Z) <= 1e-15 * max(1.0, 9 * C * Z)
    lo = mu - 40 * sig
    norm, _ = integrate.quad(lambda l: mx.truncated_pdf(l, C, Z), lo, Z, limit=400, epsabs=1e-14, epsrel=1e-13)
    inj, _ = integrate.quad(lambda l: mx.truncated_pdf(l, C, Z) * math.exp(l), lo, Z, limit=400, epsabs=1e-14,
                            epsrel=1e-13)
    assert abs(norm - 1) < 1e-11 and abs(inj - 1) < 1e-11
    assert mx.truncated_pdf(Z + 1e-9, C, Z) == 0.0


def test_truncated_gaussian_reduces_to_the_gaussian_when_the_cut_is_far():
    """c -> 0 at fixed Z puts the cut many sigma above the mean: mu -> -sigma^2/2."""
    for c in (1e-4, 1e-3):
        mu, sig = mx.truncated_params(c, 2.0)
        g_mu, g_sig = mx.gaussian_params(c, 2.0)
        assert abs(mu - g_mu) <= 1e-12 and sig == g_sig
    # at the paper's c the cut moves the mean up, and less for larger Z relative to sigma
    mu2, s2 = mx.truncated_params(C, math.log(2))
    assert mu2 > mx.gaussian_params(C, math.log(2))[0]


def test_truncated_gaussian_cgf_slope_saturates_at_Z():
    """d/dt K(t; Z) tends to the upper end of the support, lambda_max = Z (appendix).
    K'(t) is the mean of the tilted density, a normal of mean mu + t sigma^2 cut at
    Z: scipy's truncated normal gives it; quadrature checks it at moderate t; for
    large t it approaches Z as Z - s2/D + 2 s2^2/D^3, D = mu + t s2 - Z, s2 = sigma^2
    (the asymptotic series of the normal's Mills ratio)."""
    from scipy.stats import truncnorm
    Z = math.log(4)
    mu, sig = mx.truncated_params(C, Z)
    prev = -math.inf
    for t in (0.5, 1.0, 10.0, 100.0, 1000.0):
        m = mu + t * sig * sig
        with np.errstate(invalid="ignore"):
            k1 = float(truncnorm(-np.inf, (Z - m) / sig, loc=m, scale=sig).stats(moments="m"))
        if t <= 10:
            num, _ = integrate.quad(lambda l: l * mx.truncated_pdf(l, C, Z) * math.exp(t * (l - Z)), mu - 40 * sig, Z,
                                    limit=400, epsabs=0, epsrel=1e-10)
            den, _ = integrate.quad(lambda l: mx.truncated_pdf(l, C, Z) * math.exp(t * (l - Z)), mu - 40 * sig, Z,
                                    limit=400, epsabs=0, epsrel=1e-10)
            assert abs(num / den - k1) < 1e-9
        assert prev < k1 < Z
        prev = k1
        if t >= 100:
            D, s2 = m - Z, sig * sig
            tol = 20 * s2 ** 3 / D ** 5 + 1e-12 if t <= 100 else 1e-7   # scipy's far-tail mean: ~1e-8
            assert abs((Z - k1) - (s2 / D - 2 * s2 * s2 / D ** 3)) < tol
    assert prev > Z - 1.1e-3


def test_truncated_weights_are_bin_masses_of_the_density():
    """Mode 3 weights = quadrature of the truncated density over each member's bin;
    members above the cut get nothing; they sum to 1."""
    lam = paper_lambda_grid()
    for Z in (math.log(2), math.log(8)):
        w = mx.weights(lam, C, Z, mode=3)
        assert abs(sum(w) - 1) < 1e-14
        edges = mx.cell_edges(lam, 0)
        mu, sig = mx.truncated_params(C, Z)
        for (a, b), wi, l in zip(edges, w, lam):
            if a >= Z:
                assert wi == 0.0
                continue
            lo = max(a, mu - 40 * sig)
            hi = min(b, Z)
            ref, _ = integrate.quad(lambda x: mx.truncated_pdf(x, C, Z), lo, hi, epsabs=1e-16, epsrel=1e-12) \
                if hi > lo else (0.0, 0.0)
            assert abs(wi - ref) <= 1e-12 * max(ref, 1e-300) + 1e-17, (l, wi, ref)
    assert mx.weights(lam, C, 0.0, mode=3)[lam.index(0.0)] == 1.0


# ---------------------------------------------------------------- scale gap from R_lambda
def test_rlambda_from_means_closed_form():
    """u' = 1, eps = 15 nu gives lambda_T = 1 and R_lambda = 1/nu."""
    nu = 0.01
    assert abs(mx.rlambda_from_means(1.5, 15 * nu, nu) - 1 / nu) < 1e-12


def test_prefactor_fit_recovers_an_exact_power_law_and_ignores_negative_lambda():
    lam = paper_lambda_grid()
    A = 63.0
    rls = [A * math.exp(l / 6) * (1.0 if l >= 0 else 7.0) for l in lam]   # lambda < 0 members must not count
    assert abs(mx.rlambda_prefactor(lam, rls) - A) < 1e-12 * A
    # log-least-squares with fixed slope: geometric mean of R e^(-lambda/6) over lambda >= 0
    rls2 = [A * math.exp(l / 6) * (1.1 if i % 2 else 1 / 1.1) for i, l in enumerate(lam)]
    sel = [(l, r) for l, r in zip(lam, rls2) if l >= 0]
    gm = math.exp(sum(math.log(r) - l / 6 for l, r in sel) / len(sel))
    assert abs(mx.rlambda_prefactor(lam, rls2) - gm) < 1e-12 * gm
    with pytest.raises(ValueError):
        mx.rlambda_prefactor([-1.0, -0.5], [10.0, 12.0])


def test_scale_gap_reproduces_the_reference_table():
    """Table II from Table I's central member: the ens256 centre (R = 63, box 4 pi)
    against references in boxes 8, 16, 32 pi (Z = ln 2, ln 4, ln 8) predicts
    R_lambda,ref = 63 e^(2Z/3) = 100, 159, 252 against the printed 103, 173, 261
    (within 10 %: the printed centre is one member, not the fit); an exponent of
    1/3 or 4/3 instead of 2/3 would miss by a factor 1.3-16."""
    r_ens = GOLD["ens256_rlambda_central"]["value"]
    for Z, r_ref in zip((math.log(2), math.log(4), math.log(8)), GOLD["reference_rlambda"]["value"]):
        z = mx.scale_gap(r_ref, r_ens)
        assert abs(z - Z) < 0.15
        assert abs(r_ens * math.exp(2 * Z / 3) - r_ref) / r_ref < 0.10
    assert mx.scale_gap(r_ens, r_ens) == 0.0


# ---------------------------------------------------------------- lambda density from the CGF
def test_cf_inversion_of_the_quadratic_cgf_is_the_gaussian():
    """exp(K(i omega; Z)) with K = 9cZ (t^2 - t)/2 (quadratic exponents) inverts to
    the Gaussian of eq. (gaussian_lambda_pdf)."""
    Z, M, h, lam0 = math.log(8), 1024, 0.02, -10.24
    om = mx.cf_omegas(M, h)
    t = 1j * om
    phi = np.exp(9 * C * Z * (t * t - t) / 2)
    pdf = mx.lambda_pdf_from_cf(phi, lam0, h)
    lam = lam0 + h * np.arange(M)
    ref = np.array([mx.lambda_pdf(l, C, Z) for l in lam])
    assert np.max(np.abs(pdf - ref)) < 1e-12 * ref.max()


def test_cf_inversion_of_a_shifted_gamma_cgf():
    """A skewed family with K linear in Z and K(1; Z) = 0: lambda = s - G with G
    Gamma-distributed (shape aZ, rate b), K(t) = aZ [t ln(1 + 1/b) - ln(1 + t/b)];
    scipy's gamma density gives the exact P."""
    from scipy import stats
    a, b, Z = 3.0, 4.0, 1.5
    s = a * Z * math.log(1 + 1 / b)
    M, h, lam0 = 4096, 0.005, -12.0
    t = 1j * mx.cf_omegas(M, h)
    phi = np.exp(a * Z * (t * math.log(1 + 1 / b) - np.log(1 + t / b)))
    pdf = mx.lambda_pdf_from_cf(phi, lam0, h)
    lam = lam0 + h * np.arange(M)
    ref = stats.gamma(a * Z, scale=1 / b).pdf(s - lam)
    assert np.max(np.abs(pdf - ref)) < 2e-6 * ref.max()          # the density's kink-free tail limits the rule
    # injection constraint of the exact density
    inj, _ = integrate.quad(lambda x: stats.gamma(a * Z, scale=1 / b).pdf(s - x) * math.exp(x), -40, s, limit=200)
    assert abs(inj - 1) < 1e-10


def test_table_weights_integrate_the_piecewise_linear_density():
    """A triangle density on [0, 2] tabulated exactly: bins integrate it exactly."""
    h, lam0 = 0.5, -1.0
    pdf = [0.0, 0.0, 0.0, 0.5, 1.0, 0.5, 0.0, -0.1]         # lambda = -1 .. 2.5; last sample clamps to 0
    lams = [0.25, 1.0, 1.75]
    w = mx.weights_from_table(lams, pdf, lam0, h)
    # bins (-inf, 0.625), [0.625, 1.375), [1.375, inf); triangle area 1
    F = lambda x: 0.0 if x <= 0 else (x * x / 2 if x <= 1 else (1 - (2 - x) ** 2 / 2 if x < 2 else 1.0))
    ref = [F(0.625), F(1.375) - F(0.625), 1 - F(1.375)]
    assert np.allclose(w, ref, rtol=1e-15, atol=1e-16)


def test_table_weights_of_the_gaussian_table_approach_the_gaussian_bin_masses():
    lam = paper_lambda_grid()
    Z, h, lam0 = math.log(8), 0.001, -12.0
    grid = lam0 + h * np.arange(24001)
    pdf = [mx.lambda_pdf(l, C, Z) for l in grid]
    w = mx.weights_from_table(lam, pdf, lam0, h)
    ref = mx.weights(lam, C, Z, mode=0)
    assert np.max(np.abs(np.array(w) - ref)) < 1e-7
