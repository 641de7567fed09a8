"""Pins of the oracle's ensemble-mixture arithmetic against the paper's printed
numbers (tests/golden/paper_values.json), closed forms and quadrature."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

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


def test_cost_saving_matches_paper():
    g = GOLD["cost_saving"]
    r = mx.cost_ratio(g["rlambda_ref"], g["rlambda_ens"], g["n"])
    assert float(f"{r:.1e}") == g["value"]
