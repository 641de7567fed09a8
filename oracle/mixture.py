"""Ensemble mixture of member statistics (oracle side, FP64, plain Python).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows arXiv 2506.23712:
  * ensemble hypothesis, eq. (ensemble_hypothesis): a statistic at scale gap Z
    is the average over lambda, weighted by P(lambda; Z), of the statistic of a
    member with injection e^lambda * eps_bar;
  * PDFs superpose the same way, eq. (pdf_superposition);
  * quadratic (log-normal) exponents zeta_p = p/3 - c (p^2 - 3p)/2,
    eq. (quadratic_scaling_exponents), give a Gaussian P(lambda; Z) with mean
    -9cZ/2 and variance 9cZ, eq. (gaussian_lambda_pdf);
  * each member is given the probability mass of its lambda bin (the sentence
    after eq. gaussian_lambda_pdf); any average is then a weighted sum;
  * skewness / flatness predictions are ratios of mixed moments
    (section "Modeling choices", eq. def_skewness_flatness and the skewness
    prediction that follows it);
  * Z follows R_lambda,ref ~ exp(2Z/3), eq. (Rlambda_Z_relation).

Readings (the paper is silent): members are sorted by lambda and the bin of a
member is bounded by the midpoints to its neighbours; the two end bins are open
to -inf / +inf (mode 0), or closed at half a spacing and renormalised (mode 1);
mode 2 is self-normalised importance weighting P(lambda_i; Z) / q(lambda_i) for
members whose lambda were drawn from a normal density q; mode 3 takes the bin
masses (open end bins) of the truncated Gaussian of the appendix,
eq. (truncated_gaussian): variance 9cZ, support lambda <= Z, its mean mu(Z) the
root of the mean-injection constraint (eq. mean_injection_constraint).

The scale gap from a target Reynolds number (section "Benchmarking the method
against DNS data", eq. Rlambda_Z_relation): with C_eps constant, eq.
(Re_definition) at fixed L and nu gives Re ~ e^(lambda/3) across the members, and
R_lambda ~ Re^(1/2) ~ e^(lambda/6).  Fitting C_eps to the members with
lambda >= 0 is then a fit of A in R_lambda = A e^(lambda/6) (slope fixed, least
squares in log R_lambda); the reference at scale gap Z has Re larger by
e^(4Z/3), so R_lambda,ref = A e^(2Z/3) and Z = (3/2) ln(R_lambda,ref / A).
A member's R_lambda is formed from its time-averaged energy and dissipation,
R_lambda = (2<E>/3) sqrt(15 / (nu <D>)).
"""
from __future__ import annotations

import math
from typing import Sequence


def gaussian_params(c: float, Z: float) -> tuple[float, float]:
    """(mean, standard deviation) of P(lambda; Z) for quadratic exponents."""
    return -4.5 * c * Z, math.sqrt(9.0 * c * Z)


def lambda_pdf(lam: float, c: float, Z: float) -> float:
    """P(lambda; Z), eq. (gaussian_lambda_pdf)."""
    mu, sig = gaussian_params(c, Z)
    return math.exp(-(lam - mu) ** 2 / (2.0 * sig * sig)) / (sig * math.sqrt(2.0 * math.pi))


def _mass(a: float, b: float, mu: float, sig: float) -> float:
    """Normal probability of [a, b); tails use erfc so small masses keep their digits."""
    r = 1.0 / (sig * math.sqrt(2.0))

    def upper(x):   # P(X >= x)
        return 0.5 * math.erfc((x - mu) * r) if x != math.inf else 0.0

    def lower(x):   # P(X < x)
        return 0.5 * math.erfc((mu - x) * r) if x != -math.inf else 0.0

    if a >= mu:
        return upper(a) - upper(b)
    if b <= mu:
        return lower(b) - lower(a)
    return 1.0 - lower(a) - upper(b)


def _phi(x: float) -> float:
    """Standard normal distribution function."""
    return 0.5 * math.erfc(-x / math.sqrt(2.0))


def truncated_params(c: float, Z: float) -> tuple[float, float]:
    """(mu, sigma) of the truncated Gaussian, eq. (truncated_gaussian): sigma^2 = 9cZ
    and mu(Z) such that the density N exp(-(lambda - mu)^2 / (2 sigma^2)) on
    lambda <= Z has int P e^lambda = 1.  For a normal truncated at Z,
    int P e^lambda = exp(mu + sigma^2/2) Phi((Z - mu - sigma^2)/sigma) / Phi((Z - mu)/sigma);
    its logarithm g(mu) grows with mu, is negative at mu = -sigma^2/2 (the
    untruncated root) and tends to Z > 0 as mu grows: bisection on it."""
    if Z <= 0.0:
        return 0.0, 0.0
    sig = math.sqrt(9.0 * c * Z)
    s2 = sig * sig

    def g(mu):
        return mu + 0.5 * s2 + math.log(_phi((Z - mu - s2) / sig)) - math.log(_phi((Z - mu) / sig))

    lo = -0.5 * s2
    step = max(sig, 1e-3)
    hi = lo + step
    while g(hi) <= 0.0:
        lo, hi = hi, hi + step
        step *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if g(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi), sig


def truncated_pdf(lam: float, c: float, Z: float) -> float:
    """P(lambda; Z) of eq. (truncated_gaussian), normalised on lambda <= Z."""
    mu, sig = truncated_params(c, Z)
    if lam > Z:
        return 0.0
    return math.exp(-(lam - mu) ** 2 / (2 * sig * sig)) / (sig * math.sqrt(2 * math.pi) * _phi((Z - mu) / sig))


def cell_edges(lams: Sequence[float], mode: int = 0) -> list[tuple[float, float]]:
    """Bin [a_i, b_i) of each member (input order kept)."""
    order = sorted(range(len(lams)), key=lambda i: lams[i])
    s = [lams[i] for i in order]
    n = len(s)
    edges = [None] * n
    for r in range(n):
        a = 0.5 * (s[r - 1] + s[r]) if r > 0 else None
        b = 0.5 * (s[r] + s[r + 1]) if r < n - 1 else None
        if a is None:
            a = -math.inf if (mode == 0 or n == 1) else s[r] - (b - s[r])
        if b is None:
            b = math.inf if (mode == 0 or n == 1) else s[r] + (s[r] - a)
        edges[order[r]] = (a, b)
    return edges


def weights(lams: Sequence[float], c: float, Z: float, mode: int = 0,
            q_sigma: float | None = None) -> list[float]:
    """Mixture weight of each member (same order as ``lams``)."""
    n = len(lams)
    if n == 0:
        return []
    if mode == 2:
        if Z <= 0:
            raise ValueError("importance weights need Z > 0")
        mu, sig = gaussian_params(c, Z)
        raw = []
        for l in lams:
            p = math.exp(-(l - mu) ** 2 / (2 * sig * sig)) / sig
            q = math.exp(-l * l / (2 * q_sigma * q_sigma)) / q_sigma
            raw.append(p / q)
        s = sum(raw)
        return [r / s for r in raw]
    edges = cell_edges(lams, 0 if mode == 3 else mode)
    if Z <= 0.0:                       # P(lambda; 0) = delta(lambda)
        return [1.0 if (a <= 0.0 < b) else 0.0 for a, b in edges]
    if mode == 3:                      # truncated Gaussian: mass of [a, b) cut at Z
        mu, sig = truncated_params(c, Z)
        tot = _mass(-math.inf, Z, mu, sig)
        return [(_mass(a, min(b, Z), mu, sig) / tot if a < Z else 0.0) for a, b in edges]
    mu, sig = gaussian_params(c, Z)
    w = [_mass(a, b, mu, sig) for a, b in edges]
    if mode == 1:
        s = sum(w)
        w = [x / s for x in w]
    return w


def z_from_rlambda(r_target: float, r_anchor: float, z_anchor: float) -> float:
    """Scale gap for a target R_lambda, from R_lambda ~ exp(2Z/3) through an anchor."""
    return z_anchor + 1.5 * math.log(r_target / r_anchor)


def lambda_pdf_from_cf(phi, lam0: float, h: float):
    """Density P(lambda) on the grid lambda_j = lam0 + j h (j = 0 .. M-1) from
    samples of its characteristic function phi_k = exp(K(i omega_k; Z)), the
    cumulant generating function (eq. cumulant_generating_function) at imaginary
    argument, omega_k = 2 pi f_k with f_k numpy's FFT frequencies of M points at
    spacing h (section "Modeling choices": the two-sided Laplace transform is
    inverted by a Fourier transform).  P_j = Re sum_k phi_k e^(-i omega_k lambda_j) / (M h):
    the rectangle rule of the inverse Fourier integral, one FFT (numpy's)."""
    import numpy as np
    phi = np.asarray(phi, dtype=np.complex128)
    M = phi.shape[0]
    omega = 2.0 * np.pi * np.fft.fftfreq(M, d=h)
    return np.real(np.fft.fft(phi * np.exp(-1j * omega * lam0))) / (M * h)


def cf_omegas(M: int, h: float):
    """The frequencies omega_k at which lambda_pdf_from_cf expects its samples."""
    import numpy as np
    return 2.0 * np.pi * np.fft.fftfreq(M, d=h)


def weights_from_table(lams: Sequence[float], pdf: Sequence[float], lam0: float, h: float) -> list[float]:
    """Member weights from a tabulated lambda density: negative samples (ringing of
    the Fourier inversion) set to zero, the density linear between samples and
    zero outside the table, each member the integral over its bin (mode-0 bins:
    midpoints, open end bins), normalised by the sum of the bin integrals."""
    p = [max(0.0, float(v)) for v in pdf]
    M = len(p)

    def integral(a, b):
        tot = 0.0
        for s in range(M - 1):
            x0, x1 = lam0 + s * h, lam0 + (s + 1) * h
            lo, hi = max(a, x0), min(b, x1)
            if hi <= lo:
                continue
            f = lambda x: p[s] + (p[s + 1] - p[s]) * (x - x0) / h
            tot += (hi - lo) * 0.5 * (f(lo) + f(hi))
        return tot

    raw = [integral(a, b) for a, b in cell_edges(lams, 0)]
    s = sum(raw)
    return [r / s for r in raw]


def rlambda_from_means(e_mean: float, d_mean: float, nu: float) -> float:
    """Taylor-scale Reynolds number from time-averaged energy and dissipation:
    u'^2 = 2<E>/3, lambda_T = sqrt(15 nu u'^2 / <D>), R_lambda = u' lambda_T / nu."""
    up2 = 2.0 * e_mean / 3.0
    return up2 * math.sqrt(15.0 / (nu * d_mean))


def rlambda_prefactor(lams: Sequence[float], rls: Sequence[float]) -> float:
    """A of R_lambda = A e^(lambda/6), least squares in log over members with lambda >= 0."""
    xs = [math.log(r) - l / 6.0 for l, r in zip(lams, rls) if l >= 0.0]
    if not xs:
        raise ValueError("no member with lambda >= 0")
    return math.exp(sum(xs) / len(xs))


def scale_gap(r_ref: float, prefactor: float) -> float:
    """Z with R_lambda,ref = A e^(2Z/3), eq. (Rlambda_Z_relation)."""
    return 1.5 * math.log(r_ref / prefactor)


def mix(ws: Sequence[float], values: Sequence[Sequence[float]]) -> list[float]:
    """sum_i w_i values_i, elementwise, members summed in the given order."""
    out = [0.0] * len(values[0])
    for w, v in zip(ws, values):
        for j, x in enumerate(v):
            out[j] += w * x
    return out


def skewness(m2: float, m3: float) -> float:
    """S = <x^3> / <x^2>^(3/2) of a zero-mean variable (eq. def_skewness_flatness)."""
    return m3 / m2 ** 1.5


def flatness(m2: float, m4: float) -> float:
    """F = <x^4> / <x^2>^2 of a zero-mean variable (eq. def_skewness_flatness)."""
    return m4 / (m2 * m2)


def hyperflatness(m2: float, m6: float) -> float:
    """H = <x^6> / <x^2>^3 of a zero-mean variable (eq. def_skewness_flatness)."""
    return m6 / (m2 * m2 * m2)


def cost_ratio(r_ref: float, r_ens: float, n: int) -> float:
    """Cost of one full DNS over the cost of the ensemble, (R_ref/R_ens)^5 / n."""
    return (r_ref / r_ens) ** 5 / n
