"""FP32 and FP64 runs of the same member agree statistically: mean dissipation
and the QR-PDF, with bias-corrected and accelerated (BCa) bootstrap intervals
over non-overlapping windows of about one integral time (the error-bar
procedure the paper uses for its reference data, Fig. 4 and Fig. 8 captions).
Both runs start from the same seeded field and decorrelate by chaos; the
two-sample bootstrap compares their window means."""
import math

import numpy as np
import pytest
from scipy import stats as sps

pytestmark = pytest.mark.gpu

N, NU, EPS, DT = 64, 0.03, 1.0, 0.005
TRANSIENT, WINDOW, NWIN, EVERY = 1000, 200, 24, 10
HK = dict(qr_bins=96, q_lo=-6.0, q_hi=6.0, r_lo=-6.0, r_hi=6.0, log_bins=256, log10_lo=-6.0,
          log10_hi=3.0, a_bins=256, a_lo=-20.0, a_hi=20.0, eps_ref=EPS, nu_ref=NU)


def integral_time(orc, uhat):
    """T = L/u' with L = (pi / (2 u'^2)) sum_k E(k)/k and u'^2 = 2E/3 (shell sums)."""
    mz, my, mx = orc.modes(N)
    k = np.sqrt((mz * mz + my * my + mx * mx).astype(float))
    w = np.ones(N // 2 + 1); w[1:] = 2
    e_mode = 0.5 * np.sum(np.abs(uhat) ** 2, axis=0) * w
    E = e_mode.sum()
    up2 = 2 * E / 3
    L = math.pi / (2 * up2) * np.sum(e_mode[k > 0] / k[k > 0])
    return L / math.sqrt(up2)


def test_fp32_and_fp64_statistics_agree_within_bootstrap_intervals(orc):
    import paper_2506_23712_amd as ens
    h = ens.HistSpec(**HK)
    E = ens.Ensemble(hist=h)
    m64 = E.add_member(ens.MemberSpec(n=N, nu=NU, eps_ref=EPS, kf_hi=2.5, dt=DT, precision="fp64", seed=9))
    m32 = E.add_member(ens.MemberSpec(n=N, nu=NU, eps_ref=EPS, kf_hi=2.5, dt=DT, precision="fp32", seed=9))
    E.step(TRANSIENT)
    T = integral_time(orc, m64.state().cpu().numpy())
    print(f"integral time {T:.3f}, window {WINDOW * DT:.3f}")
    assert 0.4 * T <= WINDOW * DT <= 3.0 * T          # windows of about one integral time
    eps_w = {32: [], 64: []}
    pdf_w = {32: [], 64: []}
    for _ in range(NWIN):
        m64.reset_stats(); m32.reset_stats()
        for s in range(WINDOW // EVERY):
            E.step(EVERY)
            E.accumulate_stats()
        for bits, m in ((64, m64), (32, m32)):
            counts, mom, npts = m.stats()
            eps_w[bits].append(mom[12].item() / npts * EPS)
            qr = h.split(counts.numpy())["qr"].astype(float)
            pdf_w[bits].append(qr / npts)
    E.close()
    rng = np.random.default_rng(0)
    e32, e64 = np.array(eps_w[32]), np.array(eps_w[64])
    # stationary mean dissipation equals the injection rate (within the window scatter)
    for e in (e32, e64):
        ci = sps.bootstrap((e,), np.mean, method="BCa", confidence_level=0.99, random_state=rng).confidence_interval
        assert ci.low <= EPS * 1.15 and ci.high >= EPS * 0.85, ci
    diff = sps.bootstrap((e32, e64), lambda a, b: np.mean(a) - np.mean(b), method="BCa", confidence_level=0.95,
                         random_state=rng).confidence_interval
    print(f"<eps> fp32 {e32.mean():.4f}  fp64 {e64.mean():.4f}  95% BCa CI of difference [{diff.low:.4f}, {diff.high:.4f}]")
    assert diff.low <= 0.0 <= diff.high
    # QR-PDF: bins holding >= 0.05% of the samples; 99% BCa intervals of the difference
    p32, p64 = np.array(pdf_w[32]), np.array(pdf_w[64])
    mean_p = 0.5 * (p32.mean(0) + p64.mean(0))
    bins = np.argwhere(mean_p >= 5e-4)
    inside = 0
    for (i, j) in bins:
        a, b = p32[:, i, j], p64[:, i, j]
        ci = sps.bootstrap((a, b), lambda x, y: np.mean(x) - np.mean(y), method="BCa", confidence_level=0.99,
                           random_state=rng).confidence_interval
        inside += ci.low <= 0.0 <= ci.high
    frac = inside / len(bins)
    print(f"QR-PDF: {len(bins)} bins tested, {inside} with 0 inside the 99% interval ({frac:.3f})")
    assert len(bins) >= 30 and frac >= 0.95
