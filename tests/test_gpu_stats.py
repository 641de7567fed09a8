"""Parity of the gradient statistics and of the ensemble mixture with the oracle."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HK = dict(qr_bins=64, q_lo=-30.0, q_hi=30.0, r_lo=-60.0, r_hi=60.0, log_bins=512, log10_lo=-8.0,
          log10_hi=5.0, a_bins=1024, a_lo=-100.0, a_hi=100.0, eps_ref=0.1, nu_ref=0.02)


# FP32 statistics (FP32 gradient transforms, values and sums in FP64) against
# the oracle's FP64 statistics of the same field.  Gradient errors of FP32
# transforms: about 6e-8 (the FP32 rounding of i k_j u_i) times a few per
# transform pass, relative to the field's largest gradient; the allowance
# for samples near a bin edge takes 1e-5 of max|A_ij| (oracle grad_tol), and
# moment sums, at most sixth powers of those values, agree to 5e-5 of their
# scale.
FP32_GRAD_TOL = 1e-5
FP32_MOMENT_TOL = 5e-5


def moment_scales(rm, npts):
    """Size against which each moment sum is compared.  Sums that vanish by
    symmetry (odd moments, <Q>, <R>, Tr A) are measured against the
    Cauchy-Schwarz bound sqrt(M_(p-1) M_(p+1)) of their absolute sum."""
    sc = np.zeros(26)
    for base, cnt in ((0, 3 * npts), (6, 6 * npts)):
        M = [cnt] + [rm[base + p] for p in range(6)]        # M[p] = sum x^p
        for p in range(1, 7):
            sc[base + p - 1] = abs(M[p]) if p % 2 == 0 else np.sqrt(M[p - 1] * M[p + 1]) if p < 6 else abs(M[p])
        sc[base + 4] = np.sqrt(M[4] * M[6])
    for base in (12, 16):
        sc[base:base + 4] = np.abs(rm[base:base + 4])
    sc[20] = np.sqrt(npts * rm[24]); sc[21] = np.sqrt(npts * rm[25])
    sc[22] = rm[22]; sc[23] = rm[22]; sc[24] = rm[24]; sc[25] = rm[25]
    return sc


def counts_close(got, ref, near):
    """Counts must agree except for points whose bin coordinate sits within
    rounding of an edge (the oracle counts those)."""
    diff = int(np.abs(got.astype(np.int64) - ref.astype(np.int64)).sum())
    assert diff <= 2 * int(near), (diff, int(near))


@pytest.mark.parametrize("n,steps,prec", [(32, 20, "fp64"), (64, 5, "fp64"), (16, 3, "fp64")])
def test_snapshot_statistics_match_oracle(orc, n, steps, prec):
    import paper_2506_23712_amd as ens
    E = ens.Ensemble(hist=ens.HistSpec(**HK))
    spec = ens.MemberSpec(n=n, nu=0.02, eps_ref=0.1, kf_hi=2.0, dt=0.01, seed=3 + n, precision=prec)
    m = E.add_member(spec)
    E.step(steps)
    E.accumulate_stats()
    counts, mom, npts = m.stats()
    state = m.state().cpu().numpy()
    E.close()
    h = orc.Hist(**HK)
    om = orc.Member(n=n, nu=0.02, eps=0.1, kf_hi=2.0, dt=0.01)
    rc, rm, near, _ = orc.stats(om, h, state)           # same field on both sides
    got = h.split(counts.numpy().astype(np.uint64))
    ref = h.split(rc)
    assert npts == n ** 3
    for k, name in enumerate(("qr", "log_eps", "log_ens", "a_long", "a_trans")):
        counts_close(np.concatenate([got[name].ravel(), got[name + "_special"]]),
                     np.concatenate([ref[name].ravel(), ref[name + "_special"]]), near[k])
    m = mom.numpy()
    tol = moment_scales(rm, n ** 3)
    for i in range(26):
        assert abs(m[i] - rm[i]) <= 1e-11 * tol[i], (i, m[i], rm[i], tol[i])


@pytest.mark.parametrize("n,steps", [(32, 20), (64, 10), (128, 4)])
def test_fp32_snapshot_statistics_match_oracle(orc, n, steps):
    """FP32 members (FP32 gradient transforms, values, bins and sums in FP64):
    the statistics of the member's field against the oracle's FP64 statistics
    of the same field (its state read back), at sizes that use each FP32
    exchange layout of the statistics kernel (128^3: 8-line rows)."""
    import paper_2506_23712_amd as ens
    E = ens.Ensemble(hist=ens.HistSpec(**HK))
    spec = ens.MemberSpec(n=n, nu=0.02, eps_ref=0.1, kf_hi=2.0, dt=0.0, cfl=0.5, seed=5 + n, precision="fp32")
    m = E.add_member(spec)
    E.step(steps)
    E.accumulate_stats()
    counts, mom, npts = m.stats()
    state = m.state().cpu().numpy()
    E.close()
    h = orc.Hist(**HK)
    om = orc.Member(n=n, nu=0.02, eps=0.1, kf_hi=2.0, dt=0.0, cfl=0.5)
    rc, rm, near, _ = orc.stats(om, h, state, grad_tol=FP32_GRAD_TOL)
    got, ref = h.split(counts.numpy().astype(np.uint64)), h.split(rc)
    assert npts == n ** 3
    for k, name in enumerate(("qr", "log_eps", "log_ens", "a_long", "a_trans")):
        counts_close(np.concatenate([got[name].ravel(), got[name + "_special"]]),
                     np.concatenate([ref[name].ravel(), ref[name + "_special"]]), near[k])
    mm = mom.numpy()
    sc = moment_scales(rm, n ** 3)
    for i in range(26):
        assert abs(mm[i] - rm[i]) <= FP32_MOMENT_TOL * sc[i], (i, mm[i], rm[i], sc[i])


def test_statistics_accumulate_and_reset(orc):
    import paper_2506_23712_amd as ens
    E = ens.Ensemble(hist=ens.HistSpec(**HK))
    m = E.add_member(ens.MemberSpec(n=32, nu=0.02, eps_ref=0.1, kf_hi=2.0, dt=0.01, seed=8))
    E.accumulate_stats()
    c1, m1, p1 = m.stats()
    E.accumulate_stats()
    c2, m2, p2 = m.stats()
    assert p2 == 2 * p1 and np.array_equal(c2.numpy(), 2 * c1.numpy())
    assert np.allclose(m2.numpy(), 2 * m1.numpy(), rtol=1e-15, atol=0)
    m.reset_stats()
    c3, m3, p3 = m.stats()
    assert p3 == 0 and not c3.numpy().any() and not m3.numpy().any()
    E.close()


def test_mixture_matches_oracle(orc):
    import paper_2506_23712_amd as ens
    from oracle import mixture as mx
    lams = [0.6, -0.9, 0.0, 1.5, -2.2]
    hs = ens.HistSpec(**HK)
    E = ens.Ensemble(hist=hs)
    ms = [E.add_member(ens.MemberSpec(n=16, nu=0.02, eps_ref=0.1, lam=l, kf_hi=2.0, dt=0.01, seed=50 + i))
          for i, l in enumerate(lams)]
    E.step(3)
    E.accumulate_stats()
    states = [m.state().cpu().numpy() for m in ms]
    h = orc.Hist(**HK)
    per = []
    for l, s in zip(lams, states):
        c, mom, near, _ = orc.stats(orc.Member(n=16, nu=0.02, eps=0.1 * math.exp(l), kf_hi=2.0, dt=0.01), h, s)
        per.append((c, mom))
    for mode, Z in ((0, math.log(8)), (1, math.log(4)), (0, 0.0), (2, math.log(2)), (3, math.log(8)),
                    (3, math.log(2)), (3, 0.0), (3, 6.0)):
        res = E.mix(0.023, Z, mode=mode, q_sigma=math.sqrt(2))
        w = mx.weights(lams, 0.023, Z, mode=mode, q_sigma=math.sqrt(2))
        assert np.allclose(res["weights"].numpy(), w, rtol=1e-13, atol=1e-16)
        npts = 16 ** 3
        area = (60 / 64) * (120 / 64)
        pdfs = [h.split(c)["qr"].ravel() / (npts * area) for c, _ in per]
        ref = np.array(mx.mix(w, pdfs))
        assert np.allclose(res["qr"].numpy().ravel(), ref, rtol=1e-12, atol=1e-300)
        means = [[mom[i] / (npts * (3 if i < 6 else 6 if i < 12 else 1)) for i in range(26)] for _, mom in per]
        mm = np.array(mx.mix(w, means))
        scale = np.max([moment_scales(mom, npts) / np.array([3 * npts] * 6 + [6 * npts] * 6 + [npts] * 14)
                        for _, mom in per], axis=0)
        assert np.all(np.abs(res["moments"].numpy()[:26] - mm) <= 1e-11 * scale)
        assert math.isclose(res["S_long"], mx.skewness(mm[1], mm[2]), rel_tol=1e-10)
        assert math.isclose(res["F_trans"], mx.flatness(mm[7], mm[9]), rel_tol=1e-10)
    E.close()


def test_scale_gap_from_snapshot_averaged_rlambda(orc):
    """Snapshot sums of E and D land in moments [26..28]; the scale gap for a
    target R_lambda follows the oracle's fit of R_lambda = A e^(lambda/6) over
    the members with lambda >= 0 and Z = (3/2) ln(R_ref / A)."""
    import paper_2506_23712_amd as ens
    from oracle import mixture as mx
    lams = [-1.0, 0.0, 0.5, 1.0, 2.0]
    nu = 0.02
    E = ens.Ensemble(hist=ens.HistSpec(**HK))
    ms = [E.add_member(ens.MemberSpec(n=16, nu=nu, eps_ref=0.1, lam=l, kf_hi=2.0, dt=0.01, seed=70 + i))
          for i, l in enumerate(lams)]
    with pytest.raises(ens.EnsError):
        E.scale_gap(100.0)                              # no snapshot yet
    sums = [[0.0, 0.0] for _ in ms]
    for _ in range(4):
        E.step(3)
        E.accumulate_stats()
        for k, m in enumerate(ms):
            d = m.diag()
            sums[k][0] += d["E"]
            sums[k][1] += d["D"]
    rls = []
    for k, m in enumerate(ms):
        _, mom, _ = m.stats()
        mom = mom.numpy()
        assert mom[26] == sums[k][0] and mom[27] == sums[k][1] and mom[28] == 4.0
        assert np.all(mom[29:] == 0)
        rls.append(mx.rlambda_from_means(mom[26] / 4, mom[27] / 4, nu))
    A = mx.rlambda_prefactor(lams, rls)
    for r_ref in (3.0, 50.0, 400.0):
        res = E.scale_gap(r_ref)
        assert np.allclose(res["rlambda"], rls, rtol=1e-14, atol=0)
        assert math.isclose(res["prefactor"], A, rel_tol=1e-14)
        assert math.isclose(res["Z"], mx.scale_gap(r_ref, A), rel_tol=1e-13, abs_tol=1e-14)
    # only the lambda < 0 member: no fit
    with pytest.raises(ens.EnsError):
        E.scale_gap(100.0, members=ms[:1])
    ms[1].reset_stats()
    with pytest.raises(ens.EnsError):
        E.scale_gap(100.0)
    E.close()


@pytest.mark.parametrize("M,family", [(1024, "quadratic"), (4096, "gamma"), (1000, "quadratic")])
def test_lambda_density_from_characteristic_function_matches_oracle(M, family):
    import torch
    import paper_2506_23712_amd as ens
    from oracle import mixture as mx
    if family == "quadratic":
        c, Z, h, lam0 = 0.023, math.log(8), 0.02, -10.0
        t = 1j * mx.cf_omegas(M, h)
        phi = np.exp(9 * c * Z * (t * t - t) / 2)
    else:
        a, b, Z, h, lam0 = 3.0, 4.0, 1.5, 0.005, -12.0
        t = 1j * mx.cf_omegas(M, h)
        phi = np.exp(a * Z * (t * math.log(1 + 1 / b) - np.log(1 + t / b)))
    got = ens.lambda_pdf_from_cf(torch.from_numpy(phi).cuda(), lam0, h).cpu().numpy()
    ref = mx.lambda_pdf_from_cf(phi, lam0, h)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_mixture_with_tabulated_density_matches_oracle(orc):
    import torch
    import paper_2506_23712_amd as ens
    from oracle import mixture as mx
    lams = [0.6, -0.9, 0.0, 1.5, -2.2]
    E = ens.Ensemble(hist=ens.HistSpec(**HK))
    ms = [E.add_member(ens.MemberSpec(n=16, nu=0.02, eps_ref=0.1, lam=l, kf_hi=2.0, dt=0.01, seed=90 + i))
          for i, l in enumerate(lams)]
    E.step(3)
    E.accumulate_stats()
    M, h, lam0, c, Z = 2048, 0.01, -10.0, 0.023, math.log(8)
    t = 1j * mx.cf_omegas(M, h)
    pdf = ens.lambda_pdf_from_cf(torch.from_numpy(np.exp(9 * c * Z * (t * t - t) / 2)).cuda(), lam0, h)
    res = E.mix_table(pdf, lam0, h)
    w = mx.weights_from_table(lams, pdf.cpu().numpy().tolist(), lam0, h)
    assert np.allclose(res["weights"].numpy(), w, rtol=1e-13, atol=1e-17)
    assert abs(res["weights"].sum().item() - 1) < 1e-14
    # close to the parametric Gaussian bin masses (the table is the same density)
    g = E.mix(c, Z, mode=0)
    assert np.max(np.abs(res["weights"].numpy() - g["weights"].numpy())) < 1e-5
    # mixed QR pdf = weighted member pdfs, as in ens_mix
    h_ = orc.Hist(**HK)
    counts = [m.stats()[0].numpy().astype(np.uint64) for m in ms]
    area = (60 / 64) * (120 / 64)
    pdfs = [h_.split(cn)["qr"].ravel() / (16 ** 3 * area) for cn in counts]
    ref = np.array(mx.mix(w, pdfs))
    assert np.allclose(res["qr"].numpy().ravel(), ref, rtol=1e-12, atol=1e-300)
    with pytest.raises(ens.EnsError):
        E.mix_table(pdf[:1], lam0, h)
    E.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_member_in_a_4pi_box_steps_and_bins_like_the_oracle(orc, prec, tol):
    """The ens256 geometry: box (4 pi)^3, dk = 1/2, band [1.4, 2.3] dk, CFL
    steps from dx = 4 pi / N.  Initial field, 20 steps and a statistics
    snapshot (gradients scale with dk) against the oracle on the same box."""
    import math
    import paper_2506_23712_amd as ens
    n, box = 32, 4 * math.pi
    E = ens.Ensemble(hist=ens.HistSpec(**HK))
    spec = ens.MemberSpec(n=n, nu=0.02, eps_ref=0.1, kf_lo=1.4, kf_hi=2.3, dt=0.0, cfl=0.5, box=box,
                          precision=prec, seed=91)
    m = E.add_member(spec)
    u0 = m.state().cpu().numpy()
    ref0 = orc.init_field(n, 91, box=box)
    assert np.max(np.abs(u0 - ref0)) <= (1e-14 if prec == "fp64" else 1e-7) * np.max(np.abs(ref0))
    E.step(20)
    got = m.state().cpu().numpy()
    om = orc.Member(n=n, nu=0.02, eps=0.1, kf_lo=1.4, kf_hi=2.3, dt=0.0, cfl=0.5, box=box)
    ref, rd = orc.run(om, ref0, 20)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"{prec} 4pi box: rel L2 after 20 steps {err:.2e}")
    assert err <= tol
    assert abs(m.diag()["t"] - rd[-1, 0]) <= 1e-12 * rd[-1, 0] + (0 if prec == "fp64" else 1e-6 * rd[-1, 0])
    E.accumulate_stats()
    counts, mom, npts = m.stats()
    E.close()
    h = orc.Hist(**HK)
    rc, rm, near, _ = orc.stats(om, h, got, grad_tol=0.0 if prec == "fp64" else FP32_GRAD_TOL)
    gs, rs = h.split(counts.numpy().astype(np.uint64)), h.split(rc)
    for k, name in enumerate(("qr", "log_eps", "log_ens", "a_long", "a_trans")):
        counts_close(np.concatenate([gs[name].ravel(), gs[name + "_special"]]),
                     np.concatenate([rs[name].ravel(), rs[name + "_special"]]), near[k])
    mm = mom.numpy()
    sc = moment_scales(rm, n ** 3)
    mtol = 1e-11 if prec == "fp64" else FP32_MOMENT_TOL
    for i in range(26):
        assert abs(mm[i] - rm[i]) <= mtol * sc[i], (i, mm[i], rm[i], sc[i])
