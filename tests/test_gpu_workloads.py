"""The workload recipes at their own sizes:
* 32^3 FP64, dt = 0.01, nu = 0.02, band |k| <= 2 at eps = 0.1, 100 steps, then a
  64 x 64 QR histogram -- whole-run parity with the oracle;
* 64 members at 128^3 FP64, lambda ~ N(0, 2), eps = e^lambda, nu = 0.02964,
  band |k| <= 2.5, CFL 0.5, one batched graph -- one member sampled against
  the oracle over 20 steps, statistics and the Gaussian mixture of all 64;
* the 96-member mixed FP32 benchmark workload in the benchmark's launch
  configuration -- one member per grid size sampled against the oracle over
  20 steps, and its statistics snapshot (the FP32 statistics kernels the
  benchmark times) against the oracle's statistics of the same field."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HK = dict(qr_bins=64, q_lo=-30.0, q_hi=30.0, r_lo=-60.0, r_hi=60.0, log_bins=512, log10_lo=-8.0,
          log10_hi=5.0, a_bins=1024, a_lo=-100.0, a_hi=100.0, eps_ref=0.1, nu_ref=0.02)


def test_32cubed_hundred_steps_and_qr_histogram(orc):
    import paper_2506_23712_amd as ens
    h = ens.HistSpec(**HK)
    E = ens.Ensemble(hist=h)
    m = E.add_member(ens.MemberSpec(n=32, nu=0.02, eps_ref=0.1, kf_lo=0.0, kf_hi=2.0, dt=0.01, seed=23712))
    E.step(100)
    E.accumulate_stats()
    got = m.state().cpu().numpy()
    counts, mom, npts = m.stats()
    d = m.diag()
    E.close()
    om = orc.Member(n=32, nu=0.02, eps=0.1, kf_lo=0.0, kf_hi=2.0, dt=0.01)
    ref, rd = orc.run(om, orc.init_field(32, 23712), 100)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"32^3, 100 steps: rel L2 {err:.3e}")
    assert err <= 1e-11
    assert abs(d["t"] - 1.0) <= 1e-13 and abs(d["E"] - rd[-1, 2]) <= 1e-11 * rd[-1, 2]
    oc = orc.Hist(**HK)
    rc, rm, near, _ = orc.stats(om, oc, ref)                # oracle statistics of the oracle's own field
    gq = oc.split(counts.numpy().astype(np.uint64))["qr"]
    rq = oc.split(rc)["qr"]
    diff = int(np.abs(gq.astype(np.int64) - rq.astype(np.int64)).sum())
    assert diff <= 2 * int(near[0]), (diff, near[0])
    assert npts == 32 ** 3


def test_64_members_128cubed_fp64_batch(orc):
    import paper_2506_23712_amd as ens
    from oracle import mixture as mx
    rng = np.random.default_rng(23712)
    lams = rng.normal(0.0, math.sqrt(2.0), 64)
    nu = 0.02964
    h = ens.HistSpec(**dict(HK, eps_ref=1.0, nu_ref=nu))
    E = ens.Ensemble(hist=h)
    ms = [E.add_member(ens.MemberSpec(n=128, nu=nu, eps_ref=1.0, lam=float(l), kf_hi=2.5, dt=0.0, cfl=0.5,
                                      seed=23712 + i)) for i, l in enumerate(lams)]
    E.step(20)
    sample = 17
    got = ms[sample].state().cpu().numpy()
    diags = [m.diag() for m in ms]
    E.accumulate_stats()
    res = E.mix(0.023, math.log(8), mode=2, q_sigma=math.sqrt(2.0))
    res0 = E.mix(0.023, math.log(8), mode=0)
    E.close()
    # sampled member against the oracle
    om = orc.Member(n=128, nu=nu, eps=math.exp(lams[sample]), kf_hi=2.5, dt=0.0, cfl=0.5)
    ref, rd = orc.run(om, orc.init_field(128, 23712 + sample), 20)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"128^3 member {sample} (lambda {lams[sample]:.3f}): rel L2 after 20 steps {err:.3e}")
    assert err <= 1e-11
    # per-member device dt from each member's own CFL, injection e^lambda
    for l, d in zip(lams, diags):
        assert not d["diverged"] and abs(d["cfl"] - 0.5) <= 1e-12
        assert abs(d["inj"] - math.exp(l)) <= 1e-12 * math.exp(l)
    assert len({round(d["dt"], 15) for d in diags}) > 32
    # mixture weights: importance weights for the drawn lambdas, bin masses for sorted cells
    w2 = mx.weights(list(lams), 0.023, math.log(8), mode=2, q_sigma=math.sqrt(2.0))
    w0 = mx.weights(list(lams), 0.023, math.log(8), mode=0)
    assert np.allclose(res["weights"].numpy(), w2, rtol=1e-12, atol=1e-300)
    assert np.allclose(res0["weights"].numpy(), w0, rtol=1e-12, atol=1e-300)
    # the mixed QR pdf integrates to the weighted in-range fraction (<= 1)
    area = (60 / 64) * (120 / 64)
    total = float(res0["qr"].sum()) * area
    assert 0.0 < total <= 1.0 + 1e-12


@pytest.mark.timeout(900)
def test_benchmark_workload_sampled_against_the_oracle(orc):
    """The 96-member mixed FP32 workload exactly as the benchmark launches it
    (autotuned variants, one captured graph per step): after 20 steps, one
    member of each grid size (64^3, 128^3 and the largest-lambda 256^3 member)
    against 20 FP64 oracle steps from the same field (FP32 bound 2e-5), then
    the statistics snapshot of all 96 against the oracle's statistics of each
    sampled member's field: counts equal except for samples within the FP32
    gradient tolerance of a bin edge, moment sums to the FP32 bound."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    import paper_2506_23712_amd as ens
    specs = bench.ens96_specs(ens)
    E = ens.Ensemble(hist=bench.hist_for(ens, 0.03395), graphs=True)
    ms = [E.add_member(s) for s in specs]
    E.autotune()
    from test_gpu_stats import FP32_GRAD_TOL, FP32_MOMENT_TOL, moment_scales, counts_close
    picks = [next(i for i, s in enumerate(specs) if s.n == n) for n in (64, 128)] + [len(specs) - 1]
    assert specs[picks[2]].n == 256
    u0 = {i: ms[i].state().cpu().numpy() for i in picks}
    E.step(20)
    got = {i: ms[i].state().cpu().numpy() for i in picks}
    dts = {i: ms[i].diag()["t"] for i in picks}
    E.accumulate_stats()                                    # the snapshot of the timed loop
    stats = {i: ms[i].stats() for i in picks}
    assert not any(m.diag()["diverged"] for m in ms)
    E.close()
    hb = bench.hist_for(ens, 0.03395)
    oh = orc.Hist(**{k: getattr(hb, k) for k in orc.Hist.__dataclass_fields__})
    for i in picks:
        s = specs[i]
        om = orc.Member(n=s.n, nu=s.nu, eps=s.eps_ref * math.exp(s.lam), kf_lo=s.kf_lo, kf_hi=s.kf_hi, dt=s.dt,
                        cfl=s.cfl)
        ref, rd = orc.run(om, u0[i], 20)
        err = float(np.linalg.norm(got[i] - ref) / np.linalg.norm(ref))
        print(f"member {i} ({s.n}^3, lambda {s.lam:+.2f}): rel L2 after 20 steps {err:.2e}, "
              f"t {dts[i]:.6f} vs {rd[-1, 0]:.6f}", flush=True)
        assert err <= 2e-5
        assert abs(dts[i] - rd[-1, 0]) <= 2e-5 * rd[-1, 0]
        counts, mom, npts = stats[i]
        assert npts == s.n ** 3
        rc, rm, near, _ = orc.stats(om, oh, got[i], grad_tol=FP32_GRAD_TOL)
        gs, rs = oh.split(counts.numpy().astype(np.uint64)), oh.split(rc)
        for k, name in enumerate(("qr", "log_eps", "log_ens", "a_long", "a_trans")):
            counts_close(np.concatenate([gs[name].ravel(), gs[name + "_special"]]),
                         np.concatenate([rs[name].ravel(), rs[name + "_special"]]), near[k])
        mm = mom.numpy()
        sc = moment_scales(rm, s.n ** 3)
        for j in range(26):
            assert abs(mm[j] - rm[j]) <= FP32_MOMENT_TOL * sc[j], (i, j, mm[j], rm[j], sc[j])
