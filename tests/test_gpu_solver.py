"""Parity of the HIP solver with the CPU oracle (same seeded inputs), and
invariants at the full 256^3 size."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TAU = 2 * math.pi


def ens_mod():
    import paper_2506_23712_amd as ens
    return ens


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make(n, nu, eps, kf_lo, kf_hi, dt, cfl=0.5, prec="fp64", seed=23712, lam=0.0, visc=0, graphs=True, hist=None):
    ens = ens_mod()
    E = ens.Ensemble(hist=hist, graphs=graphs)
    m = E.add_member(ens.MemberSpec(n=n, nu=nu, eps_ref=eps, lam=lam, kf_lo=kf_lo, kf_hi=kf_hi, dt=dt, cfl=cfl,
                                    precision=prec, seed=seed, visc_mode=visc))
    return E, m


def oracle_member(n, nu, eps, kf_lo, kf_hi, dt, cfl=0.5, visc=0):
    import oracle
    return oracle.Member(n=n, nu=nu, eps=eps, kf_lo=kf_lo, kf_hi=kf_hi, dt=dt, cfl=cfl, visc_mode=visc)


@pytest.mark.parametrize("n", [16, 32, 64, 128])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_initial_field_matches_oracle(orc, n, prec):
    E, m = make(n, 0.02, 0.1, 0, 2, 0.01, prec=prec, seed=1000 + n)
    got = m.state().cpu().numpy()
    ref = orc.init_field(n, 1000 + n, k_peak=2.0, e0=0.5)
    tol = 1e-14 if prec == "fp64" else 1e-7
    assert rel(got, ref) <= tol
    E.close()


def test_state_roundtrip_and_truncation(orc):
    import torch
    n = 32
    E, m = make(n, 0.02, 0.1, 0, 2, 0.01)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, n, n, n // 2 + 1)) + 1j * rng.standard_normal((3, n, n, n // 2 + 1))
    m.set_state(torch.from_numpy(x))
    got = m.state().cpu().numpy()
    mask = orc.retained_mask(n)
    assert np.array_equal(got[:, mask], x[:, mask])
    assert np.all(got[:, ~mask] == 0)
    E.close()


CASES = {
    # name: (n, nu, eps, kf_lo, kf_hi, dt, cfl)
    "c1_32_fixed_dt": (32, 0.02, 0.1, 0.0, 2.0, 0.01, 0.5),
    "n16_cfl": (16, 0.05, 0.3, 0.0, 2.5, 0.0, 0.5),
    "n64_cfl_band_paper": (64, 0.01, 1.0, 1.4, 2.3, 0.0, 0.5),
    "n128_cfl": (128, 0.02964, 1.0, 0.0, 2.5, 0.0, 0.5),
    "n32_band_integer_edges": (32, 0.02, 0.1, 1.0, 2.0, 0.005, 0.5),   # |m|^2 = 1 and 4 in the band
}


@pytest.mark.parametrize("case", list(CASES))
def test_twenty_steps_match_oracle_fp64(orc, case):
    n, nu, eps, lo, hi, dt, cfl = CASES[case]
    steps = 20
    E, m = make(n, nu, eps, lo, hi, dt, cfl, seed=77 + n)
    E.step(steps)
    got = m.state().cpu().numpy()
    d = m.diag()
    u0 = orc.init_field(n, 77 + n)
    ref, rd = orc.run(oracle_member(n, nu, eps, lo, hi, dt, cfl), u0, steps)
    err = rel(got, ref)
    print(f"{case}: rel L2 after {steps} steps = {err:.3e}")
    assert err <= 1e-11
    assert abs(d["t"] - rd[-1, 0]) <= 1e-12 * rd[-1, 0]
    assert abs(d["E"] - rd[-1, 2]) <= 1e-12 * rd[-1, 2]
    assert abs(d["D"] - rd[-1, 3]) <= 1e-11 * rd[-1, 3]
    assert abs(d["dt"] - rd[-1, 1]) <= 1e-12 * rd[-1, 1]
    assert abs(d["umax"] - rd[-1, 6]) <= 1e-12 * rd[-1, 6]
    assert abs(d["E_f"] - rd[-1, 5]) <= 1e-12 * rd[-1, 5]
    assert d["step"] == steps and not d["diverged"]
    E.close()


def test_explicit_viscous_variant_matches_oracle(orc):
    n, nu, eps = 32, 0.02, 0.1
    E, m = make(n, nu, eps, 0.0, 2.0, 0.01, visc=1, seed=5)
    E.step(10)
    ref, _ = orc.run(oracle_member(n, nu, eps, 0.0, 2.0, 0.01, visc=1), orc.init_field(n, 5), 10)
    assert rel(m.state().cpu().numpy(), ref) <= 1e-11
    E.close()


@pytest.mark.parametrize("n", [32, 64])
def test_twenty_steps_fp32_within_bound(orc, n):
    nu, eps = (0.02, 0.1) if n == 32 else (0.01, 1.0)
    dt = 0.01 if n == 32 else 0.0
    E, m = make(n, nu, eps, 0.0, 2.0, dt, prec="fp32", seed=31 + n)
    E.step(20)
    ref, _ = orc.run(oracle_member(n, nu, eps, 0.0, 2.0, dt), orc.init_field(n, 31 + n), 20)
    err = rel(m.state().cpu().numpy(), ref)
    print(f"fp32 n={n}: rel L2 after 20 steps = {err:.3e}")
    assert err <= 2e-5
    E.close()


FUSED = {
    # name: (n, nu, eps, kf_lo, kf_hi, dt, prec, tolerance after 20 steps)
    "n16_fp64": (16, 0.05, 0.3, 0.0, 2.5, 0.0, "fp64", 1e-11),
    "n32_fp64_fixed_dt": (32, 0.02, 0.1, 0.0, 2.0, 0.01, "fp64", 1e-11),
    "n64_fp64_band_paper": (64, 0.01, 1.0, 1.4, 2.3, 0.0, "fp64", 1e-11),
    "n128_fp64": (128, 0.02964, 1.0, 0.0, 2.5, 0.0, "fp64", 1e-11),
    "n64_fp32_band_paper": (64, 0.01, 1.0, 1.4, 2.3, 0.0, "fp32", 2e-5),
    "n128_fp32": (128, 0.02964, 1.0, 0.0, 2.5, 0.0, "fp32", 2e-5),
}


@pytest.mark.parametrize("case", list(FUSED))
def test_fused_z_forward_matches_oracle(orc, case):
    """z forward variant 1: stages 0 and 1 also perform the next stage's z
    inverse from the updated velocity in registers (two z-inverse launches
    fewer per step).  Twenty steps against the oracle, in graph and direct
    launches."""
    n, nu, eps, lo, hi, dt, prec, tol = FUSED[case]
    ref, rd = orc.run(oracle_member(n, nu, eps, lo, hi, dt), orc.init_field(n, 91 + n), 20)
    for graphs in (True, False):
        E, m = make(n, nu, eps, lo, hi, dt, prec=prec, seed=91 + n, graphs=graphs)
        E.set_variant("zfwd_update", n, prec, 1)
        E.step(20)
        err = rel(m.state().cpu().numpy(), ref)
        d = m.diag()
        print(f"{case} graphs={graphs}: rel L2 after 20 steps = {err:.3e}")
        assert err <= tol
        assert abs(d["E"] - rd[-1, 2]) <= 10 * tol * rd[-1, 2]
        assert d["step"] == 20 and not d["diverged"]
        E.close()


@pytest.mark.parametrize("n,prec,count", [(256, "fp32", 25), (128, "fp32", 24), (64, "fp32", 47), (256, "fp64", 1),
                                          (512, "fp32", 1), (1024, "fp32", 1)])
def test_fused_z_forward_agrees_with_separate_passes(n, prec, count):
    """The fused z forward against the separate z inverse on the benchmark's
    batch shapes, three steps: the same operations up to the order of the
    inverse transform's stages, so agreement is to rounding."""
    ens = ens_mod()
    finals = []
    for variant in (0, 1):
        E = ens.Ensemble()
        ms = [E.add_member(ens.MemberSpec(n=n, nu=0.03395 * (256 / n) ** (4 / 3), eps_ref=1.0, lam=0.3 * i - 1.0,
                                          kf_hi=2.5, dt=0.0, cfl=0.5, precision=prec, seed=800 + i))
              for i in range(count)]
        E.set_variant("zfwd_update", n, prec, variant)
        E.step(3)
        pick = sorted({0, count // 2, count - 1})
        finals.append([ms[i].state().cpu().numpy() for i in pick])
        E.close()
    tol = 2e-6 if prec == "fp32" else 1e-13
    for a, b in zip(finals[0], finals[1]):
        err = rel(b, a)
        print(f"{n} {prec} x{count}: fused vs separate rel L2 {err:.2e}")
        assert err <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_steps_of_one_call_agree_with_single_step_calls(orc, prec):
    """Inside one ens_step call every step but the last performs the next
    step's first z inverse in its last z forward.  Stepping 1, 2, 3 or 12
    steps per call (graphs and direct launches) gives the oracle's trajectory,
    and the same one to rounding."""
    n, nu, eps, steps = 64, 0.01, 1.0, 12
    ref, _ = orc.run(oracle_member(n, nu, eps, 1.4, 2.3, 0.0), orc.init_field(n, 17), steps)
    tol = 1e-11 if prec == "fp64" else 2e-5
    finals = []
    for chunk in (1, 2, 3, 12):
        for graphs in (True, False):
            E, m = make(n, nu, eps, 1.4, 2.3, 0.0, prec=prec, seed=17, graphs=graphs)
            for _ in range(steps // chunk):
                E.step(chunk)
            got = m.state().cpu().numpy()
            err = rel(got, ref)
            print(f"{prec} {chunk} steps per call, graphs={graphs}: rel L2 {err:.3e}")
            assert err <= tol and m.diag()["step"] == steps
            finals.append(got)
            E.close()
    for g in finals[1:]:
        assert rel(g, finals[0]) <= (1e-13 if prec == "fp64" else 2e-6)


def test_graph_and_direct_launch_agree_bitwise():
    outs = []
    for graphs in (True, False):
        E, m = make(32, 0.02, 0.1, 0.0, 2.0, 0.0, graphs=graphs, seed=9)
        E.step(7)
        outs.append(m.state().cpu().numpy())
        E.close()
    assert np.array_equal(outs[0], outs[1])


def test_graph_modes_agree_bitwise_on_mixed_groups():
    """Direct launches, one graph per step and the graph with one branch per
    group (three groups: 32^3 FP64, 64^3 FP64, 64^3 FP32), replayed several
    times with eager work and synchronisations between the replays."""
    ens = ens_mod()
    specs = [ens.MemberSpec(n=32, nu=0.02, eps_ref=0.1, lam=-0.5, kf_hi=2.0, seed=31),
             ens.MemberSpec(n=64, nu=0.02, eps_ref=0.1, lam=0.4, kf_hi=2.0, seed=32),
             ens.MemberSpec(n=64, nu=0.02, eps_ref=0.1, lam=0.0, kf_hi=2.0, seed=33, precision="fp32"),
             ens.MemberSpec(n=32, nu=0.02, eps_ref=0.1, lam=1.0, kf_hi=2.0, seed=34)]
    outs = {}
    for mode in (0, 1, 2):
        E = ens.Ensemble(graphs=mode)
        ms = [E.add_member(s) for s in specs]
        states = []
        for rep in range(3):
            E.step(2)
            states.append([m.state().cpu().numpy() for m in ms])   # eager copies, host sync between replays
        outs[mode] = (states, [m.diag()["t"] for m in ms])
        E.close()
    for mode in (1, 2):
        for a, b in zip(outs[0][0], outs[mode][0]):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
        assert outs[0][1] == outs[mode][1]
    # switching the mode of a live context drops its graphs and keeps stepping
    # identically (the same steps per call: where a call ends decides where
    # a step hands its last z inverse to the next, which rounds differently)
    E = ens.Ensemble(graphs=2)
    ms = [E.add_member(s) for s in specs]
    E.step(2)
    E.set_graph_mode(1)
    E.step(2)
    E.step(2)
    assert np.array_equal(ms[1].state().cpu().numpy(), outs[0][0][2][1])
    with pytest.raises(ens.EnsError):
        E.set_graph_mode(3)
    E.close()


def test_repeat_runs_are_bitwise_identical():
    outs = []
    for _ in range(2):
        E, m = make(64, 0.01, 1.0, 0.0, 2.5, 0.0, seed=4)
        E.step(5)
        outs.append((m.state().cpu().numpy(), m.diag()["E"]))
        E.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


def test_batched_members_equal_single_runs():
    ens = ens_mod()
    specs = [ens.MemberSpec(n=32, nu=0.02, eps_ref=0.1, lam=l, kf_hi=2.0, dt=0.0, cfl=0.5, seed=100 + i)
             for i, l in enumerate([-1.0, 0.0, 0.7])]
    specs.append(ens.MemberSpec(n=64, nu=0.02, eps_ref=0.1, lam=0.3, kf_hi=2.0, dt=0.0, cfl=0.5, seed=200,
                                precision="fp32"))
    E = ens.Ensemble()
    ms = [E.add_member(s) for s in specs]
    E.step(4)
    batched = [m.state().cpu().numpy() for m in ms]
    E.close()
    for s, b in zip(specs, batched):
        E1 = ens.Ensemble()
        m1 = E1.add_member(s)
        E1.step(4)
        assert np.array_equal(m1.state().cpu().numpy(), b)
        E1.close()


def test_full_size_256_invariants(orc):
    """256^3 at the benchmark's configuration: properties that hold at any size."""
    n, nu = 256, 4.594e-3
    E, m = make(n, nu, 1.0, 0.0, 2.5, 0.0, 0.5, seed=23712)
    E.step(3)
    u = m.state().cpu().numpy()
    d = m.diag()
    assert orc.divergence_ratio(u) <= 1e-13
    assert np.all(u[:, ~orc.retained_mask(n)] == 0)
    assert abs(orc.energy(u) - d["E"]) <= 1e-12 * d["E"]
    assert abs(orc.dissipation(u, nu) - d["D"]) <= 1e-11 * d["D"]
    assert abs(d["inj"] - 1.0) <= 1e-14 and abs(d["cfl"] - 0.5) <= 1e-12
    p = u[:, :, :, 0]
    mirrored = np.conj(p[:, (-np.arange(n)) % n][:, :, (-np.arange(n)) % n])
    assert np.max(np.abs(p - mirrored)) <= 1e-13 * np.max(np.abs(p))
    E.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_kernel_variant_matches_oracle(orc, prec):
    """Each compiled variant of each transform pass: 8 or 16 values per
    thread; the y/z passes' variants 2 and 3 with twice the lines per
    workgroup; the streamed x pass."""
    n, nu, eps = 64, 0.01, 1.0
    ref, _ = orc.run(oracle_member(n, nu, eps, 0.0, 2.5, 0.0), orc.init_field(n, 12), 5)
    tol = 1e-12 if prec == "fp64" else 2e-5
    for variant in (0, 1, 2, 3):
        E, m = make(n, nu, eps, 0.0, 2.5, 0.0, prec=prec, seed=12)
        for p in ("zinv", "yinv", "xpass", "yfwd"):
            E.set_variant(p, n, prec, variant)
        E.step(5)
        err = rel(m.state().cpu().numpy(), ref)
        print(f"{prec} variant {variant}: rel L2 {err:.3e}")
        assert err <= tol
        E.close()


@pytest.mark.parametrize("n,prec,count", [(128, "fp32", 6), (128, "fp64", 3), (256, "fp32", 25), (64, "fp32", 47),
                                          (256, "fp64", 1), (512, "fp32", 1), (64, "fp64", 5)])
def test_streamed_xpass_agrees_with_classic(n, prec, count):
    """The persistent streamed x passes on long tile ranges per workgroup
    (batches of the benchmark's shapes) against the classic 8-value kernel:
    variant 2 (8 values per thread), 3 (FP32: 16), and the wave-private
    variants 4 (16 FP32 / 8 FP64 values) and 5 (8 / 4), whose exchanges never
    leave a wave, and 6 (as 4, inputs staged pairwise through two buffers).  All perform the same operations; the compiler may fuse
    multiply-adds differently, so agreement is to rounding: a tile staged
    wrongly, read before its copy landed or exchanged without ordering would
    differ at O(1)."""
    ens = ens_mod()
    finals = []
    variants = ((0, 2, 3) if prec == "fp32" and 128 <= n <= 512 else (0, 2)) + (4, 5, 6)
    for variant in variants:
        E = ens.Ensemble()
        ms = [E.add_member(ens.MemberSpec(n=n, nu=0.03395, eps_ref=1.0, lam=0.3 * i - 1.0, kf_hi=2.5, dt=0.0, cfl=0.5,
                                          precision=prec, seed=700 + i)) for i in range(count)]
        E.set_variant("xpass", n, prec, variant)
        E.step(2)
        pick = sorted({0, count // 2, count - 1})
        finals.append(([ms[i].state().cpu().numpy() for i in pick], [m.diag()["dt"] for m in ms]))
        E.close()
    tol = 2e-6 if prec == "fp32" else 1e-13
    for k in range(1, len(variants)):
        for a, b in zip(finals[0][0], finals[k][0]):
            err = rel(b, a)
            worst = float(np.max(np.abs(b - a)) / np.max(np.abs(a)))
            print(f"{n} {prec} x{count} variant {variants[k]}: rel L2 {err:.2e}, max {worst:.2e}")
            assert err <= tol and worst <= 5 * tol
        assert np.allclose(finals[k][1], finals[0][1], rtol=tol, atol=0)   # per-member CFL steps


def test_autotune_keeps_state_and_writes_cache(tmp_path):
    E, m = make(32, 0.02, 0.1, 0.0, 2.0, 0.01, seed=3)
    before = m.state().cpu().numpy()
    cache = tmp_path / "variants.txt"
    table = E.autotune(cache_path=str(cache))
    assert np.array_equal(m.state().cpu().numpy(), before)
    assert set(table.values()) <= {0, 1, 2, 3, 4, 5, 6} and len(table) == 5
    assert table["zfwd_update:32:fp64"] == 1          # not timed (it updates the state): the default, fused
    text = cache.read_text()
    assert "zinv:32:fp64" in text and "zfwd_update" not in text
    E.close()
