"""Edge cases of the stepping path on the GPU: degenerate fields, empty and
invalid requests, and a closed form that holds at any size (a single Fourier
mode has no nonlinear term and, outside the forcing band, decays exactly by
the viscous factor)."""
import ctypes
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def ens_mod():
    import paper_2506_23712_amd as ens
    return ens


@pytest.mark.parametrize("n,prec", [(16, "fp64"), (64, "fp32"), (256, "fp64"), (256, "fp32")])
def test_single_mode_decays_by_the_viscous_factor(n, prec):
    """u = (0, a, 0) e^{i m x} with m = (3, 0, 0) is a steady Euler solution
    (u.grad u = 0 and it is divergence free): one RK3 step with the integrating
    factor multiplies it by exp(-nu |k|^2 dt) exactly, at every grid size.
    Without injection (eps = 0): the linear band forcing eps / (2 E_f) u is
    singular for a band without energy, and would blow the round-off that the
    transforms leave in the band up to the injection rate."""
    import torch
    ens = ens_mod()
    nu, dt = 0.05, 0.01
    E = ens.Ensemble()
    m = E.add_member(ens.MemberSpec(n=n, nu=nu, eps_ref=0.0, kf_lo=0.0, kf_hi=1.5, dt=dt, precision=prec, seed=1))
    u = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    u[1, 0, 0, 3] = 0.25 - 0.5j
    m.set_state(torch.from_numpy(u))
    E.step(4)
    got = m.state().cpu().numpy()
    E.close()
    want = u * math.exp(-nu * 9.0 * 4 * dt)
    tol = 1e-14 if prec == "fp64" else 1e-6
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(u))


@pytest.mark.parametrize("n,prec", [(32, "fp64"), (32, "fp32"), (256, "fp64"), (256, "fp32")])
def test_single_off_band_mode_with_injection_is_not_forced(n, prec):
    """The same mode with eps > 0: the band holds only the rounding the
    transforms leave there, at most 1e-10 of the field's energy, so it counts
    as empty on both sides (no forcing, no injection, flag bit 1); the mode
    decays by the viscous factor over 20 steps, as in the oracle."""
    import torch
    import oracle
    ens = ens_mod()
    nu, dt, steps = 0.05, 0.01, 20
    E = ens.Ensemble()
    m = E.add_member(ens.MemberSpec(n=n, nu=nu, eps_ref=1.0, kf_lo=0.0, kf_hi=2.5, dt=dt, precision=prec, seed=1))
    u = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    u[1, 0, 0, 3] = 0.25 - 0.5j
    m.set_state(torch.from_numpy(u))
    E.step(steps)
    got = m.state().cpu().numpy()
    d = m.diag()
    E.close()
    assert d["inj"] == 0.0 and (d["flags"] & 2) and not d["diverged"]
    want = u * math.exp(-nu * 9.0 * steps * dt)
    tol = 1e-13 if prec == "fp64" else 2e-6
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(u))
    if n == 32:
        ref, diag = oracle.run(oracle.Member(n=n, nu=nu, eps=1.0, kf_lo=0.0, kf_hi=2.5, dt=dt), u, steps)
        assert np.all(diag[:, 4] == 0)
        assert np.linalg.norm(got - ref) <= (1e-13 if prec == "fp64" else 2e-6) * np.linalg.norm(ref)


def test_zero_field_with_fixed_dt_stays_zero_and_cfl_reports_no_velocity():
    import torch
    ens = ens_mod()
    E = ens.Ensemble()
    a = E.add_member(ens.MemberSpec(n=32, nu=0.02, eps_ref=1.0, kf_hi=2.5, dt=0.01, seed=2))
    b = E.add_member(ens.MemberSpec(n=32, nu=0.02, eps_ref=1.0, kf_hi=2.5, dt=0.0, cfl=0.5, seed=3))
    z = torch.zeros((3, 32, 32, 17), dtype=torch.complex128)
    a.set_state(z)
    b.set_state(z)
    E.step(2, members=[a])
    assert np.all(a.state().cpu().numpy() == 0)              # no band energy: no forcing, no flow
    da = a.diag()
    assert not da["diverged"] and da["E"] == 0.0 and abs(da["t"] - 0.02) < 1e-15
    E.step(1, members=[b])
    assert b.diag()["diverged"]                              # no CFL velocity: flagged, not a fault
    E.close()


def test_zero_steps_and_invalid_requests_change_nothing():
    import paper_2506_23712_amd as ens
    from paper_2506_23712_amd import _lib
    E = ens.Ensemble()
    m = E.add_member(ens.MemberSpec(n=32, nu=0.02, eps_ref=1.0, kf_hi=2.5, seed=4))
    before = m.state().cpu().numpy()
    E.step(0)
    assert np.array_equal(m.state().cpu().numpy(), before) and m.diag()["step"] == 0
    L = _lib.lib()
    ids = (ctypes.c_int32 * 2)(m.id, m.id)
    assert L.ens_step(E.ctx, ids, 0, 1, None) == _lib.ENS_E_INVALID          # empty list
    assert L.ens_step(E.ctx, ids, 2, 1, None) == _lib.ENS_E_INVALID          # duplicate member
    bad = (ctypes.c_int32 * 1)(99)
    assert L.ens_step(E.ctx, bad, 1, 1, None) == _lib.ENS_E_INVALID          # unknown member
    assert L.ens_step(E.ctx, ids, 1, -1, None) == _lib.ENS_E_INVALID         # negative step count
    with pytest.raises(ens.EnsError):
        E.add_member(ens.MemberSpec(n=48, nu=0.02))                          # not a supported size
    with pytest.raises(ens.EnsError):
        E.add_member(ens.MemberSpec(n=1024, nu=0.02, precision="fp64"))      # 1024^3 is FP32 only
    with pytest.raises(ens.EnsError):
        E.add_member(ens.MemberSpec(n=32, nu=0.02, dt=0.0, cfl=0.0))         # no time step rule
    # a workspace one byte short is refused before anything is written
    import torch
    spec = ens.MemberSpec(n=32, nu=0.02, seed=5)
    need = E.workspace_bytes(spec)
    ws = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    mid = ctypes.c_int32(-1)
    d = spec.desc()
    st = L.ens_member_init(E.ctx, ctypes.byref(d), ctypes.c_void_p(ws.data_ptr()), need - 1, None, ctypes.byref(mid))
    assert st == _lib.ENS_E_OOM and mid.value == -1
    assert np.array_equal(m.state().cpu().numpy(), before)
    E.close()


def _hermitian_part(u):
    """Hermitian part of the m_x = 0 plane of a half spectrum (the rest is
    Hermitian by construction)."""
    n = u.shape[1]
    h = u.copy()
    p = u[:, :, :, 0]
    h[:, :, :, 0] = 0.5 * (p + np.conj(p[:, (-np.arange(n)) % n][:, :, (-np.arange(n)) % n]))
    return h


@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_band_part_breaking_hermitian_symmetry_is_not_forced(orc, prec, fused):
    """A part of the m_x = 0 plane that breaks the Hermitian symmetry of a real
    field (i r added at both modes of a pair in the band) is invisible in
    physical space.  The oracle's forcing ignores it; the library removes it
    from the band at every stage.  The Hermitian parts of both results agree,
    and the library's band plane is Hermitian after the step."""
    import torch
    ens = ens_mod()
    n, nu, dt = 32, 0.02, 0.005
    u = orc.init_field(n, 41)
    pairs = (((1, 1), (0.03, -0.02, 0.01)), ((2, 0), (0.0, 0.025, -0.04)), ((-1, 2), (0.01, 0.01, 0.02)))
    for (my, mz), r in pairs:
        for c in range(3):
            u[c, mz % n, my % n, 0] += 1j * r[c]
            u[c, (-mz) % n, (-my) % n, 0] += 1j * r[c]
    E = ens.Ensemble()
    m = E.add_member(ens.MemberSpec(n=n, nu=nu, eps_ref=0.1, kf_lo=1.4, kf_hi=2.3, dt=dt, precision=prec, seed=41))
    # fused: the z inverse of stages 1 and 2 runs inside the z forward, on the
    # velocity before the band step removes the broken part
    E.set_variant("zfwd_update", n, prec, fused)
    m.set_state(torch.from_numpy(u))
    E.step(3)
    got = m.state().cpu().numpy()
    E.close()
    ref, _ = orc.run(orc.Member(n=n, nu=nu, eps=0.1, kf_lo=1.4, kf_hi=2.3, dt=dt), u, 3)
    tol = 1e-13 if prec == "fp64" else 2e-6
    hg, hr = _hermitian_part(got), _hermitian_part(ref)
    assert np.max(np.abs(hg - hr)) <= tol * np.max(np.abs(hr))
    # the band modes of the library's plane: Hermitian to rounding (the last
    # stage's update adds rounding only); the oracle keeps the broken part
    for (my, mz), _ in pairs:
        a, b = got[:, mz % n, my % n, 0], got[:, (-mz) % n, (-my) % n, 0]
        assert np.max(np.abs(a - np.conj(b))) <= tol * np.max(np.abs(hr))
        a, b = ref[:, mz % n, my % n, 0], ref[:, (-mz) % n, (-my) % n, 0]
        assert np.max(np.abs(a - np.conj(b))) > 0.01


def test_mean_flow_is_carried_but_neither_forced_nor_counted_in_the_band(orc):
    """A uniform flow (the m = 0 mode) with a band starting at 0: it advects the
    field and enters the CFL velocity, but it is not part of the band (E_f,
    forcing), and it keeps its value.  Five steps against the oracle."""
    import torch
    ens = ens_mod()
    n, nu, steps = 32, 0.02, 5
    u = orc.init_field(n, 53)
    u[:, 0, 0, 0] = (0.3, -0.2, 0.45)
    E = ens.Ensemble()
    m = E.add_member(ens.MemberSpec(n=n, nu=nu, eps_ref=0.1, kf_lo=0.0, kf_hi=2.0, dt=0.0, cfl=0.5,
                                    precision="fp64", seed=53))
    m.set_state(torch.from_numpy(u))
    E.step(steps)
    got = m.state().cpu().numpy()
    d = m.diag()
    E.close()
    ref, rd = orc.run(orc.Member(n=n, nu=nu, eps=0.1, kf_lo=0.0, kf_hi=2.0, dt=0.0, cfl=0.5), u, steps)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.array_equal(got[:, 0, 0, 0], u[:, 0, 0, 0])
    assert abs(d["E_f"] - rd[-1, 5]) <= 1e-12 * rd[-1, 5]
    assert abs(d["umax"] - rd[-1, 6]) <= 1e-12 * rd[-1, 6]
    assert abs(d["inj"] - 0.1) <= 1e-14


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_long_forced_run_keeps_the_invisible_parts_at_rounding(prec):
    """Regression test for the band forcing: 20 000 CFL steps of a forced 32^3
    member (several hundred time units).  The divergent part of u and the part
    of the m_x = 0 plane that breaks Hermitian symmetry get no tendency from
    the projected nonlinear term; a forcing that acted on them would grow them
    from rounding at about eps/(2 E_f) - nu k^2 per time unit (e^100 and more
    over this run).  Both stay at rounding level, and the energy stays finite."""
    ens = ens_mod()
    n = 32
    E = ens.Ensemble()
    m = E.add_member(ens.MemberSpec(n=n, nu=0.05, eps_ref=1.0, kf_lo=1.4, kf_hi=2.3, dt=0.0, cfl=0.5,
                                    precision=prec, seed=77))
    E.step(20000)
    d = m.diag()
    u = m.state().cpu().numpy()
    E.close()
    assert not d["diverged"] and d["t"] > 100.0 and 0.0 < d["E"] < 50.0
    k = np.fft.fftfreq(n, 1.0 / n)
    mz, my, mx = np.meshgrid(k, k, np.arange(n // 2 + 1), indexing="ij")
    k2 = mx * mx + my * my + mz * mz
    k2[0, 0, 0] = 1.0
    w = np.where(mx > 0, 1.0, 0.5)
    e_tot = float(np.sum(w * np.sum(np.abs(u) ** 2, axis=0)))
    kd = mx * u[0] + my * u[1] + mz * u[2]
    e_div = float(np.sum(w * np.abs(kd) ** 2 / k2))
    p = u[:, :, :, 0]
    anti = 0.5 * (p - np.conj(p[:, (-np.arange(n)) % n][:, :, (-np.arange(n)) % n]))
    e_anti = 0.5 * float(np.sum(np.abs(anti) ** 2))
    lim = 1e-20 if prec == "fp64" else 1e-8
    print(f"{prec}: t = {d['t']:.0f}, E = {d['E']:.3f}, divergent {e_div / e_tot:.2e}, broken symmetry {e_anti / e_tot:.2e}")
    assert e_div / e_tot <= lim and e_anti / e_tot <= lim
