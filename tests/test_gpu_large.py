"""Full-size grids (256^3 FP64, 512^3 FP64, 1024^3 FP32): parity on a field
whose solution the oracle computes exactly on a small grid, and invariants
that hold at any size."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def tg_small():
    """Taylor-Green velocity in the canonical layout on an 8^3 grid (library FFT)."""
    n = 8
    x = np.arange(n) * 2 * np.pi / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.stack([np.sin(X) * np.cos(Y) * np.cos(Z), -np.cos(X) * np.sin(Y) * np.cos(Z), 0 * X])
    return np.stack([np.fft.rfftn(u[c]) / n ** 3 for c in range(3)])


def embed(small, n, device):
    """Copy every mode of a small canonical field into an n^3 canonical field on the device."""
    import torch
    ns = small.shape[1]
    big = torch.zeros((3, n, n, n // 2 + 1), dtype=torch.complex128, device=device)
    for iz in range(ns):
        for iy in range(ns):
            for ix in range(ns // 2 + 1):
                v = small[:, iz, iy, ix]
                if not np.any(np.abs(v) > 0):
                    continue
                mz = iz if iz <= ns // 2 else iz - ns
                my = iy if iy <= ns // 2 else iy - ns
                big[:, mz % n, my % n, ix] = torch.from_numpy(v).to(device)
    return big


def box(field, n, B):
    """Modes |m_i| <= B of an n^3 canonical field, laid out as the canonical field of a 3B+? grid."""
    import torch
    idx = torch.tensor(list(range(B + 1)) + list(range(n - B, n)), device=field.device)
    sub = field.index_select(1, idx).index_select(2, idx)[..., : B + 1]
    return sub.cpu().numpy()


@pytest.mark.parametrize("n,prec,tol", [(256, "fp64", 1e-12), (512, "fp64", 1e-12), (1024, "fp32", 2e-5)])
def test_one_step_of_taylor_green_matches_oracle_at_full_size(orc, n, prec, tol):
    import torch
    import paper_2506_23712_amd as ens
    nu, eps, dt, B = 0.01, 0.1, 0.01, 8
    small = tg_small()
    print(f"case n={n} {prec}", flush=True)
    E = ens.Ensemble()
    m = E.add_member(ens.MemberSpec(n=n, nu=nu, eps_ref=eps, kf_hi=2.0, dt=dt, precision=prec))
    big = embed(small, n, E.device)
    m.set_state(big)
    del big
    E.step(1)
    out = m.state()
    got = box(out, n, B)
    total = float((out.abs() ** 2).sum())
    del out
    torch.cuda.empty_cache()
    # oracle on 32^3: after one RK3 step the field holds |m_i| <= 8 < K = 10, untruncated on both grids
    ref32, _ = orc.run(orc.Member(n=32, nu=nu, eps=eps, kf_hi=2.0, dt=dt), embed_np(small, 32), 1)
    ref = box_np(ref32, 32, B)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    outside = (total - float(np.sum(np.abs(got) ** 2))) / total
    print(f"n={n} {prec}: rel L2 on |m|<=8 = {err:.3e}, energy fraction outside = {outside:.2e}")
    assert err <= tol
    assert abs(outside) <= (1e-24 if prec == "fp64" else 1e-10)
    d = m.diag()
    assert abs(d["inj"] - eps) <= 1e-15 and d["step"] == 1
    E.close()


def embed_np(small, n):
    ns = small.shape[1]
    big = np.zeros((3, n, n, n // 2 + 1), complex)
    for iz in range(ns):
        for iy in range(ns):
            mz = iz if iz <= ns // 2 else iz - ns
            my = iy if iy <= ns // 2 else iy - ns
            big[:, mz % n, my % n, : ns // 2 + 1] = small[:, iz, iy, :]
    return big


def box_np(field, n, B):
    idx = list(range(B + 1)) + list(range(n - B, n))
    return field[:, idx][:, :, idx][..., : B + 1]


def test_1024_fp32_invariants_and_statistics(orc):
    """1024^3 FP32 (the largest single-member configuration): two CFL steps from
    the seeded field, then invariants on the device and one statistics snapshot."""
    import torch
    import paper_2506_23712_amd as ens
    n, nu = 1024, 1.5e-3
    h = ens.HistSpec(qr_bins=256, log_bins=512, a_bins=1024, eps_ref=1.0, nu_ref=nu)
    E = ens.Ensemble(hist=h)
    m = E.add_member(ens.MemberSpec(n=n, nu=nu, eps_ref=1.0, kf_hi=2.5, dt=0.0, cfl=0.5, precision="fp32"))
    E.step(2)
    d = m.diag()
    assert not d["diverged"] and d["step"] == 2
    assert abs(d["cfl"] - 0.5) <= 1e-12 and abs(d["inj"] - 1.0) <= 1e-14
    u = m.state()
    k = torch.fft.fftfreq(n, 1.0 / n, dtype=torch.float64, device=u.device)
    kx = torch.arange(n // 2 + 1, dtype=torch.float64, device=u.device)
    div = (kx[None, None, :] * u[0] + k[None, :, None] * u[1] + k[:, None, None] * u[2]).abs().max().item()
    amp = u.abs().max().item() * (n // 3) * math.sqrt(3)
    assert div <= 1e-5 * amp
    w = torch.ones(n // 2 + 1, dtype=torch.float64, device=u.device); w[1:] = 2
    energy = 0.5 * float(((u.abs() ** 2).sum(dim=0) * w).sum())
    assert abs(energy - d["E"]) <= 1e-5 * d["E"]
    del u
    torch.cuda.empty_cache()
    E.accumulate_stats()
    counts, mom, npts = m.stats()
    assert npts == n ** 3
    split = h.split(counts.numpy())
    assert int(split["a_long"].sum() + split["a_long_special"].sum()) == 3 * n ** 3
    tau2 = nu / 1.0
    # nu <omega^2> = <eps> = D (within FP32 transform rounding)
    mean_eps = mom[12].item() / n ** 3
    mean_ens = mom[16].item() / n ** 3
    assert abs(mean_eps - d["D"]) <= 1e-4 * d["D"] and abs(mean_ens - d["D"]) <= 1e-4 * d["D"]
    assert abs(mom[20].item()) / n ** 3 <= 1e-4 * mom[22].item() / n ** 3
    E.close()
