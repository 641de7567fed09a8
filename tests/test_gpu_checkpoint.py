"""Checkpoint and resume on the GPU: a run split at a step boundary into two
contexts (the second loading the first's .npz file) ends bitwise where the
uninterrupted run ends -- velocity, diagnostics record, histogram counts and
moment sums -- for FP64 and FP32 members, CFL and fixed time steps, with
statistics snapshots before and after the split."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _specs(ens):
    return [ens.MemberSpec(n=32, nu=0.02, eps_ref=0.1, lam=-0.4, kf_lo=1.4, kf_hi=2.3, dt=0.0, cfl=0.5, seed=61),
            ens.MemberSpec(n=64, nu=0.02, eps_ref=0.1, lam=0.5, kf_lo=1.4, kf_hi=2.3, dt=0.0, cfl=0.5, seed=62,
                           precision="fp32"),
            ens.MemberSpec(n=32, nu=0.02, eps_ref=0.1, lam=0.0, kf_hi=2.0, dt=0.01, seed=63)]


def _hist(ens):
    return ens.HistSpec(qr_bins=64, log_bins=128, a_bins=256, eps_ref=0.1, nu_ref=0.02)


def _leg(E, ms, steps):
    for _ in range(steps // 10):
        E.step(10, members=ms)
        E.accumulate_stats(members=ms)


def _final(ms):
    out = []
    for m in ms:
        counts, mom, npts = m.stats()
        d = m.diag()
        out.append((m.state().cpu().numpy(), {k: v for k, v in d.items()}, counts.numpy(), mom.numpy(), npts))
    return out


def test_split_run_resumes_bitwise(tmp_path):
    import paper_2506_23712_amd as ens
    # uninterrupted
    E = ens.Ensemble(hist=_hist(ens))
    ms = [E.add_member(s) for s in _specs(ens)]
    _leg(E, ms, 30)
    _leg(E, ms, 30)
    ref = _final(ms)
    E.close()
    # first leg, checkpoint, new context, second leg
    E = ens.Ensemble(hist=_hist(ens))
    ms = [E.add_member(s) for s in _specs(ens)]
    _leg(E, ms, 30)
    path = str(tmp_path / "ck.npz")
    E.save_checkpoint(path)
    E.close()
    E2, ms2 = ens.Ensemble.load_checkpoint(path)
    assert [m.spec for m in ms2] == _specs(ens)
    assert all(m.diag()["step"] == 30 for m in ms2)
    _leg(E2, ms2, 30)
    got = _final(ms2)
    E2.close()
    for (u, d, c, mo, n), (ur, dr, cr, mr, nr) in zip(got, ref):
        assert np.array_equal(u, ur)
        assert d == dr
        assert np.array_equal(c, cr) and np.array_equal(mo, mr) and n == nr
    assert ref[0][1]["step"] == 60 and ref[0][4] == 6 * 32 ** 3


def test_restore_refuses_bad_records_and_other_histograms(tmp_path):
    import paper_2506_23712_amd as ens
    from paper_2506_23712_amd import _lib
    E = ens.Ensemble(hist=_hist(ens))
    m = E.add_member(_specs(ens)[0])
    E.step(3)
    ck = m.checkpoint()
    d = _lib.Diag.from_buffer_copy(ck["diag"])
    L = _lib.lib()
    for field, value in (("t", -1.0), ("t", float("nan")), ("step", -2), ("reserved", 1)):
        bad = _lib.Diag.from_buffer_copy(ck["diag"])
        setattr(bad, field, value)
        assert L.ens_member_set_diag(E.ctx, m.id, ctypes.byref(bad), None) == _lib.ENS_E_INVALID
    assert m.diag()["step"] == 3 and m.diag()["t"] == d.t                 # nothing written
    E.close()
    # a context with other histogram axes cannot take these statistics
    E = ens.Ensemble(hist=ens.HistSpec(qr_bins=32, log_bins=128, a_bins=256, eps_ref=0.1, nu_ref=0.02))
    m2 = E.add_member(_specs(ens)[0])
    with pytest.raises(ValueError):
        m2.restore(ck)
    E.close()
    # no histogram descriptor: the statistics call is refused
    E = ens.Ensemble()
    m3 = E.add_member(_specs(ens)[0])
    assert L.ens_set_stats(E.ctx, m3.id, None, None, None) == _lib.ENS_E_STATE
    m3.restore({"state": ck["state"], "diag": ck["diag"]})
    assert m3.diag()["step"] == 3
    E.close()
