"""The mixture entry point that allocates nothing (its member table is the
library's static device array) against ens_mix, the entry point it varies:
bitwise equal results on two calls in a row, the second with fewer members
(so that table entries of the first call stay behind in the array), and the
size limit refused on the host."""
import ctypes
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HK = dict(qr_bins=32, q_lo=-30.0, q_hi=30.0, r_lo=-60.0, r_hi=60.0, log_bins=128, log10_lo=-8.0,
          log10_hi=5.0, a_bins=128, a_lo=-100.0, a_hi=100.0, eps_ref=0.1, nu_ref=0.02)


def _mix_via_abi(E, members, fn, c, Z, mode, q_sigma):
    import torch
    from paper_2506_23712_amd import _lib
    L = _lib.lib()
    n = ctypes.c_size_t()
    _lib.check(L.ens_mix_len(E.ctx, len(members), ctypes.byref(n)))
    out = torch.full((n.value,), float("nan"), dtype=torch.float64, device="cuda")
    ids = (ctypes.c_int32 * len(members))(*[m.id for m in members])
    st = getattr(L, fn)(E.ctx, ids, len(members), c, Z, mode, q_sigma, ctypes.c_void_p(out.data_ptr()),
                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(st)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_mixture_equals_ens_mix_on_two_calls():
    import paper_2506_23712_amd as ens
    from paper_2506_23712_amd import _lib
    E = ens.Ensemble(hist=ens.HistSpec(**HK))
    lams = [-2.0 + 0.5 * i for i in range(9)]
    ms = [E.add_member(ens.MemberSpec(n=16, nu=0.02, eps_ref=0.1, lam=l, kf_hi=2.0, dt=0.01, seed=40 + i))
          for i, l in enumerate(lams)]
    E.step(3)
    E.accumulate_stats()
    E.step(2)
    E.accumulate_stats()
    calls = [(ms, 0.023, math.log(8), 0, 1.0),              # all nine members, open end bins
             (ms[2:7][::-1], 0.023, math.log(4), 1, 1.0)]   # then five, in another order, closed end bins
    for sel, c, Z, mode, qs in calls:
        ref = _mix_via_abi(E, sel, "ens_mix", c, Z, mode, qs)
        got = _mix_via_abi(E, sel, "ens_mix_noalloc", c, Z, mode, qs)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref)                      # same kernels, same inputs: bitwise
        assert abs(got[:len(sel)].sum() - 1.0) <= 1e-14      # weights
    # the binding's switch reaches the same entry point
    a, b = E.mix(0.023, math.log(2), noalloc=True), E.mix(0.023, math.log(2))
    assert np.array_equal(a["qr"].numpy(), b["qr"].numpy()) and a["S_long"] == b["S_long"]
    # sizes beyond the static table are refused on the host, before any copy
    L = _lib.lib()
    big = (ctypes.c_int32 * (_lib.ENS_MIX_STATIC_MAX + 1))(*range(_lib.ENS_MIX_STATIC_MAX + 1))
    assert L.ens_mix_noalloc(E.ctx, big, _lib.ENS_MIX_STATIC_MAX + 1, 0.023, 1.0, 0, 1.0,
                             ctypes.c_void_p(16), None) == _lib.ENS_E_INVALID
    assert b"static mixture table" in L.ens_last_error()
    E.close()
