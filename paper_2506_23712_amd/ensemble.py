"""Python view of the ensemble: members, stepping, statistics and the mixture.

Every computation happens in libensdns (HIP kernels for gfx950); this module
allocates device memory with torch, passes raw pointers and the current HIP
stream, and wraps results as tensors / dicts.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field

import torch

from . import _lib
from ._lib import check, lib


@dataclass
class MemberSpec:
    """One member: DNS at injection exp(lambda) * eps_ref, fixed band, viscosity nu."""
    n: int
    nu: float
    eps_ref: float = 1.0
    lam: float = 0.0
    kf_lo: float = 0.0
    kf_hi: float = 2.5
    dt: float = 0.0            # > 0 fixed step, else CFL step
    cfl: float = 0.5
    precision: str = "fp64"    # "fp64" or "fp32"
    box: float = 2 * math.pi
    seed: int = 23712
    k_peak: float = 2.0
    e0: float = 0.5
    visc_mode: int = 0

    def desc(self) -> _lib.MemberDesc:
        p = {"fp64": _lib.ENS_FP64, "fp32": _lib.ENS_FP32}[self.precision]
        return _lib.MemberDesc(self.n, p, self.box, self.nu, self.eps_ref, self.lam, self.kf_lo, self.kf_hi,
                               self.dt, self.cfl, self.seed, self.k_peak, self.e0, self.visc_mode, 0)


@dataclass
class HistSpec:
    """Histogram axes, in units of the reference (lambda = 0) member."""
    qr_bins: int = 64
    q_lo: float = -30.0
    q_hi: float = 30.0
    r_lo: float = -60.0
    r_hi: float = 60.0
    log_bins: int = 512
    log10_lo: float = -8.0
    log10_hi: float = 5.0
    a_bins: int = 1024
    a_lo: float = -100.0
    a_hi: float = 100.0
    eps_ref: float = 1.0
    nu_ref: float = 0.01

    def desc(self) -> _lib.HistDesc:
        return _lib.HistDesc(self.qr_bins, self.q_lo, self.q_hi, self.r_lo, self.r_hi, self.log_bins,
                             self.log10_lo, self.log10_hi, self.a_bins, self.a_lo, self.a_hi,
                             self.eps_ref, self.nu_ref)

    def split(self, counts):
        """Split a flat counts vector into named histograms (bins, specials)."""
        q, l, a = self.qr_bins, self.log_bins, self.a_bins
        out, o = {}, 0
        for name, nb in (("qr", q * q), ("log_eps", l), ("log_ens", l), ("a_long", a), ("a_trans", a)):
            out[name] = counts[o:o + nb]
            out[name + "_special"] = counts[o + nb:o + nb + 3]
            o += nb + 3
        out["qr"] = out["qr"].reshape(q, q)
        return out


def _stream_ptr() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ids(members) -> ctypes.Array:
    ids = [m.id for m in members]
    return (ctypes.c_int32 * len(ids))(*ids)


class Member:
    def __init__(self, ens: "Ensemble", spec: MemberSpec, mid: int, workspace: torch.Tensor):
        self.ens, self.spec, self.id, self.workspace = ens, spec, mid, workspace

    @property
    def n(self) -> int:
        return self.spec.n

    def state(self) -> torch.Tensor:
        """Velocity in the canonical layout: complex128 (3, N, N, N/2+1) on the device."""
        n = self.spec.n
        out = torch.empty((3, n, n, n // 2 + 1), dtype=torch.complex128, device=self.ens.device)
        check(lib().ens_member_get_state(self.ens.ctx, self.id, ctypes.c_void_p(out.data_ptr()), _stream_ptr()))
        return out

    def set_state(self, uhat: torch.Tensor) -> None:
        n = self.spec.n
        u = uhat.to(device=self.ens.device, dtype=torch.complex128).contiguous()
        if tuple(u.shape) != (3, n, n, n // 2 + 1):
            raise ValueError(f"state must have shape (3, {n}, {n}, {n // 2 + 1})")
        check(lib().ens_member_set_state(self.ens.ctx, self.id, ctypes.c_void_p(u.data_ptr()), _stream_ptr()))
        self._keep = u      # alive until the copy has run on the stream
        torch.cuda.current_stream().synchronize()

    def diag(self) -> dict:
        d = _lib.Diag()
        st = lib().ens_get_diag(self.ens.ctx, self.id, ctypes.byref(d))
        out = {name: getattr(d, name) for name, _ in _lib.Diag._fields_ if name != "reserved"}
        if st not in (_lib.ENS_OK, _lib.ENS_E_DIVERGED):
            check(st)
        out["diverged"] = st == _lib.ENS_E_DIVERGED
        return out

    def stats(self):
        """(counts uint64 tensor, moments float64 tensor, grid points summed)."""
        n = ctypes.c_size_t()
        check(lib().ens_stats_len(self.ens.ctx, ctypes.byref(n)))
        counts = torch.zeros(n.value, dtype=torch.int64)
        mom = torch.zeros(_lib.ENS_NMOM, dtype=torch.float64)
        npts = ctypes.c_uint64()
        check(lib().ens_get_stats(self.ens.ctx, self.id,
                                  ctypes.cast(counts.data_ptr(), ctypes.POINTER(ctypes.c_uint64)),
                                  ctypes.cast(mom.data_ptr(), ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(npts)))
        return counts, mom, npts.value

    def reset_stats(self) -> None:
        check(lib().ens_reset_stats(self.ens.ctx, self.id, _stream_ptr()))

    # ------------------------------------------------------------ checkpoints
    def checkpoint(self) -> dict:
        """Host copy of everything the member carries between steps: velocity
        (canonical layout, complex128), the diagnostics record (time, step
        count, ...) and, with a histogram descriptor, the statistics sums."""
        d = _lib.Diag()
        st = lib().ens_get_diag(self.ens.ctx, self.id, ctypes.byref(d))
        if st not in (_lib.ENS_OK, _lib.ENS_E_DIVERGED):
            check(st)
        out = {"state": self.state().cpu().numpy(), "diag": bytes(d)}
        if self.ens.hist is not None:
            counts, mom, _ = self.stats()
            out["counts"] = counts.numpy().astype("uint64")
            out["moments"] = mom.numpy()
        return out

    def restore(self, ck: dict) -> None:
        """Continue from `checkpoint()` output of a member of the same spec."""
        import numpy as np
        self.set_state(torch.from_numpy(np.asarray(ck["state"])))
        d = _lib.Diag.from_buffer_copy(bytes(ck["diag"]))
        check(lib().ens_member_set_diag(self.ens.ctx, self.id, ctypes.byref(d), _stream_ptr()))
        if "counts" in ck and self.ens.hist is not None:
            counts = np.ascontiguousarray(ck["counts"], dtype=np.uint64)
            mom = np.ascontiguousarray(ck["moments"], dtype=np.float64)
            n = ctypes.c_size_t()
            check(lib().ens_stats_len(self.ens.ctx, ctypes.byref(n)))
            if counts.size != n.value or mom.size != _lib.ENS_NMOM:
                raise ValueError("statistics of the checkpoint do not match this context's histograms")
            check(lib().ens_set_stats(self.ens.ctx, self.id,
                                      counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                      mom.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_ptr()))

    def spectrum(self, nshell: int | None = None) -> torch.Tensor:
        """Shell energy spectrum E[s], s = 0 .. nshell-1 (float64 on the device);
        by default every shell that holds retained modes."""
        if nshell is None:
            nshell = int(math.isqrt(3 * (self.spec.n // 3) ** 2)) + 2
        out = torch.empty(nshell, dtype=torch.float64, device=self.ens.device)
        check(lib().ens_spectrum(self.ens.ctx, self.id, nshell, ctypes.c_void_p(out.data_ptr()), _stream_ptr()))
        return out

    def integral_scales(self) -> torch.Tensor:
        """(E, u', L, T) as float64 on the device: energy, rms velocity, integral
        length and integral time from mode sums."""
        out = torch.empty(4, dtype=torch.float64, device=self.ens.device)
        check(lib().ens_integral_scales(self.ens.ctx, self.id, ctypes.c_void_p(out.data_ptr()), _stream_ptr()))
        return out

    def refine_from(self, src: "Member") -> None:
        """Take src's field on this member's (finer or equal) grid: retained modes
        of src kept, the rest zero; time and diagnostics carried over."""
        if src.ens is not self.ens:
            raise ValueError("both members must belong to the same ensemble")
        check(lib().ens_member_refine(self.ens.ctx, src.id, self.id, _stream_ptr()))


class Ensemble:
    def __init__(self, hist: HistSpec | None = None, device: int = 0, graphs: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required (libensdns has no CPU path)")
        self.device = torch.device("cuda", device)
        self.hist = hist
        L = lib()
        self.ctx = ctypes.c_void_p()
        hd = hist.desc() if hist is not None else None
        with torch.cuda.device(self.device):
            check(L.ens_create(ctypes.byref(self.ctx), device, ctypes.byref(hd) if hd is not None else None))
            check(L.ens_set_graphs(self.ctx, int(graphs)))
        self.members: list[Member] = []

    # ---------------------------------------------------------------- members
    def set_graph_mode(self, mode: int) -> None:
        """0 direct launches, 1 one graph per step, 2 the same with a branch per group."""
        check(lib().ens_set_graphs(self.ctx, mode))

    def workspace_bytes(self, spec: MemberSpec) -> int:
        b = ctypes.c_size_t()
        d = spec.desc()
        check(lib().ens_member_workspace_bytes(self.ctx, ctypes.byref(d), ctypes.byref(b)))
        return b.value

    def add_member(self, spec: MemberSpec) -> Member:
        nbytes = self.workspace_bytes(spec)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        d = spec.desc()
        mid = ctypes.c_int32()
        check(lib().ens_member_init(self.ctx, ctypes.byref(d), ctypes.c_void_p(ws.data_ptr() + off), nbytes,
                                    _stream_ptr(), ctypes.byref(mid)))
        m = Member(self, spec, mid.value, ws)
        self.members.append(m)
        return m

    # ------------------------------------------------------------ checkpoints
    def save_checkpoint(self, path: str, members=None, extra: dict | None = None) -> None:
        """Write the members' checkpoints, their specs and the histogram spec to
        one .npz file (plain arrays and JSON text; nothing pickled); `extra`
        (JSON-serialisable) is stored beside them for the caller."""
        import dataclasses
        import json
        import numpy as np
        ms = members if members is not None else self.members
        # the kernel variants in use: results are bitwise only under the same ones
        arrays = {"specs": np.array(json.dumps([dataclasses.asdict(m.spec) for m in ms])),
                  "hist": np.array(json.dumps(dataclasses.asdict(self.hist) if self.hist is not None else None)),
                  "variants": np.array(json.dumps(self.variants(ms))),
                  "extra": np.array(json.dumps(extra))}
        for k, m in enumerate(ms):
            ck = m.checkpoint()
            arrays[f"m{k}_state"] = ck["state"]
            arrays[f"m{k}_diag"] = np.frombuffer(ck["diag"], dtype=np.uint8)
            if "counts" in ck:
                arrays[f"m{k}_counts"] = ck["counts"]
                arrays[f"m{k}_moments"] = ck["moments"]
        np.savez(path, **arrays)

    @staticmethod
    def read_checkpoint_extra(path: str):
        """The `extra` object a checkpoint was written with (None if none)."""
        import json
        import numpy as np
        with np.load(path, allow_pickle=False) as z:
            return json.loads(str(z["extra"])) if "extra" in z.files else None

    @classmethod
    def load_checkpoint(cls, path: str, device: int = 0, graphs: bool = True):
        """New context and members from `save_checkpoint` output; returns
        (ensemble, members in the saved order)."""
        import json
        import numpy as np
        with np.load(path, allow_pickle=False) as z:
            specs = [MemberSpec(**s) for s in json.loads(str(z["specs"]))]
            h = json.loads(str(z["hist"]))
            E = cls(hist=HistSpec(**h) if h is not None else None, device=device, graphs=graphs)
            for key, v in json.loads(str(z["variants"])).items():
                pass_name, n, prec = key.split(":")
                E.set_variant(pass_name, int(n), prec, int(v))
            ms = []
            for k, spec in enumerate(specs):
                m = E.add_member(spec)
                ck = {"state": z[f"m{k}_state"], "diag": z[f"m{k}_diag"].tobytes()}
                if f"m{k}_counts" in z:
                    ck["counts"], ck["moments"] = z[f"m{k}_counts"], z[f"m{k}_moments"]
                m.restore(ck)
                ms.append(m)
        return E, ms

    # ----------------------------------------------------------------- stepping
    def step(self, nsteps: int = 1, members=None) -> None:
        ms = members if members is not None else self.members
        check(lib().ens_step(self.ctx, _ids(ms), len(ms), nsteps, _stream_ptr()))

    def profile_step(self, members=None) -> dict:
        ms = members if members is not None else self.members
        out = (ctypes.c_double * _lib.ENS_NPASS)()
        check(lib().ens_profile_step(self.ctx, _ids(ms), len(ms), _stream_ptr(), out))
        return dict(zip(_lib.PASS_NAMES, list(out)))

    def autotune(self, members=None, cache_path: str | None = None) -> dict:
        """Pick the fastest kernel variant per (pass, n, precision); returns the table."""
        ms = members if members is not None else self.members
        cp = cache_path.encode() if cache_path else None
        check(lib().ens_autotune(self.ctx, _ids(ms), len(ms), _stream_ptr(), cp))
        return self.variants(ms)

    def variants(self, members=None) -> dict:
        """Kernel variant in use per (pass, n, precision) of the members' sizes."""
        ms = members if members is not None else self.members
        out = {}
        for n, prec in sorted({(m.spec.n, m.spec.precision) for m in ms}):
            p = _lib.ENS_FP32 if prec == "fp32" else _lib.ENS_FP64
            for pid in (1, 2, 3, 4, 5):
                v = ctypes.c_int32()
                check(lib().ens_get_variant(self.ctx, pid, n, p, ctypes.byref(v)))
                out[f"{_lib.PASS_NAMES[pid]}:{n}:{prec}"] = v.value
        return out

    def set_variant(self, pass_name: str, n: int, precision: str, variant: int) -> None:
        p = _lib.ENS_FP32 if precision == "fp32" else _lib.ENS_FP64
        check(lib().ens_set_variant(self.ctx, _lib.PASS_NAMES.index(pass_name), n, p, variant))

    # --------------------------------------------------------------- statistics
    def accumulate_stats(self, members=None) -> None:
        ms = members if members is not None else self.members
        check(lib().ens_accumulate_stats(self.ctx, _ids(ms), len(ms), _stream_ptr()))

    def mix(self, c: float, Z: float, mode: int = 0, q_sigma: float = 1.0, members=None,
            noalloc: bool = False) -> dict:
        """Gaussian mixture of the members' statistics; noalloc=True uses the
        entry point whose member table is the library's static device array
        (the output tensor is still allocated here, by the caller)."""
        ms = members if members is not None else self.members
        out = self._mix_out(len(ms))
        fn = lib().ens_mix_noalloc if noalloc else lib().ens_mix
        check(fn(self.ctx, _ids(ms), len(ms), c, Z, mode, q_sigma, ctypes.c_void_p(out.data_ptr()), _stream_ptr()))
        return self._split_mix(out, len(ms))

    def mix_table(self, pdf: torch.Tensor, lam0: float, dlam: float, members=None) -> dict:
        """Mixture with weights from a tabulated lambda density (float64 device
        tensor sampled at lam0 + j dlam); same result layout as mix()."""
        ms = members if members is not None else self.members
        p = pdf.to(device=self.device, dtype=torch.float64).contiguous()
        out = self._mix_out(len(ms))
        check(lib().ens_mix_table(self.ctx, _ids(ms), len(ms), ctypes.c_void_p(p.data_ptr()), p.numel(), lam0, dlam,
                                  ctypes.c_void_p(out.data_ptr()), _stream_ptr()))
        return self._split_mix(out, len(ms))

    def _mix_out(self, count: int) -> torch.Tensor:
        n = ctypes.c_size_t()
        check(lib().ens_mix_len(self.ctx, count, ctypes.byref(n)))
        return torch.zeros(n.value, dtype=torch.float64, device=self.device)

    def _split_mix(self, out: torch.Tensor, count: int) -> dict:
        o = out.cpu()
        h = self.hist
        q, l, a, k = h.qr_bins, h.log_bins, h.a_bins, count
        res, pos = {}, 0
        for name, size in (("weights", k), ("qr", q * q), ("log_eps", l), ("log_ens", l), ("a_long", a),
                           ("a_trans", a), ("moments", _lib.ENS_NMOM), ("derived", 8)):
            res[name] = o[pos:pos + size]
            pos += size
        res["qr"] = res["qr"].reshape(q, q)
        d = res["derived"]
        res.update(S_long=float(d[0]), F_long=float(d[1]), H_long=float(d[2]), F_trans=float(d[3]),
                   H_trans=float(d[4]), mean_eps=float(d[5]), mean_ens=float(d[6]))
        return res

    def scale_gap(self, rlambda_ref: float, members=None) -> dict:
        """Z for a target R_lambda from the members' snapshot-averaged R_lambda
        (prefactor A of R_lambda = A e^(lambda/6) fitted over lambda >= 0)."""
        ms = members if members is not None else self.members
        Z, A = ctypes.c_double(), ctypes.c_double()
        rl = (ctypes.c_double * len(ms))()
        check(lib().ens_scale_gap(self.ctx, _ids(ms), len(ms), rlambda_ref, ctypes.byref(Z), ctypes.byref(A), rl))
        return {"Z": Z.value, "prefactor": A.value, "rlambda": list(rl)}

    def close(self) -> None:
        if self.ctx:
            torch.cuda.synchronize(self.device)
            lib().ens_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lambda_pdf_from_cf(phi: torch.Tensor, lam0: float, dlam: float) -> torch.Tensor:
    """Lambda density on lam0 + j dlam from exp(K(i omega_k; Z)) sampled at the FFT
    frequencies omega_k = 2 pi f_k / (M dlam) (complex128 device tensor of M values)."""
    if phi.dim() != 1 or not phi.is_cuda or phi.dtype != torch.complex128:
        raise ValueError("phi must be a 1-D complex128 device tensor")
    p = phi.contiguous()
    out = torch.empty(p.numel(), dtype=torch.float64, device=p.device)
    check(lib().ens_lambda_pdf_from_cf(ctypes.c_void_p(p.data_ptr()), p.numel(), lam0, dlam,
                                       ctypes.c_void_p(out.data_ptr()), _stream_ptr()))
    return out


def fft_pencils(x: torch.Tensor, sign: int) -> torch.Tensor:
    """Batched FFT of the columns of a (n, lines) complex device tensor (unnormalised)."""
    if x.dim() != 2 or not x.is_cuda:
        raise ValueError("x must be a 2-D device tensor (n, lines)")
    if x.dtype == torch.complex128:
        prec = _lib.ENS_FP64
    elif x.dtype == torch.complex64:
        prec = _lib.ENS_FP32
    else:
        raise ValueError("x must be complex64 or complex128")
    x = x.contiguous()
    out = torch.empty_like(x)
    check(lib().ens_fft_pencils(x.shape[0], prec, sign, x.shape[1], ctypes.c_void_p(x.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), _stream_ptr()))
    return out
