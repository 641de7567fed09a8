"""CPU FP64 oracle for the ensemble-DNS hot path (arXiv 2506.23712).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product package never imports
it.  It shares no code with the GPU library; the only thing both sides agree on
is the published definition of the counter-based generator (splitmix64) that
seeds initial fields, and the documented data layouts.

The numerical core is ``oracle.c`` (plain loops, own radix-2 FFT, OpenMP over
lines); this module marshals numpy arrays in and out of it.  The ensemble
mixture (a small amount of scalar math) lives in ``oracle.mixture``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _SO)
    return _SO


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("visc_mode", ctypes.c_int32),
                ("box", ctypes.c_double), ("nu", ctypes.c_double), ("eps", ctypes.c_double),
                ("kf_lo", ctypes.c_double), ("kf_hi", ctypes.c_double),
                ("dt", ctypes.c_double), ("cfl", ctypes.c_double)]


class HistDesc(ctypes.Structure):
    _fields_ = [("qr_bins", ctypes.c_int32), ("q_lo", ctypes.c_double), ("q_hi", ctypes.c_double),
                ("r_lo", ctypes.c_double), ("r_hi", ctypes.c_double),
                ("log_bins", ctypes.c_int32), ("log10_lo", ctypes.c_double), ("log10_hi", ctypes.c_double),
                ("a_bins", ctypes.c_int32), ("a_lo", ctypes.c_double), ("a_hi", ctypes.c_double),
                ("eps_ref", ctypes.c_double), ("nu_ref", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.or_fft1d.argtypes = [ctypes.c_int, dp, ctypes.c_int]
        L.or_fft3d.argtypes = [ctypes.c_int, dp, ctypes.c_int]
        L.or_init_field.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                    ctypes.c_double, ctypes.c_double, dp]
        L.or_rhs.argtypes = [ctypes.POINTER(Params), dp, dp, ctypes.c_int, dp]
        L.or_run.argtypes = [ctypes.POINTER(Params), dp, ctypes.c_int, ctypes.c_double, dp]
        L.or_stats.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(HistDesc), dp, u64p, dp, u64p, dp,
                               ctypes.c_double]
        L.or_counts_len.argtypes = [ctypes.POINTER(HistDesc)]
        L.or_counts_len.restype = ctypes.c_long
        L.or_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.or_splitmix64.restype = ctypes.c_uint64
        L.or_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


# --------------------------------------------------------------------------- FFT
def fft1d(x: np.ndarray, sign: int) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    if lib().or_fft1d(a.size, _dp(a), sign) != 0:
        raise ValueError("or_fft1d: bad size or sign")
    return a


def fft3d(x: np.ndarray, sign: int) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    n = a.shape[0]
    assert a.shape == (n, n, n)
    if lib().or_fft3d(n, _dp(a), sign) != 0:
        raise ValueError("or_fft3d: bad size or sign")
    return a


# ----------------------------------------------------------------- field layout
def canonical_shape(n: int):
    return (3, n, n, n // 2 + 1)


def modes(n: int, box: float = 2 * np.pi):
    """Integer mode numbers (m_z, m_y, m_x) broadcastable to the canonical layout."""
    m = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    m[n // 2] = n // 2
    mz = m[:, None, None]
    my = m[None, :, None]
    mx = np.arange(n // 2 + 1, dtype=np.int64)[None, None, :]
    return mz, my, mx


def retained_mask(n: int) -> np.ndarray:
    K = n // 3
    mz, my, mx = modes(n)
    return (np.abs(mz) <= K) & (np.abs(my) <= K) & (np.abs(mx) <= K)


def energy(uhat: np.ndarray) -> float:
    """(1/2) sum over the full spectrum of |u_hat|^2 (weight 2 for m_x > 0)."""
    w = np.ones(uhat.shape[-1]); w[1:] = 2.0
    return 0.5 * float(np.sum(np.abs(uhat) ** 2 * w))


def dissipation(uhat: np.ndarray, nu: float, box: float = 2 * np.pi) -> float:
    n = uhat.shape[1]
    dk = 2 * np.pi / box
    mz, my, mx = modes(n)
    k2 = dk * dk * (mz * mz + my * my + mx * mx)
    w = np.ones(uhat.shape[-1]); w[1:] = 2.0
    return nu * float(np.sum(k2 * np.abs(uhat) ** 2 * w))


def divergence_ratio(uhat: np.ndarray, box: float = 2 * np.pi) -> float:
    """max |k . u_hat| / max(|k| |u_hat|)."""
    n = uhat.shape[1]
    dk = 2 * np.pi / box
    mz, my, mx = modes(n)
    kd = dk * (mx * uhat[0] + my * uhat[1] + mz * uhat[2])
    kk = dk * np.sqrt((mz * mz + my * my + mx * mx).astype(float))
    den = np.max(kk * np.sqrt(np.sum(np.abs(uhat) ** 2, axis=0)))
    return float(np.max(np.abs(kd)) / den) if den > 0 else 0.0


# ---------------------------------------------------------- spectral diagnostics
def shell_index(m2):
    """Shell s of integer |m|^2 = m2: s - 1/2 <= |m| < s + 1/2 (no ties: |m|^2 is
    an integer and (s + 1/2)^2 never is)."""
    return np.floor(np.sqrt(np.asarray(m2, dtype=np.float64)) + 0.5).astype(np.int64)


def spectrum(uhat: np.ndarray, nshell: int) -> np.ndarray:
    """Shell energy spectrum of a field in the canonical layout, the quantity of
    the paper's energy-spectra figure (section describing the ensemble
    simulations): E[s] = (1/2) sum of |u_hat_m|^2 over the full spectrum for
    the modes of shell s (|m| in units of the wavenumber spacing; weight 2 for
    m_x > 0 in the half-spectrum layout).  Shells s >= nshell are dropped."""
    n = uhat.shape[1]
    mz, my, mx = modes(n)
    s = np.broadcast_to(shell_index(mz * mz + my * my + mx * mx), uhat.shape[1:])
    w = np.ones(uhat.shape[-1]); w[1:] = 2.0
    e = 0.5 * np.sum(uhat.real ** 2 + uhat.imag ** 2, axis=0) * w
    keep = s < nshell
    return np.bincount(s[keep].ravel(), weights=e[keep].ravel(), minlength=nshell)[:nshell]


def integral_scales(uhat: np.ndarray, box: float = 2 * np.pi):
    """(E, u', L, T) of a field in the canonical layout: the energy, the rms
    velocity u' = sqrt(2E/3), the integral length L = pi / (2 u'^2) times the
    sum over modes of e_m / |k_m| (the discrete form of the integral of E(k)/k),
    and the integral time T = L / u' that the paper measures run lengths and
    bootstrap windows in.  Sums over the full spectrum, e_m = |u_hat_m|^2 / 2."""
    n = uhat.shape[1]
    mz, my, mx = modes(n)
    m2 = np.broadcast_to(mz * mz + my * my + mx * mx, uhat.shape[1:]).astype(np.float64)
    w = np.ones(uhat.shape[-1]); w[1:] = 2.0
    e = 0.5 * np.sum(uhat.real ** 2 + uhat.imag ** 2, axis=0) * w
    E = float(e.sum())
    up2 = 2.0 * E / 3.0
    dk = 2 * np.pi / box
    nz = m2 > 0
    L = float(np.pi / (2 * up2) * np.sum(e[nz] / (dk * np.sqrt(m2[nz])))) if up2 > 0 else 0.0
    up = float(np.sqrt(up2))
    return E, up, L, (L / up if up > 0 else 0.0)


def refine(uhat: np.ndarray, n_big: int) -> np.ndarray:
    """Spectral refinement onto a finer grid (the paper replaces its most
    intense ensemble members by identical simulations at twice the resolution,
    section on extrapolating to the frontier): every retained mode |m_i| <= n/3
    of the n^3 field keeps its value on the n_big^3 grid, every other mode is
    zero.  Canonical layout in and out."""
    n = uhat.shape[1]
    K = n // 3
    if n_big < n:
        raise ValueError("refinement needs n_big >= n")
    out = np.zeros(canonical_shape(n_big), dtype=np.complex128)
    m = np.arange(-K, K + 1)
    src = m % n
    dst = m % n_big
    out[:, dst[:, None, None], dst[None, :, None], np.arange(K + 1)[None, None, :]] = \
        uhat[:, src[:, None, None], src[None, :, None], np.arange(K + 1)[None, None, :]]
    return out


# ----------------------------------------------------------------------- solver
@dataclass
class Member:
    """One ensemble member: grid, box, viscosity, injection, band, time step."""
    n: int
    nu: float
    eps: float
    kf_lo: float = 0.0
    kf_hi: float = 2.0
    dt: float = 0.01
    cfl: float = 0.5
    box: float = 2 * np.pi
    visc_mode: int = 0

    def params(self) -> Params:
        return Params(self.n, self.visc_mode, self.box, self.nu, self.eps,
                      self.kf_lo, self.kf_hi, self.dt, self.cfl)


def init_field(n: int, seed: int, k_peak: float = 2.0, e0: float = 0.5,
               box: float = 2 * np.pi) -> np.ndarray:
    out = np.zeros(canonical_shape(n), dtype=np.complex128)
    if lib().or_init_field(n, box, seed, k_peak, e0, _dp(out)) != 0:
        raise ValueError("or_init_field: bad arguments")
    return out


T_NONLINEAR, T_FORCING, T_VISCOUS = 1, 2, 4


def rhs(m: Member, uhat: np.ndarray, terms: int = T_NONLINEAR | T_FORCING):
    """G(u_hat) in the canonical layout; info = (E_f, injection, umax, imag ratio)."""
    u = np.ascontiguousarray(uhat, dtype=np.complex128)
    g = np.zeros_like(u)
    info = np.zeros(4)
    p = m.params()
    if lib().or_rhs(ctypes.byref(p), _dp(u), _dp(g), terms, _dp(info)) != 0:
        raise ValueError("or_rhs: bad arguments")
    return g, info


DIAG_NAMES = ("t", "dt", "E", "D", "inj", "E_f", "umax", "cfl")


def run(m: Member, uhat: np.ndarray, nsteps: int, t0: float = 0.0):
    """Advance ``nsteps`` RK3 steps; returns (u_hat, diag[nsteps, 8])."""
    u = np.ascontiguousarray(uhat, dtype=np.complex128).copy()
    diag = np.zeros((max(nsteps, 1), len(DIAG_NAMES)))
    p = m.params()
    rc = lib().or_run(ctypes.byref(p), _dp(u), nsteps, t0, _dp(diag))
    if rc != 0:
        raise RuntimeError(f"or_run failed ({rc})")
    return u, diag[:nsteps]


@dataclass
class Hist:
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

    def desc(self) -> HistDesc:
        return HistDesc(self.qr_bins, self.q_lo, self.q_hi, self.r_lo, self.r_hi,
                        self.log_bins, self.log10_lo, self.log10_hi,
                        self.a_bins, self.a_lo, self.a_hi, self.eps_ref, self.nu_ref)

    def split(self, counts: np.ndarray) -> dict:
        """Split a flat counts vector into named histograms (bins, specials)."""
        q, l, a = self.qr_bins, self.log_bins, self.a_bins
        out, o = {}, 0
        for name, nb in (("qr", q * q), ("log_eps", l), ("log_ens", l), ("a_long", a), ("a_trans", a)):
            out[name] = counts[o:o + nb]
            out[name + "_special"] = counts[o + nb:o + nb + 3]
            o += nb + 3
        out["qr"] = out["qr"].reshape(q, q)
        return out


NMOM = 32


def stats(m: Member, h: Hist, uhat: np.ndarray, grad_tol: float = 0.0):
    """Gradient statistics of one snapshot: (counts, moments, near_edge, max|Tr A|).

    near_edge[k] counts the samples of histogram k (QR, log eps, log Omega,
    A_L, A_T) whose bin may differ on a path that rounds differently: bin
    coordinate within 1e-9 (relative) of an edge, or, with grad_tol > 0,
    within the first-order change caused by gradient errors up to
    grad_tol * max|A_ij| (the bound a path with FP32 transforms is held to)."""
    u = np.ascontiguousarray(uhat, dtype=np.complex128)
    d = h.desc()
    counts = np.zeros(int(lib().or_counts_len(ctypes.byref(d))), dtype=np.uint64)
    mom = np.zeros(NMOM)
    near = np.zeros(5, dtype=np.uint64)
    trmax = np.zeros(1)
    p = m.params()
    rc = lib().or_stats(ctypes.byref(p), ctypes.byref(d), _dp(u),
                        counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _dp(mom),
                        near.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _dp(trmax), float(grad_tol))
    if rc != 0:
        raise ValueError("or_stats: bad arguments")
    return counts, mom, near, float(trmax[0])


def splitmix64(seed: int, counter: int) -> int:
    return int(lib().or_splitmix64(seed, counter))
