// ens_internal.h -- types shared by the host side and the kernels of libensdns.
// Not part of the public ABI (include/ens.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/ens.h"

namespace ens {

// The linear band forcing eps/(2 E_f) u is singular as E_f -> 0.  A band
// holding no more than this fraction of the member's energy at the start of
// the step (the energy of the previous step's end, or of the field as set)
// is treated as empty and not forced: rounding puts about 1e-30 (FP64) or
// 1e-13 (FP32) of the energy into a band that should be empty.
constexpr double kForceEmptyFrac = 1e-10;

// Per-member scalars kept in device memory.  `diag` is what ens_get_diag
// returns; the rest carries values between kernels of one step.
struct DevState {
    ens_diag diag;
    double Ef;                       // band energy of the current stage (FP64)
    double dt;                       // time step of the current step
    unsigned long long umax_bits;    // max(|u|+|v|+|w|) as bits of a non-negative double
    double e_init;                   // energy of the raw initial field (init only)
    double pad[4];
};

// Pitch of the x-mode (fastest) index of the statistics pass's pencil
// buffers, which its z/y inverses write in runs of one 128-byte line per
// position: K + 1 rounded up to whole lines (16 FP32 / 8 FP64 complex
// values), the pad entries written as zeros, so that every store covers whole
// lines.  A line shared by two workgroups, each writing part of it, is
// written back twice at far lower bandwidth.  `cbytes` is the size of one
// complex value.  Where the padding would exceed 1/8 of a row (short rows:
// n <= 64 FP32, n <= 32 FP64) the rows are left unpadded.  (The time-step
// passes need no pad: their lines are numbered so that every run they store
// is a whole number of lines; see MemberDev.)
__host__ __device__ constexpr int kx_pitch(int K, int cbytes) {
    const int per = 128 / cbytes, px = (K + 1 + per - 1) / per * per;
    return 8 * (px - (K + 1)) <= K + 1 ? px : K + 1;
}

__host__ __device__ constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }

// Plane pitch of the state arrays (u_hat and the RK register, [3][2K+1 (kz)]
// [ZP]): the (2K+1)(K+1) modes of one kz plane rounded up to whole 128-byte
// lines, so that every plane and every field starts on a line and the z-line
// tiles of the z passes (16 FP32 / 8 FP64 consecutive lines of a plane) load
// and store whole lines.  The pad entries of a plane are never read.
__host__ __device__ constexpr int state_pitch(int K, int cbytes) {
    const int per = 128 / cbytes, p = (2 * K + 1) * (K + 1);
    return (p + per - 1) / per * per;
}

// Everything a kernel needs to know about one member (lives in a device
// table owned by the library; pointers refer to the caller's workspace).
// KX = K + 1 x-modes, NZLS = (2K+1) KX modes per z plane, ZP = state_pitch,
// NYL = n KX; the y-pencil buffers hold blocks of ZB consecutive z rows,
// BL = ZB KX values per position, ZB the fewest rows that fill whole 128-byte
// lines (8 FP32 / 4 FP64 at n = 256).  Layouts of a time step (x-mode index
// fastest, no row pad): every y/z pass numbers its lines so that a
// workgroup's consecutive lines are consecutive in the buffer it writes, and
// a run of 16 (FP32) / 8 (FP64) lines per position is one whole 128-byte line.
struct MemberDev {
    void *uh;          // velocity  [3][2K+1 (kz)][ZP: 2K+1 (ky) x K+1 (kx), then pad] complex
    void *q;           // RK register, same layout
    void *bufA;        // z-inverse out [5][n (z)][ZP] (planes as in uh, pad zeroed) /
                       // x-pass out [3][n / ZB][n (y)][ZB (z)][KX] (the rows of its input)
    void *bufB;        // y-inverse out [6][n / ZB][n (y)][BL = ZB (z) x KX] /
                       // y-forward out [3][n / ZB][2K+1 (ky)][BL]
                       // (statistics: [6][n][2K+1][PX] and [9][n][n][PX], PX = kx_pitch)
    DevState *st;      // diag.E: energy at the end of the last step (or of the field as set)
    double *partials;  // per-workgroup FP64 partial sums
    unsigned long long *counts;   // statistics counters
    double *moments;              // ENS_NMOM sums
    double nu, eps_m, kf_lo2, kf_hi2, dt_fixed, cfl, box, dk;
    int n, K, prec, visc_mode;
    int px;            // x-mode pitch PX of the statistics pass's buffers
    int zp;            // state plane pitch ZP = state_pitch(K, complex size)
};

// Host-visible geometry of one member.
struct Geom {
    int n, K, px;
    long long nzl;     // z-lines of the statistics pass's buffers = (2K+1) PX (pad lines included)
    long long zp;      // state plane pitch ZP
    long long S;       // state elements per component = (2K+1) ZP (pad entries included)
    long long nyl;     // y-lines of the time-step buffers = n (K+1)
};

inline Geom make_geom(int n, int prec) {
    Geom g;
    g.n = n; g.K = n / 3;
    g.px = kx_pitch(g.K, prec == ENS_FP32 ? 8 : 16);
    g.nzl = (long long)(2 * g.K + 1) * g.px;
    g.zp = state_pitch(g.K, prec == ENS_FP32 ? 8 : 16);
    g.S = (long long)(2 * g.K + 1) * g.zp;
    g.nyl = (long long)n * (g.K + 1);
    return g;
}

// Histogram geometry (from ens_hist_desc).
struct HistGeom {
    int qb, lb, ab;
    long long n_counts;
    long long off_qr, off_le, off_lw, off_al, off_at;
};

inline HistGeom make_hist_geom(const ens_hist_desc &h) {
    HistGeom g;
    g.qb = h.qr_bins; g.lb = h.log_bins; g.ab = h.a_bins;
    g.off_qr = 0;
    g.off_le = (long long)g.qb * g.qb + 3;
    g.off_lw = g.off_le + g.lb + 3;
    g.off_al = g.off_lw + g.lb + 3;
    g.off_at = g.off_al + g.ab + 3;
    g.n_counts = g.off_at + g.ab + 3;
    return g;
}

// Passes timed by ens_profile_step.
enum Pass { P_BAND = 0, P_ZINV = 1, P_YINV = 2, P_XPASS = 3, P_YFWD = 4, P_ZFWD = 5, P_END = 6 };

// Launchers (defined in the .hip files).  `mem` points to a device array of
// `count` MemberDev of one size n and precision; grids cover all of them.
// `variant` selects a compiled kernel variant (0: 8 values per thread,
// 1: 16 values per thread; y/z passes 2, 3: the same with twice the lines
// per workgroup; x pass 2 to 6: the streamed and wave-private passes, see
// ens_autotune in ens.h; z forward 1: fused with the next stage's z inverse,
// 2 (not selectable by callers): the last stage too, for a step followed by
// another in the same call) for passes with pass_variants(pass) > 1.
hipError_t launch_pass(int pass, int variant, int n, int prec, const MemberDev *mem, int count, int stage,
                       const void *tw, hipStream_t s);
int pass_variants(int pass);
int default_variant(int pass, int n, int prec);

hipError_t launch_init_field(int n, int prec, const MemberDev *mem, uint64_t seed, double k_peak, double e0, hipStream_t s);
hipError_t launch_set_state(int n, int prec, const MemberDev *mem, const double *src, hipStream_t s);
hipError_t launch_get_state(int n, int prec, const MemberDev *mem, double *dst, hipStream_t s);

hipError_t launch_grad_zinv(int n, int prec, const MemberDev *mem, int count, const void *tw, hipStream_t s);
hipError_t launch_grad_yinv(int n, int prec, const MemberDev *mem, int count, const void *tw, hipStream_t s);
hipError_t launch_grad_xstats(int n, int prec, const MemberDev *mem, int count, const ens_hist_desc &h,
                              const double *ledge, const void *tw, hipStream_t s);
hipError_t launch_stats_reduce(int n, int prec, const MemberDev *mem, int count, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, long long n, unsigned long long v, hipStream_t s);
hipError_t launch_fill_f64(double *p, long long n, double v, hipStream_t s);

hipError_t launch_fft_pencils(int n, int prec, int sign, long long lines, const void *in, void *out,
                              const void *tw, hipStream_t s);

hipError_t launch_mix(const MemberDev *const *members_host, const double *lambdas, int count,
                      const ens_hist_desc &h, double c, double Z, int mode, double q_sigma,
                      double *out, void *scratch, hipStream_t s);

size_t mix_scratch_bytes(int count);
int mix_max_members();
// Mixture with the member table in the library's static device array (no
// allocation).  mix_static_setup(device) takes that array's device address on
// `device`, which must be current; launch_mix_static uses it.
hipError_t mix_static_setup(int device);
size_t mix_static_bytes();
hipError_t launch_mix_static(int device, const MemberDev *const *members_host, const double *lambdas, int count,
                             const ens_hist_desc &h, double c, double Z, int mode, double q_sigma, double *out,
                             hipStream_t s);

// Number of workgroups that write FP64 partials, per member.
long long zfwd_blocks(int n, int prec);
long long xstats_blocks(int n);
bool stats_hist_fits(const ens_hist_desc &h);   // 1-D histograms and log edges fit the statistics kernel's LDS
long long init_blocks(int n);

}  // namespace ens
