/*
 * ens.h -- C ABI of libensdns: an ensemble of forced, periodic-box,
 * incompressible Navier-Stokes simulations, time-stepped by the Fourier
 * pseudo-spectral method on one AMD Instinct MI355X (gfx950), with the
 * velocity-gradient statistics and the Gaussian-in-lambda mixture of
 * arXiv 2506.23712 (Bentkamp & Wilczek, "Predicting any small-scale
 * statistics of high-Reynolds-number turbulence using ensemble simulations").
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every function returns ens_status (0 = ENS_OK, < 0 = error) and never
 *    throws or aborts.  ens_last_error() gives a thread-local message for the
 *    last failing call.
 *  - Arguments are validated before anything is changed: an ENS_E_INVALID
 *    return leaves the context as it was.  A failing HIP call returns
 *    ENS_E_HIP and poisons the context; after that only ens_destroy is allowed.
 *  - The caller owns all device memory (workspaces, input and output arrays)
 *    and keeps it alive until ens_destroy.  The library owns host metadata,
 *    HIP graphs and small device tables (twiddles, member table) only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    are asynchronous on that stream unless the comment says they synchronise.
 *  - Grid: N points per direction on [0, L)^3, Delta k = 2 pi / L, wavevector
 *    k = Delta k * m.  Retained set D: |m_x|, |m_y|, |m_z| <= K = floor(N/3)
 *    (cubic 2/3 truncation; the paper does not state its dealiasing rule).
 *  - Canonical spectral layout (set/get state): FP64 complex interleaved
 *    [3][N (m_z)][N (m_y)][N/2+1 (m_x)], m_x contiguous, FFT index order
 *    (index i > N/2 means m = i - N), zero outside D, forward normalisation
 *    u_hat = N^-3 sum_x u(x) exp(-i k.x).
 */
#ifndef ENS_H
#define ENS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ENS_OK = 0,
    ENS_E_INVALID = -1,      /* bad argument; nothing changed */
    ENS_E_OOM = -2,          /* a workspace is smaller than required */
    ENS_E_HIP = -3,          /* a HIP call failed; the context is poisoned */
    ENS_E_UNSUPPORTED = -4,  /* valid request this library does not provide */
    ENS_E_STATE = -5,        /* call not allowed in the current state */
    ENS_E_DIVERGED = -6      /* a member has non-finite energy or no CFL velocity */
} ens_status;

enum { ENS_FP64 = 0, ENS_FP32 = 1 };

typedef struct ens_ctx ens_ctx;   /* opaque, owned by the library */

/* One ensemble member: a DNS at (L, e^lambda eps_ref, nu) with a fixed forcing
 * band (section "Description of the ensemble simulations": same band and
 * viscosity across the ensemble, injection e^lambda times that of the central
 * member; band [1.4, 2.3] Delta k and CFL 0.2 in the paper). */
typedef struct {
    int32_t  n;          /* grid points per direction: 16, 32, 64, 128, 256, 512, 1024 */
    int32_t  precision;  /* ENS_FP64 or ENS_FP32 for transforms and right-hand side;
                            band energy, dt, reductions and accumulators are FP64 */
    double   box;        /* L > 0 */
    double   nu;         /* kinematic viscosity >= 0 */
    double   eps_ref;    /* injection of the central member */
    double   lambda;     /* this member injects eps_m = exp(lambda) * eps_ref */
    double   kf_lo, kf_hi;  /* forcing band in units of Delta k, inclusive:
                               0 < |m|^2 and kf_lo^2 <= |m|^2 <= kf_hi^2 */
    double   dt;         /* > 0: fixed time step; <= 0: CFL step */
    double   cfl;        /* dt = cfl * (L/N) / max_x(|u|+|v|+|w|) from the stage-1 field */
    uint64_t seed;       /* initial field seed (splitmix64, see ens_member_init) */
    double   k_peak;     /* initial shell spectrum k^4 exp(-2 (k/k_peak)^2) */
    double   e0;         /* initial energy (1/2) sum |u_hat|^2 */
    int32_t  visc_mode;  /* 0: integrating factor (exact viscous decay), 1: explicit */
    int32_t  reserved;   /* must be 0 */
} ens_member_desc;

/* Histogram axes for the gradient statistics.  All members bin on the same
 * absolute axes, in units of the reference (lambda = 0) member:
 * tau = sqrt(nu_ref/eps_ref), <Tr S^2>_ref = eps_ref / (2 nu_ref),
 * Q* = Q/<TrS^2>_ref, R* = R/<TrS^2>_ref^(3/2), eps* = eps/eps_ref,
 * Omega* = omega^2 nu_ref/eps_ref, A* = A tau. */
typedef struct {
    int32_t qr_bins;  double q_lo, q_hi, r_lo, r_hi;    /* joint Q*-R* histogram */
    int32_t log_bins; double log10_lo, log10_hi;        /* log10 eps*, log10 Omega* */
    int32_t a_bins;   double a_lo, a_hi;                /* pooled A*_ii and A*_ij (i != j) */
    double  eps_ref, nu_ref;
} ens_hist_desc;

/* Per-member diagnostics (FP64), refreshed at the end of every step. */
typedef struct {
    double  t, dt;       /* time after the last step, and that step's dt */
    double  E, D;        /* (1/2) sum |u_hat|^2 and nu sum k^2 |u_hat|^2 after the step */
    double  inj;         /* injection rate of the last stage-1 forcing (= eps_m) */
    double  E_f;         /* band energy at stage 1 of the last step */
    double  umax;        /* max_x(|u|+|v|+|w|) at stage 1 of the last step */
    double  cfl;         /* dt * umax / dx */
    double  rlambda;     /* u'^2 sqrt(15/(nu D)), u'^2 = 2E/3 */
    double  kmax_eta;    /* K Delta k (nu^3/D)^(1/4) */
    int64_t step;        /* steps taken */
    int32_t flags;       /* bit 0: non-finite energy, bit 1: zero band energy,
                            bit 2: zero CFL velocity */
    int32_t reserved;
} ens_diag;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  `h` fixes the histogram axes of
 * every member (may be NULL: statistics calls then return ENS_E_STATE); its
 * ranges must be finite with hi > lo and its reference scales finite and
 * positive, else ENS_E_INVALID before any device call. */
ens_status ens_create(ens_ctx **out, int device, const ens_hist_desc *h);

/* Free host metadata, graphs and device tables.  Caller memory is not freed. */
ens_status ens_destroy(ens_ctx *ctx);

/* Thread-local message of the last failing call ("" if none). */
const char *ens_last_error(void);

/* 1: capture one RK step of a member set as a HIP graph and replay it
 * (default); 2: the same graph with one branch per group of members of equal
 * grid size and precision, so that the groups' kernels may run side by side;
 * 0: launch kernels directly.  Changing the mode synchronises the device and
 * drops the graphs captured so far.  ENS_E_INVALID for other values. */
ens_status ens_set_graphs(ens_ctx *ctx, int32_t mode);

/* ---------------------------------------------------------------- members */

/* Device bytes one member needs (state, RK register, transform buffers,
 * statistics accumulators), for the context's histogram axes. */
ens_status ens_member_workspace_bytes(const ens_ctx *ctx, const ens_member_desc *d,
                                      size_t *bytes);

/* Register a member on caller device memory `dev_workspace` (>= the size from
 * ens_member_workspace_bytes, 256-byte aligned) and fill its initial field:
 * for every retained half-space mode, six normal deviates from splitmix64
 * (output number c of a generator seeded with d->seed, where
 * c = (((m_z+2048)*4096 + (m_y+2048))*4096 + (m_x+2048))*8 + j, j = 0..5,
 * uniform ((x>>11)+0.5)*2^-53, Box-Muller pairs (j, j+1)) form a complex
 * 3-vector a; a is projected perpendicular to k and scaled to length
 * sqrt(E(|k|)/(4 pi |k|^2)), E(k) = k^4 exp(-2 (k/k_peak)^2); the m_x = 0 plane
 * is made Hermitian; finally the field is scaled to energy e0.  Statistics are
 * zeroed, t = 0.  Runs on the GPU on `stream`.  The paper only requires members
 * to be forced homogeneous isotropic turbulence at a prescribed injection rate
 * (section "Description of the ensemble simulations"). */
ens_status ens_member_init(ens_ctx *ctx, const ens_member_desc *d, void *dev_workspace,
                           size_t bytes, void *stream, int32_t *member_id);

/* Replace member m's velocity with a device array in the canonical layout
 * (modes outside D are ignored; m_x = 0 entries are used as given). */
ens_status ens_member_set_state(ens_ctx *ctx, int32_t m, const double *dev_uhat, void *stream);

/* Write member m's velocity into a device array in the canonical layout. */
ens_status ens_member_get_state(ens_ctx *ctx, int32_t m, double *dev_uhat, void *stream);

/* ------------------------------------------------------------ time stepping */

/* Advance `count` members by `nsteps` steps of the low-storage integrating-
 * factor RK3 (Williamson 2N coefficients A = (0,-5/9,-153/128),
 * B = (1/3,15/16,8/15); q <- E_s (A_s q + dt G(u)), u <- E_s u + B_s q with
 * E_s = exp(-nu k^2 h_s dt), h = (1/3,5/12,1/4)).  G = P(u x omega + f):
 * rotational nonlinear term by inverse transforms of u and omega = i k x u,
 * forward transform truncated to D, band forcing f = eps_m / (2 E_f) u on the
 * band with E_f its FP64 energy at the stage (the paper's forcing amplifies
 * band coefficients every step so that the injection rate is fixed, section
 * "Description of the ensemble simulations"), projection perpendicular to k
 * of the sum.  The velocity is real and solenoidal; parts of the stored
 * spectrum that are not (rounding) would be invisible to the nonlinear term
 * and grow under the linear forcing, so the forcing is projected with the
 * nonlinear term and, at every stage, the band's part of the m_x = 0 plane
 * is made Hermitian in place before E_f is summed.
 * Members may differ in N and precision.  Device-side dt: members with dt <= 0
 * take the CFL step from their stage-1 field.  With the fused z forward
 * (pass 5 variant 1, the default for n <= 512) every step of a call but the
 * last also performs the next step's first z inverse, so splitting the same
 * steps into calls differently changes results at the rounding level; the
 * same sequence of calls is bitwise reproducible.  Asynchronous on `stream`. */
ens_status ens_step(ens_ctx *ctx, const int32_t *members, int32_t count, int32_t nsteps,
                    void *stream);

/* Same as one ens_step, launched without graphs, with HIP events around every
 * kernel on `stream`; synchronises.  ms_out[p] (p < ENS_NPASS) receives the
 * summed kernel time of pass p: 0 band energy, 1 z inverse + curl,
 * 2 y inverse, 3 x fused (c2r, u x omega, r2c), 4 y forward,
 * 5 z forward + projection + forcing + update, 6 end-of-step reduction.
 * With the fused z forward (pass 5 variant 1) the z inverse of stages 2 and
 * 3 runs inside pass 5 and is counted there. */
#define ENS_NPASS 7
ens_status ens_profile_step(ens_ctx *ctx, const int32_t *members, int32_t count, void *stream,
                            double *ms_out);

/* Diagnostics of member m (synchronises the stream of the member's last call). */
ens_status ens_get_diag(ens_ctx *ctx, int32_t m, ens_diag *out);

/* ---------------------------------------------------------------- tuning */

/* Time the compiled variants of the transform passes (1 z inverse, 2 y
 * inverse, 3 x pass, 4 y forward; variant 0 = 8, 1 = 16 complex values per
 * thread; z inverse, y inverse and y forward variants 2 and 3 = 8 and 16
 * values per thread with twice the lines per workgroup (two 128-byte lines
 * per position) where the thread budget allows, else as 0 and 1; x pass
 * variant 2 = persistent workgroups streaming their inputs by
 * direct-to-LDS loads, 8 values per thread, the same as variant 0 for n < 64;
 * variant 3 = the same with 16 values per thread for FP32 and 128 <= n <= 512,
 * else variant 2; variants 4 and 5 = the streamed pass with one wave per
 * workgroup and every transform exchange inside the wave, 16 or 8 (FP32) /
 * 8 or 4 (FP64) values per thread, n >= 64, else variant 2; variant 6 =
 * variant 4 with its inputs staged pairwise through two buffers, less LDS
 * per wave)
 * on the grid sizes and precisions of `members`, and keep the fastest
 * per (pass, n, precision) for later steps (the x pass timed in its place,
 * each launch after the y inverse that writes its inputs).  Only scratch buffers are written:
 * member state is unchanged.  `cache_path` (may be NULL) names a text file of
 * "pass:n:precision variant" lines: entries found there are used without
 * timing, and the file is rewritten with the full table.  Synchronises. */
ens_status ens_autotune(ens_ctx *ctx, const int32_t *members, int32_t count, void *stream,
                        const char *cache_path);

/* Force / query the variant of one (pass, n, precision).  Invalidates graphs.
 * Besides the timed passes above, pass 5 (z forward + update) has two
 * variants, chosen by default and not timed by ens_autotune (it updates the
 * state): 0 = the z inverse of every RK stage is a launch of its own; 1 = the
 * z forward of the first two stages also performs the next stage's z inverse
 * from the velocity it has just updated, so each step reads the velocity back
 * once instead of three times, and inside one ens_step call of several steps
 * the last stage does the same for the next step (default for n <= 512). */
ens_status ens_set_variant(ens_ctx *ctx, int32_t pass, int32_t n, int32_t precision, int32_t variant);
ens_status ens_get_variant(const ens_ctx *ctx, int32_t pass, int32_t n, int32_t precision, int32_t *variant);

/* --------------------------------------------------------------- statistics */

/* Accumulate one snapshot of velocity-gradient statistics per member from its
 * current field: A_ij = d_j u_i (all nine, by inverse transforms of i k_j u_i),
 * Q = -Tr(A^2)/2, R = -Tr(A^3)/3 (section "Benchmarking the method against
 * DNS data"), eps = 2 nu S_ij S_ij and omega^2 (section "Extrapolating to the
 * frontier ..."), moments of gradient components to order 6 (section
 * "Modeling choices", eq. def_skewness_flatness).  Values are formed in FP64;
 * counts are uint64, sums FP64.  Bin rule: NaN -> nan counter; x < lo ->
 * underflow; b = floor((x - lo) * (nb / (hi - lo))); b >= nb -> overflow. */
ens_status ens_accumulate_stats(ens_ctx *ctx, const int32_t *members, int32_t count, void *stream);

/* Number of uint64 counters and FP64 moments per member:
 * counts = [QR qb*qb (Q-major, R fastest), outside, 0, nan]
 *          [log eps* lb, under, over, nan] [log Omega* lb, under, over, nan]
 *          [A_L ab, under, over, nan] [A_T ab, under, over, nan];
 * moments (32) = [0..5] sum A*_L^p, [6..11] sum A*_T^p (p = 1..6; 3 and 6
 * samples per point), [12..15] sum eps*^p, [16..19] sum Omega*^p (p = 1..4),
 * [20] sum Q*, [21] sum R*, [22] sum S*_ij S*_ij, [23] sum (Tr A*)^2,
 * [24] sum Q*^2, [25] sum R*^2, [26] sum over snapshots of the member's
 * energy E and [27] of its dissipation D (the values of its last step, i.e. of
 * the field the snapshot sees), [28] number of snapshots, [29..31] 0. */
#define ENS_NMOM 32
ens_status ens_stats_len(const ens_ctx *ctx, size_t *n_counts);

/* Copy member m's accumulated statistics to host memory (synchronises).
 * counts: n_counts uint64; moments: ENS_NMOM doubles; n_points: grid points summed. */
ens_status ens_get_stats(ens_ctx *ctx, int32_t m, uint64_t *counts, double *moments,
                         uint64_t *n_points);

/* Zero member m's statistics (asynchronous on `stream`). */
ens_status ens_reset_stats(ens_ctx *ctx, int32_t m, void *stream);

/* ------------------------------------------------------------ checkpointing */

/* Members run for tens of integral times after their transient (section
 * "Description of the ensemble simulations"), which a long run may have to
 * split over several processes.  A member's checkpoint at a step boundary is
 * its velocity (ens_member_get_state), its ens_diag record (ens_get_diag:
 * time, step count, last dt, diagnostics, flags) and its statistics sums
 * (ens_get_stats).  Restored into a member of the same descriptor, in a
 * context of the same histogram descriptor, with ens_member_set_state and the
 * two calls below, the member continues bitwise as the uninterrupted run
 * would: between steps the RK register holds nothing the next step reads,
 * and the band energy and the CFL velocity are recomputed by that step. */

/* Restore member m's clock and diagnostics from a record `d` that
 * ens_get_diag returned.  Refuses (ENS_E_INVALID, nothing written) a record
 * with a negative or non-finite time, a negative step count or reserved != 0.
 * Host record; returns after the copy has completed on `stream`. */
ens_status ens_member_set_diag(ens_ctx *ctx, int32_t m, const ens_diag *d, void *stream);

/* Replace member m's statistics sums with host arrays as ens_get_stats
 * returns them: `counts` (ens_stats_len entries) and `moments` (ENS_NMOM
 * entries); either may be NULL to keep that part.  Needs a histogram
 * descriptor (ENS_E_STATE otherwise).  Returns after the copies have
 * completed on `stream`. */
ens_status ens_set_stats(ens_ctx *ctx, int32_t m, const uint64_t *counts, const double *moments, void *stream);

/* ------------------------------------------------------------------ mixture */

/* Mix the statistics of `count` members with Gaussian weights in lambda
 * (eq. ensemble_hypothesis and eq. pdf_superposition; P(lambda; Z) Gaussian
 * with mean -9cZ/2 and variance 9cZ for quadratic exponents with parameter c,
 * eq. gaussian_lambda_pdf; each member gets the mass of its lambda bin).
 * Bins: members sorted by lambda, edges at midpoints; mode 0: end bins open to
 * +-inf; mode 1: end bins closed at half a spacing, weights renormalised;
 * mode 2: w_i proportional to P(lambda_i; Z)/q(lambda_i), q = N(0, q_sigma^2);
 * mode 3: the truncated Gaussian of the appendix (eq. truncated_gaussian:
 * variance 9cZ, support lambda <= Z, its mean set on the host by bisection so
 * that the mean-injection constraint, eq. mean_injection_constraint, holds),
 * bins as in mode 0, each member the mass of its bin below Z.
 * Z = 0 puts all weight on the member whose bin holds lambda = 0.
 * Mixed moments [26..31] are 0 (the snapshot sums of E and D are per member).
 * Writes to device memory `dev_out` (FP64, ens_mix_len elements):
 *   [weights: count][QR pdf: qb*qb][log eps* pdf: lb][log Omega* pdf: lb]
 *   [A_L pdf: ab][A_T pdf: ab][mixed mean moments: ENS_NMOM]
 *   [S(A_L), F(A_L), H(A_L), F(A_T), H(A_T), <eps*>, <Omega*>, 0]
 * Member pdfs are count / (n_samples * bin width (area for QR)), with
 * n_samples including under/overflow; mixed = sum_i w_i pdf_i in sorted-lambda
 * order; moments likewise from per-member means.  Runs on the GPU.  The member
 * table of a call lives in a device buffer the context owns (grown, after a
 * device synchronisation, when a call needs more): ens_mix and ens_mix_table
 * calls of one context are ordered on one stream, but calls on streams whose
 * kernels may run at once race. */
ens_status ens_mix_len(const ens_ctx *ctx, int32_t count, size_t *n_out);
ens_status ens_mix(ens_ctx *ctx, const int32_t *members, int32_t count, double c, double Z,
                   int32_t weight_mode, double q_sigma, double *dev_out, void *stream);

/* Mixture as ens_mix for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no device memory is allocated; the member table that ens_mix
 * keeps in a buffer the library allocates lives instead in a fixed
 * file-scope device array of ENS_MIX_STATIC_MAX entries (48 bytes each,
 * about 48 KiB), one copy on each GPU the library runs on, held until the
 * process ends.  Arguments, output layout and results are those of ens_mix
 * (bitwise equal on the same input); count > ENS_MIX_STATIC_MAX returns
 * ENS_E_INVALID.  Each call rewrites every table entry it reads (nothing of an
 * earlier call is used), but all calls on one GPU share the array: calls that
 * overlap on one GPU (concurrent calls from several threads, or on several
 * streams whose kernels may run at once) race.  Synchronises the members'
 * streams and `stream` (as ens_mix does) before enqueuing the mixture kernels
 * on `stream`. */
#define ENS_MIX_STATIC_MAX 1023
ens_status ens_mix_noalloc(ens_ctx *ctx, const int32_t *members, int32_t count, double c, double Z,
                           int32_t weight_mode, double q_sigma, double *dev_out, void *stream);

/* Mixture as ens_mix, with each member's weight the mass of its lambda bin
 * (bins of mode 0: midpoints, open end bins) under a tabulated lambda density
 * instead of a parametric one: for any exponent parameterisation whose lambda
 * distribution follows from its cumulant generating function (eqs.
 * exponents_KZ_1 and cumulant_generating_function; section "Modeling choices").
 * dev_pdf: table_len FP64 samples in device memory at lam0 + j dlam; negative
 * samples count as zero, the density is linear between samples and zero
 * outside the table; weights are normalised to sum to 1.  Output layout as
 * ens_mix.  Errors: ENS_E_INVALID for bad ids, table_len < 2, dlam <= 0, null
 * pointers; ENS_E_STATE without a histogram descriptor. */
ens_status ens_mix_table(ens_ctx *ctx, const int32_t *members, int32_t count, const double *dev_pdf,
                         int32_t table_len, double lam0, double dlam, double *dev_out, void *stream);

/* Lambda density from its characteristic function: the two-sided Laplace
 * transform exp(K(t; Z)) of eq. cumulant_generating_function evaluated at
 * t = i omega and inverted by a Fourier transform (section "Modeling
 * choices").  dev_phi: table_len complex FP64 values (re, im interleaved) of
 * exp(K(i omega_k; Z)) at omega_k = 2 pi f_k / (table_len dlam), f_k = k for
 * k < table_len/2 and k - table_len otherwise (the FFT frequency order);
 * dev_pdf (table_len doubles) receives
 *   P(lam0 + j dlam) = Re sum_k phi_k exp(-i omega_k (lam0 + j dlam)) / (table_len dlam),
 * the rectangle rule of the inverse Fourier integral, summed directly in a
 * fixed order (deterministic).  Asynchronous on `stream`.  Errors:
 * ENS_E_INVALID for table_len outside [2, 65536], dlam <= 0 or null pointers. */
ens_status ens_lambda_pdf_from_cf(const double *dev_phi, int32_t table_len, double lam0, double dlam,
                                  double *dev_pdf, void *stream);

/* Scale gap Z for a target Taylor-scale Reynolds number (section
 * "Benchmarking the method against DNS data", eq. Rlambda_Z_relation, with
 * C_eps constant as in eq. Re_definition).  Each member's R_lambda is formed
 * from its snapshot-averaged energy and dissipation (moments [26..28]):
 * R_lambda = (2<E>/3) sqrt(15 / (nu <D>)).  C_eps constant makes
 * Re ~ e^(lambda/3) across members at fixed L and nu, so R_lambda = A e^(lambda/6);
 * A is fitted (least squares in ln R_lambda, slope fixed) over the members
 * with lambda >= 0, and Z = (3/2) ln(rlambda_ref / A) (negative if the target
 * is below the fitted central value).  Host outputs: *Z_out, *prefactor_out
 * (= A) and, if not NULL, rlambda_out[count] (each member's R_lambda, in the
 * order given).  Synchronises.  Errors: ENS_E_INVALID for bad ids, a
 * non-positive target or no member with lambda >= 0; ENS_E_STATE without a
 * histogram descriptor or for a member with no snapshot. */
ens_status ens_scale_gap(ens_ctx *ctx, const int32_t *members, int32_t count, double rlambda_ref,
                         double *Z_out, double *prefactor_out, double *rlambda_out);

/* ---------------------------------------------------- spectral diagnostics */

/* Shell energy spectrum of member m (the energy spectra of the ensemble
 * members shown in the paper's figure of energy spectra, section "Description
 * of the ensemble simulations"): E[s] = sum over the retained modes with
 * s - 1/2 <= |m| < s + 1/2 of (1/2)|u_hat_m|^2 over the full spectrum, |m| in
 * units of the wavenumber spacing, s = 0 .. nshell-1 (shells beyond the
 * retained set are zero).  FP64, written to device memory `dev_out` (nshell
 * doubles, caller-owned), asynchronous on `stream`.  Deterministic (fixed
 * summation order).  Errors:
 * ENS_E_INVALID for a bad member, nshell < 1 or a null pointer. */
ens_status ens_spectrum(ens_ctx *ctx, int32_t m, int32_t nshell, double *dev_out, void *stream);

/* Energy, rms velocity, integral length and integral time of member m, the
 * scales that set the run lengths and the bootstrap windows of one integral
 * time (section "Description of the ensemble simulations", tables of the
 * ensemble and reference runs).  Sums over the retained modes of the full
 * spectrum, e_m = (1/2)|u_hat_m|^2, |k_m| = dk |m|:
 *   dev_out[0] = E = sum e_m,  dev_out[1] = u' = sqrt(2E/3),
 *   dev_out[2] = L = pi / (2 u'^2) * sum_{m != 0} e_m / |k_m|,  dev_out[3] = T = L / u'
 * (L = T = 0 for a zero field).  FP64 into device memory (4 doubles,
 * caller-owned), asynchronous on `stream`; uses the member's own partial-sum
 * area, so it is ordered with the member's steps only on one stream.
 * Deterministic.  Errors: ENS_E_INVALID for a bad member or a null pointer. */
ens_status ens_integral_scales(ens_ctx *ctx, int32_t m, double *dev_out, void *stream);

/* Spectral refinement (section "Extrapolating to the frontier of current
 * turbulence simulations": the most intense members are replaced by identical
 * simulations at twice the resolution): member dst, on a grid n_dst >= n_src
 * with the same box, takes member src's field (every retained mode of src
 * keeps its value, every other mode is zero; FP32 <-> FP64 conversion as the
 * precisions require); dst's RK register is cleared and src's time, step count
 * and diagnostics are carried over.  Both members must exist; the physics
 * parameters of dst are its own.  Asynchronous on `stream`.  Errors: ENS_E_INVALID for bad ids, src == dst,
 * n_dst < n_src or a different box. */
ens_status ens_member_refine(ens_ctx *ctx, int32_t src, int32_t dst, void *stream);

/* ------------------------------------------------------------- primitives */

/* Batched complex FFT of `lines` lines of length n (16..1024, power of two)
 * in the pencil layout the solver's y/z passes use: element j of line l at
 * index j*lines + l (lines contiguous), complex interleaved, FP64 or FP32.
 * sign -1: X[k] = sum_j x[j] exp(-2 pi i jk/n); +1: exp(+...); unnormalised.
 * in and out are device pointers and may be equal. */
ens_status ens_fft_pencils(int32_t n, int32_t precision, int32_t sign, int64_t lines,
                           const void *dev_in, void *dev_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ENS_H */
