/*
 * oracle.c -- plain, slow, FP64 CPU reference for the ensemble-DNS hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark.  The product
 * library never links, loads or calls it, and it shares no code, header,
 * table or constant with the GPU library.
 *
 * What it computes (arXiv 2506.23712, "Predicting any small-scale statistics
 * of high-Reynolds-number turbulence using ensemble simulations"):
 *   - one member DNS: statistically stationary, forced, periodic-box,
 *     incompressible Navier-Stokes at viscosity nu, with a forcing that
 *     amplifies the Fourier coefficients of a low-wavenumber band each step so
 *     that the injection rate equals e^lambda * eps_bar
 *     (section "Description of the ensemble simulations", first paragraph;
 *     box / band / CFL in the paragraph after Table II);
 *   - the velocity-gradient statistics that the ensemble hypothesis mixes:
 *     A_ij = d_j u_i, Q = -Tr(A^2)/2 and R = -Tr(A^3)/3 (section "Benchmarking
 *     the method against DNS data", QR-PDF paragraph), dissipation
 *     eps = 2 nu Tr(S^2) and enstrophy omega^2 (section "Extrapolating to the
 *     frontier ...", extreme-gradient paragraph), and gradient moments up to
 *     order 6 (section "Modeling choices", eq. def_skewness_flatness).
 *
 * The paper does not state its DNS numerics; the readings taken here are:
 * Fourier pseudo-spectral method on [0,L)^3, cubic 2/3 truncation
 * |m_x|,|m_y|,|m_z| <= floor(N/3), rotational nonlinear term u x omega,
 * solenoidal projection, linear band forcing f = eps/(2 E_f) u on the band
 * (E_f evaluated at every Runge-Kutta stage; f acts on the Hermitian part of
 * the spectrum and is projected together with the nonlinear term, which
 * changes nothing for the spectrum of a real solenoidal field; a band that
 * holds no more than FORCE_EMPTY_FRAC of the member's energy at the start of
 * the step counts as empty and is not forced), integrating-factor low-storage
 * (Williamson 2N) RK3 with A = (0,-5/9,-153/128), B = (1/3,15/16,8/15),
 * and CFL time step dt = cfl * dx / max(|u|+|v|+|w|) from the stage-1 field.
 *
 * Data structures are deliberately naive: full complex N^3 arrays in
 * [z][y][x] order (x fastest), an iterative radix-2 FFT with twiddles
 * computed directly as cos/sin(2 pi j/N) (no recurrence), and loops over all
 * points.  Spectral fields are exchanged in the canonical layout
 * [3][N (m_z)][N (m_y)][N/2+1 (m_x)] complex (FFT index order, m > N/2 means
 * m - N), forward normalised as u_hat = N^-3 sum_x u(x) exp(-i k.x).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

#define OR_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------ */
/* Parameters (mirrored by a ctypes Structure in oracle/__init__.py)         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;          /* grid points per direction, power of two */
    int32_t visc_mode;  /* 0: integrating factor, 1: explicit viscous term */
    double box;         /* L; Delta k = 2 pi / L */
    double nu;          /* kinematic viscosity */
    double eps;         /* injection rate e^lambda * eps_bar */
    double kf_lo, kf_hi;/* forcing band in units of Delta k, inclusive */
    double dt;          /* > 0: fixed step; <= 0: CFL step */
    double cfl;
} or_params;

typedef struct {
    int32_t qr_bins;  double q_lo, q_hi, r_lo, r_hi;
    int32_t log_bins; double log10_lo, log10_hi;
    int32_t a_bins;   double a_lo, a_hi;
    double eps_ref, nu_ref;   /* units of the reference (lambda = 0) member */
} or_hist_desc;

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* FFT                                                                       */
/* ------------------------------------------------------------------------ */
static int is_pow2(int n) { return n >= 2 && (n & (n - 1)) == 0; }

/* tw[j] = exp(sign * 2 pi i j / n), each entry evaluated directly. */
static cplx *make_twiddles(int n, int sign) {
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)(n / 2 + 1));
    for (int j = 0; j <= n / 2; j++) {
        double a = 2.0 * OR_PI * (double)j / (double)n;
        tw[j] = cos(a) + I * ((double)sign * sin(a));
    }
    return tw;
}

/* In-place radix-2 decimation-in-time transform of one contiguous line:
 * a[k] <- sum_j a[j] exp(sign * 2 pi i j k / n), unnormalised. */
static void fft_line(cplx *a, int n, const cplx *tw) {
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len >> 1, step = n / len;
        for (int i = 0; i < n; i += len) {
            for (int k = 0; k < half; k++) {
                cplx x = a[i + k];
                cplx y = a[i + k + half] * tw[k * step];
                a[i + k] = x + y;
                a[i + k + half] = x - y;
            }
        }
    }
}

int or_fft1d(int n, double *data, int sign) {
    if (!is_pow2(n) || (sign != 1 && sign != -1)) return -1;
    cplx *tw = make_twiddles(n, sign);
    fft_line((cplx *)data, n, tw);
    free(tw);
    return 0;
}

/* 3-D transform of a full [z][y][x] complex array, one axis after another. */
static void fft3d(cplx *a, int n, int sign) {
    cplx *tw = make_twiddles(n, sign);
    const long nn = (long)n * n;
    #pragma omp parallel
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        #pragma omp for schedule(static)
        for (long line = 0; line < nn; line++) fft_line(a + line * n, n, tw);
        #pragma omp for schedule(static)
        for (long line = 0; line < nn; line++) {           /* y lines */
            long z = line / n, x = line % n;
            for (int y = 0; y < n; y++) buf[y] = a[(z * n + y) * n + x];
            fft_line(buf, n, tw);
            for (int y = 0; y < n; y++) a[(z * n + y) * n + x] = buf[y];
        }
        #pragma omp for schedule(static)
        for (long line = 0; line < nn; line++) {           /* z lines */
            for (int z = 0; z < n; z++) buf[z] = a[(long)z * nn + line];
            fft_line(buf, n, tw);
            for (int z = 0; z < n; z++) a[(long)z * nn + line] = buf[z];
        }
        free(buf);
    }
    free(tw);
}

int or_fft3d(int n, double *data, int sign) {
    if (!is_pow2(n) || (sign != 1 && sign != -1)) return -1;
    fft3d((cplx *)data, n, sign);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Spectral grid helpers                                                     */
/* ------------------------------------------------------------------------ */
static inline int mode_of(int i, int n) { return i <= n / 2 ? i : i - n; }

typedef struct {
    int n, K;
    long n3;
    double dk;
} grid_t;

static grid_t make_grid(int n, double box) {
    grid_t g;
    g.n = n; g.K = n / 3; g.n3 = (long)n * n * n;
    g.dk = 2.0 * OR_PI / box;
    return g;
}

static inline int retained(const grid_t *g, int mx, int my, int mz) {
    return abs(mx) <= g->K && abs(my) <= g->K && abs(mz) <= g->K;
}

/* canonical [3][n][n][n/2+1] -> three full [z][y][x] arrays (Hermitian fill) */
static void canon_to_full(const grid_t *g, const cplx *can, cplx *full[3]) {
    const int n = g->n, nh = n / 2 + 1;
    for (int c = 0; c < 3; c++) {
        const cplx *src = can + (long)c * n * n * nh;
        cplx *dst = full[c];
        #pragma omp parallel for schedule(static)
        for (int z = 0; z < n; z++)
            for (int y = 0; y < n; y++)
                for (int x = 0; x < n; x++) {
                    cplx v;
                    if (x < nh) v = src[((long)z * n + y) * nh + x];
                    else {
                        int xs = n - x, ys = (n - y) % n, zs = (n - z) % n;
                        v = conj(src[((long)zs * n + ys) * nh + xs]);
                    }
                    dst[((long)z * n + y) * n + x] = v;
                }
    }
}

static void full_to_canon(const grid_t *g, cplx *const full[3], cplx *can) {
    const int n = g->n, nh = n / 2 + 1;
    for (int c = 0; c < 3; c++) {
        cplx *dst = can + (long)c * n * n * nh;
        const cplx *src = full[c];
        for (int z = 0; z < n; z++)
            for (int y = 0; y < n; y++)
                for (int x = 0; x < nh; x++)
                    dst[((long)z * n + y) * nh + x] = src[((long)z * n + y) * n + x];
    }
}

static cplx *alloc_c(long n) { return (cplx *)calloc((size_t)n, sizeof(cplx)); }

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: splitmix64 (Steele, Lea & Flood 2014, in    */
/* the form published by S. Vigna).  Output number c of a generator seeded    */
/* with s is mix(s + (c+1) * 0x9E3779B97F4A7C15).                             */
/* ------------------------------------------------------------------------ */
static uint64_t sm64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t or_splitmix64(uint64_t seed, uint64_t counter) { return sm64(seed, counter); }

/* uniform in (0,1): the top 53 bits, offset by half a step */
static double unif(uint64_t bits) { return ((double)(bits >> 11) + 0.5) * 0x1.0p-53; }

/* Counter of normal deviate j (0..5) of mode (mx,my,mz). */
static uint64_t mode_counter(int mx, int my, int mz, int j) {
    uint64_t a = (uint64_t)(mz + 2048), b = (uint64_t)(my + 2048), c = (uint64_t)(mx + 2048);
    return (((a * 4096u + b) * 4096u + c) * 8u) + (uint64_t)j;
}

/* ------------------------------------------------------------------------ */
/* Initial field: seeded random solenoidal u_hat with shell spectrum         */
/* E(k) ~ k^4 exp(-2 (k/k_peak)^2), truncated to the retained set, Hermitian */
/* on the m_x = 0 plane, rescaled so that (1/2) sum_full |u_hat|^2 = e0.     */
/* Steps: 6 Box-Muller normals per half-space mode -> complex 3-vector a ->   */
/* a - k (k.a)/k^2 -> a * sqrt(E(|k|) / (4 pi |k|^2)) / |a| -> mirror.        */
/* ------------------------------------------------------------------------ */
static void init_mode(const grid_t *g, uint64_t seed, double kp, int mx, int my, int mz, cplx out[3]) {
    double gn[6];
    for (int p = 0; p < 3; p++) {
        double u1 = unif(sm64(seed, mode_counter(mx, my, mz, 2 * p)));
        double u2 = unif(sm64(seed, mode_counter(mx, my, mz, 2 * p + 1)));
        double r = sqrt(-2.0 * log(u1));
        gn[2 * p] = r * cos(2.0 * OR_PI * u2);
        gn[2 * p + 1] = r * sin(2.0 * OR_PI * u2);
    }
    cplx a[3] = { gn[0] + I * gn[1], gn[2] + I * gn[3], gn[4] + I * gn[5] };
    double k[3] = { g->dk * mx, g->dk * my, g->dk * mz };
    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    cplx kd = k[0] * a[0] + k[1] * a[1] + k[2] * a[2];
    for (int c = 0; c < 3; c++) a[c] -= k[c] * kd / k2;
    double na = sqrt(creal(a[0] * conj(a[0]) + a[1] * conj(a[1]) + a[2] * conj(a[2])));
    double kk = sqrt(k2);
    double ek = kk * kk * kk * kk * exp(-2.0 * (kk / kp) * (kk / kp));
    double amp = sqrt(ek / (4.0 * OR_PI * k2));
    for (int c = 0; c < 3; c++) out[c] = na > 0.0 ? a[c] * (amp / na) : 0.0;
}

static int positive_half(int mx, int my, int mz) {
    return mx > 0 || (mx == 0 && (my > 0 || (my == 0 && mz > 0)));
}

int or_init_field(int n, double box, uint64_t seed, double k_peak, double e0, double *out_can) {
    if (!is_pow2(n) || n < 8 || box <= 0 || k_peak <= 0 || e0 < 0) return -1;
    grid_t g = make_grid(n, box);
    const int nh = n / 2 + 1;
    cplx *can = (cplx *)out_can;
    memset(can, 0, sizeof(cplx) * (size_t)3 * n * n * nh);
    for (int z = 0; z < n; z++)
        for (int y = 0; y < n; y++)
            for (int x = 0; x < nh; x++) {
                int mx = mode_of(x, n), my = mode_of(y, n), mz = mode_of(z, n);
                if (!retained(&g, mx, my, mz)) continue;
                if (mx == 0 && my == 0 && mz == 0) continue;
                cplx v[3];
                if (positive_half(mx, my, mz)) init_mode(&g, seed, k_peak, mx, my, mz, v);
                else {          /* m_x = 0 plane, negative half: mirror of -m */
                    init_mode(&g, seed, k_peak, -mx, -my, -mz, v);
                    for (int c = 0; c < 3; c++) v[c] = conj(v[c]);
                }
                for (int c = 0; c < 3; c++) can[(((long)c * n + z) * n + y) * nh + x] = v[c];
            }
    /* energy over the full spectrum: weight 2 for m_x > 0 */
    double E = 0.0;
    for (int c = 0; c < 3; c++)
        for (int z = 0; z < n; z++)
            for (int y = 0; y < n; y++)
                for (int x = 0; x < nh; x++) {
                    cplx v = can[(((long)c * n + z) * n + y) * nh + x];
                    double w = (x == 0) ? 0.5 : 1.0;
                    E += w * creal(v * conj(v));
                }
    if (E > 0.0) {
        double s = sqrt(e0 / E);
        for (long i = 0; i < (long)3 * n * n * nh; i++) can[i] *= s;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    grid_t g;
    or_params p;
    cplx *u[3], *w[3], *nl[3];    /* physical-space work (complex storage) */
    double eref;                  /* energy of the field at the start of the step */
} rhs_work;

/* The linear band forcing eps/(2 E_f) u is singular as E_f -> 0: a band that
 * holds only rounding-level energy would be amplified to inject eps.  The
 * paper's forcing amplifies the band's existing coefficients; with nothing
 * there it has nothing to amplify.  A band holding no more than this fraction
 * of the member's energy at the start of the step is not forced.  Rounding
 * puts about 1e-30 (FP64) or 1e-13 (FP32 transforms) of the energy in a band
 * that should be empty; a developed field holds a sizeable fraction there. */
#define FORCE_EMPTY_FRAC 1e-10

static double field_energy(long n3, cplx *const uh[3]) {
    double e = 0.0;
    for (long i = 0; i < n3; i++)
        for (int c = 0; c < 3; c++) e += 0.5 * creal(uh[c][i] * conj(uh[c][i]));
    return e;
}

static void work_alloc(rhs_work *W, const or_params *p) {
    W->p = *p;
    W->g = make_grid(p->n, p->box);
    W->eref = 0.0;
    for (int c = 0; c < 3; c++) {
        W->u[c] = alloc_c(W->g.n3); W->w[c] = alloc_c(W->g.n3); W->nl[c] = alloc_c(W->g.n3);
    }
}

static void work_free(rhs_work *W) {
    for (int c = 0; c < 3; c++) { free(W->u[c]); free(W->w[c]); free(W->nl[c]); }
}

static inline void kvec(const grid_t *g, long idx, int *m, double *k) {
    int n = g->n;
    int x = (int)(idx % n), y = (int)((idx / n) % n), z = (int)(idx / ((long)n * n));
    m[0] = mode_of(x, n); m[1] = mode_of(y, n); m[2] = mode_of(z, n);
    k[0] = g->dk * m[0]; k[1] = g->dk * m[1]; k[2] = g->dk * m[2];
}

static int in_band(const or_params *p, const int m[3]) {
    long m2 = (long)m[0] * m[0] + (long)m[1] * m[1] + (long)m[2] * m[2];
    if (m2 == 0) return 0;
    double d = (double)m2;
    return d >= p->kf_lo * p->kf_lo && d <= p->kf_hi * p->kf_hi;
}

/* The velocity is a real field, so its spectrum has u(-k) = conj u(k).  A
 * part of the stored spectrum that breaks this is invisible in physical space
 * (the nonlinear term never sees it); the forcing acts on the Hermitian part
 * (u(k) + conj u(-k)) / 2 only, so that such a part is not amplified. */
static inline cplx herm(const grid_t *g, const cplx *f, long i) {
    const int n = g->n;
    const long x = i % n, y = (i / n) % n, z = i / ((long)n * n);
    const long j = (((n - z) % n) * n + (n - y) % n) * n + (n - x) % n;
    return 0.5 * (f[i] + conj(f[j]));
}

/* band energy E_f = (1/2) sum over band modes of the full spectrum (of its
 * Hermitian part) */
static double band_energy(const rhs_work *W, cplx *const uh[3]) {
    double ef = 0.0;
    for (long i = 0; i < W->g.n3; i++) {
        int m[3]; double k[3];
        kvec(&W->g, i, m, k);
        if (!in_band(&W->p, m)) continue;
        for (int c = 0; c < 3; c++) {
            cplx h = herm(&W->g, uh[c], i);
            ef += 0.5 * creal(h * conj(h));
        }
    }
    return ef;
}

enum { T_NONLINEAR = 1, T_FORCING = 2, T_VISCOUS = 4 };

/* info[0] = E_f, info[1] = injection sum Re(u^* . f), info[2] = max(|u|+|v|+|w|),
 * info[3] = max |Im u| / max |Re u| over the inverse transforms (a check). */
static void rhs_eval(rhs_work *W, cplx *const uh[3], cplx *G[3], int terms, double info[4]) {
    const grid_t *g = &W->g;
    const long n3 = g->n3;
    const double inv_n3 = 1.0 / (double)n3;
    double umax = 0.0, maxre = 0.0, maxim = 0.0;
    for (int c = 0; c < 3; c++) memset(G[c], 0, sizeof(cplx) * (size_t)n3);

    /* u_hat -> u, omega_hat = i k x u_hat -> omega (inverse transforms); always
     * evaluated so that the CFL velocity is available. */
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n3; i++) {
        int m[3]; double k[3];
        kvec(g, i, m, k);
        cplx a = uh[0][i], b = uh[1][i], cz = uh[2][i];
        W->u[0][i] = a; W->u[1][i] = b; W->u[2][i] = cz;
        W->w[0][i] = I * (k[1] * cz - k[2] * b);
        W->w[1][i] = I * (k[2] * a - k[0] * cz);
        W->w[2][i] = I * (k[0] * b - k[1] * a);
    }
    for (int c = 0; c < 3; c++) { fft3d(W->u[c], g->n, +1); fft3d(W->w[c], g->n, +1); }
    for (long i = 0; i < n3; i++) {
        double s = 0.0;
        for (int c = 0; c < 3; c++) {
            s += fabs(creal(W->u[c][i]));
            if (fabs(creal(W->u[c][i])) > maxre) maxre = fabs(creal(W->u[c][i]));
            if (fabs(cimag(W->u[c][i])) > maxim) maxim = fabs(cimag(W->u[c][i]));
            if (fabs(cimag(W->w[c][i])) > maxim) maxim = fabs(cimag(W->w[c][i]));
        }
        if (s > umax) umax = s;
    }

    if (terms & T_NONLINEAR) {
        /* n = u x omega in physical space (real parts), then forward transform */
        #pragma omp parallel for schedule(static)
        for (long i = 0; i < n3; i++) {
            double u0 = creal(W->u[0][i]), u1 = creal(W->u[1][i]), u2 = creal(W->u[2][i]);
            double w0 = creal(W->w[0][i]), w1 = creal(W->w[1][i]), w2 = creal(W->w[2][i]);
            W->nl[0][i] = u1 * w2 - u2 * w1;
            W->nl[1][i] = u2 * w0 - u0 * w2;
            W->nl[2][i] = u0 * w1 - u1 * w0;
        }
        for (int c = 0; c < 3; c++) fft3d(W->nl[c], g->n, -1);
        /* normalise, truncate to the retained set, project onto k-perpendicular */
        #pragma omp parallel for schedule(static)
        for (long i = 0; i < n3; i++) {
            int m[3]; double k[3];
            kvec(g, i, m, k);
            if (!retained(g, m[0], m[1], m[2])) continue;
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            if (k2 == 0.0) continue;
            cplx nh[3];
            for (int c = 0; c < 3; c++) nh[c] = W->nl[c][i] * inv_n3;
            cplx kd = k[0] * nh[0] + k[1] * nh[1] + k[2] * nh[2];
            for (int c = 0; c < 3; c++) G[c][i] += nh[c] - k[c] * kd / k2;
        }
    }

    /* The forcing enters the right-hand side through the same projection as
     * the nonlinear term (the pressure removes the divergent part of every
     * non-viscous term); for a solenoidal field P u = u. */
    double ef = band_energy(W, uh), inj = 0.0;
    if ((terms & T_FORCING) && ef > FORCE_EMPTY_FRAC * W->eref) {
        double fac = W->p.eps / (2.0 * ef);
        for (long i = 0; i < n3; i++) {
            int m[3]; double k[3];
            kvec(g, i, m, k);
            if (!in_band(&W->p, m)) continue;
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            if (k2 == 0.0) continue;
            cplx h[3];
            for (int c = 0; c < 3; c++) h[c] = herm(g, uh[c], i);
            cplx kd = k[0] * h[0] + k[1] * h[1] + k[2] * h[2];
            for (int c = 0; c < 3; c++) {
                cplx f = fac * (h[c] - k[c] * kd / k2);
                G[c][i] += f;
                inj += creal(conj(uh[c][i]) * f);
            }
        }
    }
    if (terms & T_VISCOUS) {
        #pragma omp parallel for schedule(static)
        for (long i = 0; i < n3; i++) {
            int m[3]; double k[3];
            kvec(g, i, m, k);
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            for (int c = 0; c < 3; c++) G[c][i] -= W->p.nu * k2 * uh[c][i];
        }
    }
    if (info) {
        info[0] = ef; info[1] = inj; info[2] = umax;
        info[3] = maxre > 0.0 ? maxim / maxre : 0.0;
    }
}

int or_rhs(const or_params *p, const double *uhat_can, double *g_can, int terms, double *info) {
    if (!is_pow2(p->n) || p->n < 8) return -1;
    rhs_work W; work_alloc(&W, p);
    cplx *uh[3], *G[3];
    for (int c = 0; c < 3; c++) { uh[c] = alloc_c(W.g.n3); G[c] = alloc_c(W.g.n3); }
    canon_to_full(&W.g, (const cplx *)uhat_can, uh);
    W.eref = field_energy(W.g.n3, uh);
    rhs_eval(&W, uh, G, terms, info);
    full_to_canon(&W.g, G, (cplx *)g_can);
    for (int c = 0; c < 3; c++) { free(uh[c]); free(G[c]); }
    work_free(&W);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Time stepping: Williamson's 2N-storage RK3 applied to the integrating-    */
/* factor variable exp(nu k^2 t) u_hat, written for the pair (u_hat, q):      */
/*   E_s = exp(-nu k^2 h_s dt),  h = (1/3, 5/12, 1/4)  (stage-time gaps)     */
/*   q   <- E_s (A_s q + dt G(u_hat))                                         */
/*   u_hat <- E_s u_hat + B_s q                                               */
/* visc_mode 1 is the same scheme with the viscous term explicit in G.       */
/* ------------------------------------------------------------------------ */
static const double RK_A[3] = { 0.0, -5.0 / 9.0, -153.0 / 128.0 };
static const double RK_B[3] = { 1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0 };
static const double RK_H[3] = { 1.0 / 3.0, 5.0 / 12.0, 1.0 / 4.0 };

enum { D_T, D_DT, D_E, D_DISS, D_INJ, D_EF, D_UMAX, D_CFL, D_NDIAG };

int or_ndiag(void) { return D_NDIAG; }

/* diag (per step, D_NDIAG doubles): t, dt, E, D, injection (stage 1),
 * E_f (stage 1), umax (stage 1), cfl number dt*umax/dx; E and D after the step. */
int or_run(const or_params *p, double *uhat_can, int nsteps, double t0, double *diag) {
    if (!is_pow2(p->n) || p->n < 8 || nsteps < 0) return -1;
    rhs_work W; work_alloc(&W, p);
    const grid_t *g = &W.g;
    const long n3 = g->n3;
    cplx *uh[3], *q[3], *G[3];
    for (int c = 0; c < 3; c++) { uh[c] = alloc_c(n3); q[c] = alloc_c(n3); G[c] = alloc_c(n3); }
    canon_to_full(g, (const cplx *)uhat_can, uh);
    const int terms = T_NONLINEAR | T_FORCING | (p->visc_mode == 1 ? T_VISCOUS : 0);
    const double dx = p->box / p->n;
    double t = t0;
    int rc = 0;
    W.eref = field_energy(n3, uh);
    for (int step = 0; step < nsteps; step++) {
        double dt = p->dt, info0[4] = { 0 };
        for (int s = 0; s < 3; s++) {
            double info[4];
            rhs_eval(&W, uh, G, terms, info);
            if (s == 0) {
                memcpy(info0, info, sizeof(info0));
                if (p->dt <= 0.0) {
                    if (!(info[2] > 0.0)) { rc = -6; goto done; }
                    dt = p->cfl * dx / info[2];
                }
            }
            #pragma omp parallel for schedule(static)
            for (long i = 0; i < n3; i++) {
                int m[3]; double k[3];
                kvec(g, i, m, k);
                double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                if (p->visc_mode == 1) {
                    for (int c = 0; c < 3; c++) {
                        q[c][i] = RK_A[s] * q[c][i] + dt * G[c][i];
                        uh[c][i] = uh[c][i] + RK_B[s] * q[c][i];
                    }
                } else {
                    double e = exp(-p->nu * k2 * RK_H[s] * dt);
                    for (int c = 0; c < 3; c++) {
                        q[c][i] = e * (RK_A[s] * q[c][i] + dt * G[c][i]);
                        uh[c][i] = e * uh[c][i] + RK_B[s] * q[c][i];
                    }
                }
            }
        }
        t += dt;
        double E = 0.0, D = 0.0;
        for (long i = 0; i < n3; i++) {
            int m[3]; double k[3];
            kvec(g, i, m, k);
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            for (int c = 0; c < 3; c++) {
                double a2 = creal(uh[c][i] * conj(uh[c][i]));
                E += 0.5 * a2; D += p->nu * k2 * a2;
            }
        }
        W.eref = E;                        /* the next step's empty-band threshold */
        if (diag) {
            double *d = diag + (long)step * D_NDIAG;
            d[D_T] = t; d[D_DT] = dt; d[D_E] = E; d[D_DISS] = D;
            d[D_INJ] = info0[1]; d[D_EF] = info0[0]; d[D_UMAX] = info0[2];
            d[D_CFL] = dt * info0[2] / dx;
        }
    }
done:
    full_to_canon(g, uh, (cplx *)uhat_can);
    for (int c = 0; c < 3; c++) { free(uh[c]); free(q[c]); free(G[c]); }
    work_free(&W);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Velocity-gradient statistics of one snapshot                               */
/* ------------------------------------------------------------------------ */
/* Bin rule (shared definition, restated independently by the GPU library):
 *   NaN -> nan counter; x < lo -> underflow; b = floor((x - lo) * (nb / (hi - lo)));
 *   b >= nb -> overflow; else bin b.
 * Counts layout (uint64):
 *   QR  : qb*qb bins (Q-major, R fastest) + [outside, 0, nan]
 *   logE: lb + [under, over, nan]    (x = log10(eps/eps_ref); eps <= 0 -> under)
 *   logW: lb + [under, over, nan]    (x = log10(omega^2 nu_ref/eps_ref))
 *   A_L : ab + [under, over, nan]    (A_ii tau_ref, three per point)
 *   A_T : ab + [under, over, nan]    (A_ij tau_ref, i != j, six per point)
 * Moments (double, 32): [0..5] sum A_L*^p, [6..11] sum A_T*^p (p = 1..6),
 *   [12..15] sum eps*^p, [16..19] sum Omega*^p (p = 1..4), [20] sum Q*,
 *   [21] sum R*, [22] sum S*_ij S*_ij, [23] sum (Tr A*)^2, [24] sum Q*^2,
 *   [25] sum R*^2, [26..31] zero.
 * Starred quantities use the reference member: tau = sqrt(nu_ref/eps_ref),
 *   Q* = Q / <TrS^2>_ref, R* = R / <TrS^2>_ref^(3/2), <TrS^2>_ref = eps_ref/(2 nu_ref).
 * near_edge[5]: samples (QR and the log histograms: points; the component
 *   histograms: each A_ij) whose bin coordinate lies within rounding of an
 *   integer (a bin edge), i.e. whose bin may legitimately differ on a path that
 *   rounds differently.  "Within rounding" is 1e-9 relative to the coordinate
 *   (FP64 paths), or, with grad_tol > 0, the first-order change of the
 *   coordinate under a perturbation of every gradient component by
 *   dA = grad_tol * max |A_ij| over the field (FP32 transforms): |dA_ij| <= dA
 *   gives |dQ| <= 3|A| dA, |dR| <= 3|A|^2 dA (|.| the Frobenius norm),
 *   |d eps| <= 12 nu |S| dA, |d omega_i| <= 2 dA, hence
 *   |d omega^2| <= 4 sqrt(3) |omega| dA + 12 dA^2, and d log10 x = dx / (x ln 10). */
#define OR_NMOM 32

static long counts_len(const or_hist_desc *h) {
    return (long)h->qr_bins * h->qr_bins + 2L * h->log_bins + 2L * h->a_bins + 15;
}

long or_counts_len(const or_hist_desc *h) { return counts_len(h); }
int or_nmom(void) { return OR_NMOM; }

/* frac within max(1e-9 |frac|, dfrac) of an integer */
static int near_edge(double frac, double dfrac) {
    double r = nearbyint(frac);
    return fabs(frac - r) <= fmax(1e-9 * fmax(1.0, fabs(frac)), dfrac);
}

/* returns bin in [0,nb), or -1 under, -2 over, -3 nan; *amb += 1 if the bin
 * coordinate is within dx (absolute, in units of x) of an edge */
static int bin1(double x, double lo, double hi, int nb, double dx, int *amb) {
    if (x != x) return -3;
    double frac = (x - lo) * ((double)nb / (hi - lo));
    if (frac > -0.5 && frac < nb + 0.5 && near_edge(frac, dx * ((double)nb / (hi - lo)))) *amb += 1;
    if (x < lo) return -1;
    double b = floor(frac);
    if (b >= (double)nb) return -2;
    return (int)b;
}

/* Compensated (Neumaier) accumulation of the moment sums: the sums are over up
 * to 10^8 samples whose terms span many orders of magnitude (sixth powers), and
 * a plain running sum drops every term below half an ulp of itself. */
static inline void kadd(double *s, double *c, double x) {
    const double t = *s + x;
    *c += fabs(*s) >= fabs(x) ? (*s - t) + x : (x - t) + *s;
    *s = t;
}

static void add1(uint64_t *h, int nb, int b) {
    if (b >= 0) h[b]++;
    else if (b == -1) h[nb]++;
    else if (b == -2) h[nb + 1]++;
    else h[nb + 2]++;
}

int or_stats(const or_params *p, const or_hist_desc *h, const double *uhat_can,
             uint64_t *counts, double *moments, uint64_t *near, double *trace_max, double grad_tol) {
    if (!is_pow2(p->n) || p->n < 8) return -1;
    if (h->qr_bins <= 0 || h->log_bins <= 0 || h->a_bins <= 0) return -1;
    grid_t g = make_grid(p->n, p->box);
    const long n3 = g.n3;
    cplx *uh[3];
    for (int c = 0; c < 3; c++) uh[c] = alloc_c(n3);
    canon_to_full(&g, (const cplx *)uhat_can, uh);
    cplx *A[9];   /* A[3*i + j] = d_j u_i */
    for (int ij = 0; ij < 9; ij++) {
        int i = ij / 3, j = ij % 3;
        A[ij] = alloc_c(n3);
        for (long idx = 0; idx < n3; idx++) {
            int m[3]; double k[3];
            kvec(&g, idx, m, k);
            A[ij][idx] = I * k[j] * uh[i][idx];
        }
        fft3d(A[ij], g.n, +1);
    }
    const int qb = h->qr_bins, lb = h->log_bins, ab = h->a_bins;
    uint64_t *hq = counts, *hle = hq + (long)qb * qb + 3, *hlw = hle + lb + 3;
    uint64_t *hal = hlw + lb + 3, *hat = hal + ab + 3;
    memset(counts, 0, sizeof(uint64_t) * (size_t)counts_len(h));
    memset(moments, 0, sizeof(double) * OR_NMOM);
    memset(near, 0, sizeof(uint64_t) * 5);
    const double tau = sqrt(h->nu_ref / h->eps_ref);
    const double trs_ref = h->eps_ref / (2.0 * h->nu_ref);
    double tmax = 0.0, amax = 0.0;
    if (grad_tol > 0.0)
        for (int ij = 0; ij < 9; ij++)
            for (long idx = 0; idx < n3; idx++) amax = fmax(amax, fabs(creal(A[ij][idx])));
    const double dA = grad_tol * amax;
    double comp[OR_NMOM] = { 0 };              /* compensations of the moment sums */
    for (long idx = 0; idx < n3; idx++) {
        double a[3][3];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) a[i][j] = creal(A[3 * i + j][idx]);
        double tr = a[0][0] + a[1][1] + a[2][2];
        if (fabs(tr) > tmax) tmax = fabs(tr);
        double q = 0.0, r = 0.0, ss = 0.0;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                q += a[i][j] * a[j][i];
                double s = 0.5 * (a[i][j] + a[j][i]);
                ss += s * s;
                for (int k = 0; k < 3; k++) r += a[i][j] * a[j][k] * a[k][i];
            }
        q *= -0.5; r *= -1.0 / 3.0;
        double w0 = a[2][1] - a[1][2], w1 = a[0][2] - a[2][0], w2 = a[1][0] - a[0][1];
        double w2s = w0 * w0 + w1 * w1 + w2 * w2;
        double epsv = 2.0 * p->nu * ss;
        double qs = q / trs_ref, rs = r / pow(trs_ref, 1.5);
        double es = epsv / h->eps_ref, ws = w2s * h->nu_ref / h->eps_ref;
        /* first-order bounds of the changes under gradient errors <= dA */
        double fa2 = 0.0;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) fa2 += a[i][j] * a[i][j];
        const double dq = 3.0 * sqrt(fa2) * dA / trs_ref, dr = 3.0 * fa2 * dA / pow(trs_ref, 1.5);
        const double de = 12.0 * p->nu * sqrt(ss) * dA / h->eps_ref;
        const double dw = (4.0 * sqrt(3.0) * sqrt(w2s) * dA + 12.0 * dA * dA) * h->nu_ref / h->eps_ref;
        const double ln10 = log(10.0);
        /* QR joint histogram */
        int amb = 0, amb2 = 0;
        int bq = bin1(qs, h->q_lo, h->q_hi, qb, dq, &amb);
        int br = bin1(rs, h->r_lo, h->r_hi, qb, dr, &amb);
        if (qs != qs || rs != rs) hq[(long)qb * qb + 2]++;
        else if (bq < 0 || br < 0) hq[(long)qb * qb]++;
        else hq[(long)bq * qb + br]++;
        if (amb) near[0]++;
        /* log histograms (a value within its error of zero: ambiguous) */
        amb = 0;
        add1(hle, lb, es > 0.0 ? bin1(log10(es), h->log10_lo, h->log10_hi, lb, de >= es ? INFINITY : de / (es * ln10), &amb)
                               : (es != es ? -3 : -1));
        if (amb || (dA > 0.0 && !(es > de))) near[1]++;
        amb = 0;
        add1(hlw, lb, ws > 0.0 ? bin1(log10(ws), h->log10_lo, h->log10_hi, lb, dw >= ws ? INFINITY : dw / (ws * ln10), &amb)
                               : (ws != ws ? -3 : -1));
        if (amb || (dA > 0.0 && !(ws > dw))) near[2]++;
        /* gradient components */
        amb = 0; amb2 = 0;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double x = a[i][j] * tau;
                double xp = 1.0;
                if (i == j) {
                    add1(hal, ab, bin1(x, h->a_lo, h->a_hi, ab, dA * tau, &amb));
                    for (int pw = 0; pw < 6; pw++) { xp *= x; kadd(&moments[pw], &comp[pw], xp); }
                } else {
                    add1(hat, ab, bin1(x, h->a_lo, h->a_hi, ab, dA * tau, &amb2));
                    for (int pw = 0; pw < 6; pw++) { xp *= x; kadd(&moments[6 + pw], &comp[6 + pw], xp); }
                }
            }
        near[3] += (uint64_t)amb;
        near[4] += (uint64_t)amb2;
        double ep = 1.0, wp = 1.0;
        for (int pw = 0; pw < 4; pw++) {
            ep *= es; wp *= ws;
            kadd(&moments[12 + pw], &comp[12 + pw], ep); kadd(&moments[16 + pw], &comp[16 + pw], wp);
        }
        kadd(&moments[20], &comp[20], qs); kadd(&moments[21], &comp[21], rs);
        kadd(&moments[22], &comp[22], ss * tau * tau);
        kadd(&moments[23], &comp[23], tr * tr * tau * tau);
        kadd(&moments[24], &comp[24], qs * qs); kadd(&moments[25], &comp[25], rs * rs);
    }
    for (int k = 0; k < OR_NMOM; k++) moments[k] += comp[k];
    if (trace_max) *trace_max = tmax;
    for (int c = 0; c < 3; c++) free(uh[c]);
    for (int ij = 0; ij < 9; ij++) free(A[ij]);
    return 0;
}
