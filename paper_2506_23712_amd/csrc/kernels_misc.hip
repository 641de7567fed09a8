// kernels_misc.hip -- member initial field, canonical-layout state exchange,
// device fills, and the stand-alone batched pencil FFT.
#include "ens_internal.h"
#include "fft.hpp"

namespace ens {

template <typename P> using L2 = LdsT<P>;

// ------------------------------------------------------------------ RNG
// splitmix64 (Steele, Lea & Flood 2014; constants as published by S. Vigna):
// output number c of a generator seeded with s is mix(s + (c + 1) * gamma).
__device__ __forceinline__ unsigned long long sm64(unsigned long long seed, unsigned long long c) {
    unsigned long long z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double u01(unsigned long long x) { return ((double)(x >> 11) + 0.5) * 0x1.0p-53; }
__device__ __forceinline__ unsigned long long ctr(int mx, int my, int mz, int j) {
    return ((((unsigned long long)(mz + 2048) * 4096ull + (unsigned long long)(my + 2048)) * 4096ull +
             (unsigned long long)(mx + 2048)) * 8ull) + (unsigned long long)j;
}

// Unscaled initial coefficient of a half-space mode (m_x, m_y, m_z) != 0.
__device__ void init_coeff(unsigned long long seed, double dk, double kp, int mx, int my, int mz, double out[6]) {
    const double PI = 3.14159265358979323846;
    double g[6];
#pragma unroll
    for (int p = 0; p < 3; p++) {
        const double a = u01(sm64(seed, ctr(mx, my, mz, 2 * p)));
        const double b = u01(sm64(seed, ctr(mx, my, mz, 2 * p + 1)));
        const double r = sqrt(-2.0 * log(a));
        g[2 * p] = r * cos(2.0 * PI * b);
        g[2 * p + 1] = r * sin(2.0 * PI * b);
    }
    const double kx = dk * mx, ky = dk * my, kz = dk * mz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    // complex a = (g0 + i g1, g2 + i g3, g4 + i g5); a <- a - k (k.a)/k^2
    const double dr = (kx * g[0] + ky * g[2] + kz * g[4]) / k2;
    const double di = (kx * g[1] + ky * g[3] + kz * g[5]) / k2;
    g[0] -= kx * dr; g[1] -= kx * di;
    g[2] -= ky * dr; g[3] -= ky * di;
    g[4] -= kz * dr; g[5] -= kz * di;
    const double na = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + g[3] * g[3] + g[4] * g[4] + g[5] * g[5]);
    const double kk = sqrt(k2);
    const double ek = kk * kk * kk * kk * exp(-2.0 * (kk / kp) * (kk / kp));
    const double amp = sqrt(ek / (4.0 * PI * k2));
    const double f = na > 0.0 ? amp / na : 0.0;
#pragma unroll
    for (int i = 0; i < 6; i++) out[i] = g[i] * f;
}

// Coefficient of retained mode (iz, iy, kx) in storage order (Hermitian fill
// of the m_x = 0 plane from the mirrored positive-half mode).
__device__ void init_mode(const MemberDev &md, unsigned long long seed, double kp, long long s, double out[6]) {
    const int K = md.K;
    const long long nzl = (long long)(2 * K + 1) * (K + 1);
    const int iz = (int)(s / nzl);
    const int rem = (int)(s % nzl);
    const int iy = rem / (K + 1), mx = rem % (K + 1);
    const int my = iy <= K ? iy : iy - (2 * K + 1);
    const int mz = iz <= K ? iz : iz - (2 * K + 1);
    if (mx == 0 && my == 0 && mz == 0) {
        for (int i = 0; i < 6; i++) out[i] = 0.0;
        return;
    }
    const bool pos = mx > 0 || (my > 0 || (my == 0 && mz > 0));
    if (pos) {
        init_coeff(seed, md.dk, kp, mx, my, mz, out);
    } else {
        init_coeff(seed, md.dk, kp, -mx, -my, -mz, out);
        out[1] = -out[1]; out[3] = -out[3]; out[5] = -out[5];
    }
}

template <int NT>
__device__ __forceinline__ double bsum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// pass 1: FP64 energy partials of the unscaled field
__global__ void __launch_bounds__(256) k_init_energy(const MemberDev *__restrict__ mp, unsigned long long seed, double kp) {
    __shared__ double red[256];
    const MemberDev &md = *mp;
    const int K = md.K;
    const long long S = (long long)(2 * K + 1) * (2 * K + 1) * (K + 1);
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (s < S) {
        double c[6];
        init_mode(md, seed, kp, s, c);
        const int mx = (int)(s % (K + 1));
        double a = 0.0;
        for (int i = 0; i < 6; i++) a += c[i] * c[i];
        e = (mx > 0 ? 1.0 : 0.5) * a;
    }
    const double b = bsum<256>(e, red);
    if (threadIdx.x == 0) md.partials[blockIdx.x] = b;
}

// pass 2: total energy, scale, fresh diagnostics (one workgroup)
__global__ void __launch_bounds__(256) k_init_reduce(const MemberDev *__restrict__ mp, int nblocks, double e0) {
    __shared__ double red[256];
    const MemberDev &md = *mp;
    double e = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += 256) e += md.partials[i];
    const double E = bsum<256>(e, red);
    if (threadIdx.x == 0) {
        DevState *st = md.st;
        st->e_init = E > 0.0 ? sqrt(e0 / E) : 0.0;
        st->Ef = 0.0; st->dt = 0.0; st->umax_bits = 0ull;
        st->diag.t = 0.0; st->diag.dt = 0.0; st->diag.E = e0; st->diag.D = 0.0;
        st->diag.inj = 0.0; st->diag.E_f = 0.0; st->diag.umax = 0.0; st->diag.cfl = 0.0;
        st->diag.rlambda = 0.0; st->diag.kmax_eta = 0.0; st->diag.step = 0; st->diag.flags = 0;
        st->diag.reserved = 0;
    }
}

// pass 3: regenerate, scale, store; zero the RK register
template <typename P>
__global__ void __launch_bounds__(256) k_init_store(const MemberDev *__restrict__ mp, unsigned long long seed, double kp) {
    const MemberDev &md = *mp;
    const int K = md.K;
    const long long S = (long long)(2 * K + 1) * (2 * K + 1) * (K + 1);
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= S) return;
    double c[6];
    init_mode(md, seed, kp, s, c);
    const double f = md.st->e_init;
    L2<P> *u = reinterpret_cast<L2<P> *>(md.uh);
    L2<P> *q = reinterpret_cast<L2<P> *>(md.q);
    const long long nzl = (long long)(2 * K + 1) * (K + 1), zp = md.zp, Sp = (2 * K + 1) * zp;
    const long long at = (s / nzl) * zp + s % nzl;          // storage index of mode s
    for (int comp = 0; comp < 3; comp++) {
        L2<P> v; v.x = (P)(c[2 * comp] * f); v.y = (P)(c[2 * comp + 1] * f);
        u[comp * Sp + at] = v;
        L2<P> z; z.x = P(0); z.y = P(0);
        q[comp * Sp + at] = z;
    }
}

long long init_blocks(int n) {
    const int K = n / 3;
    const long long S = (long long)(2 * K + 1) * (2 * K + 1) * (K + 1);
    return (S + 255) / 256;
}

hipError_t launch_init_field(int n, int prec, const MemberDev *mem, uint64_t seed, double k_peak, double e0, hipStream_t s) {
    const unsigned nb = (unsigned)init_blocks(n);
    k_init_energy<<<nb, 256, 0, s>>>(mem, seed, k_peak);
    k_init_reduce<<<1, 256, 0, s>>>(mem, (int)nb, e0);
    if (prec == ENS_FP32) k_init_store<float><<<nb, 256, 0, s>>>(mem, seed, k_peak);
    else k_init_store<double><<<nb, 256, 0, s>>>(mem, seed, k_peak);
    return hipGetLastError();
}

// ------------------------------------------------------------ state exchange
// canonical [3][N][N][N/2+1] FP64 complex  <->  storage [3][2K+1][ZP], a plane
// holding [2K+1 (ky)][K+1 (kx)] then pad entries (written as zeros here)
template <typename P>
__global__ void __launch_bounds__(256) k_set_state(const MemberDev *__restrict__ mp, const double *__restrict__ src) {
    const MemberDev &md = *mp;
    const int n = md.n, K = md.K, nh = n / 2 + 1;
    const long long nzl = (long long)(2 * K + 1) * (K + 1), zp = md.zp;
    const long long S = (2 * K + 1) * zp;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= 3 * S) return;
    const int comp = (int)(i / S);
    const long long s = i % S;
    const int iz = (int)(s / zp), rem = (int)(s % zp);
    L2<P> v; v.x = P(0); v.y = P(0);
    if (rem < nzl) {
        const int iy = rem / (K + 1), kx = rem % (K + 1);
        const int zi = iz <= K ? iz : iz - (2 * K + 1) + n;
        const int yi = iy <= K ? iy : iy - (2 * K + 1) + n;
        const long long ci = (((long long)comp * n + zi) * n + yi) * nh + kx;
        v.x = (P)src[2 * ci]; v.y = (P)src[2 * ci + 1];
    }
    reinterpret_cast<L2<P> *>(md.uh)[i] = v;
    L2<P> z; z.x = P(0); z.y = P(0);
    reinterpret_cast<L2<P> *>(md.q)[i] = z;
}

template <typename P>
__global__ void __launch_bounds__(256) k_get_state(const MemberDev *__restrict__ mp, double *__restrict__ dst) {
    const MemberDev &md = *mp;
    const int n = md.n, K = md.K, nh = n / 2 + 1;
    const long long zp = md.zp;
    const long long S = (2 * K + 1) * zp;
    const long long total = 3LL * n * n * nh;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const int kx = (int)(i % nh);
    const int yi = (int)((i / nh) % n);
    const int zi = (int)((i / ((long long)nh * n)) % n);
    const int comp = (int)(i / ((long long)nh * n * n));
    const int my = yi <= n / 2 ? yi : yi - n, mz = zi <= n / 2 ? zi : zi - n;
    double re = 0.0, im = 0.0;
    if (kx <= K && my >= -K && my <= K && mz >= -K && mz <= K) {
        const int iy = my >= 0 ? my : my + 2 * K + 1, iz = mz >= 0 ? mz : mz + 2 * K + 1;
        L2<P> v = reinterpret_cast<const L2<P> *>(md.uh)[comp * S + iz * zp + (long long)iy * (K + 1) + kx];
        re = (double)v.x; im = (double)v.y;
    }
    dst[2 * i] = re;
    dst[2 * i + 1] = im;
}

hipError_t launch_set_state(int n, int prec, const MemberDev *mem, const double *src, hipStream_t s) {
    const long long S = make_geom(n, prec).S;
    const unsigned nb = (unsigned)((3 * S + 255) / 256);
    if (prec == ENS_FP32) k_set_state<float><<<nb, 256, 0, s>>>(mem, src);
    else k_set_state<double><<<nb, 256, 0, s>>>(mem, src);
    return hipGetLastError();
}

hipError_t launch_get_state(int n, int prec, const MemberDev *mem, double *dst, hipStream_t s) {
    const long long total = 3LL * n * n * (n / 2 + 1);
    const unsigned nb = (unsigned)((total + 255) / 256);
    if (prec == ENS_FP32) k_get_state<float><<<nb, 256, 0, s>>>(mem, dst);
    else k_get_state<double><<<nb, 256, 0, s>>>(mem, dst);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fills
__global__ void k_fill_u64(unsigned long long *p, long long n, unsigned long long v) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) p[i] = v;
}
__global__ void k_fill_f64(double *p, long long n, double v) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) p[i] = v;
}
hipError_t launch_fill_u64(unsigned long long *p, long long n, unsigned long long v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long nb = (n + 255) / 256;
    k_fill_u64<<<(unsigned)(nb < 4096 ? nb : 4096), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, long long n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long nb = (n + 255) / 256;
    k_fill_f64<<<(unsigned)(nb < 4096 ? nb : 4096), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------- batched pencil FFT
// element j of line l at j * lines + l
template <typename P, int N, int DIR>
__global__ void __launch_bounds__(256) k_fft_pencils(long long lines, const L2<P> *__restrict__ in, L2<P> *out,
                                                     const Cx<P> *__restrict__ tw) {
    constexpr int E = 16, M = N / E, T = 256 / M;
    __shared__ L2<P> lds[N * T];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const long long L = (long long)blockIdx.x * T + l;
    const bool valid = L < lines;
    Cx<P> v[E];
#pragma unroll
    for (int m = 0; m < E; m++) {
        if (valid) { L2<P> x = in[(long long)(t + M * m) * lines + L]; v[m] = {x.x, x.y}; }
        else v[m] = czero<P>();
    }
    line_fft<P, N, E, T, DIR>(v, lds, l, t, tw);
    if (valid) {
#pragma unroll
        for (int s = 0; s < E; s++) {
            L2<P> x; x.x = v[s].re; x.y = v[s].im;
            out[(long long)Plan<N, E>::out_pos(t, s) * lines + L] = x;
        }
    }
}

template <typename P, int N>
static hipError_t pencils_n(int sign, long long lines, const void *in, void *out, const void *tw, hipStream_t s) {
    constexpr int T = 256 / (N / 16);
    const unsigned nb = (unsigned)((lines + T - 1) / T);
    const L2<P> *ip = reinterpret_cast<const L2<P> *>(in);
    L2<P> *op = reinterpret_cast<L2<P> *>(out);
    const Cx<P> *twp = reinterpret_cast<const Cx<P> *>(tw);
    if (sign < 0) k_fft_pencils<P, N, -1><<<nb, 256, 0, s>>>(lines, ip, op, twp);
    else k_fft_pencils<P, N, +1><<<nb, 256, 0, s>>>(lines, ip, op, twp);
    return hipGetLastError();
}

template <typename P>
static hipError_t pencils_p(int n, int sign, long long lines, const void *in, void *out, const void *tw, hipStream_t s) {
    switch (n) {
    case 16: return pencils_n<P, 16>(sign, lines, in, out, tw, s);
    case 32: return pencils_n<P, 32>(sign, lines, in, out, tw, s);
    case 64: return pencils_n<P, 64>(sign, lines, in, out, tw, s);
    case 128: return pencils_n<P, 128>(sign, lines, in, out, tw, s);
    case 256: return pencils_n<P, 256>(sign, lines, in, out, tw, s);
    case 512: return pencils_n<P, 512>(sign, lines, in, out, tw, s);
    case 1024: return pencils_n<P, 1024>(sign, lines, in, out, tw, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fft_pencils(int n, int prec, int sign, long long lines, const void *in, void *out,
                              const void *tw, hipStream_t s) {
    return prec == ENS_FP32 ? pencils_p<float>(n, sign, lines, in, out, tw, s)
                            : pencils_p<double>(n, sign, lines, in, out, tw, s);
}

}  // namespace ens
