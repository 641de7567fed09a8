// kernels_step.hip -- one Runge-Kutta stage of the pseudo-spectral right-hand
// side and update, for a batch of members of one grid size and precision.
//
// Data flow of a stage (K = N/3, retained set |m_i| <= K, half space m_x >= 0):
//   band   : E_f = (1/2) sum_band |u_hat|^2 (FP64)                (tiny kernel)
//   zinv   : u_hat_c -> Z^-1[u_hat_c], Z^-1[i k_z u_hat_c]         5 fields
//   yinv   : -> u_x,u_y,u_z, omega_x,omega_y,omega_z  (y physical)   6 fields
//   xpass  : c2r along x, n = u x omega, r2c along x, keep m_x <= K  3 fields
//   yfwd   : forward along y, keep |m_y| <= K                         3 fields
//   zfwd   : forward along z, keep |m_z| <= K, project, force, RK update
//   end    : FP64 reduction of E and D partials, diagnostics, time
// Pencils of the y/z passes are lines of one (x-mode, other-coordinate) pair;
// the x-mode index is the fastest in memory, so consecutive lanes of a
// workgroup read consecutive complex words.
#include "ens_internal.h"
#include "fft.hpp"

namespace ens {

template <typename P> using L2 = LdsT<P>;

template <typename P> __device__ __forceinline__ Cx<P> ldc(const void *base, long long i) {
    L2<P> v = reinterpret_cast<const L2<P> *>(base)[i];
    return {v.x, v.y};
}
template <typename P> __device__ __forceinline__ void stc(void *base, long long i, Cx<P> c) {
    L2<P> v; v.x = c.re; v.y = c.im;
    reinterpret_cast<L2<P> *>(base)[i] = v;
}

__device__ __forceinline__ int mode_of(int n, int N) { return n <= N / 2 ? n : n - N; }

// FP64 block sum with a fixed combination order (deterministic).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------ pass configs
template <int N> struct Cfg {
    static constexpr int K = N / 3;
    static constexpr long long NZL = (long long)(2 * K + 1) * (K + 1);
    static constexpr long long S = (long long)(2 * K + 1) * NZL;
    static constexpr long long NYL = (long long)N * (K + 1);
    // y/z inverse and y forward: 16 values per thread, 256 threads
    static constexpr int E16 = 16, M16 = N / 16, T16 = 256 / M16;
    // x pass and z forward: 8 values per thread
    static constexpr int E8 = 8, M8 = N / 8, TX = 256 / M8;          // x pass: 256 threads
    static constexpr int TZ = (512 / M8) < 1 ? 1 : 512 / M8;          // z forward: 512 threads
};

// ================================================================== band
// One workgroup per member: E_f over the forcing band (FP64, fixed order).
template <typename P>
__global__ void __launch_bounds__(256) k_band_energy(const MemberDev *__restrict__ mems, int stage) {
    __shared__ double red[256];
    const MemberDev &md = mems[blockIdx.x];
    const int K = md.K;
    const long long nzl = (long long)(2 * K + 1) * (K + 1);
    const long long S = (long long)(2 * K + 1) * nzl;
    int B = (int)floor(sqrt(md.kf_hi2));
    if (B > K) B = K;
    const int W = 2 * B + 1;
    const long long ncand = (long long)(B + 1) * W * W;
    double acc = 0.0;
    for (long long c = threadIdx.x; c < ncand; c += 256) {
        const int mx = (int)(c % (B + 1));
        const int my = (int)((c / (B + 1)) % W) - B;
        const int mz = (int)(c / ((long long)(B + 1) * W)) - B;
        const int m2 = mx * mx + my * my + mz * mz;
        if (m2 == 0 || (double)m2 < md.kf_lo2 || (double)m2 > md.kf_hi2) continue;
        const int iy = my >= 0 ? my : my + 2 * K + 1, iz = mz >= 0 ? mz : mz + 2 * K + 1;
        const long long idx = (long long)iz * nzl + (long long)iy * (K + 1) + mx;
        const double w = mx > 0 ? 1.0 : 0.5;
#pragma unroll
        for (int comp = 0; comp < 3; comp++) {
            Cx<P> v = ldc<P>(md.uh, comp * S + idx);
            acc += w * ((double)v.re * (double)v.re + (double)v.im * (double)v.im);
        }
    }
    const double ef = block_sum<256>(acc, red);
    if (threadIdx.x == 0) {
        md.st->Ef = ef;
        if (stage == 0) {
            md.st->diag.E_f = ef;
            md.st->diag.inj = ef > 0.0 ? md.eps_m : 0.0;
            md.st->umax_bits = 0ull;
            if (!(ef > 0.0) && md.eps_m != 0.0) md.st->diag.flags |= 2;
        }
    }
}

// ================================================================== zinv
// z-lines L = iy (K+1) + kx of the retained (m_y, m_x) pairs.
// out (bufA) [5][N (z)][NZL]: U_x, U_y, U_z, W_x = Z^-1[i k_z u_x], W_y = Z^-1[i k_z u_y]
template <typename P, int N>
__global__ void __launch_bounds__(256) k_zinv(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ tw) {
    using C = Cfg<N>;
    constexpr int E = C::E16, M = C::M16, T = C::T16, K = C::K;
    __shared__ L2<P> lds[N * T];
    const MemberDev &md = mems[blockIdx.y];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const long long L = (long long)blockIdx.x * T + l;
    const bool valid = L < C::NZL;
    const P dk = (P)md.dk;
    Cx<P> a[E], b[E];
#pragma unroll
    for (int c = 0; c < 3; c++) {
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int mz = mode_of(t + M * m, N);
            const bool keep = valid && mz >= -K && mz <= K;
            const int iz = mz >= 0 ? mz : mz + 2 * K + 1;
            a[m] = keep ? ldc<P>(md.uh, c * C::S + iz * C::NZL + L) : czero<P>();
        }
        if (c < 2) {
#pragma unroll
            for (int m = 0; m < E; m++) b[m] = mul_i(cscale(a[m], dk * (P)mode_of(t + M * m, N)));
            line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
            if (valid) {
#pragma unroll
                for (int s = 0; s < E; s++)
                    stc<P>(md.bufA, ((3 + c) * N + Plan<N, E>::out_pos(t, s)) * C::NZL + L, b[s]);
            }
        }
        line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
        if (valid) {
#pragma unroll
            for (int s = 0; s < E; s++) stc<P>(md.bufA, (c * N + Plan<N, E>::out_pos(t, s)) * C::NZL + L, a[s]);
        }
    }
}

// ================================================================== yinv
// y-lines L = z (K+1) + kx.  in bufA [5][N][NZL]; out bufB [6][N (z)][N (y)][K+1]:
// u_x, u_y, u_z, omega_x, omega_y, omega_z
template <typename P, int N>
__global__ void __launch_bounds__(256) k_yinv(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ tw) {
    using C = Cfg<N>;
    constexpr int E = C::E16, M = C::M16, T = C::T16, K = C::K;
    __shared__ L2<P> lds[N * T];
    const MemberDev &md = mems[blockIdx.y];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const long long L = (long long)blockIdx.x * T + l;
    const bool valid = L < C::NYL;
    const long long z = valid ? L / (K + 1) : 0;
    const int kx = valid ? (int)(L % (K + 1)) : 0;
    const P dk = (P)md.dk;
    const P kxv = dk * (P)kx;
    auto in_idx = [&](int f, int iy) -> long long { return (f * N + z) * C::NZL + (long long)iy * (K + 1) + kx; };
    auto out_idx = [&](int f, int y) -> long long { return ((f * N + z) * N + y) * (long long)(K + 1) + kx; };
    auto load = [&](Cx<P> *v, int f) {
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int my = mode_of(t + M * m, N);
            const bool keep = valid && my >= -K && my <= K;
            v[m] = keep ? ldc<P>(md.bufA, in_idx(f, my >= 0 ? my : my + 2 * K + 1)) : czero<P>();
        }
    };
    auto store = [&](const Cx<P> *v, int f) {
        if (valid) {
#pragma unroll
            for (int s = 0; s < E; s++) stc<P>(md.bufB, out_idx(f, Plan<N, E>::out_pos(t, s)), v[s]);
        }
    };
    Cx<P> a[E], b[E];
    // 1: b = Y^-1[i k_y U_x] (kept), u_x
    load(a, 0);
#pragma unroll
    for (int m = 0; m < E; m++) b[m] = mul_i(cscale(a[m], dk * (P)mode_of(t + M * m, N)));
    line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
    line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
    store(a, 0);
    // 2: u_y, omega_z = i k_x u_y - d_y u_x
    load(a, 1);
    line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
    store(a, 1);
#pragma unroll
    for (int s = 0; s < E; s++) b[s] = mul_i(cscale(a[s], kxv)) - b[s];
    store(b, 5);
    // 3: omega_x = Y^-1[i k_y U_z - W_y], omega_y = Y^-1[W_x - i k_x U_z], u_z
    load(a, 2);
    load(b, 4);
#pragma unroll
    for (int m = 0; m < E; m++) b[m] = mul_i(cscale(a[m], dk * (P)mode_of(t + M * m, N))) - b[m];
    line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
    store(b, 3);
    load(b, 3);
#pragma unroll
    for (int m = 0; m < E; m++) b[m] = b[m] - mul_i(cscale(a[m], kxv));
    line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
    store(b, 4);
    line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
    store(a, 2);
}

// ================================================================== xpass
// Rows R = z N + y.  in bufB [6][N][N][K+1]; out bufA [3][N][N][K+1] = x-transform
// (unnormalised) of n = u x omega, truncated to m_x <= K.
// Stage 0 also folds max(|u|+|v|+|w|) into st->umax_bits.
template <typename P, int N>
__global__ void __launch_bounds__(256) k_xpass(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ tw, int stage) {
    using C = Cfg<N>;
    constexpr int E = C::E8, M = C::M8, T = C::TX, K = C::K;
    __shared__ L2<P> lds[N * T];
    __shared__ double redmax[256 / 64];
    const MemberDev &md = mems[blockIdx.y];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const long long R = (long long)blockIdx.x * T + l;
    const long long plane = (long long)N * N;
    auto in_idx = [&](int f, int kx) -> long long { return (f * plane + R) * (K + 1) + kx; };
    P ph[6][E];
    Cx<P> v[E];
#pragma unroll
    for (int pr = 0; pr < 3; pr++) {
        const int fa = 2 * pr, fb = 2 * pr + 1;
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int n = t + M * m;
            if (n == 0) {
                Cx<P> A = ldc<P>(md.bufB, in_idx(fa, 0)), B = ldc<P>(md.bufB, in_idx(fb, 0));
                v[m] = {A.re, B.re};
            } else if (n <= K) {
                Cx<P> A = ldc<P>(md.bufB, in_idx(fa, n)), B = ldc<P>(md.bufB, in_idx(fb, n));
                v[m] = {A.re - B.im, A.im + B.re};
            } else if (n >= N - K) {
                Cx<P> A = ldc<P>(md.bufB, in_idx(fa, N - n)), B = ldc<P>(md.bufB, in_idx(fb, N - n));
                v[m] = {A.re + B.im, B.re - A.im};
            } else {
                v[m] = czero<P>();
            }
        }
        line_fft<P, N, E, T, +1>(v, lds, l, t, tw);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[fa][s] = v[s].re; ph[fb][s] = v[s].im; }
    }
    // ph: 0 u_x, 1 u_y, 2 u_z, 3 omega_x, 4 omega_y, 5 omega_z
    if (stage == 0) {
        P mx = P(0);
#pragma unroll
        for (int s = 0; s < E; s++) {
            P a = fabs(ph[0][s]) + fabs(ph[1][s]) + fabs(ph[2][s]);
            mx = a > mx ? a : mx;
        }
        double dm = (double)mx;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            double o = __shfl_xor(dm, off, 64);
            dm = o > dm ? o : dm;
        }
        if ((threadIdx.x & 63) == 0) redmax[threadIdx.x >> 6] = dm;
    }
    Cx<P> d1[E], d2[E];
#pragma unroll
    for (int s = 0; s < E; s++) {
        const P nx = ph[1][s] * ph[5][s] - ph[2][s] * ph[4][s];
        const P ny = ph[2][s] * ph[3][s] - ph[0][s] * ph[5][s];
        const P nz = ph[0][s] * ph[4][s] - ph[1][s] * ph[3][s];
        d1[s] = {nx, ny};
        d2[s] = {nz, P(0)};
    }
    line_fft_T<P, N, E, T, -1>(d1, lds, l, t, tw);      // d1[m] = D1[t + M m]
    line_fft_T<P, N, E, T, -1>(d2, lds, l, t, tw);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; m++) lds_put<P>(lds, (t + M * m) * T + l, d1[m]);
    __syncthreads();
    if (stage == 0 && threadIdx.x == 0) {
        double dm = redmax[0];
        for (int w = 1; w < 256 / 64; w++) dm = redmax[w] > dm ? redmax[w] : dm;
        atomicMax(&md.st->umax_bits, (unsigned long long)__double_as_longlong(dm));
    }
#pragma unroll
    for (int m = 0; m < E; m++) {
        const int k = t + M * m;
        if (k <= K) {
            const Cx<P> a = d1[m];
            const Cx<P> b = lds_get<P>(lds, ((N - k) % N) * T + l);
            const P h = P(0.5);
            Cx<P> nxk = {h * (a.re + b.re), h * (a.im - b.im)};
            Cx<P> nyk = {h * (a.im + b.im), h * (b.re - a.re)};
            stc<P>(md.bufA, (0 * plane + R) * (K + 1) + k, nxk);
            stc<P>(md.bufA, (1 * plane + R) * (K + 1) + k, nyk);
            stc<P>(md.bufA, (2 * plane + R) * (K + 1) + k, d2[m]);
        }
    }
}

// ================================================================== yfwd
// y-lines L = z (K+1) + kx.  in bufA [3][N][N][K+1]; out bufB [3][N (z)][2K+1][K+1]
template <typename P, int N>
__global__ void __launch_bounds__(256) k_yfwd(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ tw) {
    using C = Cfg<N>;
    constexpr int E = C::E16, M = C::M16, T = C::T16, K = C::K;
    __shared__ L2<P> lds[N * T];
    const MemberDev &md = mems[blockIdx.y];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const long long L = (long long)blockIdx.x * T + l;
    const bool valid = L < C::NYL;
    const long long z = valid ? L / (K + 1) : 0;
    const int kx = valid ? (int)(L % (K + 1)) : 0;
    Cx<P> a[E];
#pragma unroll
    for (int f = 0; f < 3; f++) {
#pragma unroll
        for (int m = 0; m < E; m++)
            a[m] = valid ? ldc<P>(md.bufA, ((f * N + z) * N + (t + M * m)) * (long long)(K + 1) + kx) : czero<P>();
        line_fft<P, N, E, T, -1>(a, lds, l, t, tw);
        if (valid) {
#pragma unroll
            for (int s = 0; s < E; s++) {
                const int my = mode_of(Plan<N, E>::out_pos(t, s), N);
                if (my >= -K && my <= K) {
                    const int iy = my >= 0 ? my : my + 2 * K + 1;
                    stc<P>(md.bufB, (f * N + z) * C::NZL + (long long)iy * (K + 1) + kx, a[s]);
                }
            }
        }
    }
}

// ================================================================== zfwd + update
// z-lines L = iy (K+1) + kx.  in bufB [3][N][NZL].  Forward along z, keep
// |m_z| <= K, normalise by N^-3, project, add band forcing, RK stage update.
template <typename P, int N>
__global__ void __launch_bounds__(512) k_zfwd_update(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ tw, int stage) {
    using C = Cfg<N>;
    constexpr int E = C::E8, M = C::M8, T = C::TZ, K = C::K;
    constexpr int NT = T * M;
    static_assert(NT * sizeof(double) <= N * T * sizeof(L2<P>), "reduction scratch reuses the FFT LDS");
    __shared__ L2<P> lds[N * T];
    double *red = reinterpret_cast<double *>(lds);
    const MemberDev &md = mems[blockIdx.y];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const long long L = (long long)blockIdx.x * T + l;
    const bool valid = L < C::NZL;
    const int iy = valid ? (int)(L / (K + 1)) : 0;
    const int kx = valid ? (int)(L % (K + 1)) : 0;
    const int my = iy <= K ? iy : iy - (2 * K + 1);
    Cx<P> a[3][E];
#pragma unroll
    for (int f = 0; f < 3; f++) {
#pragma unroll
        for (int m = 0; m < E; m++)
            a[f][m] = valid ? ldc<P>(md.bufB, (f * N + (t + M * m)) * C::NZL + L) : czero<P>();
        line_fft<P, N, E, T, -1>(a[f], lds, l, t, tw);
    }
    // time step of this RK step
    double dt;
    if (md.dt_fixed > 0.0) dt = md.dt_fixed;
    else if (stage == 0) {
        const double um = __longlong_as_double((long long)md.st->umax_bits);
        dt = um > 0.0 ? md.cfl * (md.box / N) / um : 0.0;
    } else dt = md.st->dt;
    if (stage == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        md.st->dt = dt;
        if (!(dt > 0.0)) md.st->diag.flags |= 4;
    }
    const double Ef = md.st->Ef;
    const P ffac = (P)(Ef > 0.0 ? md.eps_m / (2.0 * Ef) : 0.0);
    const double RKA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    const double RKB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    const double RKH[3] = {1.0 / 3.0, 5.0 / 12.0, 1.0 / 4.0};
    const P As = (P)RKA[stage], Bs = (P)RKB[stage], Pdt = (P)dt;
    const double nh = md.nu * RKH[stage] * dt * md.dk * md.dk;   // exponent per |m|^2
    const P inv_n3 = (P)(1.0 / ((double)N * N * N));
    const P dk = (P)md.dk, nu = (P)md.nu;
    double eacc = 0.0, dacc = 0.0;
    if (valid) {
#pragma unroll
        for (int s = 0; s < E; s++) {
            const int mz = mode_of(Plan<N, E>::out_pos(t, s), N);
            if (mz < -K || mz > K) continue;
            const int iz = mz >= 0 ? mz : mz + 2 * K + 1;
            const long long idx = (long long)iz * C::NZL + L;
            const int m2 = kx * kx + my * my + mz * mz;
            const P kxv = dk * (P)kx, kyv = dk * (P)my, kzv = dk * (P)mz;
            const P k2 = kxv * kxv + kyv * kyv + kzv * kzv;
            Cx<P> u[3], g[3];
#pragma unroll
            for (int c = 0; c < 3; c++) u[c] = ldc<P>(md.uh, c * C::S + idx);
            if (m2 == 0) {
                g[0] = g[1] = g[2] = czero<P>();
            } else {
                Cx<P> n0 = cscale(a[0][s], inv_n3), n1 = cscale(a[1][s], inv_n3), n2 = cscale(a[2][s], inv_n3);
                const P ik2 = P(1) / k2;
                Cx<P> kn = cscale(n0, kxv) + cscale(n1, kyv) + cscale(n2, kzv);
                g[0] = n0 - cscale(kn, kxv * ik2);
                g[1] = n1 - cscale(kn, kyv * ik2);
                g[2] = n2 - cscale(kn, kzv * ik2);
                if ((double)m2 >= md.kf_lo2 && (double)m2 <= md.kf_hi2) {
#pragma unroll
                    for (int c = 0; c < 3; c++) g[c] = g[c] + cscale(u[c], ffac);
                }
            }
            if (md.visc_mode == 1) {
#pragma unroll
                for (int c = 0; c < 3; c++) g[c] = g[c] - cscale(u[c], nu * k2);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    Cx<P> q = stage == 0 ? czero<P>() : ldc<P>(md.q, c * C::S + idx);
                    q = cscale(q, As) + cscale(g[c], Pdt);
                    u[c] = u[c] + cscale(q, Bs);
                    stc<P>(md.q, c * C::S + idx, q);
                    stc<P>(md.uh, c * C::S + idx, u[c]);
                }
            } else {
                const P es = (P)exp(-nh * (double)m2);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    Cx<P> q = stage == 0 ? czero<P>() : ldc<P>(md.q, c * C::S + idx);
                    q = cscale(cscale(q, As) + cscale(g[c], Pdt), es);
                    u[c] = cscale(u[c], es) + cscale(q, Bs);
                    stc<P>(md.q, c * C::S + idx, q);
                    stc<P>(md.uh, c * C::S + idx, u[c]);
                }
            }
            if (stage == 2) {
                const double w = kx > 0 ? 1.0 : 0.5;
                double e2 = 0.0;
#pragma unroll
                for (int c = 0; c < 3; c++) e2 += (double)u[c].re * (double)u[c].re + (double)u[c].im * (double)u[c].im;
                eacc += w * e2;
                dacc += w * e2 * (double)m2;
            }
        }
    }
    if (stage == 2) {
        __syncthreads();                     // LDS of the last transform is reused below
        const double es = block_sum<NT>(eacc, red);
        const double ds = block_sum<NT>(dacc, red);
        if (threadIdx.x == 0) {
            md.partials[2 * blockIdx.x] = es;
            md.partials[2 * blockIdx.x + 1] = ds;
        }
    }
}

// ================================================================== end of step
template <int N>
__global__ void __launch_bounds__(256) k_end_step(const MemberDev *__restrict__ mems, int nblocks) {
    __shared__ double red[256];
    const MemberDev &md = mems[blockIdx.x];
    double e = 0.0, d = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += 256) { e += md.partials[2 * i]; d += md.partials[2 * i + 1]; }
    const double E = block_sum<256>(e, red);
    const double Dm2 = block_sum<256>(d, red);
    if (threadIdx.x == 0) {
        DevState *st = md.st;
        const double dt = st->dt;
        const double D = 2.0 * md.nu * md.dk * md.dk * Dm2;
        const double um = __longlong_as_double((long long)st->umax_bits);
        st->diag.t += dt;
        st->diag.dt = dt;
        st->diag.E = E;
        st->diag.D = D;
        st->diag.umax = um;
        st->diag.cfl = dt * um / (md.box / N);
        st->diag.rlambda = (D > 0.0 && md.nu > 0.0) ? (2.0 * E / 3.0) * sqrt(15.0 / (md.nu * D)) : 0.0;
        st->diag.kmax_eta = D > 0.0 ? md.K * md.dk * pow(md.nu * md.nu * md.nu / D, 0.25) : 0.0;
        st->diag.step += 1;
        if (!isfinite(E)) st->diag.flags |= 1;
    }
}

// ================================================================== launchers
template <typename P, int N>
static hipError_t run_pass(int pass, const MemberDev *mem, int count, int stage, const void *tw, hipStream_t s) {
    using C = Cfg<N>;
    const Cx<P> *twp = reinterpret_cast<const Cx<P> *>(tw);
    switch (pass) {
    case P_ZINV: {
        dim3 g((unsigned)((C::NZL + C::T16 - 1) / C::T16), count);
        k_zinv<P, N><<<g, 256, 0, s>>>(mem, twp);
        break;
    }
    case P_YINV: {
        dim3 g((unsigned)((C::NYL + C::T16 - 1) / C::T16), count);
        k_yinv<P, N><<<g, 256, 0, s>>>(mem, twp);
        break;
    }
    case P_XPASS: {
        dim3 g((unsigned)((long long)N * N / C::TX), count);
        k_xpass<P, N><<<g, 256, 0, s>>>(mem, twp, stage);
        break;
    }
    case P_YFWD: {
        dim3 g((unsigned)((C::NYL + C::T16 - 1) / C::T16), count);
        k_yfwd<P, N><<<g, 256, 0, s>>>(mem, twp);
        break;
    }
    case P_ZFWD: {
        dim3 g((unsigned)((C::NZL + C::TZ - 1) / C::TZ), count);
        k_zfwd_update<P, N><<<g, C::TZ * C::M8, 0, s>>>(mem, twp, stage);
        break;
    }
    case P_END: {
        k_end_step<N><<<count, 256, 0, s>>>(mem, (int)((C::NZL + C::TZ - 1) / C::TZ));
        break;
    }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename P>
static hipError_t dispatch_n(int n, int pass, const MemberDev *mem, int count, int stage, const void *tw, hipStream_t s) {
    switch (n) {
    case 16: return run_pass<P, 16>(pass, mem, count, stage, tw, s);
    case 32: return run_pass<P, 32>(pass, mem, count, stage, tw, s);
    case 64: return run_pass<P, 64>(pass, mem, count, stage, tw, s);
    case 128: return run_pass<P, 128>(pass, mem, count, stage, tw, s);
    case 256: return run_pass<P, 256>(pass, mem, count, stage, tw, s);
    default: return hipErrorInvalidValue;
    }
}

static hipError_t dispatch(int n, int prec, int pass, const MemberDev *mem, int count, int stage, const void *tw, hipStream_t s) {
    return prec == ENS_FP32 ? dispatch_n<float>(n, pass, mem, count, stage, tw, s)
                            : dispatch_n<double>(n, pass, mem, count, stage, tw, s);
}

hipError_t launch_band_energy(int n, int prec, const MemberDev *mem, int count, int stage, hipStream_t s) {
    (void)n;
    if (prec == ENS_FP32) k_band_energy<float><<<count, 256, 0, s>>>(mem, stage);
    else k_band_energy<double><<<count, 256, 0, s>>>(mem, stage);
    return hipGetLastError();
}
hipError_t launch_zinv(int n, int prec, const MemberDev *mem, int count, const void *tw, hipStream_t s) {
    return dispatch(n, prec, P_ZINV, mem, count, 0, tw, s);
}
hipError_t launch_yinv(int n, int prec, const MemberDev *mem, int count, int nfields, const void *tw, hipStream_t s) {
    (void)nfields;
    return dispatch(n, prec, P_YINV, mem, count, 0, tw, s);
}
hipError_t launch_xpass(int n, int prec, const MemberDev *mem, int count, int stage, const void *tw, hipStream_t s) {
    return dispatch(n, prec, P_XPASS, mem, count, stage, tw, s);
}
hipError_t launch_yfwd(int n, int prec, const MemberDev *mem, int count, const void *tw, hipStream_t s) {
    return dispatch(n, prec, P_YFWD, mem, count, 0, tw, s);
}
hipError_t launch_zfwd_update(int n, int prec, const MemberDev *mem, int count, int stage, const void *tw, hipStream_t s) {
    return dispatch(n, prec, P_ZFWD, mem, count, stage, tw, s);
}
hipError_t launch_end_step(int n, int prec, const MemberDev *mem, int count, hipStream_t s) {
    return dispatch(n, prec, P_END, mem, count, 0, nullptr, s);
}

long long zfwd_blocks(int n) {
    const int K = n / 3;
    const long long nzl = (long long)(2 * K + 1) * (K + 1);
    const int TZ = 512 / (n / 8) < 1 ? 1 : 512 / (n / 8);
    return (nzl + TZ - 1) / TZ;
}

}  // namespace ens
