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
// Pencils of the y/z passes are lines of one (x-mode, other-coordinate) pair,
// numbered with the x-mode fastest and in the order of the buffer the pass
// writes, so that a workgroup's consecutive lines are consecutive complex
// words at every position and its stores cover whole 128-byte lines with no
// row padding (its loads may straddle lines: the neighbouring workgroups, on
// the same XCD, read the rest of them).  Every buffer is addressed as a
// workgroup-uniform base pointer per field plus a 32-bit per-lane offset, and
// the loads of the next transform are issued before the current one is
// computed, so that HBM latency overlaps the butterflies.
#include "ens_internal.h"
#include "fft.hpp"
#include "gmem.hpp"

namespace ens {

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
// E = complex values per thread (a line of N uses N/E threads).  Variants of
// E are compiled for the pencil passes and the x pass; the host picks one per
// (pass, N, precision) from its tuning table.
template <typename P, int N, int E_, int TM = 1> struct Cfg {
    static constexpr int K = N / 3, KX = K + 1;                 // x-modes kept
    static constexpr int NZLS = (2 * K + 1) * KX;               // z-lines: modes of a z plane
    static constexpr int ZP = state_pitch(K, (int)sizeof(Cx<P>));  // plane pitch (whole 128-byte lines)
    static constexpr int S = (2 * K + 1) * ZP;                  // state elements per component
    static constexpr int NYL = N * KX;                          // y-lines
    // y-pencil buffers are blocked by z: ZB consecutive z rows (BL = ZB (K+1)
    // lines, the fewest that fill whole 128-byte lines) are stored together,
    // position by position, so that a pass's position stride is BL values
    // (5.5 KB at N = 256) instead of the whole y-line count
    static constexpr int TLB = 128 / (int)sizeof(Cx<P>);
    static constexpr int ZB = TLB / gcd_int(KX, TLB), BL = ZB * KX;
    // element of line L at position p of a y-pencil buffer with NP positions
    __device__ static constexpr uint32_t yel(int L, int p, int NP) {
        return (uint32_t)(L / BL) * (uint32_t)(NP * BL) + (uint32_t)p * BL + (uint32_t)(L % BL);
    }
    static constexpr int E = E_ > N ? N : E_;
    static constexpr int M = N / E;
    // Lines per workgroup of the y/z pencil passes: at least 256 threads and
    // at least one 128-byte line per position (16 FP32 / 8 FP64 consecutive
    // lines, a multiple of which is where every tile starts), so that every
    // store covers whole lines; at most 1024 threads (512
    // with 16 values per thread, so that a wave may use 256 VGPRs); gfx950
    // gives a workgroup up to 160 KiB of LDS.
    static constexpr int TL = 128 / (int)sizeof(Cx<P>);
    static constexpr int MAXT = E >= 16 ? 512 : 1024;             // 16 values/thread: keep 256 VGPRs available
    // TM > 1 (autotuner variants 2, 3 of the y/z passes): TM times as many
    // lines, i.e. TM whole lines per position, where the thread budget above
    // allows it (not for 16 FP64 values per thread, which would spill)
    static constexpr int T1 = N <= 256 ? (256 / M > TL ? 256 / M : TL) : (TL * M <= MAXT ? TL : MAXT / M);
    static constexpr int T = (T1 * TM * M <= MAXT && !(sizeof(P) == 8 && E >= 16)) ? T1 * TM : T1;
    static constexpr int NT = T * M;
    // z/y inverse passes: waves per SIMD the register budget is cut for
    static constexpr int PMINW = (sizeof(P) == 4 && E == 16 && NT == 256) ? 3 : 1;
    static constexpr int TX = 256 / M;                          // x pass: 256 threads
    // z forward + update: 8 values per thread, 512 threads up to N = 256;
    // 16 values per thread and the pencil rule above for longer lines
    static constexpr int EZ = N <= 256 ? 8 : 16, MZ = N / EZ;
    static constexpr int TZ = N <= 256 ? ((512 / MZ) < 1 ? 1 : 512 / MZ) : (TL * MZ <= 512 ? TL : 512 / MZ);
    static constexpr int NTZ = TZ * MZ;
    // z forward + update, waves per SIMD the register budget is cut for: two
    // 512-thread workgroups per compute unit (4 waves per SIMD) in FP32; the
    // FP64 update keeps its registers
    static constexpr int ZMINB = (sizeof(P) == 4 && NTZ == 512 && EZ == 8) ? 4 : 1;
};

// ================================================================== band
// One workgroup per member: the band's part of the m_x = 0 plane made
// Hermitian, then E_f over the forcing band (FP64, fixed order).
template <typename P>
__global__ void __launch_bounds__(256) k_band_energy(const MemberDev *__restrict__ mems, int stage) {
    __shared__ double red[256];
    const MemberDev &md = mems[blockIdx.x];
    const int K = md.K;
    const long long zp = md.zp;
    const long long S = (long long)(2 * K + 1) * zp;
    int B = (int)floor(sqrt(md.kf_hi2));
    if (B > K) B = K;
    const int W = 2 * B + 1;
    const long long ncand = (long long)(B + 1) * W * W;
    // The velocity is real, so the m_x = 0 plane of its half spectrum is
    // Hermitian: u(0, -m_y, -m_z) = conj u(0, m_y, m_z).  A part breaking
    // that is invisible to the nonlinear term, and the linear forcing would
    // amplify it in the band; the band's part of the plane is made Hermitian
    // here (one thread per pair) before E_f is summed.
    for (int c = (int)threadIdx.x; c < W * W; c += 256) {
        const int my = c % W - B, mz = c / W - B;
        const int m2 = my * my + mz * mz;
        if (!(mz > 0 || (mz == 0 && my > 0)) || (double)m2 < md.kf_lo2 || (double)m2 > md.kf_hi2) continue;
        const int iy = my >= 0 ? my : my + 2 * K + 1, iz = mz;
        const int jy = my > 0 ? 2 * K + 1 - my : -my, jz = mz > 0 ? 2 * K + 1 - mz : 0;
        const uint32_t i1 = (uint32_t)((long long)iz * zp + (long long)iy * (K + 1));
        const uint32_t i2 = (uint32_t)((long long)jz * zp + (long long)jy * (K + 1));
#pragma unroll
        for (int comp = 0; comp < 3; comp++) {
            const Fld<P> F(md.uh, comp * S);
            const Cx<P> a = F.ld(i1), b = F.ld(i2);
            const Cx<P> h = {P(0.5) * (a.re + b.re), P(0.5) * (a.im - b.im)};
            F.st(i1, h);
            F.st(i2, {h.re, -h.im});
        }
    }
    __syncthreads();
    double acc = 0.0;
    for (long long c = threadIdx.x; c < ncand; c += 256) {
        const int mx = (int)(c % (B + 1));
        const int my = (int)((c / (B + 1)) % W) - B;
        const int mz = (int)(c / ((long long)(B + 1) * W)) - B;
        const int m2 = mx * mx + my * my + mz * mz;
        if (m2 == 0 || (double)m2 < md.kf_lo2 || (double)m2 > md.kf_hi2) continue;
        const int iy = my >= 0 ? my : my + 2 * K + 1, iz = mz >= 0 ? mz : mz + 2 * K + 1;
        const long long idx = (long long)iz * zp + (long long)iy * (K + 1) + mx;
        const double w = mx > 0 ? 1.0 : 0.5;
#pragma unroll
        for (int comp = 0; comp < 3; comp++) {
            Cx<P> v = Fld<P>(md.uh, comp * S).ld((uint32_t)idx);
            acc += w * ((double)v.re * (double)v.re + (double)v.im * (double)v.im);
        }
    }
    const double ef = block_sum<256>(acc, red);
    if (threadIdx.x == 0) {
        // A band holding no more than kForceEmptyFrac of the energy the field
        // had at the start of the step (diag.E) is empty: the linear forcing,
        // eps/(2 E_f) u, would otherwise amplify rounding-level band modes to
        // inject eps.  Ef = 0 tells the update to add no forcing.
        const bool forced = ef > kForceEmptyFrac * md.st->diag.E;
        md.st->Ef = forced ? ef : 0.0;
        if (stage == 0) {
            md.st->diag.E_f = ef;
            md.st->diag.inj = forced ? md.eps_m : 0.0;
            md.st->umax_bits = 0ull;
            if (!forced && md.eps_m != 0.0) md.st->diag.flags |= 2;
        }
    }
}

// Loads of one pencil (E values of line L at positions t + M m), truncated:
// position p holds mode m = p or p - N; only |m| <= K is stored, at index
// m (m >= 0) or m + 2K + 1, with stride `stride` between stored modes.
template <typename P, int N, int E>
__device__ __forceinline__ void load_trunc(Cx<P> *v, const Fld<P> &f, uint32_t base, uint32_t stride, int t, bool valid) {
    constexpr int K = N / 3, M = N / E;
#pragma unroll
    for (int m = 0; m < E; m++) {
        const int mm = mode_of(t + M * m, N);
        const bool keep = valid && mm >= -K && mm <= K;
        const uint32_t im = (uint32_t)(mm >= 0 ? mm : mm + 2 * K + 1);
        v[m] = keep ? f.ld(base + im * stride) : czero<P>();
    }
}

// ================================================================== zinv
// z-lines L = iy (K+1) + kx, the (m_y, m_x) pairs numbered as in a state
// plane; lines NZLS..ZP-1 (a plane's pad) carry zeros.  in u_hat
// [3][2K+1][ZP]; out (bufA) [5][N (z)][ZP]:
// U_x, U_y, U_z, W_x = Z^-1[i k_z u_x], W_y = Z^-1[i k_z u_y]
template <typename P, int N, int EV, int TM = 1>
__global__ void __launch_bounds__((Cfg<P, N, EV, TM>::NT), (Cfg<P, N, EV, TM>::PMINW)) k_zinv(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ twg) {
    using C = Cfg<P, N, EV, TM>;
    constexpr int E = C::E, M = C::M, T = C::T, ZP = C::ZP;
    __shared__ LdsT<P> lds[N * T];
    __shared__ Cx<P> tw[twiddle_span(N, E)];               // twiddles in LDS: no global load inside the transforms
    for (int i = (int)threadIdx.x; i < twiddle_span(N, E); i += (int)blockDim.x) tw[i] = twg[i];
    unsigned tile, mem_i;
    xcd_tile(tile, mem_i);
    const MemberDev &md = mems[mem_i];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const int L = tile * T + l;
    const bool inb = L < ZP;                                    // output line (written)
    const bool valid = L < C::NZLS;                             // retained line (read)
    const uint32_t Ls = valid ? (uint32_t)L : 0u;               // the line in the state
    const P dk = (P)md.dk;
    auto kz = [&](int m) { return dk * (P)mode_of(t + M * m, N); };
    auto store = [&](const Cx<P> *v, int f) {
        if (inb) {
            const Fld<P> o(md.bufA, (long long)f * N * ZP);
#pragma unroll
            for (int s = 0; s < E; s++) o.st((uint32_t)Plan<N, E>::out_pos(t, s) * ZP + L, v[s]);
        }
    };
    Cx<P> a[E], b[E], p[E];
    load_trunc<P, N, E>(a, Fld<P>(md.uh, 0), Ls, C::ZP, t, valid);
    load_trunc<P, N, E>(p, Fld<P>(md.uh, C::S), Ls, C::ZP, t, valid);
#pragma unroll
    for (int m = 0; m < E; m++) b[m] = mul_i(cscale(a[m], kz(m)));
    line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
    store(b, 3);
    line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
    store(a, 0);
#pragma unroll
    for (int m = 0; m < E; m++) a[m] = p[m];
    load_trunc<P, N, E>(p, Fld<P>(md.uh, 2 * C::S), Ls, C::ZP, t, valid);
#pragma unroll
    for (int m = 0; m < E; m++) b[m] = mul_i(cscale(a[m], kz(m)));
    line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
    store(b, 4);
    line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
    store(a, 1);
    line_fft<P, N, E, T, +1>(p, lds, l, t, tw);
    store(p, 2);
}

// ================================================================== yinv
// y-lines L = z (K+1) + kx.  in bufA [5][N (z)][ZP] (line L at iy (K+1) of
// plane z); out bufB [6][N / ZB][N (y)][BL] (Cfg::yel):
// u_x, u_y, u_z, omega_x, omega_y, omega_z
template <typename P, int N, int EV, int TM = 1>
__global__ void __launch_bounds__((Cfg<P, N, EV, TM>::NT)) k_yinv(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ twg) {
    using C = Cfg<P, N, EV, TM>;
    constexpr int E = C::E, M = C::M, T = C::T, KX = C::KX, ZP = C::ZP, NYL = C::NYL;
    __shared__ LdsT<P> lds[N * T];
    __shared__ Cx<P> tw[twiddle_span(N, E)];               // twiddles in LDS: no global load inside the transforms
    for (int i = (int)threadIdx.x; i < twiddle_span(N, E); i += (int)blockDim.x) tw[i] = twg[i];
    unsigned tile, mem_i;
    xcd_tile(tile, mem_i);
    const MemberDev &md = mems[mem_i];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const int L = tile * T + l;
    const bool inb = L < NYL;
    const int z = inb ? L / KX : 0;
    const int kx = inb ? L % KX : 0;
    const bool valid = inb;
    const P dk = (P)md.dk;
    const P kxv = dk * (P)kx;
    const uint32_t in_base = (uint32_t)z * ZP + kx;              // + iy (K+1)
    const uint32_t out_base = C::yel(inb ? L : 0, 0, N);          // + y BL
    auto ky = [&](int m) { return dk * (P)mode_of(t + M * m, N); };
    auto load = [&](Cx<P> *v, int f) {
        load_trunc<P, N, E>(v, Fld<P>(md.bufA, (long long)f * N * ZP), in_base, KX, t, valid);
    };
    auto store = [&](const Cx<P> *v, int f) {
        if (inb) {
            const Fld<P> o(md.bufB, (long long)f * N * NYL);
#pragma unroll
            for (int s = 0; s < E; s++) o.st(out_base + (uint32_t)Plan<N, E>::out_pos(t, s) * C::BL, v[s]);
        }
    };
    Cx<P> a[E], b[E], p[E];
    load(a, 0);                                   // U_x
    load(p, 1);                                   // prefetch U_y
    // b = Y^-1[i k_y U_x] = d_y u_x (kept), then u_x
#pragma unroll
    for (int m = 0; m < E; m++) b[m] = mul_i(cscale(a[m], ky(m)));
    line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
    line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
    store(a, 0);
    // u_y and omega_z = i k_x u_y - d_y u_x
#pragma unroll
    for (int m = 0; m < E; m++) a[m] = p[m];
    load(p, 2);                                   // prefetch U_z
    line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
    store(a, 1);
#pragma unroll
    for (int s = 0; s < E; s++) b[s] = mul_i(cscale(a[s], kxv)) - b[s];
    store(b, 5);
    // omega_x = Y^-1[i k_y U_z - W_y], omega_y = Y^-1[W_x - i k_x U_z], u_z
#pragma unroll
    for (int m = 0; m < E; m++) a[m] = p[m];
    load(b, 4);                                   // W_y
    load(p, 3);                                   // prefetch W_x
#pragma unroll
    for (int m = 0; m < E; m++) b[m] = mul_i(cscale(a[m], ky(m))) - b[m];
    line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
    store(b, 3);
#pragma unroll
    for (int m = 0; m < E; m++) b[m] = p[m] - mul_i(cscale(a[m], kxv));
    line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
    store(b, 4);
    line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
    store(a, 2);
}

// ================================================================== xpass
// Rows R = y N + z of K+1 x-modes.  in bufB [6][N][N][K+1]; out bufA
// [3][N][N][K+1] = x-transform (unnormalised) of n = u x omega, truncated to
// m_x <= K.
// The T rows of a workgroup are contiguous in every field, so inputs are
// copied into LDS (and outputs out of it) with linear, fully coalesced
// accesses; the next field pair is fetched into registers while the current
// pair is transformed.  Stage 0 also folds max(|u|+|v|+|w|) into st->umax_bits.
template <typename P, int N, int EV>
__global__ void __launch_bounds__(256) k_xpass(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ twg, int stage) {
    using C = Cfg<P, N, EV>;
    constexpr int E = C::E, M = C::M, T = C::TX, K = C::K, KX = C::KX;
    constexpr long long FS = (long long)N * N * KX;           // elements per input field
    constexpr long long FSO = (long long)N * N * KX;          // elements per output field
    constexpr int RW = T * KX;                                 // elements of the tile per input field
    constexpr int RWO = T * KX;                                // elements of the tile per output field
    // staged rows are K + 2 apart in LDS when K + 1 is a multiple of 16, so
    // that the rows of a wave fall in different banks
    constexpr int LP = KX % 16 == 0 ? KX + 1 : KX, RWL = T * LP;
    constexpr int PER = (RW + 255) / 256;                      // staged elements per thread per field
    __shared__ LdsT<P> lds[N * T];
    __shared__ Cx<P> tw[twiddle_span(N, E)];               // twiddles in LDS: no global load inside the transforms
    for (int i = (int)threadIdx.x; i < twiddle_span(N, E); i += (int)blockDim.x) tw[i] = twg[i];
    __shared__ LdsT<P> sb[2 * RWL];                            // staged pair / two output fields
    __shared__ double redmax[256 / 64];
    unsigned tile, mem_i;
    xcd_tile(tile, mem_i);
    const MemberDev &md = mems[mem_i];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const uint32_t tb = tile * RW;                             // first element of the tile in a field
    Cx<P> st[2][PER];
    auto fetch = [&](int fa) {                                 // global -> registers, linear
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const Fld<P> f(md.bufB, (fa + h) * FS);
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const int e = threadIdx.x + 256 * i;
                st[h][i] = e < RW ? f.ld(tb + e) : czero<P>();
            }
        }
    };
    auto park = [&]() {                                        // registers -> LDS
#pragma unroll
        for (int h = 0; h < 2; h++)
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const int e = threadIdx.x + 256 * i;
                if (e < RW) lds_put<P>(sb, h * RWL + e + (LP - KX) * (e / KX), st[h][i]);
            }
    };
    // packed two-for-one spectrum of the staged pair: C = A + i B, Hermitian fill
    auto gather = [&](Cx<P> *v) {
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int n = t + M * m;
            const bool lo = n <= K, hi = n >= N - K;
            const int kx = lo ? n : N - n;
            Cx<P> A = czero<P>(), B = czero<P>();
            if (lo || hi) { A = lds_get<P>(sb, l * LP + kx); B = lds_get<P>(sb, RWL + l * LP + kx); }
            if (n == 0) v[m] = {A.re, B.re};
            else if (lo) v[m] = {A.re - B.im, A.im + B.re};
            else v[m] = {A.re + B.im, B.re - A.im};            // zero pairs stay zero
        }
    };
    P ph[6][E];
    Cx<P> v[E];
    fetch(0);
    park();
#pragma unroll
    for (int pr = 0; pr < 3; pr++) {
        __syncthreads();                                       // staged pair visible
        gather(v);
        if (pr < 2) fetch(2 * pr + 2);                         // next pair in flight during the transform
        line_fft<P, N, E, T, +1, 0, RowLay<P, T>, truncated_slots(N, E, K)>(v, lds, l, t, tw);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[2 * pr][s] = v[s].re; ph[2 * pr + 1][s] = v[s].im; }
        if (pr < 2) {
            __syncthreads();                                   // every thread has gathered
            park();
        }
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
    for (int m = 0; m < E; m++)          // the split reads only the partner positions 0 and >= N - K
        if (m == 0 || M * m + M - 1 >= N - K) lds_put<P>(lds, (t + M * m) * T + l, d1[m]);
    __syncthreads();
    if (stage == 0 && threadIdx.x == 0) {
        double dm = redmax[0];
        for (int w = 1; w < 256 / 64; w++) dm = redmax[w] > dm ? redmax[w] : dm;
        atomicMax(&md.st->umax_bits, (unsigned long long)__double_as_longlong(dm));
    }
    // split D1 into the x-spectra of n_x and n_y; stage all three in LDS:
    // n_x, n_y -> sb (free since the last gather), n_z -> lds rows after D1 reads
    Cx<P> ox[E], oy[E];
#pragma unroll
    for (int m = 0; m < E; m++) {
        const int k = t + M * m;
        if (k <= K) {
            const Cx<P> a = d1[m];
            const Cx<P> b = lds_get<P>(lds, ((N - k) % N) * T + l);
            const P h = P(0.5);
            ox[m] = {h * (a.re + b.re), h * (a.im - b.im)};
            oy[m] = {h * (a.im + b.im), h * (b.re - a.re)};
        }
    }
    __syncthreads();                                           // D1 partner reads done
#pragma unroll
    for (int m = 0; m < E; m++) {
        const int k = t + M * m;
        if (k <= K) {
            lds_put<P>(sb, l * (K + 1) + k, ox[m]);
            lds_put<P>(sb, RWO + l * (K + 1) + k, oy[m]);
            lds_put<P>(lds, l * (K + 1) + k, d2[m]);
        }
    }
    __syncthreads();
    const Fld<P> o0(md.bufA, 0), o1(md.bufA, FSO), o2(md.bufA, 2 * FSO);
    const uint32_t tbo = tile * RWO;
#pragma unroll
    for (int i = 0; i < (RWO + 255) / 256; i++) {
        const int e = threadIdx.x + 256 * i;
        if (e < RWO) {
            o0.st(tbo + e, lds_get<P>(sb, e));
            o1.st(tbo + e, lds_get<P>(sb, RWO + e));
            o2.st(tbo + e, lds_get<P>(lds, e));
        }
    }
}

// ------------------------------------------------------ pipelined x pass
// The same computation as k_xpass, organised for streaming: a persistent
// workgroup walks a contiguous range of row tiles of one member.  Its six input
// fields arrive by direct-to-LDS loads into two staging buffers (fields 0-2 and
// 3-5 of a tile), and the next tile's fields are requested as soon as a buffer
// has been read, so HBM reads stay in flight through the transforms, the
// product and the stores without holding registers.  Twiddles are read from
// LDS, since a global load consumed inside the loop would wait for every
// earlier copy (vector-memory operations complete in order).  Outputs are
// staged in LDS and written with linear 16-byte stores.
template <typename P, int N, int E_> struct XCfg {
    static constexpr int K = N / 3, E = E_ > N ? N : E_, M = N / E;
    static constexpr int CS = (int)sizeof(Cx<P>), CPV = 16 / CS;
    static constexpr int RQ = K + 1;                           // row pitch in HBM and in the LDS staging
    // FP32: each thread keeps its twiddles in registers; FP64: a table in LDS
    // (registers would cost the second wave per SIMD)
    static constexpr bool REGTW = sizeof(P) == 4;
    static constexpr int NTW = REGTW ? 1 : twiddle_span(N, E);
    static constexpr long long lds_bytes(int t) {
        const long long rs = (long long)t * RQ, ro = (long long)t * (K + 1);
        const long long xl = (long long)N * t > 3 * ro ? (long long)N * t : 3 * ro;
        return (6 * rs + xl + NTW) * CS + 64;
    }
    // rows per tile: the most (at most 256 threads) whose LDS lets three
    // workgroups share a compute unit, else the fewest with one full wave
    static constexpr int pick_t() {
        int t = 256 / M;
        while (t > 1 && (t * M > 64) && lds_bytes(t) > 53248) t /= 2;
        return t < 1 ? 1 : t;
    }
    static constexpr int T = pick_t(), NTH = M * T;
    static constexpr int RW = T * RQ;                      // elements of a tile per field (contiguous in HBM)
    static constexpr int RV = RW / CPV;                    // 16-byte vectors read per field tile
    static constexpr int RWO = T * (K + 1);                // elements written per field tile (rows of K + 1)
    static constexpr int RVO = RWO / CPV;
    static constexpr int D3 = dma_tile_ops<3, RV, NTH>();     // copies per wave per staging buffer
    static constexpr int S = dma_tile_ops<3, RVO, NTH>();     // 16-byte stores per wave per tile
    static constexpr int XL = N * T > 3 * RWO ? N * T : 3 * RWO;
    static constexpr int TILES = N * N / T;
    // waves per SIMD the register budget is cut for: what the LDS allows
    // (workgroups per compute unit times waves per workgroup, over 4 SIMDs),
    // at most 3 (FP32) or 2 (FP64)
    static constexpr int WG_LDS = (int)(163840 / ((lds_bytes(T) + 511) / 512 * 512));
    static constexpr int W_LDS = WG_LDS * (NTH / 64) / 4;
    static constexpr int W_MAX = sizeof(P) == 4 ? 3 : 2;
    static constexpr int MINB = W_LDS < 1 ? 1 : (W_LDS < W_MAX ? W_LDS : W_MAX);
    static_assert(RW % CPV == 0 && RWO % CPV == 0 && NTH % 64 == 0 && RV >= 64 && RVO >= 64 && D3 + S < 64,
                  "x-pass tile shape");
};

template <typename P, int N, int EV>
__global__ void __launch_bounds__((XCfg<P, N, EV>::NTH), (XCfg<P, N, EV>::MINB)) k_xpass_dma(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ tw, int stage) {
    using C = XCfg<P, N, EV>;
    constexpr int E = C::E, M = C::M, T = C::T, K = C::K, NTH = C::NTH, RW = C::RW, RQ = C::RQ;
    constexpr int RWO = C::RWO, RVO = C::RVO;
    constexpr long long FSB = (long long)N * N * RQ * C::CS;         // bytes per input field
    constexpr long long FSBO = (long long)N * N * (K + 1) * C::CS;   // bytes per output field
    __shared__ __attribute__((aligned(16))) LdsT<P> slot0[3 * RW];
    __shared__ __attribute__((aligned(16))) LdsT<P> slot1[3 * RW];
    __shared__ __attribute__((aligned(16))) LdsT<P> lds[C::XL];
    __shared__ Cx<P> twl[C::NTW];
    unsigned chunk, mem_i;
    xcd_tile(chunk, mem_i);
    const MemberDev &md = mems[mem_i];
    const int t0 = (int)((long long)chunk * C::TILES / gridDim.x);
    const int t1 = (int)((long long)(chunk + 1) * C::TILES / gridDim.x);
    if (t0 >= t1) return;                                     // uniform over the workgroup
    const int l = (int)threadIdx.x % T, t = (int)threadIdx.x / T;
    TwRegs<P, N, E> twr;
    if constexpr (C::REGTW) twr.load(tw, t);
    else for (int i = (int)threadIdx.x; i < C::NTW; i += NTH) twl[i] = tw[i];
    const auto &twx = [&]() -> const auto & {
        if constexpr (C::REGTW) return twr;
        else return twl;
    }();
    const char *inb = (const char *)md.bufB;
    char *outb = (char *)md.bufA;
    auto request = [&](LdsT<P> *dst, int tile, int f0) {      // fields f0..f0+2 of `tile`
        dma_tile<3, C::RV, NTH>(dst, inb + (long long)f0 * FSB + (long long)tile * RW * C::CS, FSB);
    };
    // packed two-for-one spectrum of fields (fa, fb): C = A + i B, Hermitian
    // fill.  Position n = t + M m; whole segments [M m, M m + M) below K, above
    // N - K or in between are sorted out at compile time.
    auto gather = [&](Cx<P> *v, const LdsT<P> *fa, const LdsT<P> *fb) {
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int n = t + M * m;
            const int r = l * RQ;
            if (M * m > K && M * m + M - 1 < N - K) {
                v[m] = czero<P>();
            } else if (m > 0 && M * m + M - 1 <= K) {
                const Cx<P> A = lds_get<P>(fa, r + n), B = lds_get<P>(fb, r + n);
                v[m] = {A.re - B.im, A.im + B.re};
            } else if (M * m >= N - K) {
                const Cx<P> A = lds_get<P>(fa, r + N - n), B = lds_get<P>(fb, r + N - n);
                v[m] = {A.re + B.im, B.re - A.im};
            } else {
                const bool lo = n <= K, hi = n >= N - K;
                const int kx = lo ? n : N - n;
                Cx<P> A = czero<P>(), B = czero<P>();
                if (lo || hi) { A = lds_get<P>(fa, r + kx); B = lds_get<P>(fb, r + kx); }
                if (n == 0) v[m] = {A.re, B.re};
                else if (lo) v[m] = {A.re - B.im, A.im + B.re};
                else v[m] = {A.re + B.im, B.re - A.im};
            }
        }
    };
    P umx = P(0);
    Cx<P> v[E];
    // Write the tile staged in lds ([3][T][K+1], contiguous in the output) with
    // 16-byte stores in wave-sized chunks of 64 vectors (the same count per
    // wave; the last chunk of a field is moved back onto its end).
    typedef float F4 __attribute__((ext_vector_type(4)));
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const unsigned lane16 = (threadIdx.x & 63u) * 16u;
    auto store_tile = [&](int tile, bool zero) {
        constexpr int NCF = (RVO + 63) / 64, NCH = 3 * NCF, NW = NTH / 64;
#pragma unroll
        for (int j = 0; j < C::S; j++) {
            int c = j * NW + wave;
            c = c < NCH ? c : NCH - 1;
            const int f = c / NCF, q = c - f * NCF;
            const int st = q * 64 < RVO - 64 ? q * 64 : RVO - 64;
            const F4 x = zero ? F4{0.f, 0.f, 0.f, 0.f} : *(const F4 *)((const char *)lds + (f * RVO + st) * 16 + lane16);
            ENS_GLOBAL char *dst = (ENS_GLOBAL char *)outb + f * FSBO + (long long)tile * RWO * C::CS + st * 16;
            *(ENS_GLOBAL F4 *)(dst + lane16) = x;
        }
    };
    // Wait accounting (vector-memory operations complete in issue order): in
    // the loop, fields 0-2 of a tile are followed by its fields 3-5 (D3 copies)
    // and the previous tile's S stores, fields 3-5 by those stores.  The
    // prologue reproduces that order by writing zeros to the first tile's
    // output (overwritten by the same threads later).  Requests are issued
    // unconditionally (the last tile re-requests itself) and the first pair of
    // the next tile is read at the end of the loop body, so that every read of
    // a staging buffer sees one fixed history of copies.
    request(slot0, t0, 0);
    request(slot1, t0, 3);
    store_tile(t0, true);
    wait_vm<C::D3 + C::S>();                                   // fields 0-2 of the first tile
    lds_barrier();
    gather(v, slot0, slot0 + RW);
    for (int tile = t0; tile < t1; tile++) {
        const bool more = tile + 1 < t1;
        P ph[6][E];
        line_fft<P, N, E, T, +1, 1, RowLay<P, T>, truncated_slots(N, E, K)>(v, lds, l, t, twx);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[0][s] = v[s].re; ph[1][s] = v[s].im; }
        wait_vm<C::S>();                                       // fields 3-5
        lds_barrier();
        gather(v, slot0 + 2 * RW, slot1);
        lds_barrier();                                         // slot0 read by every wave
        request(slot0, more ? tile + 1 : tile, 0);
        line_fft<P, N, E, T, +1, 1, RowLay<P, T>, truncated_slots(N, E, K)>(v, lds, l, t, twx);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[2][s] = v[s].re; ph[3][s] = v[s].im; }
        gather(v, slot1 + RW, slot1 + 2 * RW);
        lds_barrier();                                         // slot1 read by every wave
        request(slot1, more ? tile + 1 : tile, 3);
        line_fft<P, N, E, T, +1, 1, RowLay<P, T>, truncated_slots(N, E, K)>(v, lds, l, t, twx);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[4][s] = v[s].re; ph[5][s] = v[s].im; }
        // ph: 0 u_x, 1 u_y, 2 u_z, 3 omega_x, 4 omega_y, 5 omega_z
        if (stage == 0) {
#pragma unroll
            for (int s = 0; s < E; s++) {
                const P a = fabs(ph[0][s]) + fabs(ph[1][s]) + fabs(ph[2][s]);
                umx = a > umx ? a : umx;
            }
        }
        Cx<P> d1[E], d2[E];
#pragma unroll
        for (int s = 0; s < E; s++) {
            d1[s] = {ph[1][s] * ph[5][s] - ph[2][s] * ph[4][s], ph[2][s] * ph[3][s] - ph[0][s] * ph[5][s]};
            d2[s] = {ph[0][s] * ph[4][s] - ph[1][s] * ph[3][s], P(0)};
        }
        line_fft_T<P, N, E, T, -1, true>(d1, lds, l, t, twx);        // d1[m] = D1[t + M m]
        line_fft_T<P, N, E, T, -1, true>(d2, lds, l, t, twx);
        lds_barrier();
#pragma unroll
        for (int m = 0; m < E; m++)          // the split reads only the partner positions 0 and >= N - K
            if (m == 0 || M * m + M - 1 >= N - K) lds_put<P>(lds, (t + M * m) * T + l, d1[m]);
        lds_barrier();
        // split D1 into the x-spectra of n_x and n_y
        Cx<P> ox[E], oy[E];
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int k = t + M * m;
            if (M * m <= K && (M * m + M - 1 <= K || k <= K)) {
                const Cx<P> a = d1[m];
                const Cx<P> b = lds_get<P>(lds, ((N - k) % N) * T + l);
                const P h = P(0.5);
                ox[m] = {h * (a.re + b.re), h * (a.im - b.im)};
                oy[m] = {h * (a.im + b.im), h * (b.re - a.re)};
            }
        }
        lds_barrier();                                         // partner reads done
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int k = t + M * m;
            if (M * m <= K && (M * m + M - 1 <= K || k <= K)) {
                lds_put<P>(lds, l * (K + 1) + k, ox[m]);
                lds_put<P>(lds, RWO + l * (K + 1) + k, oy[m]);
                lds_put<P>(lds, 2 * RWO + l * (K + 1) + k, d2[m]);
            }
        }
        lds_barrier();
        store_tile(tile, false);
        if (more) {                                            // first pair of the next tile
            wait_vm<C::D3 + C::S>();                           // its fields 0-2 precede 3-5 and the stores
            lds_barrier();
            gather(v, slot0, slot0 + RW);
        }
    }
    wait_vm<0>();                                              // no copy into LDS outlives the workgroup
    if (stage == 0) {
        double dm = (double)umx;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(dm, off, 64);
            dm = o > dm ? o : dm;
        }
        if ((threadIdx.x & 63) == 0) atomicMax(&md.st->umax_bits, (unsigned long long)__double_as_longlong(dm));
    }
}

// ------------------------------------------------------ wave-private x pass
// The streamed x pass with every workgroup one wave: a tile is the R = 64 / M
// rows whose transforms the wave's lanes hold (lane = row * M + thread), so
// every exchange of the transforms stays inside the wave.  The LDS executes
// one wave's operations in issue order, so no exchange needs an s_barrier or
// an LDS wait, only a compiler fence (stage barrier kind 2); rows are XOR
// swizzled per 128-byte block (WaveLay) so that the strided and the
// consecutive exchange patterns both spread over all banks.  The wave copies
// its own inputs (direct-to-LDS) and stores its own outputs, so the only
// waits left are the exact vector-memory counts of the copies and an LDS wait
// before a staging buffer is handed back to the copies.
// Whether the wave-private x pass has a valid tile for (N, E, complex size):
// a line within one wave, whole 16-byte vectors per output tile, at least one
// wave-sized copy per field and a vector-memory count that fits its counter.
constexpr bool xwave_ok(int N, int E, int CS) {
    const int M = N / (E > N ? N : E), K = N / 3, CPV = 16 / CS;
    if (M > 64 || 64 % M != 0) return false;
    const int R = 64 / M, RWO = R * (K + 1), RV = RWO / CPV;
    if (RWO % CPV != 0 || RV < 64) return false;
    const int D3 = 3 * ((RV + 63) / 64), S = 3 * ((RWO / CPV + 63) / 64);
    return D3 + S < 64;
}

template <typename P, int N, int E_> struct XWCfg {
    static constexpr int K = N / 3, E = E_ > N ? N : E_, M = N / E;
    static constexpr int R = 64 / M;                           // rows per tile (one wave)
    static constexpr int CS = (int)sizeof(Cx<P>), CPV = 16 / CS;
    static constexpr int RQ = K + 1;                           // row pitch in HBM and in the LDS staging
    static constexpr bool REGTW = sizeof(P) == 4;               // FP32: twiddles in registers
    static constexpr int NTW = REGTW ? 1 : twiddle_span(N, E);
    static constexpr int RW = R * RQ, RV = RW / CPV;            // a tile's elements / 16-byte vectors per field
    static constexpr int RWO = R * (K + 1), RVO = RWO / CPV;
    static constexpr int D3 = dma_tile_ops<3, RV, 64>();          // copies per staging buffer
    static constexpr int S = dma_tile_ops<3, RVO, 64>();          // 16-byte stores per tile
    static constexpr int XL = N * R > 3 * RWO ? N * R : 3 * RWO;
    static constexpr int TILES = N * N / R;
    static constexpr long long LDS_BYTES = (6LL * RW + XL + NTW) * CS + 64;
    // waves per SIMD the register budget is cut for: what the LDS allows (one
    // wave per workgroup, four SIMDs per compute unit), at most 4
    static constexpr int WPS = (int)(163840 / ((LDS_BYTES + 511) / 512 * 512)) / 4;
    static constexpr int MINW = WPS < 1 ? 1 : (WPS > 4 ? 4 : WPS);
    static_assert(M <= 64 && 64 % M == 0, "a line must fit one wave");
    static_assert(RW % CPV == 0 && RWO % CPV == 0 && RV >= 64 && RVO >= 64 && D3 + S < 64, "x-pass tile shape");
};

template <typename P, int N, int EV>
__global__ void __launch_bounds__(64, (XWCfg<P, N, EV>::MINW)) k_xpass_wave(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ tw, int stage) {
    using C = XWCfg<P, N, EV>;
    using LY = WaveLay<P, N>;
    constexpr int E = C::E, M = C::M, R = C::R, K = C::K, RW = C::RW, RQ = C::RQ;
    constexpr int RWO = C::RWO, RVO = C::RVO;
    constexpr long long FSB = (long long)N * N * RQ * C::CS;         // bytes per input field
    constexpr long long FSBO = (long long)N * N * (K + 1) * C::CS;   // bytes per output field
    __shared__ __attribute__((aligned(16))) LdsT<P> slot0[3 * RW];
    __shared__ __attribute__((aligned(16))) LdsT<P> slot1[3 * RW];
    __shared__ __attribute__((aligned(16))) LdsT<P> lds[C::XL];
    __shared__ Cx<P> twl[C::NTW];
    unsigned chunk, mem_i;
    xcd_tile(chunk, mem_i);
    const MemberDev &md = mems[mem_i];
    const int t0 = (int)((long long)chunk * C::TILES / gridDim.x);
    const int t1 = (int)((long long)(chunk + 1) * C::TILES / gridDim.x);
    if (t0 >= t1) return;                                     // uniform over the wave
    const int t = (int)threadIdx.x % M, l = (int)threadIdx.x / M;
    TwRegs<P, N, E> twr;
    if constexpr (C::REGTW) twr.load(tw, t);
    else for (int i = (int)threadIdx.x; i < C::NTW; i += 64) twl[i] = tw[i];
    wave_fence();
    const auto &twx = [&]() -> const auto & {
        if constexpr (C::REGTW) return twr;
        else return twl;
    }();
    const char *inb = (const char *)md.bufB;
    char *outb = (char *)md.bufA;
    auto request = [&](LdsT<P> *dst, int tile, int f0) {      // fields f0..f0+2 of the tile's R rows
        dma_tile<3, C::RV, 64>(dst, inb + (long long)f0 * FSB + (long long)tile * RW * C::CS, FSB);
    };
    // packed two-for-one spectrum of fields (fa, fb), as in the streamed x pass
    auto gather = [&](Cx<P> *v, const LdsT<P> *fa, const LdsT<P> *fb) {
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int n = t + M * m;
            const int r = l * RQ;
            if (M * m > K && M * m + M - 1 < N - K) {
                v[m] = czero<P>();
            } else if (m > 0 && M * m + M - 1 <= K) {
                const Cx<P> A = lds_get<P>(fa, r + n), B = lds_get<P>(fb, r + n);
                v[m] = {A.re - B.im, A.im + B.re};
            } else if (M * m >= N - K) {
                const Cx<P> A = lds_get<P>(fa, r + N - n), B = lds_get<P>(fb, r + N - n);
                v[m] = {A.re + B.im, B.re - A.im};
            } else {
                const bool lo = n <= K, hi = n >= N - K;
                const int kx = lo ? n : N - n;
                Cx<P> A = czero<P>(), B = czero<P>();
                if (lo || hi) { A = lds_get<P>(fa, r + kx); B = lds_get<P>(fb, r + kx); }
                if (n == 0) v[m] = {A.re, B.re};
                else if (lo) v[m] = {A.re - B.im, A.im + B.re};
                else v[m] = {A.re + B.im, B.re - A.im};
            }
        }
    };
    P umx = P(0);
    Cx<P> v[E];
    typedef float F4 __attribute__((ext_vector_type(4)));
    const unsigned lane16 = (threadIdx.x & 63u) * 16u;
    // the tile's outputs staged in lds ([3][R][K+1], contiguous in the output)
    // leave in wave-sized chunks of 64 vectors, the last chunk of a field moved
    // back onto its end
    auto store_tile = [&](int tile, bool zero) {
        constexpr int NCF = (RVO + 63) / 64, NCH = 3 * NCF;
#pragma unroll
        for (int c = 0; c < NCH; c++) {
            const int f = c / NCF, q = c - f * NCF;
            const int st = q * 64 < RVO - 64 ? q * 64 : RVO - 64;
            const F4 x = zero ? F4{0.f, 0.f, 0.f, 0.f} : *(const F4 *)((const char *)lds + (f * RVO + st) * 16 + lane16);
            ENS_GLOBAL char *dst = (ENS_GLOBAL char *)outb + f * FSBO + (long long)tile * RWO * C::CS + st * 16;
            *(ENS_GLOBAL F4 *)(dst + lane16) = x;
        }
    };
    static_assert(C::S == 3 * ((RVO + 63) / 64), "store count");
    // Wait accounting as in the streamed x pass (vector-memory operations
    // complete in issue order; requests are unconditional, the prologue writes
    // zeros to the first tile's output to reproduce the loop's order).
    request(slot0, t0, 0);
    request(slot1, t0, 3);
    store_tile(t0, true);
    wait_vm<C::D3 + C::S>();                                   // fields 0-2 of the first tile
    wave_fence();
    gather(v, slot0, slot0 + RW);
    for (int tile = t0; tile < t1; tile++) {
        const bool more = tile + 1 < t1;
        P ph[6][E];
        line_fft<P, N, E, R, +1, 2, LY, truncated_slots(N, E, K)>(v, lds, l, t, twx);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[0][s] = v[s].re; ph[1][s] = v[s].im; }
        wait_vm<C::S>();                                       // fields 3-5
        wave_fence();
        gather(v, slot0 + 2 * RW, slot1);
        lds_wait();                                            // slot0 read
        request(slot0, more ? tile + 1 : tile, 0);
        line_fft<P, N, E, R, +1, 2, LY, truncated_slots(N, E, K)>(v, lds, l, t, twx);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[2][s] = v[s].re; ph[3][s] = v[s].im; }
        gather(v, slot1 + RW, slot1 + 2 * RW);
        lds_wait();                                            // slot1 read
        request(slot1, more ? tile + 1 : tile, 3);
        line_fft<P, N, E, R, +1, 2, LY, truncated_slots(N, E, K)>(v, lds, l, t, twx);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[4][s] = v[s].re; ph[5][s] = v[s].im; }
        // ph: 0 u_x, 1 u_y, 2 u_z, 3 omega_x, 4 omega_y, 5 omega_z
        if (stage == 0) {
#pragma unroll
            for (int s = 0; s < E; s++) {
                const P a = fabs(ph[0][s]) + fabs(ph[1][s]) + fabs(ph[2][s]);
                umx = a > umx ? a : umx;
            }
        }
        Cx<P> d1[E], d2[E];
#pragma unroll
        for (int s = 0; s < E; s++) {
            d1[s] = {ph[1][s] * ph[5][s] - ph[2][s] * ph[4][s], ph[2][s] * ph[3][s] - ph[0][s] * ph[5][s]};
            d2[s] = {ph[0][s] * ph[4][s] - ph[1][s] * ph[3][s], P(0)};
        }
        line_fft_T<P, N, E, R, -1, 2, LY>(d1, lds, l, t, twx);        // d1[m] = D1[t + M m]
        line_fft_T<P, N, E, R, -1, 2, LY>(d2, lds, l, t, twx);
        wave_fence();
#pragma unroll
        for (int m = 0; m < E; m++)          // the split reads only the partner positions 0 and >= N - K
            if (m == 0 || M * m + M - 1 >= N - K) lds_put<P>(lds, LY::slot(t + M * m, l), d1[m]);
        wave_fence();
        // split D1 into the x-spectra of n_x and n_y
        Cx<P> ox[E], oy[E];
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int k = t + M * m;
            if (M * m <= K && (M * m + M - 1 <= K || k <= K)) {
                const Cx<P> a = d1[m];
                const Cx<P> b = lds_get<P>(lds, LY::slot((N - k) % N, l));
                const P h = P(0.5);
                ox[m] = {h * (a.re + b.re), h * (a.im - b.im)};
                oy[m] = {h * (a.im + b.im), h * (b.re - a.re)};
            }
        }
        wave_fence();
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int k = t + M * m;
            if (M * m <= K && (M * m + M - 1 <= K || k <= K)) {
                lds_put<P>(lds, l * (K + 1) + k, ox[m]);
                lds_put<P>(lds, RWO + l * (K + 1) + k, oy[m]);
                lds_put<P>(lds, 2 * RWO + l * (K + 1) + k, d2[m]);
            }
        }
        wave_fence();
        store_tile(tile, false);
        if (more) {                                            // first pair of the next tile
            wait_vm<C::D3 + C::S>();
            wave_fence();
            gather(v, slot0, slot0 + RW);
        }
    }
    wait_vm<0>();                                              // no copy into LDS outlives the workgroup
    if (stage == 0) {
        double dm = (double)umx;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(dm, off, 64);
            dm = o > dm ? o : dm;
        }
        if (threadIdx.x == 0) atomicMax(&md.st->umax_bits, (unsigned long long)__double_as_longlong(dm));
    }
}

// Wave-private x pass with the six input fields staged as three pairs through
// two buffers of two fields each (instead of two buffers of three): pair q of
// the wave's sequence (3 per tile) goes to buffer q mod 2 and is requested as
// soon as pair q - 2 has been read from it, so two pairs are resident or in
// flight at any time.  A third less staging LDS per wave than k_xpass_wave
// (19.5 against 24.8 KB for 256-point FP32 rows), so that eight one-wave
// workgroups share a compute unit, two per SIMD, where six leave two SIMDs
// with a single wave.
template <typename P, int N, int E_> struct XW2Cfg {
    using B = XWCfg<P, N, E_>;
    static constexpr int D2 = dma_tile_ops<2, B::RV, 64>();    // copies per pair
    static constexpr long long LDS_BYTES = (4LL * B::RW + B::XL + B::NTW) * B::CS + 64;
    static constexpr int WPS = (int)(163840 / ((LDS_BYTES + 511) / 512 * 512)) / 4;
    static constexpr int MINW = WPS < 1 ? 1 : (WPS > 4 ? 4 : WPS);
    static_assert(D2 + B::S < 64, "vector-memory count of the x-pass tile");
};

template <typename P, int N, int EV>
__global__ void __launch_bounds__(64, (XW2Cfg<P, N, EV>::MINW)) k_xpass_wave2(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ tw, int stage) {
    using C = XWCfg<P, N, EV>;
    using C2 = XW2Cfg<P, N, EV>;
    using LY = WaveLay<P, N>;
    constexpr int E = C::E, M = C::M, R = C::R, K = C::K, RW = C::RW, RQ = C::RQ;
    constexpr int RWO = C::RWO, RVO = C::RVO, D2 = C2::D2, S = C::S;
    constexpr long long FSB = (long long)N * N * RQ * C::CS;         // bytes per input field
    constexpr long long FSBO = (long long)N * N * (K + 1) * C::CS;   // bytes per output field
    __shared__ __attribute__((aligned(16))) LdsT<P> slotA[2 * RW];
    __shared__ __attribute__((aligned(16))) LdsT<P> slotB[2 * RW];
    __shared__ __attribute__((aligned(16))) LdsT<P> lds[C::XL];
    __shared__ Cx<P> twl[C::NTW];
    unsigned chunk, mem_i;
    xcd_tile(chunk, mem_i);
    const MemberDev &md = mems[mem_i];
    const int t0 = (int)((long long)chunk * C::TILES / gridDim.x);
    const int t1 = (int)((long long)(chunk + 1) * C::TILES / gridDim.x);
    if (t0 >= t1) return;                                     // uniform over the wave
    const int t = (int)threadIdx.x % M, l = (int)threadIdx.x / M;
    TwRegs<P, N, E> twr;
    if constexpr (C::REGTW) twr.load(tw, t);
    else for (int i = (int)threadIdx.x; i < C::NTW; i += 64) twl[i] = tw[i];
    wave_fence();
    const auto &twx = [&]() -> const auto & {
        if constexpr (C::REGTW) return twr;
        else return twl;
    }();
    const char *inb = (const char *)md.bufB;
    char *outb = (char *)md.bufA;
    auto slot = [&](int i) -> LdsT<P> * { return i ? slotB : slotA; };
    auto request = [&](LdsT<P> *dst, int tile, int pair) {    // fields 2 pair, 2 pair + 1 of the tile's R rows
        dma_tile<2, C::RV, 64>(dst, inb + (long long)(2 * pair) * FSB + (long long)tile * RW * C::CS, FSB);
    };
    auto gather = [&](Cx<P> *v, const LdsT<P> *fa, const LdsT<P> *fb) {
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int n = t + M * m;
            const int r = l * RQ;
            if (M * m > K && M * m + M - 1 < N - K) {
                v[m] = czero<P>();
            } else if (m > 0 && M * m + M - 1 <= K) {
                const Cx<P> A = lds_get<P>(fa, r + n), B = lds_get<P>(fb, r + n);
                v[m] = {A.re - B.im, A.im + B.re};
            } else if (M * m >= N - K) {
                const Cx<P> A = lds_get<P>(fa, r + N - n), B = lds_get<P>(fb, r + N - n);
                v[m] = {A.re + B.im, B.re - A.im};
            } else {
                const bool lo = n <= K, hi = n >= N - K;
                const int kx = lo ? n : N - n;
                Cx<P> A = czero<P>(), B = czero<P>();
                if (lo || hi) { A = lds_get<P>(fa, r + kx); B = lds_get<P>(fb, r + kx); }
                if (n == 0) v[m] = {A.re, B.re};
                else if (lo) v[m] = {A.re - B.im, A.im + B.re};
                else v[m] = {A.re + B.im, B.re - A.im};
            }
        }
    };
    P umx = P(0);
    Cx<P> v[E];
    typedef float F4 __attribute__((ext_vector_type(4)));
    const unsigned lane16 = (threadIdx.x & 63u) * 16u;
    auto store_tile = [&](int tile, bool zero) {
        constexpr int NCF = (RVO + 63) / 64, NCH = 3 * NCF;
#pragma unroll
        for (int c = 0; c < NCH; c++) {
            const int f = c / NCF, q = c - f * NCF;
            const int st = q * 64 < RVO - 64 ? q * 64 : RVO - 64;
            const F4 x = zero ? F4{0.f, 0.f, 0.f, 0.f} : *(const F4 *)((const char *)lds + (f * RVO + st) * 16 + lane16);
            ENS_GLOBAL char *dst = (ENS_GLOBAL char *)outb + f * FSBO + (long long)tile * RWO * C::CS + st * 16;
            *(ENS_GLOBAL F4 *)(dst + lane16) = x;
        }
    };
    // Wait accounting (vector-memory operations complete in issue order).  The
    // wave's pair requests R(q), q = 3 (tile - t0) + j, and its tile stores
    // S(tile) are issued in the order ... R(3u+1) S(u-1) R(3u+2) R(3u+3) R(3u+4)
    // S(u) ..., so before reading pair 0 of tile u at most D2 + S operations
    // issued after it may be outstanding, before pair 1 S + D2, before pair 2
    // D2.  The prologue writes zeros to the first tile's output to reproduce
    // that order; requests past the last tile repeat the last tile's pairs.
    request(slot(0), t0, 0);
    request(slot(1), t0, 1);
    store_tile(t0, true);
    wait_vm<D2 + S>();                                         // pair 0 of the first tile
    wave_fence();
    gather(v, slot(0), slot(0) + RW);
    for (int tile = t0; tile < t1; tile++) {
        const int u = (tile - t0) & 1;                         // pairs 0, 1, 2 of this tile in slots u, 1 - u, u
        const bool more = tile + 1 < t1;
        const int nxt = more ? tile + 1 : tile;
        P ph[6][E];
        lds_wait();                                            // pair 0 read
        request(slot(u), tile, 2);
        line_fft<P, N, E, R, +1, 2, LY, truncated_slots(N, E, K)>(v, lds, l, t, twx);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[0][s] = v[s].re; ph[1][s] = v[s].im; }
        wait_vm<S + D2>();                                     // pair 1
        wave_fence();
        gather(v, slot(1 - u), slot(1 - u) + RW);
        lds_wait();                                            // pair 1 read
        request(slot(1 - u), nxt, 0);
        line_fft<P, N, E, R, +1, 2, LY, truncated_slots(N, E, K)>(v, lds, l, t, twx);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[2][s] = v[s].re; ph[3][s] = v[s].im; }
        wait_vm<D2>();                                         // pair 2
        wave_fence();
        gather(v, slot(u), slot(u) + RW);
        lds_wait();                                            // pair 2 read
        request(slot(u), nxt, 1);
        line_fft<P, N, E, R, +1, 2, LY, truncated_slots(N, E, K)>(v, lds, l, t, twx);
#pragma unroll
        for (int s = 0; s < E; s++) { ph[4][s] = v[s].re; ph[5][s] = v[s].im; }
        // ph: 0 u_x, 1 u_y, 2 u_z, 3 omega_x, 4 omega_y, 5 omega_z
        if (stage == 0) {
#pragma unroll
            for (int s = 0; s < E; s++) {
                const P a = fabs(ph[0][s]) + fabs(ph[1][s]) + fabs(ph[2][s]);
                umx = a > umx ? a : umx;
            }
        }
        Cx<P> d1[E], d2[E];
#pragma unroll
        for (int s = 0; s < E; s++) {
            d1[s] = {ph[1][s] * ph[5][s] - ph[2][s] * ph[4][s], ph[2][s] * ph[3][s] - ph[0][s] * ph[5][s]};
            d2[s] = {ph[0][s] * ph[4][s] - ph[1][s] * ph[3][s], P(0)};
        }
        line_fft_T<P, N, E, R, -1, 2, LY>(d1, lds, l, t, twx);        // d1[m] = D1[t + M m]
        line_fft_T<P, N, E, R, -1, 2, LY>(d2, lds, l, t, twx);
        wave_fence();
#pragma unroll
        for (int m = 0; m < E; m++)          // the split reads only the partner positions 0 and >= N - K
            if (m == 0 || M * m + M - 1 >= N - K) lds_put<P>(lds, LY::slot(t + M * m, l), d1[m]);
        wave_fence();
        Cx<P> ox[E], oy[E];
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int k = t + M * m;
            if (M * m <= K && (M * m + M - 1 <= K || k <= K)) {
                const Cx<P> a = d1[m];
                const Cx<P> b = lds_get<P>(lds, LY::slot((N - k) % N, l));
                const P h = P(0.5);
                ox[m] = {h * (a.re + b.re), h * (a.im - b.im)};
                oy[m] = {h * (a.im + b.im), h * (b.re - a.re)};
            }
        }
        wave_fence();
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int k = t + M * m;
            if (M * m <= K && (M * m + M - 1 <= K || k <= K)) {
                lds_put<P>(lds, l * (K + 1) + k, ox[m]);
                lds_put<P>(lds, RWO + l * (K + 1) + k, oy[m]);
                lds_put<P>(lds, 2 * RWO + l * (K + 1) + k, d2[m]);
            }
        }
        wave_fence();
        store_tile(tile, false);
        if (more) {                                            // pair 0 of the next tile, in slot 1 - u
            wait_vm<D2 + S>();
            wave_fence();
            gather(v, slot(1 - u), slot(1 - u) + RW);
        }
    }
    wait_vm<0>();                                              // no copy into LDS outlives the workgroup
    if (stage == 0) {
        double dm = (double)umx;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(dm, off, 64);
            dm = o > dm ? o : dm;
        }
        if (threadIdx.x == 0) atomicMax(&md.st->umax_bits, (unsigned long long)__double_as_longlong(dm));
    }
}

// ================================================================== yfwd
// y-lines L = z (K+1) + kx.  in bufA [3][N / ZB][N (y)][BL] (the x-pass
// rows); out bufB [3][N / ZB][2K+1 (m_y)][BL]
template <typename P, int N, int EV, int TM = 1>
__global__ void __launch_bounds__((Cfg<P, N, EV, TM>::NT)) k_yfwd(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ twg) {
    using C = Cfg<P, N, EV, TM>;
    constexpr int E = C::E, M = C::M, T = C::T, K = C::K, NYL = C::NYL;
    constexpr long long FS = (long long)N * NYL;
    __shared__ LdsT<P> lds[N * T];
    __shared__ Cx<P> tw[twiddle_span(N, E)];               // twiddles in LDS: no global load inside the transforms
    for (int i = (int)threadIdx.x; i < twiddle_span(N, E); i += (int)blockDim.x) tw[i] = twg[i];
    unsigned tile, mem_i;
    xcd_tile(tile, mem_i);
    const MemberDev &md = mems[mem_i];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const int L = tile * T + l;
    const bool inb = L < NYL;
    const bool valid = inb;
    const uint32_t in_base = C::yel(inb ? L : 0, 0, N);           // + y BL
    const uint32_t out_base = C::yel(inb ? L : 0, 0, 2 * K + 1);  // + m_y BL
    auto load = [&](Cx<P> *v, int f) {
        const Fld<P> in(md.bufA, f * FS);
#pragma unroll
        for (int m = 0; m < E; m++) v[m] = valid ? in.ld(in_base + (uint32_t)(t + M * m) * C::BL) : czero<P>();
    };
    Cx<P> a[E], p[E];
    load(a, 0);
#pragma unroll
    for (int f = 0; f < 3; f++) {
        if (f < 2) load(p, f + 1);
        line_fft<P, N, E, T, -1>(a, lds, l, t, tw);
        if (inb) {
            const Fld<P> o(md.bufB, (long long)f * (2 * K + 1) * NYL);
#pragma unroll
            for (int s = 0; s < E; s++) {
                const int my = mode_of(Plan<N, E>::out_pos(t, s), N);
                if (my >= -K && my <= K) o.st(out_base + (uint32_t)(my >= 0 ? my : my + 2 * K + 1) * C::BL, a[s]);
            }
        }
        if (f < 2) {
#pragma unroll
            for (int m = 0; m < E; m++) a[m] = p[m];
        }
    }
}

// ================================================================== zfwd + update
// z-lines L = iy (K+1) + kx of the state; in bufB [3][N / ZB][2K+1][BL]
// line L's position z is at block z / ZB, row iy, entry (z mod ZB)(K+1) + kx.
// Forward along z, keep |m_z| <= K, normalise by N^-3, project, add band
// forcing, RK stage update.
// The RK stage is a template parameter: no run-time branches on it.
// FUSE: the kernel also performs the next stage's z inverse (k_zinv's five
// outputs in bufA) from the updated velocity it holds in registers, so that
// the next stage does not read the velocity back; in the last stage, the z
// inverse of the next step's first stage.  That velocity is the one before
// the next stage's band step makes the band's part of the m_x = 0 plane
// Hermitian; the part it removes is invisible to the x pass, which takes
// only the real part at m_x = 0.
template <typename P, int N, int stage, bool FUSE = false>
__global__ void __launch_bounds__((Cfg<P, N, 8>::NTZ), (Cfg<P, N, 8>::ZMINB)) k_zfwd_update(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ twg) {
    using C = Cfg<P, N, 8>;
    constexpr int E = C::EZ, M = C::MZ, T = C::TZ, K = C::K, KX = C::KX, NYL = C::NYL, S = C::S;
    constexpr int ZB = C::ZB, BL = C::BL;
    constexpr int NT = C::NTZ;
    static_assert(NT * sizeof(double) <= N * T * sizeof(LdsT<P>), "reduction scratch reuses the FFT LDS");
    __shared__ LdsT<P> lds[N * T];
    __shared__ Cx<P> tw[twiddle_span(N, E)];               // twiddles in LDS: no global load inside the transforms
    __shared__ double ezt[N];                               // exp(-nh m_z^2) by position
    for (int i = (int)threadIdx.x; i < twiddle_span(N, E); i += (int)blockDim.x) tw[i] = twg[i];
    double *red = reinterpret_cast<double *>(lds);
    unsigned tile, mem_i;
    xcd_tile(tile, mem_i);
    const MemberDev &md = mems[mem_i];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const int L = tile * T + l;
    const bool valid = L < C::NZLS;
    const int iy = valid ? L / (K + 1) : 0;
    const int kx = valid ? L % (K + 1) : 0;
    const uint32_t Lz = (uint32_t)iy * BL + (uint32_t)kx;      // position 0 of the line in bufB
    const int my = iy <= K ? iy : iy - (2 * K + 1);
    // time step of this RK step
    double dt;
    if (md.dt_fixed > 0.0) dt = md.dt_fixed;
    else if (stage == 0) {
        const double um = __longlong_as_double((long long)md.st->umax_bits);
        dt = um > 0.0 ? md.cfl * (md.box / N) / um : 0.0;
    } else dt = md.st->dt;
    if (stage == 0 && tile == 0 && threadIdx.x == 0) {
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
    // integrating factor exp(-nh |m|^2) = exp(-nh (m_x^2 + m_y^2)) exp(-nh m_z^2):
    // one exponential per line and a table of the m_z factors per workgroup
    for (int i = (int)threadIdx.x; i < N; i += NT) {
        const double mz = (double)mode_of(i, N);
        ezt[i] = exp(-nh * mz * mz);
    }
    const double exy = exp(-nh * (double)(kx * kx + my * my));
    Cx<P> a[3][E];
#pragma unroll
    for (int f = 0; f < 3; f++) {
        const Fld<P> in(md.bufB, (long long)f * (2 * K + 1) * NYL);
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int z = t + M * m;
            a[f][m] = valid ? in.ld((uint32_t)(z / ZB) * (uint32_t)((2 * K + 1) * BL) + (uint32_t)(z % ZB) * KX + Lz)
                            : czero<P>();
        }
    }
#pragma unroll
    for (int f = 0; f < 3; f++) line_fft<P, N, E, T, -1>(a[f], lds, l, t, tw);
    __syncthreads();
    const P inv_n3 = (P)(1.0 / ((double)N * N * N));
    const P dk = (P)md.dk, nu = (P)md.nu;
    const double kf_lo2 = md.kf_lo2, kf_hi2 = md.kf_hi2;
    const bool explicit_visc = md.visc_mode == 1;
    const Fld<P> U[3] = {Fld<P>(md.uh, 0), Fld<P>(md.uh, S), Fld<P>(md.uh, 2 * S)};
    const Fld<P> Q[3] = {Fld<P>(md.q, 0), Fld<P>(md.q, S), Fld<P>(md.q, 2 * S)};
    double eacc = 0.0, dacc = 0.0;
    if (valid) {
        // stage 0 (no RK register to read) takes the outputs in pairs: the
        // state loads of a pair are issued before its arithmetic (from a
        // valid address for a mode that is not kept, whose value is then
        // discarded), so that their latencies overlap; stages 1 and 2 take
        // one output at a time (pairs with their register loads spill)
        constexpr int HB = stage == 0 ? 2 : 1;
#pragma unroll
        for (int s0 = 0; s0 < E; s0 += HB) {
            Cx<P> ub[HB][3], qb[HB][3];
#pragma unroll
            for (int j = 0; j < HB; j++) {
                const int mz = mode_of(Plan<N, E>::out_pos(t, s0 + j), N);
                const bool keep = mz >= -K && mz <= K;
                const uint32_t idx = (uint32_t)(keep ? (mz >= 0 ? mz : mz + 2 * K + 1) : 0) * C::ZP + L;
#pragma unroll
                for (int c = 0; c < 3; c++) ub[j][c] = U[c].ld(idx);
#pragma unroll
                for (int c = 0; c < 3; c++) qb[j][c] = stage == 0 ? czero<P>() : Q[c].ld(idx);
            }
#pragma unroll
            for (int j = 0; j < HB; j++) {
                const int s = s0 + j;
                const int pz = Plan<N, E>::out_pos(t, s);
                const int mz = mode_of(pz, N);
                if (mz < -K || mz > K) {
                    if constexpr (FUSE) a[0][s] = a[1][s] = a[2][s] = czero<P>();
                    continue;
                }
                const int iz = mz >= 0 ? mz : mz + 2 * K + 1;
                const uint32_t idx = (uint32_t)iz * C::ZP + L;
                const int m2 = kx * kx + my * my + mz * mz;
                const P kxv = dk * (P)kx, kyv = dk * (P)my, kzv = dk * (P)mz;
                const P k2 = kxv * kxv + kyv * kyv + kzv * kzv;
                Cx<P> *u = ub[j], g[3];
                {
                    // the band forcing joins the nonlinear term before the projection:
                    // unprojected, it would amplify the rounding-level divergent part
                    // of u in the band at the rate eps/(2 E_f) - nu k^2 > 0
                    const P fb = ((double)m2 >= kf_lo2 && (double)m2 <= kf_hi2) ? ffac : P(0);
                    const Cx<P> n0 = cscale(a[0][s], inv_n3) + cscale(u[0], fb);
                    const Cx<P> n1 = cscale(a[1][s], inv_n3) + cscale(u[1], fb);
                    const Cx<P> n2 = cscale(a[2][s], inv_n3) + cscale(u[2], fb);
                    const P ik2 = m2 == 0 ? P(0) : P(1) / k2;
                    const Cx<P> kn = cscale(n0, kxv) + cscale(n1, kyv) + cscale(n2, kzv);
                    g[0] = n0 - cscale(kn, kxv * ik2);
                    g[1] = n1 - cscale(kn, kyv * ik2);
                    g[2] = n2 - cscale(kn, kzv * ik2);
                    if (m2 == 0) g[0] = g[1] = g[2] = czero<P>();
                }
                if (explicit_visc) {
#pragma unroll
                    for (int c = 0; c < 3; c++) g[c] = g[c] - cscale(u[c], nu * k2);
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        Cx<P> q = qb[j][c];
                        q = cscale(q, As) + cscale(g[c], Pdt);
                        u[c] = u[c] + cscale(q, Bs);
                        if (stage < 2) Q[c].st(idx, q);       // the last stage's register is never read
                        U[c].st(idx, u[c]);
                        if constexpr (FUSE) a[c][s] = u[c];
                    }
                } else {
                    const P es = (P)(exy * ezt[pz]);
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        Cx<P> q = qb[j][c];
                        q = cscale(cscale(q, As) + cscale(g[c], Pdt), es);
                        u[c] = cscale(u[c], es) + cscale(q, Bs);
                        if (stage < 2) Q[c].st(idx, q);       // the last stage's register is never read
                        U[c].st(idx, u[c]);
                        if constexpr (FUSE) a[c][s] = u[c];
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
    }
    if constexpr (FUSE) {
        // a[c][s]: the updated u_c at position out_pos(t, s), zero outside the
        // retained modes and on lines without modes; the transposed flow takes
        // that layout and returns positions t + M m.  Outputs as k_zinv's.
        const bool inb = L < C::ZP;
        auto store = [&](const Cx<P> *v, int f) {
            if (inb) {
                const Fld<P> o(md.bufA, (long long)f * N * C::ZP);
#pragma unroll
                for (int m = 0; m < E; m++) o.st((uint32_t)(t + M * m) * C::ZP + (uint32_t)L, v[m]);
            }
        };
        auto ddz = [&](Cx<P> *b, const Cx<P> *v) {
#pragma unroll
            for (int s = 0; s < E; s++) b[s] = mul_i(cscale(v[s], dk * (P)mode_of(Plan<N, E>::out_pos(t, s), N)));
        };
        Cx<P> b[E];
        ddz(b, a[0]);
        line_fft_T<P, N, E, T, +1>(b, lds, l, t, tw);
        store(b, 3);
        line_fft_T<P, N, E, T, +1>(a[0], lds, l, t, tw);
        store(a[0], 0);
        ddz(b, a[1]);
        line_fft_T<P, N, E, T, +1>(b, lds, l, t, tw);
        store(b, 4);
        line_fft_T<P, N, E, T, +1>(a[1], lds, l, t, tw);
        store(a[1], 1);
        line_fft_T<P, N, E, T, +1>(a[2], lds, l, t, tw);
        store(a[2], 2);
    }
    if (stage == 2) {
        __syncthreads();                     // LDS of the last transform is reused below
        const double es = block_sum<NT>(eacc, red);
        const double ds = block_sum<NT>(dacc, red);
        if (threadIdx.x == 0) {
            md.partials[2 * tile] = es;
            md.partials[2 * tile + 1] = ds;
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
template <typename P, int N, int EV, int TM = 1>
static hipError_t run_pencil(int pass, const MemberDev *mem, int count, int stage, const Cx<P> *tw, hipStream_t s) {
    using C = Cfg<P, N, EV, TM>;
    switch (pass) {
    case P_ZINV: k_zinv<P, N, EV, TM><<<dim3((C::ZP + C::T - 1) / C::T, count), C::NT, 0, s>>>(mem, tw); break;
    case P_YINV: k_yinv<P, N, EV, TM><<<dim3((C::NYL + C::T - 1) / C::T, count), C::NT, 0, s>>>(mem, tw); break;
    case P_XPASS: k_xpass<P, N, EV><<<dim3((unsigned)((long long)N * N / C::TX), count), 256, 0, s>>>(mem, tw, stage); break;
    case P_YFWD: k_yfwd<P, N, EV, TM><<<dim3((C::NYL + C::T - 1) / C::T, count), C::NT, 0, s>>>(mem, tw); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Persistent pipelined x pass: as many workgroups as stay resident on the
// device (occupancy times compute units), split evenly over the members.
template <typename P, int N, int EV>
static hipError_t run_xpass_dma(const MemberDev *mem, int count, int stage, const Cx<P> *tw, hipStream_t s) {
    using C = XCfg<P, N, EV>;
    static int resident = 0;                                   // workgroups per device (first call)
    if (resident == 0) {
        int dev = 0, cus = 0, occ = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_xpass_dma<P, N, EV>, C::NTH, 0);
        if (e != hipSuccess) return e;
        resident = (cus > 0 ? cus : 1) * (occ > 0 ? occ : 1);
    }
    int per = resident / (count > 0 ? count : 1);
    per = per < 1 ? 1 : (per > C::TILES ? C::TILES : per);
    k_xpass_dma<P, N, EV><<<dim3((unsigned)per, count), C::NTH, 0, s>>>(mem, tw, stage);
    return hipGetLastError();
}

// Wave-private x pass: one-wave workgroups, as many as stay resident,
// split evenly over the members.
template <typename P, int N, int EV>
static hipError_t run_xpass_wave(const MemberDev *mem, int count, int stage, const Cx<P> *tw, hipStream_t s) {
    using C = XWCfg<P, N, EV>;
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, cus = 0, occ = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_xpass_wave<P, N, EV>, 64, 0);
        if (e != hipSuccess) return e;
        resident = (cus > 0 ? cus : 1) * (occ > 0 ? occ : 1);
    }
    int per = resident / (count > 0 ? count : 1);
    per = per < 1 ? 1 : (per > C::TILES ? C::TILES : per);
    k_xpass_wave<P, N, EV><<<dim3((unsigned)per, count), 64, 0, s>>>(mem, tw, stage);
    return hipGetLastError();
}

template <typename P, int N, int EV>
static hipError_t run_xpass_wave2(const MemberDev *mem, int count, int stage, const Cx<P> *tw, hipStream_t s) {
    using C = XWCfg<P, N, EV>;
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, cus = 0, occ = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_xpass_wave2<P, N, EV>, 64, 0);
        if (e != hipSuccess) return e;
        resident = (cus > 0 ? cus : 1) * (occ > 0 ? occ : 1);
    }
    int per = resident / (count > 0 ? count : 1);
    per = per < 1 ? 1 : (per > C::TILES ? C::TILES : per);
    k_xpass_wave2<P, N, EV><<<dim3((unsigned)per, count), 64, 0, s>>>(mem, tw, stage);
    return hipGetLastError();
}

template <typename P, int N>
static hipError_t run_pass(int pass, int variant, const MemberDev *mem, int count, int stage, const void *tw, hipStream_t s) {
    using C = Cfg<P, N, 8>;
    const Cx<P> *twp = reinterpret_cast<const Cx<P> *>(tw);
    switch (pass) {
    case P_ZINV: case P_YINV: case P_XPASS: case P_YFWD:
        if (pass == P_XPASS && variant == 2) {
            if constexpr (N >= 64) return run_xpass_dma<P, N, 8>(mem, count, stage, twp, s);
            else return run_pencil<P, N, 8>(pass, mem, count, stage, twp, s);   // lines too short to stream
        }
        if (pass == P_XPASS && variant == 6) {
            // wave-private, pairs staged through two buffers: 16 (FP32) / 8 (FP64) values per thread
            constexpr int EA = sizeof(P) == 4 ? 16 : 8, CS = (int)sizeof(Cx<P>);
            if constexpr (N >= 64 && xwave_ok(N, EA, CS)) return run_xpass_wave2<P, N, EA>(mem, count, stage, twp, s);
            else if constexpr (N >= 64) return run_xpass_dma<P, N, 8>(mem, count, stage, twp, s);
            else return run_pencil<P, N, 8>(pass, mem, count, stage, twp, s);
        }
        if (pass == P_XPASS && (variant == 4 || variant == 5)) {
            // wave-private: 16 (FP32) / 8 (FP64) values per thread, or half that
            // (where that tile shape is invalid: the streamed x pass, variant 2)
            constexpr int EA = sizeof(P) == 4 ? 16 : 8, EB = EA / 2, CS = (int)sizeof(Cx<P>);
            if constexpr (N >= 64) {
                if constexpr (xwave_ok(N, EA, CS))
                    if (variant == 4) return run_xpass_wave<P, N, EA>(mem, count, stage, twp, s);
                if constexpr (xwave_ok(N, EB, CS))
                    if (variant == 5) return run_xpass_wave<P, N, EB>(mem, count, stage, twp, s);
                return run_xpass_dma<P, N, 8>(mem, count, stage, twp, s);
            } else return run_pencil<P, N, 8>(pass, mem, count, stage, twp, s);
        }
        if (pass == P_XPASS && variant == 3) {
            // streamed, 16 values per thread (one LDS exchange per 256-point
            // transform); FP32 only: FP64 would need more than 256 registers
            if constexpr (N >= 128 && N <= 512 && sizeof(P) == 4) return run_xpass_dma<P, N, 16>(mem, count, stage, twp, s);
            else if constexpr (N >= 64) return run_xpass_dma<P, N, 8>(mem, count, stage, twp, s);
            else return run_pencil<P, N, 8>(pass, mem, count, stage, twp, s);
        }
        if (pass != P_XPASS && variant == 2) return run_pencil<P, N, 8, 2>(pass, mem, count, stage, twp, s);
        if (pass != P_XPASS && variant == 3) return run_pencil<P, N, 16, 2>(pass, mem, count, stage, twp, s);
        return variant == 1 ? run_pencil<P, N, 16>(pass, mem, count, stage, twp, s)
                            : run_pencil<P, N, 8>(pass, mem, count, stage, twp, s);
    case P_ZFWD: {
        // variant 1: stages 0 and 1 also perform the next stage's z inverse;
        // variant 2 (internal, a step followed by another in the same call):
        // the last stage too, for the next step's first stage
        const dim3 grid((C::NZLS + C::TZ - 1) / C::TZ, count);
        if (stage == 0 && variant >= 1) k_zfwd_update<P, N, 0, true><<<grid, C::NTZ, 0, s>>>(mem, twp);
        else if (stage == 0) k_zfwd_update<P, N, 0><<<grid, C::NTZ, 0, s>>>(mem, twp);
        else if (stage == 1 && variant >= 1) k_zfwd_update<P, N, 1, true><<<grid, C::NTZ, 0, s>>>(mem, twp);
        else if (stage == 1) k_zfwd_update<P, N, 1><<<grid, C::NTZ, 0, s>>>(mem, twp);
        else if (variant == 2) k_zfwd_update<P, N, 2, true><<<grid, C::NTZ, 0, s>>>(mem, twp);
        else k_zfwd_update<P, N, 2><<<grid, C::NTZ, 0, s>>>(mem, twp);
        break;
    }
    case P_END:
        k_end_step<N><<<count, 256, 0, s>>>(mem, (C::NZLS + C::TZ - 1) / C::TZ);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename P>
static hipError_t dispatch_n(int n, int pass, int variant, const MemberDev *mem, int count, int stage, const void *tw, hipStream_t s) {
    switch (n) {
    case 16: return run_pass<P, 16>(pass, variant, mem, count, stage, tw, s);
    case 32: return run_pass<P, 32>(pass, variant, mem, count, stage, tw, s);
    case 64: return run_pass<P, 64>(pass, variant, mem, count, stage, tw, s);
    case 128: return run_pass<P, 128>(pass, variant, mem, count, stage, tw, s);
    case 256: return run_pass<P, 256>(pass, variant, mem, count, stage, tw, s);
    case 512: return run_pass<P, 512>(pass, variant, mem, count, stage, tw, s);
    case 1024:
        if constexpr (sizeof(P) == 4) return run_pass<P, 1024>(pass, variant, mem, count, stage, tw, s);
        else return hipErrorInvalidValue;                      // 1024^3 is FP32 only
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass(int pass, int variant, int n, int prec, const MemberDev *mem, int count, int stage,
                       const void *tw, hipStream_t s) {
    if (pass == P_BAND) {
        if (prec == ENS_FP32) k_band_energy<float><<<count, 256, 0, s>>>(mem, stage);
        else k_band_energy<double><<<count, 256, 0, s>>>(mem, stage);
        return hipGetLastError();
    }
    return prec == ENS_FP32 ? dispatch_n<float>(n, pass, variant, mem, count, stage, tw, s)
                            : dispatch_n<double>(n, pass, variant, mem, count, stage, tw, s);
}

int pass_variants(int pass) {
    if (pass == P_XPASS) return 7;
    if (pass == P_ZFWD) return 2;                               // 1: fused with the next stage's z inverse
                                                                // (2, internal: the last stage too)
    return (pass == P_ZINV || pass == P_YINV || pass == P_YFWD) ? 4 : 1;
}

int default_variant(int pass, int n, int prec) {
    if (pass == P_XPASS) return n >= 64 ? 2 : 0;               // streamed, 8 values per thread
    if (pass == P_ZINV || pass == P_YINV || pass == P_YFWD) return prec == ENS_FP32 ? 1 : 0;
    // fused z forward: 0.4-1.8 % faster per step up to n = 512 (both
    // precisions); at n = 1024 its registers spill and it gains nothing
    if (pass == P_ZFWD) return n <= 512 ? 1 : 0;
    return 0;
}

long long zfwd_blocks(int n, int prec) {
    auto blocks = [](auto cfg) { using C = decltype(cfg); return (long long)((C::NZLS + C::TZ - 1) / C::TZ); };
    const bool f = prec == ENS_FP32;
    switch (n) {
    case 16: return f ? blocks(Cfg<float, 16, 8>{}) : blocks(Cfg<double, 16, 8>{});
    case 32: return f ? blocks(Cfg<float, 32, 8>{}) : blocks(Cfg<double, 32, 8>{});
    case 64: return f ? blocks(Cfg<float, 64, 8>{}) : blocks(Cfg<double, 64, 8>{});
    case 128: return f ? blocks(Cfg<float, 128, 8>{}) : blocks(Cfg<double, 128, 8>{});
    case 256: return f ? blocks(Cfg<float, 256, 8>{}) : blocks(Cfg<double, 256, 8>{});
    case 512: return f ? blocks(Cfg<float, 512, 8>{}) : blocks(Cfg<double, 512, 8>{});
    case 1024: return blocks(Cfg<float, 1024, 8>{});
    default: return 0;
    }
}

}  // namespace ens
