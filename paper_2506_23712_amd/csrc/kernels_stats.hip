// kernels_stats.hip -- velocity-gradient statistics of a snapshot and the
// Gaussian-in-lambda ensemble mixture.
//
// Gradient transforms (K = N/3):
//   gzinv  : U_c = Z^-1[u_c], W_c = Z^-1[i k_z u_c]              -> bufA [6][N][NZL]
//   gyinv  : U_c, V_c = d_y u_c, W_c = d_z u_c (y physical)      -> bufB [9][N][N][K+1]
//   gxstats: A_c1 = X^-1[i k_x U_c], A_c2 = X^-1[V_c], A_c3 = X^-1[W_c] (c2r),
//            then per point in FP64: Q, R, eps, omega^2, histograms, moments.
#include <vector>

#include <mutex>
#include <type_traits>

#include "ens_internal.h"
#include "ens_lambda.h"
#include "fft.hpp"
#include "gmem.hpp"
#include <cmath>

namespace ens {

template <typename P> using L2 = LdsT<P>;

__device__ __forceinline__ int mode_of(int n, int N) { return n <= N / 2 ? n : n - N; }

template <typename P, int N, int EV> struct SCfg {
    static constexpr int K = N / 3;
    static constexpr int PX = kx_pitch(K, (int)sizeof(Cx<P>));   // x-mode pitch (whole 128-byte lines)
    static constexpr int NZL = (2 * K + 1) * PX;                  // z-lines of a pencil buffer
    static constexpr int NZLS = (2 * K + 1) * (K + 1);            // z-lines of the state
    static constexpr int ZP = state_pitch(K, (int)sizeof(Cx<P>));   // state plane pitch
    static constexpr int S = (2 * K + 1) * ZP;                      // state elements per component
    static constexpr int NYL = N * PX;
    static constexpr int E = EV > N ? N : EV, M = N / E;
    static constexpr int TL = 128 / (int)sizeof(Cx<P>);       // lines for 128-byte runs
    static constexpr int MAXT = E >= 16 ? 512 : 1024;
    static constexpr int T = N <= 256 ? (256 / M > TL ? 256 / M : TL) : (TL * M <= MAXT ? TL : MAXT / M);
    static constexpr int NT = T * M;
};

// values per thread of the gradient pencil passes
template <typename P> constexpr int grad_e() { return sizeof(P) == 4 ? 16 : 8; }

template <typename P, int N, int E>
__device__ __forceinline__ void gload_trunc(Cx<P> *v, const Fld<P> &f, uint32_t base, uint32_t stride, int t, bool valid) {
    constexpr int K = N / 3, M = N / E;
#pragma unroll
    for (int m = 0; m < E; m++) {
        const int mm = mode_of(t + M * m, N);
        const bool keep = valid && mm >= -K && mm <= K;
        v[m] = keep ? f.ld(base + (uint32_t)(mm >= 0 ? mm : mm + 2 * K + 1) * stride) : czero<P>();
    }
}

// ------------------------------------------------------------------ gzinv
// in u_hat [3][2K+1][ZP]; out bufA [6][N][NZL]: U_c = Z^-1[u_c] (fields
// 0..2), W_c = Z^-1[i k_z u_c] (3..5); pad lines (kx > K) carry zeros
template <typename P, int N>
__global__ void __launch_bounds__((SCfg<P, N, grad_e<P>()>::NT)) k_gzinv(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ twg) {
    using C = SCfg<P, N, grad_e<P>()>;
    constexpr int E = C::E, M = C::M, T = C::T, NZL = C::NZL;
    __shared__ LdsT<P> lds[N * T];
    __shared__ Cx<P> tw[twiddle_span(N, E)];               // twiddles in LDS: no global load inside the transforms
    for (int i = (int)threadIdx.x; i < twiddle_span(N, E); i += (int)blockDim.x) tw[i] = twg[i];
    unsigned tile, mem_i;
    xcd_tile(tile, mem_i);
    const MemberDev &md = mems[mem_i];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    const int L = tile * T + l;
    const bool inb = L < NZL;
    const int kx = L % C::PX, iy = L / C::PX;
    const bool valid = inb && kx <= C::K;
    const uint32_t Ls = valid ? (uint32_t)(iy * (C::K + 1) + kx) : 0u;   // the line in the state
    const P dk = (P)md.dk;
    auto store = [&](const Cx<P> *v, int f) {
        if (inb) {
            const Fld<P> o(md.bufA, (long long)f * N * NZL);
#pragma unroll
            for (int s = 0; s < E; s++) o.st((uint32_t)Plan<N, E>::out_pos(t, s) * NZL + L, v[s]);
        }
    };
    Cx<P> a[E], b[E], p[E];
    gload_trunc<P, N, E>(a, Fld<P>(md.uh, 0), Ls, C::ZP, t, valid);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (c < 2) gload_trunc<P, N, E>(p, Fld<P>(md.uh, (long long)(c + 1) * C::S), Ls, C::ZP, t, valid);
#pragma unroll
        for (int m = 0; m < E; m++) b[m] = mul_i(cscale(a[m], dk * (P)mode_of(t + M * m, N)));
        line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
        store(b, 3 + c);
        line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
        store(a, c);
        if (c < 2) {
#pragma unroll
            for (int m = 0; m < E; m++) a[m] = p[m];
        }
    }
}

// ------------------------------------------------------------------ gyinv
// out bufB [9][N][N][PX]: U_c (0..2), V_c = d_y u_c (3..5), W_c = d_z u_c (6..8)
template <typename P, int N>
__global__ void __launch_bounds__((SCfg<P, N, grad_e<P>()>::NT)) k_gyinv(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ twg) {
    using C = SCfg<P, N, grad_e<P>()>;
    constexpr int E = C::E, M = C::M, T = C::T, K = C::K, NZL = C::NZL;
    __shared__ LdsT<P> lds[N * T];
    __shared__ Cx<P> tw[twiddle_span(N, E)];               // twiddles in LDS: no global load inside the transforms
    for (int i = (int)threadIdx.x; i < twiddle_span(N, E); i += (int)blockDim.x) tw[i] = twg[i];
    unsigned tile, mem_i;
    xcd_tile(tile, mem_i);
    const MemberDev &md = mems[mem_i];
    const int l = threadIdx.x % T, t = threadIdx.x / T;
    constexpr int PX = C::PX;
    const int L = tile * T + l;
    const bool inb = L < C::NYL;
    const int z = inb ? L / PX : 0;
    const int kx = inb ? L % PX : 0;
    const bool valid = inb && kx <= K;
    const P dk = (P)md.dk;
    const uint32_t in_base = (uint32_t)z * NZL + kx;
    const uint32_t out_base = (uint32_t)z * N * PX + kx;
    auto load = [&](Cx<P> *v, int f) {
        gload_trunc<P, N, E>(v, Fld<P>(md.bufA, (long long)f * N * NZL), in_base, PX, t, valid);
    };
    auto store = [&](const Cx<P> *v, int f) {
        if (inb) {
            const Fld<P> o(md.bufB, (long long)f * N * N * PX);
#pragma unroll
            for (int s = 0; s < E; s++) o.st(out_base + (uint32_t)Plan<N, E>::out_pos(t, s) * PX, v[s]);
        }
    };
    Cx<P> a[E], b[E], p[E];
    load(a, 0);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        load(p, 3 + c);                                        // prefetch W_c
#pragma unroll
        for (int m = 0; m < E; m++) b[m] = mul_i(cscale(a[m], dk * (P)mode_of(t + M * m, N)));
        line_fft<P, N, E, T, +1>(b, lds, l, t, tw);
        store(b, 3 + c);
        line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
        store(a, c);
#pragma unroll
        for (int m = 0; m < E; m++) a[m] = p[m];
        if (c < 2) load(p, c + 1);                             // prefetch U_(c+1)
        line_fft<P, N, E, T, +1>(a, lds, l, t, tw);
        store(a, 6 + c);
        if (c < 2) {
#pragma unroll
            for (int m = 0; m < E; m++) a[m] = p[m];
        }
    }
}

// ----------------------------------------------------------------- gxstats
struct HistArgs {
    int qb, lb, ab;
    long long off_le, off_lw, off_al, off_at;
    double q_lo, q_scale, r_lo, r_scale, l_lo, l_scale, a_lo, a_scale;
    double tau, inv_trs, inv_trs15, inv_eps_ref, om_scale;
    int win0, win;             // QR bins [win0, win0 + win)^2 are counted in LDS, the rest globally
    int tiles_per_block;
    const double *ledge;       // lb + 1 edges 10^(l_lo + b / l_scale) of the log histograms (FP64)
    float l2s, loff;           // log10(2) l_scale and l_lo l_scale: bin estimate from log2
};

// -1 under, -2 over, -3 nan, else bin
__device__ __forceinline__ int bin_of(double x, double lo, double scale, int nb) {
    if (x != x) return -3;
    if (x < lo) return -1;
    const double b = floor((x - lo) * scale);
    if (b >= (double)nb) return -2;
    return (int)b;
}
// Bin of log10(x) for x > 0 with the decision taken in FP64 against the edge
// table: an FP32 estimate from the exponent and the hardware log2 of the
// mantissa is within a small fraction of a bin, so one comparison with each
// neighbouring edge gives floor((log10 x - lo) scale) except for x within
// rounding of an edge.  Replaces the FP64 log10 (about 80 instructions).
__device__ __forceinline__ int log_bin(double x, const double *edge, int nb, float l2s, float loff) {
    if (x < edge[0]) return -1;
    if (x >= edge[nb]) return -2;
    int e;
    const double m = frexp(x, &e);                       // x = m 2^e, m in [0.5, 1)
    const float l2 = (float)e + __log2f((float)m);
    int c = (int)floorf(l2 * l2s - loff);
    c = c < 0 ? 0 : (c > nb - 1 ? nb - 1 : c);
    if (x < edge[c]) c--;
    else if (x >= edge[c + 1]) c++;
    return c;
}
__device__ __forceinline__ int slot_1d(int b, int nb) { return b >= 0 ? b : (b == -1 ? nb : (b == -2 ? nb + 1 : nb + 2)); }
// slot_1d(bin_of(x, lo, scale, nb), nb) with fewer operations: the same FP64
// value (x - lo) scale decides the bin (truncation is floor on [0, nb))
__device__ __forceinline__ int slot_of(double x, double lo, double scale, int nb) {
    const double d = (x - lo) * scale;
    const int b = d >= (double)nb ? nb + 1 : (int)d;
    return x < lo ? nb : (d == d ? b : nb + 2);
}

// Replicated hot bins of the statistics pass: copies per bin and central bins
// of each 1-D histogram; copies per bin and central bins per axis of the QR
// histogram.
constexpr int kHotCopies1 = 8, kHotBins1 = 64, kHotCopiesQ = 8, kHotBinsQ = 16;
constexpr size_t kHotBytes = (4 * (size_t)kHotBins1 * kHotCopies1 + (size_t)kHotBinsQ * kHotBinsQ * kHotCopiesQ) * 4;

// Persistent x pass of the gradient fields: each workgroup takes row tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...; per-point values are formed in FP64;
// 1-D histograms and a central window of the QR histogram are accumulated in
// LDS (32-bit) and flushed once; moments stay in registers and are reduced
// in a fixed order to one partial per workgroup.  The register budget is
// capped at 256 so that two workgroups share a compute unit (one leaves each
// SIMD a single wave, which stalls on every dependent FP64 operation).
template <typename P, int N, int EX>
__global__ void __launch_bounds__(256, 2) k_gxstats(const MemberDev *__restrict__ mems, const Cx<P> *__restrict__ twg, HistArgs h) {
    constexpr int E = EX, M = N / E, T = 256 / M, K = N / 3;
    constexpr int PX = kx_pitch(K, (int)sizeof(Cx<P>));
    constexpr long long FS = (long long)N * N * PX;
    extern __shared__ double dyn[];                         // log edges, 1-D histograms, QR window
    double *ledge = dyn;
    unsigned int *hs = (unsigned int *)(dyn + h.lb + 1);
    __shared__ LdsT<P> lds[N * T];
    __shared__ Cx<P> tw[twiddle_span(N, E)];               // twiddles in LDS: no global load inside the transforms
    for (int i = (int)threadIdx.x; i < twiddle_span(N, E); i += (int)blockDim.x) tw[i] = twg[i];
    __shared__ double red[4][32];
    // Hot bins are replicated: the central CW bins of each 1-D histogram get
    // NC copies and the central CQ x CQ bins of the QR histogram NQ copies,
    // one per lane group (lane mod NC or NQ), so that lanes of a wavefront
    // landing in the same bin collide on one word at most 64/NC (64/NQ) ways.
    // The copies of a bin are adjacent words, i.e. in different LDS banks, so
    // that the groups hitting one hot bin do not queue on one bank.  Copies
    // are merged before the flush.
    constexpr int NC = kHotCopies1, CW = kHotBins1, NQ = kHotCopiesQ, CQ = kHotBinsQ;
    __shared__ unsigned int cen1[4][CW][NC];                // log eps, log Omega, A_L, A_T
    __shared__ unsigned int cenq[CQ * CQ][NQ];
    // QR points outside the axes and NaN points: one LDS counter each, flushed
    // once (a developed field sends whole members' points there, which as
    // global atomics on one address serialise)
    __shared__ unsigned int qspec[3];
    const MemberDev &md = mems[blockIdx.y];
    // Where a row's M threads fit one wave (N <= 256), the threads of a row are
    // consecutive lanes and the transforms exchange through wave-private LDS
    // rows (WaveLay) with no workgroup barrier; longer rows span waves and use
    // the [position][row] layout with barriers.
    constexpr bool WP = M <= 64 && 64 % M == 0;
    using LY = typename std::conditional<WP, WaveLay<P, N>, RowLay<P, T>>::type;
    const int l = WP ? (int)threadIdx.x / M : (int)threadIdx.x % T;
    const int t = WP ? (int)threadIdx.x % M : (int)threadIdx.x / T;
    const int grp = threadIdx.x & (NC - 1), grq = threadIdx.x & (NQ - 1);
    const P dk = (P)md.dk;
    const int n1d = 2 * (h.lb + 3) + 2 * (h.ab + 3);
    const int nwin = h.win * h.win;
    for (int i = threadIdx.x; i < n1d + nwin; i += 256) hs[i] = 0u;
    for (int i = threadIdx.x; i <= h.lb; i += 256) ledge[i] = h.ledge[i];
    for (int i = threadIdx.x; i < 4 * NC * CW; i += 256) (&cen1[0][0][0])[i] = 0u;
    for (int i = threadIdx.x; i < NQ * CQ * CQ; i += 256) (&cenq[0][0])[i] = 0u;
    if (threadIdx.x < 3) qspec[threadIdx.x] = 0u;
    unsigned int *h_le = hs, *h_lw = hs + (h.lb + 3), *h_al = hs + 2 * (h.lb + 3), *h_at = h_al + (h.ab + 3);
    unsigned int *h_qr = hs + n1d;
    unsigned long long *G = md.counts;
    // first bin of each replicated window (clamped inside the real bins; -1 = none)
    auto c0_of = [](double centre_bin, int nb, int w) -> int {
        if (nb < w) return -1;
        int c = (int)floor(centre_bin) - w / 2;
        return c < 0 ? 0 : (c > nb - w ? nb - w : c);
    };
    int c0[4];
    c0[0] = c0_of((log10(md.eps_m * h.inv_eps_ref) - h.l_lo) * h.l_scale, h.lb, CW);
    c0[1] = c0_of((log10(md.eps_m / md.nu * h.om_scale) - h.l_lo) * h.l_scale, h.lb, CW);
    c0[2] = c0_of((0.0 - h.a_lo) * h.a_scale, h.ab, CW);
    c0[3] = c0[2];
    if (!(md.eps_m > 0.0) || !(md.nu > 0.0)) { c0[0] = -1; c0[1] = -1; }
    const int q0 = c0_of((0.0 - h.q_lo) * h.q_scale, h.qb, CQ), r0 = c0_of((0.0 - h.r_lo) * h.r_scale, h.qb, CQ);
    // first bins of the replicated QR centre, far above every bin where there is none
    const int cq0 = q0 >= 0 && r0 >= 0 ? q0 : (1 << 30), cr0 = q0 >= 0 && r0 >= 0 ? r0 : (1 << 30);
    unsigned int *single[4] = {h_le, h_lw, h_al, h_at};
    // one LDS atomic per sample on the selected counter (a replicated hot bin
    // or the plain bin): lanes of one wave that differ in the choice do not
    // split into two atomic instructions
    // (a histogram without a replicated window gets a first bin far above
    // every slot, so that one unsigned comparison decides)
    int cw0[4];
#pragma unroll
    for (int i = 0; i < 4; i++) cw0[i] = c0[i] >= 0 ? c0[i] : (1 << 30);
    auto add1 = [&](int hist, int slot) {
        const unsigned rel = (unsigned)(slot - cw0[hist]);
        const bool hot = rel < (unsigned)CW;
        unsigned int *p = hot ? &cen1[hist][hot ? rel : 0][grp] : &single[hist][slot];
        atomicAdd(p, 1u);
    };
    double mom[26];
#pragma unroll
    for (int i = 0; i < 26; i++) mom[i] = 0.0;
    const double nu = md.nu;
    const int ntiles = N * N / T;
    __syncthreads();
    // Gradient spectra, field f = 3 c + j: j = 0 i k_x u_c (from u_c, fields 0-2
    // of bufB), j = 1 d_y u_c (fields 3-5), j = 2 d_z u_c (fields 6-8).  The raw
    // row entries of a field pair are loaded one pair ahead of their use (the
    // next tile's first pair during this tile's last transform and the
    // pointwise work), so that the loads are in flight behind the arithmetic.
    auto foff = [](int f) -> long long { return (long long)((f % 3 == 0 ? 0 : (f % 3 == 1 ? 3 : 6)) + f / 3) * FS; };
    auto load_pair = [&](int tile, int pr, Cx<P> (&ra)[E], Cx<P> (&rb)[E]) {
        const uint32_t rbase = (uint32_t)(tile * T + l) * PX;
        const int fa = 2 * pr, fb = 2 * pr + 1;
        const Fld<P> Fa(md.bufB, foff(fa)), Fb(md.bufB, fb < 9 ? foff(fb) : 0);
#pragma unroll
        for (int m = 0; m < E; m++) {
            const int n = t + M * m;
            const bool lo = n <= K, hi = n >= N - K;
            const uint32_t kx = (uint32_t)(lo ? n : N - n);
            ra[m] = czero<P>();
            rb[m] = czero<P>();
            if (lo || hi) {
                ra[m] = Fa.ld(rbase + kx);
                if (fb < 9) rb[m] = Fb.ld(rbase + kx);
            }
        }
    };
    // FP32 only: in FP64 the second pair of registers would spill
    constexpr bool PF = sizeof(P) == 4;
    Cx<P> ra[E], rb[E];
    if (PF && (int)blockIdx.x < ntiles) load_pair(blockIdx.x, 0, ra, rb);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        P g[9][E];
        Cx<P> v[E];
#pragma unroll
        for (int pr = 0; pr < 5; pr++) {
            const int fa = 2 * pr, fb = 2 * pr + 1;
            if constexpr (PF) {
                Cx<P> ca[E], cb[E];
#pragma unroll
                for (int m = 0; m < E; m++) { ca[m] = ra[m]; cb[m] = rb[m]; }
                if (pr < 4) load_pair(tile, pr + 1, ra, rb);
                else if (tile + (int)gridDim.x < ntiles) load_pair(tile + gridDim.x, 0, ra, rb);
#pragma unroll
                for (int m = 0; m < E; m++) {
                    const int n = t + M * m;
                    const bool lo = n <= K, hi = n >= N - K;
                    const P kx = (P)(lo ? n : N - n);
                    Cx<P> A = ca[m], B = cb[m];
                    if (fa % 3 == 0) A = mul_i(cscale(A, dk * kx));
                    if (fb < 9 && fb % 3 == 0) B = mul_i(cscale(B, dk * kx));
                    if (hi && !lo) { A = cconj(A); B = cconj(B); }
                    if (n == 0) { A.im = P(0); B.im = P(0); }
                    v[m] = {A.re - B.im, A.im + B.re};
                }
            } else {
                const uint32_t rbase = (uint32_t)(tile * T + l) * PX;
                auto spec = [&](int f, uint32_t kx) -> Cx<P> {
                    const Cx<P> x = Fld<P>(md.bufB, foff(f)).ld(rbase + kx);
                    return f % 3 == 0 ? mul_i(cscale(x, dk * (P)kx)) : x;
                };
#pragma unroll
                for (int m = 0; m < E; m++) {
                    const int n = t + M * m;
                    Cx<P> A = czero<P>(), B = czero<P>();
                    if (n <= K) { A = spec(fa, n); if (fb < 9) B = spec(fb, n); }
                    else if (n >= N - K) { A = cconj(spec(fa, N - n)); if (fb < 9) B = cconj(spec(fb, N - n)); }
                    if (n == 0) { A.im = P(0); B.im = P(0); }
                    v[m] = {A.re - B.im, A.im + B.re};
                }
            }
            line_fft<P, N, E, T, +1, WP ? 2 : 0, LY>(v, lds, l, t, tw);
#pragma unroll
            for (int s = 0; s < E; s++) { g[fa][s] = v[s].re; if (fb < 9) g[fb][s] = v[s].im; }
        }
#pragma unroll
        for (int s = 0; s < E; s++) {
            double a[3][3];
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) a[i][j] = (double)g[3 * i + j][s];
            const double tr = a[0][0] + a[1][1] + a[2][2];
            // Q = -tr(A^2)/2 and R = -tr(A^3)/3 from the rows of A^2
            double q = 0.0, r = 0.0;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    const double b = a[i][0] * a[0][k] + a[i][1] * a[1][k] + a[i][2] * a[2][k];
                    if (i == k) q += b;
                    r += b * a[k][i];
                }
            q *= -0.5; r *= -1.0 / 3.0;
            // S_ij S_ij: diagonal squares plus twice each off-diagonal pair
            const double s01 = a[0][1] + a[1][0], s02 = a[0][2] + a[2][0], s12 = a[1][2] + a[2][1];
            const double ss = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2] +
                              0.5 * (s01 * s01 + s02 * s02 + s12 * s12);
            const double w0 = a[2][1] - a[1][2], w1 = a[0][2] - a[2][0], w2 = a[1][0] - a[0][1];
            const double ens = w0 * w0 + w1 * w1 + w2 * w2;
            const double qs = q * h.inv_trs, rs = r * h.inv_trs15;
            const double es = 2.0 * nu * ss * h.inv_eps_ref, ws = ens * h.om_scale;
            {   // QR: replicated centre, the LDS window, the LDS outside/NaN
                // counters (one LDS atomic on the selected counter), else global
                // the bins of bin_of: in range iff !(x < lo) and (x - lo) scale < nb
                const bool nan = qs != qs || rs != rs;
                const double dq = (qs - h.q_lo) * h.q_scale, dr = (rs - h.r_lo) * h.r_scale;
                const bool inq = !(qs < h.q_lo) && dq < (double)h.qb, inr = !(rs < h.r_lo) && dr < (double)h.qb;
                const int bq = inq ? (int)dq : 0, br = inr ? (int)dr : 0;
                const bool out = !nan && !(inq && inr);
                const bool cen = !nan && !out && (unsigned)(bq - cq0) < (unsigned)CQ && (unsigned)(br - cr0) < (unsigned)CQ;
                const bool win = !nan && !out && !cen && (unsigned)(bq - h.win0) < (unsigned)h.win &&
                                 (unsigned)(br - h.win0) < (unsigned)h.win;
                if (nan || out || cen || win) {
                    unsigned int *p = nan ? &qspec[2]
                                    : out ? &qspec[0]
                                    : cen ? &cenq[(bq - q0) * CQ + (br - r0)][grq]
                                          : &h_qr[(bq - h.win0) * h.win + (br - h.win0)];
                    atomicAdd(p, 1u);
                } else {
                    atomicAdd(&G[bq * h.qb + br], 1ull);
                }
            }
            add1(0, slot_1d(es > 0.0 ? log_bin(es, ledge, h.lb, h.l2s, h.loff) : (es != es ? -3 : -1), h.lb));
            add1(1, slot_1d(ws > 0.0 ? log_bin(ws, ledge, h.lb, h.l2s, h.loff) : (ws != ws ? -3 : -1), h.lb));
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    const double x = a[i][j] * h.tau;
                    add1(i == j ? 2 : 3, slot_of(x, h.a_lo, h.a_scale, h.ab));
                    // x .. x^6 from x^2 and x^4, the odd powers fused into the sums
                    double *mo = mom + (i == j ? 0 : 6);
                    const double x2 = x * x, x4 = x2 * x2;
                    mo[0] += x; mo[1] += x2; mo[2] = fma(x2, x, mo[2]);
                    mo[3] += x4; mo[4] = fma(x4, x, mo[4]); mo[5] = fma(x4, x2, mo[5]);
                }
            {
                const double e2 = es * es, w2 = ws * ws;
                mom[12] += es; mom[13] += e2; mom[14] = fma(e2, es, mom[14]); mom[15] = fma(e2, e2, mom[15]);
                mom[16] += ws; mom[17] += w2; mom[18] = fma(w2, ws, mom[18]); mom[19] = fma(w2, w2, mom[19]);
            }
            mom[20] += qs; mom[21] += rs;
            mom[22] += ss * h.tau * h.tau;
            mom[23] += tr * tr * h.tau * h.tau;
            mom[24] += qs * qs; mom[25] += rs * rs;
        }
    }
    // merge the replicated 1-D windows into the single-copy histograms
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * CW; i += 256) {
        const int hh = i / CW, rel = i % CW;
        if (c0[hh] < 0) continue;
        unsigned int sum = 0;
#pragma unroll
        for (int c = 0; c < NC; c++) sum += cen1[hh][rel][c];
        single[hh][c0[hh] + rel] += sum;
    }
    for (int i = threadIdx.x; i < CQ * CQ; i += 256) {
        unsigned int sum = 0;
#pragma unroll
        for (int c = 0; c < NQ; c++) sum += cenq[i][c];
        if (sum) atomicAdd(&G[(long long)(q0 + i / CQ) * h.qb + (r0 + i % CQ)], (unsigned long long)sum);
    }
    if (threadIdx.x < 3 && qspec[threadIdx.x])
        atomicAdd(&G[(long long)h.qb * h.qb + threadIdx.x], (unsigned long long)qspec[threadIdx.x]);
    // deterministic reduction of the moments: wave butterfly, then waves in order
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 26; i++) {
        double x = mom[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[wave][i] = x;
    }
    __syncthreads();
    const long long pbase = ((long long)blockIdx.x) * 32;  // (the flush below is after a barrier)
    if (threadIdx.x < 32) {
        double x = 0.0;
        if (threadIdx.x < 26) x = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
        md.partials[pbase + threadIdx.x] = x;
    }
    // flush LDS histograms (non-zero bins only)
    for (int i = threadIdx.x; i < n1d + nwin; i += 256) {
        const unsigned int c = hs[i];
        if (!c) continue;
        long long gi;
        if (i < h.lb + 3) gi = h.off_le + i;
        else if (i < 2 * (h.lb + 3)) gi = h.off_lw + (i - (h.lb + 3));
        else if (i < 2 * (h.lb + 3) + h.ab + 3) gi = h.off_al + (i - 2 * (h.lb + 3));
        else if (i < n1d) gi = h.off_at + (i - 2 * (h.lb + 3) - (h.ab + 3));
        else {
            const int w = i - n1d;
            gi = (long long)(h.win0 + w / h.win) * h.qb + (h.win0 + w % h.win);
        }
        atomicAdd(&G[gi], (unsigned long long)c);
    }
}

// one workgroup per member: moments += sum over blocks (fixed order)
__global__ void __launch_bounds__(256) k_stats_reduce(const MemberDev *__restrict__ mems, long long nblocks) {
    __shared__ double red[256];
    const MemberDev &md = mems[blockIdx.x];
    for (int i = 0; i < 26; i++) {
        double x = 0.0;
        for (long long b = threadIdx.x; b < nblocks; b += 256) x += md.partials[b * 32 + i];
        red[threadIdx.x] = x;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) md.moments[i] += red[0];
        __syncthreads();
    }
    // snapshot sums of the member's energy and dissipation (its last step's
    // values, those of the field this snapshot sees) and the snapshot count
    if (threadIdx.x == 0) {
        md.moments[26] += md.st->diag.E;
        md.moments[27] += md.st->diag.D;
        md.moments[28] += 1.0;
    }
}

// Workgroups per member of the persistent statistics pass: about 2048 in
// total over the launch, at most one per row tile.
static int xstats_grid(int n, int count) {
    const int tiles = n * n / (256 / (n / 4));
    int per = (2048 + count - 1) / count;
    if (per > tiles) per = tiles;
    if (per > 512) per = 512;
    return per < 1 ? 1 : per;
}

// ---------------------------------------------------------------- launchers
// values per thread of the statistics x pass: 4 (with 8 the nine gradient
// rows, the FP64 point values and the 26 FP64 moment sums spill hundreds of
// bytes per lane at the two-workgroup register budget)
template <typename P, int N> constexpr int xstats_e() { return 4; }

template <typename P, int N>
static hipError_t stats_pass(int pass, const MemberDev *mem, int count, const ens_hist_desc *hd, const double *ledge,
                             const void *tw, hipStream_t s) {
    using C = SCfg<P, N, grad_e<P>()>;
    const Cx<P> *twp = reinterpret_cast<const Cx<P> *>(tw);
    if (pass == 0) {
        k_gzinv<P, N><<<dim3((C::NZL + C::T - 1) / C::T, count), C::NT, 0, s>>>(mem, twp);
    } else if (pass == 1) {
        k_gyinv<P, N><<<dim3((C::NYL + C::T - 1) / C::T, count), C::NT, 0, s>>>(mem, twp);
    } else if (pass == 2) {
        const ens_hist_desc &d = *hd;
        HistArgs h;
        const HistGeom g = make_hist_geom(d);
        h.qb = d.qr_bins; h.lb = d.log_bins; h.ab = d.a_bins;
        h.off_le = g.off_le; h.off_lw = g.off_lw; h.off_al = g.off_al; h.off_at = g.off_at;
        h.q_lo = d.q_lo; h.q_scale = (double)d.qr_bins / (d.q_hi - d.q_lo);
        h.r_lo = d.r_lo; h.r_scale = (double)d.qr_bins / (d.r_hi - d.r_lo);
        h.l_lo = d.log10_lo; h.l_scale = (double)d.log_bins / (d.log10_hi - d.log10_lo);
        h.a_lo = d.a_lo; h.a_scale = (double)d.a_bins / (d.a_hi - d.a_lo);
        h.tau = sqrt(d.nu_ref / d.eps_ref);
        const double trs = d.eps_ref / (2.0 * d.nu_ref);
        h.inv_trs = 1.0 / trs;
        h.inv_trs15 = 1.0 / pow(trs, 1.5);
        h.inv_eps_ref = 1.0 / d.eps_ref;
        h.om_scale = d.nu_ref / d.eps_ref;
        h.ledge = ledge;
        h.l2s = (float)(0.30102999566398119521 * h.l_scale);
        h.loff = (float)(h.l_lo * h.l_scale);
        // LDS: transform tile + reduction (static) + log edges, 1-D histograms, QR window (dynamic) <= 64 KiB
        constexpr int EX = xstats_e<P, N>(), T = 256 / (N / EX);
        const size_t stat = (size_t)N * T * sizeof(LdsT<P>) + 4 * 32 * sizeof(double) + kHotBytes + 16 +
                            (size_t)twiddle_span(N, EX) * sizeof(Cx<P>);
        const size_t n1d = 2 * (size_t)(h.lb + 3) + 2 * (size_t)(h.ab + 3);
        const size_t budget = 65536 - stat - 512;
        const size_t fixed = n1d * 4 + (size_t)(h.lb + 1) * 8;
        if (fixed > budget || !ledge) return hipErrorInvalidValue;   // rejected on the host beforehand
        int win = (int)std::sqrt((double)((budget - fixed) / 4));
        if (win > h.qb) win = h.qb;
        h.win = win;
        h.win0 = (h.qb - win) / 2;
        const size_t dyn = (size_t)(h.lb + 1) * 8 + (n1d + (size_t)win * win) * 4;
        const int per = xstats_grid(N, count);
        k_gxstats<P, N, EX><<<dim3(per, count), 256, dyn, s>>>(mem, twp, h);
    } else {
        k_stats_reduce<<<count, 256, 0, s>>>(mem, (long long)xstats_grid(N, count));
    }
    return hipGetLastError();
}

template <typename P>
static hipError_t stats_n(int n, int pass, const MemberDev *mem, int count, const ens_hist_desc *hd, const double *le,
                          const void *tw, hipStream_t s) {
    switch (n) {
    case 16: return stats_pass<P, 16>(pass, mem, count, hd, le, tw, s);
    case 32: return stats_pass<P, 32>(pass, mem, count, hd, le, tw, s);
    case 64: return stats_pass<P, 64>(pass, mem, count, hd, le, tw, s);
    case 128: return stats_pass<P, 128>(pass, mem, count, hd, le, tw, s);
    case 256: return stats_pass<P, 256>(pass, mem, count, hd, le, tw, s);
    case 512: return stats_pass<P, 512>(pass, mem, count, hd, le, tw, s);
    case 1024:
        if constexpr (sizeof(P) == 4) return stats_pass<P, 1024>(pass, mem, count, hd, le, tw, s);
        else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}
static hipError_t stats_dispatch(int n, int prec, int pass, const MemberDev *mem, int count, const ens_hist_desc *hd, const double *le,
                                 const void *tw, hipStream_t s) {
    return prec == ENS_FP32 ? stats_n<float>(n, pass, mem, count, hd, le, tw, s) : stats_n<double>(n, pass, mem, count, hd, le, tw, s);
}

hipError_t launch_grad_zinv(int n, int prec, const MemberDev *mem, int count, const void *tw, hipStream_t s) {
    return stats_dispatch(n, prec, 0, mem, count, nullptr, nullptr, tw, s);
}
hipError_t launch_grad_yinv(int n, int prec, const MemberDev *mem, int count, const void *tw, hipStream_t s) {
    return stats_dispatch(n, prec, 1, mem, count, nullptr, nullptr, tw, s);
}
hipError_t launch_grad_xstats(int n, int prec, const MemberDev *mem, int count, const ens_hist_desc &h, const double *ledge,
                              const void *tw, hipStream_t s) {
    return stats_dispatch(n, prec, 2, mem, count, &h, ledge, tw, s);
}
hipError_t launch_stats_reduce(int n, int prec, const MemberDev *mem, int count, hipStream_t s) {
    return stats_dispatch(n, prec, 3, mem, count, nullptr, nullptr, nullptr, s);
}
// upper bound of workgroup partials per member (the grid depends on the batch)
long long xstats_blocks(int /*n*/) { return 512; }
bool stats_hist_fits(const ens_hist_desc &h) {
    const size_t n1d = 2 * (size_t)(h.log_bins + 3) + 2 * (size_t)(h.a_bins + 3);
    return n1d * 4 + (size_t)(h.log_bins + 1) * 8 <= 65536 - kHotBytes - 4 * 32 * 8 - 16384 - 512 - 4096;
}

// =================================================================== mixture
struct MixIn {
    const unsigned long long *counts;
    const double *moments;
    double lambda;
    double ntot;      // samples per histogram (written by k_mix_prep)
    double w;         // weight (written by k_mix_weights)
    int order;        // member index at sorted rank (written by k_mix_weights)
    int pad;
};

struct MixTable {
    const double *p;  // tabulated lambda density (mode 4), M samples
    int M;
    double lam0, h;
};

__global__ void __launch_bounds__(256) k_mix_prep(MixIn *mi, long long nqr) {
    __shared__ unsigned long long red[256];
    unsigned long long s = 0;
    const unsigned long long *c = mi[blockIdx.x].counts;
    for (long long i = threadIdx.x; i < nqr; i += 256) s += c[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) mi[blockIdx.x].ntot = (double)red[0];
}

// normal mass of [a, b) with erfc tails
__device__ double nmass(double a, double b, double mu, double sig) {
    const double r = 1.0 / (sig * sqrt(2.0));
    auto upper = [&](double x) { return isinf(x) && x > 0 ? 0.0 : 0.5 * erfc((x - mu) * r); };
    auto lower = [&](double x) { return isinf(x) && x < 0 ? 0.0 : 0.5 * erfc((mu - x) * r); };
    if (a >= mu) return upper(a) - upper(b);
    if (b <= mu) return lower(b) - lower(a);
    return 1.0 - lower(a) - upper(b);
}

constexpr int kMaxMix = 1023;
static_assert(kMaxMix == ENS_MIX_STATIC_MAX, "the static mixture table holds the largest mixture");

// Mean of the truncated Gaussian in lambda (support lambda <= Z, variance
// 9cZ, eq. truncated_gaussian) that satisfies the mean-injection constraint.
// For a normal of mean mu cut at Z, ln int P e^lambda =
//   mu + s2/2 + ln Phi((Z - mu - s2)/s) - ln Phi((Z - mu)/s),
// increasing in mu, negative at mu = -s2/2 (the uncut root), tending to Z
// for large mu: bracketed by doubling steps, then bisected to the last bit.
static double truncated_mean(double c, double Z) {
    const double s = std::sqrt(9.0 * c * Z), s2 = s * s;
    auto lnPhi = [](double x) { return std::log(0.5 * std::erfc(-x / std::sqrt(2.0))); };
    auto g = [&](double mu) { return mu + 0.5 * s2 + lnPhi((Z - mu - s2) / s) - lnPhi((Z - mu) / s); };
    double lo = -0.5 * s2, step = std::max(s, 1e-3), hi = lo + step;
    while (g(hi) <= 0.0) { lo = hi; step *= 2.0; hi = lo + step; }
    for (int it = 0; it < 400; it++) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        (g(mid) > 0.0 ? hi : lo) = mid;
    }
    return 0.5 * (lo + hi);
}

// Integral over [a, b) of a tabulated lambda density: samples p_j at
// lam0 + j h (negative samples read as zero), linear in between, zero outside.
// Segments are visited in increasing order.
__device__ double table_mass(const MixTable &t, double a, double b) {
    const double x_end = t.lam0 + (t.M - 1) * t.h;
    const double lo = a > t.lam0 ? a : t.lam0, hi = b < x_end ? b : x_end;
    if (!(hi > lo)) return 0.0;
    int s0 = (int)floor((lo - t.lam0) / t.h), s1 = (int)floor((hi - t.lam0) / t.h);
    if (s0 < 0) s0 = 0;
    if (s1 > t.M - 2) s1 = t.M - 2;
    double acc = 0.0;
    for (int s = s0; s <= s1; s++) {
        const double x0 = t.lam0 + s * t.h, x1 = x0 + t.h;
        const double u = lo > x0 ? lo : x0, v = hi < x1 ? hi : x1;
        if (!(v > u)) continue;
        const double p0 = t.p[s] > 0.0 ? t.p[s] : 0.0, p1 = t.p[s + 1] > 0.0 ? t.p[s + 1] : 0.0;
        const double fu = p0 + (p1 - p0) * (u - x0) / t.h, fv = p0 + (p1 - p0) * (v - x0) / t.h;
        acc += (v - u) * 0.5 * (fu + fv);
    }
    return acc;
}

__global__ void __launch_bounds__(1024) k_mix_weights(MixIn *mi, int count, double c, double Z, int mode, double qs,
                                                      double mu3, MixTable tab, double *out) {
    __shared__ double raw[kMaxMix + 1];
    const int i = threadIdx.x;
    double w = 0.0;
    if (i < count) {
        const double li = mi[i].lambda;
        int rank = 0;
        double prev = -INFINITY, next = INFINITY;
        bool has_prev = false, has_next = false;
        for (int j = 0; j < count; j++) {
            const double lj = mi[j].lambda;
            const bool before = lj < li || (lj == li && j < i);
            if (before) { rank++; if (!has_prev || lj >= prev) { prev = lj; has_prev = true; } }
            else if (j != i) { if (!has_next || lj < next) { next = lj; has_next = true; } }
        }
        mi[rank].order = i;
        double a = has_prev ? 0.5 * (prev + li) : -INFINITY;
        double b = has_next ? 0.5 * (li + next) : INFINITY;
        if (mode == 1 && count > 1) {
            if (!has_prev) a = li - (b - li);
            if (!has_next) b = li + (li - a);
        }
        if (mode == 4) {
            w = table_mass(tab, a, b);
        } else if (mode == 2) {
            const double mu = -4.5 * c * Z, sig = sqrt(9.0 * c * Z);
            const double p = exp(-(li - mu) * (li - mu) / (2.0 * sig * sig)) / sig;
            const double q = exp(-li * li / (2.0 * qs * qs)) / qs;
            w = p / q;
        } else if (Z <= 0.0) {
            w = (a <= 0.0 && 0.0 < b) ? 1.0 : 0.0;
        } else if (mode == 3) {
            const double sig = sqrt(9.0 * c * Z);
            w = a < Z ? nmass(a, b < Z ? b : Z, mu3, sig) / nmass(-INFINITY, Z, mu3, sig) : 0.0;
        } else {
            w = nmass(a, b, -4.5 * c * Z, sqrt(9.0 * c * Z));
        }
    }
    raw[i] = w;
    __syncthreads();
    if (i == 0 && (mode == 1 || mode == 2 || mode == 4)) {
        double s = 0.0;
        for (int r = 0; r < count; r++) s += raw[mi[r].order];
        raw[kMaxMix] = s;    // count <= kMaxMix keeps this slot free
    }
    __syncthreads();
    if (i < count) {
        if (mode == 1 || mode == 2 || mode == 4) w = w / raw[kMaxMix];
        mi[i].w = w;
        out[i] = w;
    }
}

struct MixGeom {
    int qb, lb, ab, count;
    long long off_le, off_lw, off_al, off_at;
    double area_qr, w_l, w_a;
    long long o_qr, o_le, o_lw, o_al, o_at, o_mom, o_der;
};

__global__ void __launch_bounds__(256) k_mix_pdf(const MixIn *__restrict__ mi, MixGeom g, double *out) {
    const long long nqr = (long long)g.qb * g.qb;
    const long long total = nqr + 2LL * g.lb + 2LL * g.ab;
    const long long b = (long long)blockIdx.x * 256 + threadIdx.x;
    if (b >= total) return;
    long long src, dst;
    double width, mult;
    if (b < nqr) { src = b; dst = g.o_qr + b; width = g.area_qr; mult = 1.0; }
    else if (b < nqr + g.lb) { src = g.off_le + (b - nqr); dst = g.o_le + (b - nqr); width = g.w_l; mult = 1.0; }
    else if (b < nqr + 2 * g.lb) { const long long k = b - nqr - g.lb; src = g.off_lw + k; dst = g.o_lw + k; width = g.w_l; mult = 1.0; }
    else if (b < nqr + 2 * g.lb + g.ab) { const long long k = b - nqr - 2 * g.lb; src = g.off_al + k; dst = g.o_al + k; width = g.w_a; mult = 3.0; }
    else { const long long k = b - nqr - 2 * g.lb - g.ab; src = g.off_at + k; dst = g.o_at + k; width = g.w_a; mult = 6.0; }
    double acc = 0.0;
    for (int r = 0; r < g.count; r++) {
        const MixIn &m = mi[mi[r].order];
        const double n = m.ntot * mult;
        if (n > 0.0) acc += m.w * ((double)m.counts[src] / (n * width));
    }
    out[dst] = acc;
}

__global__ void __launch_bounds__(64) k_mix_moments(const MixIn *__restrict__ mi, MixGeom g, double *out) {
    __shared__ double mm[32];
    const int k = threadIdx.x;
    if (k < 32) {
        const double mult = k < 6 ? 3.0 : (k < 12 ? 6.0 : 1.0);
        double acc = 0.0;
        if (k < 26) {
            for (int r = 0; r < g.count; r++) {
                const MixIn &m = mi[mi[r].order];
                if (m.ntot > 0.0) acc += m.w * (m.moments[k] / (m.ntot * mult));
            }
        }
        mm[k] = acc;
        out[g.o_mom + k] = acc;
    }
    __syncthreads();
    if (k == 0) {
        double *d = out + g.o_der;
        d[0] = mm[2] / pow(mm[1], 1.5);
        d[1] = mm[3] / (mm[1] * mm[1]);
        d[2] = mm[5] / (mm[1] * mm[1] * mm[1]);
        d[3] = mm[9] / (mm[7] * mm[7]);
        d[4] = mm[11] / (mm[7] * mm[7] * mm[7]);
        d[5] = mm[12];
        d[6] = mm[16];
        d[7] = 0.0;
    }
}

size_t mix_scratch_bytes(int count) { return sizeof(MixIn) * (size_t)(count > 0 ? count : 1); }
int mix_max_members() { return kMaxMix; }

hipError_t launch_mix(const MemberDev *const *members_host, const double *lambdas, int count, const ens_hist_desc &h,
                      double c, double Z, int mode, double q_sigma, double *out, void *scratch, hipStream_t s) {
    return launch_mix_table(members_host, lambdas, count, h, c, Z, mode, q_sigma, nullptr, 0, 0.0, 0.0, out, scratch, s);
}

// Host side of the member table: pointers to each member's sums, its lambda,
// and zeros for what the kernels fill in (every entry the kernels read is
// written here, so a table left by an earlier call is never read).
static void fill_mix_table(MixIn *tbl, const MemberDev *const *members_host, const double *lambdas, int count) {
    for (int i = 0; i < count; i++) {
        tbl[i].counts = members_host[i]->counts;
        tbl[i].moments = members_host[i]->moments;
        tbl[i].lambda = lambdas[i];
        tbl[i].ntot = 0.0; tbl[i].w = 0.0; tbl[i].order = 0; tbl[i].pad = 0;
    }
}

// Copy the host table into the device table `mi` and enqueue the mixture.
// Returns after the copy has completed (the host table may then be reused);
// the kernels read `mi` asynchronously on `s`.
static hipError_t run_mix(const MixIn *tbl, MixIn *mi, int count, const ens_hist_desc &h, double c, double Z,
                          int mode, double q_sigma, const double *table, int table_len, double lam0, double dlam,
                          double *out, hipStream_t s);

hipError_t launch_mix_table(const MemberDev *const *members_host, const double *lambdas, int count,
                            const ens_hist_desc &h, double c, double Z, int mode, double q_sigma, const double *table,
                            int table_len, double lam0, double dlam, double *out, void *scratch, hipStream_t s) {
    if (count <= 0 || count > kMaxMix || !scratch) return hipErrorInvalidValue;
    if (mode == 4 && (!table || table_len < 2 || !(dlam > 0))) return hipErrorInvalidValue;
    std::vector<MixIn> tmp(count);
    fill_mix_table(tmp.data(), members_host, lambdas, count);
    return run_mix(tmp.data(), reinterpret_cast<MixIn *>(scratch), count, h, c, Z, mode, q_sigma, table, table_len,
                   lam0, dlam, out, s);
}

// ------------------------------------------------ mixture without allocation
// For callers that cannot allocate device memory: the device member table is
// this file-scope array, one copy per GPU, held until the process ends.  In
// host code `scratch` names a host-side stand-in, not the device array: its
// device address is taken once per device with hipGetSymbolAddress (at
// context creation, with that device current) and only that address is used.
static __device__ __align__(256) unsigned char scratch[kMaxMix * sizeof(MixIn)];

constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;                    // guards the two tables below
static void *g_static_dev[kMaxDevices];           // device address of `scratch`, per device
static MixIn g_static_host[kMaxMix];              // host staging of the member table

hipError_t mix_static_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_dev[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_static_dev[device] = p;
    return hipSuccess;
}

size_t mix_static_bytes() { return sizeof(scratch); }

hipError_t launch_mix_static(int device, const MemberDev *const *members_host, const double *lambdas, int count,
                             const ens_hist_desc &h, double c, double Z, int mode, double q_sigma, double *out,
                             hipStream_t s) {
    if (count <= 0 || count > kMaxMix || device < 0 || device >= kMaxDevices) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(g_static_mu);  // the host staging table is shared
    MixIn *mi = reinterpret_cast<MixIn *>(g_static_dev[device]);
    if (!mi) return hipErrorNotInitialized;
    fill_mix_table(g_static_host, members_host, lambdas, count);
    return run_mix(g_static_host, mi, count, h, c, Z, mode, q_sigma, nullptr, 0, 0.0, 0.0, out, s);
}

static hipError_t run_mix(const MixIn *tbl, MixIn *mi, int count, const ens_hist_desc &h, double c, double Z,
                          int mode, double q_sigma, const double *table, int table_len, double lam0, double dlam,
                          double *out, hipStream_t s) {
    const HistGeom hg = make_hist_geom(h);
    hipError_t e = hipMemcpyAsync(mi, tbl, sizeof(MixIn) * count, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);       // the host table may be reused on return
    if (e != hipSuccess) return e;
    k_mix_prep<<<count, 256, 0, s>>>(mi, hg.off_le);
    const double mu3 = (mode == 3 && Z > 0.0) ? truncated_mean(c, Z) : 0.0;
    MixTable tab;
    tab.p = table; tab.M = table_len; tab.lam0 = lam0; tab.h = dlam;
    k_mix_weights<<<1, 1024, 0, s>>>(mi, count, c, Z, mode, q_sigma, mu3, tab, out);
    MixGeom g;
    g.qb = hg.qb; g.lb = hg.lb; g.ab = hg.ab; g.count = count;
    g.off_le = hg.off_le; g.off_lw = hg.off_lw; g.off_al = hg.off_al; g.off_at = hg.off_at;
    g.area_qr = ((h.q_hi - h.q_lo) / h.qr_bins) * ((h.r_hi - h.r_lo) / h.qr_bins);
    g.w_l = (h.log10_hi - h.log10_lo) / h.log_bins;
    g.w_a = (h.a_hi - h.a_lo) / h.a_bins;
    g.o_qr = count;
    g.o_le = g.o_qr + (long long)hg.qb * hg.qb;
    g.o_lw = g.o_le + hg.lb;
    g.o_al = g.o_lw + hg.lb;
    g.o_at = g.o_al + hg.ab;
    g.o_mom = g.o_at + hg.ab;
    g.o_der = g.o_mom + ENS_NMOM;
    const long long total = (long long)hg.qb * hg.qb + 2LL * hg.lb + 2LL * hg.ab;
    k_mix_pdf<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(mi, g, out);
    k_mix_moments<<<1, 64, 0, s>>>(mi, g, out);
    return hipGetLastError();
}

}  // namespace ens
