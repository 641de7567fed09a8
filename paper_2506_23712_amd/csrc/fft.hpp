// fft.hpp -- workgroup-level pencil FFT engine for gfx950.
//
// A line of length N is transformed by M = N/E threads, each holding E complex
// values in registers.  The transform is a Stockham (self-sorting) radix
// sequence: the first stage has radix E, the next ones radix min(E, remaining).
// Stage s with radix r and span Ns (product of earlier radices) computes, for
// every butterfly j in [0, N/r):
//     k = j mod Ns,
//     y_m = DFT_r( x[j + m N/r] * w^(m k N/(Ns r)) ),  w = exp(DIR 2 pi i / N),
//     out[(j/Ns) Ns r + k + m Ns] = y_m.
// Thread t owns butterflies j = t + M b, b < E/r.  Between stages values
// are exchanged through LDS laid out [position][line] (lines fastest), so that
// lanes of consecutive lines touch consecutive LDS words.
//
// line_fft   : input  v[m] = x[t + M m]; output v[b r_L + m] = X[out_pos(t, b r_L + m)]
// line_fft_T : the transposed flow graph (stages reversed, twiddles after the
//              butterflies): input in out_pos layout, output v[m] = X[t + M m].
// Both compute the same DFT; using one after the other avoids a permutation.
#pragma once

#include <hip/hip_runtime.h>

namespace ens {

template <typename P> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

template <typename P> struct Cx { P re, im; };

template <typename P> __device__ __forceinline__ Cx<P> operator+(Cx<P> a, Cx<P> b) { return {a.re + b.re, a.im + b.im}; }
template <typename P> __device__ __forceinline__ Cx<P> operator-(Cx<P> a, Cx<P> b) { return {a.re - b.re, a.im - b.im}; }
template <typename P> __device__ __forceinline__ Cx<P> cmul(Cx<P> a, Cx<P> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename P> __device__ __forceinline__ Cx<P> cmulc(Cx<P> a, Cx<P> b) {   // a * conj(b)
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename P> __device__ __forceinline__ Cx<P> cscale(Cx<P> a, P s) { return {a.re * s, a.im * s}; }
template <typename P> __device__ __forceinline__ Cx<P> cconj(Cx<P> a) { return {a.re, -a.im}; }
template <typename P> __device__ __forceinline__ Cx<P> mul_i(Cx<P> a) { return {-a.im, a.re}; }       // i a
template <typename P> __device__ __forceinline__ Cx<P> czero() { return {P(0), P(0)}; }

// multiply by exp(DIR i pi / 2) = DIR i
template <int DIR, typename P> __device__ __forceinline__ Cx<P> rot90(Cx<P> a) {
    if constexpr (DIR < 0) return {a.im, -a.re};
    else return {-a.im, a.re};
}
// multiply by (cr + DIR i si)
template <int DIR, typename P> __device__ __forceinline__ Cx<P> rotc(Cx<P> a, P cr, P si) {
    if constexpr (DIR < 0) return {a.re * cr + a.im * si, a.im * cr - a.re * si};
    else return {a.re * cr - a.im * si, a.im * cr + a.re * si};
}

// cos(pi/8), sin(pi/8), sqrt(1/2)
#define ENS_C8 0.92387953251128675612818318939678828682
#define ENS_S8 0.38268343236508977172845998403039886676
#define ENS_R2 0.70710678118654752440084436210484903928

template <int DIR, typename P> __device__ __forceinline__ void dft2(Cx<P> &a, Cx<P> &b) {
    Cx<P> t = a; a = t + b; b = t - b;
}

template <typename P> __device__ __forceinline__ Cx<P> cneg(Cx<P> a) { return {-a.re, -a.im}; }

// a +- b where bit 0 of Z says a is known to be zero and bit 1 that b is
// (known zeros are the truncated modes of an inverse transform's input; the
// sums skip them)
template <int Z, typename P> __device__ __forceinline__ Cx<P> zadd(Cx<P> a, Cx<P> b) {
    if constexpr ((Z & 2) != 0) return a;
    else if constexpr ((Z & 1) != 0) return b;
    else return a + b;
}
template <int Z, typename P> __device__ __forceinline__ Cx<P> zsub(Cx<P> a, Cx<P> b) {
    if constexpr ((Z & 2) != 0) return a;
    else if constexpr ((Z & 1) != 0) return cneg(b);
    else return a - b;
}

// ZM: bit i set = input a_i is known to be zero
template <int DIR, unsigned ZM = 0u, typename P>
__device__ __forceinline__ void dft4(Cx<P> &a0, Cx<P> &a1, Cx<P> &a2, Cx<P> &a3) {
    constexpr int Z02 = (int)((ZM & 1u) | ((ZM >> 1) & 2u)), Z13 = (int)(((ZM >> 1) & 1u) | ((ZM >> 2) & 2u));
    Cx<P> t0 = zadd<Z02>(a0, a2), t1 = zsub<Z02>(a0, a2), t2 = zadd<Z13>(a1, a3), t3 = rot90<DIR>(zsub<Z13>(a1, a3));
    a0 = t0 + t2; a2 = t0 - t2; a1 = t1 + t3; a3 = t1 - t3;
}

template <int DIR, unsigned ZM = 0u, typename P> __device__ __forceinline__ void dft8(Cx<P> *v) {
    Cx<P> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    Cx<P> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    constexpr unsigned ZE = (ZM & 1u) | ((ZM >> 1) & 2u) | ((ZM >> 2) & 4u) | ((ZM >> 3) & 8u);
    constexpr unsigned ZO = ((ZM >> 1) & 1u) | ((ZM >> 2) & 2u) | ((ZM >> 3) & 4u) | ((ZM >> 4) & 8u);
    dft4<DIR, ZE>(e0, e1, e2, e3);
    dft4<DIR, ZO>(o0, o1, o2, o3);
    const P r = P(ENS_R2);
    o1 = rotc<DIR>(o1, r, r);
    o2 = rot90<DIR>(o2);
    o3 = rotc<DIR>(o3, -r, r);
    v[0] = e0 + o0; v[4] = e0 - o0;
    v[1] = e1 + o1; v[5] = e1 - o1;
    v[2] = e2 + o2; v[6] = e2 - o2;
    v[3] = e3 + o3; v[7] = e3 - o3;
}

// inputs n2, n2 + 4, n2 + 8, n2 + 12 of a 16-point mask
template <int n2> constexpr unsigned sub4(unsigned zm) {
    return ((zm >> n2) & 1u) | ((zm >> (n2 + 3)) & 2u) | ((zm >> (n2 + 6)) & 4u) | ((zm >> (n2 + 9)) & 8u);
}

template <int DIR, unsigned ZM = 0u, typename P> __device__ __forceinline__ void dft16(Cx<P> *v) {
    // 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
    Cx<P> y[4][4];
    y[0][0] = v[0]; y[0][1] = v[4]; y[0][2] = v[8]; y[0][3] = v[12];
    y[1][0] = v[1]; y[1][1] = v[5]; y[1][2] = v[9]; y[1][3] = v[13];
    y[2][0] = v[2]; y[2][1] = v[6]; y[2][2] = v[10]; y[2][3] = v[14];
    y[3][0] = v[3]; y[3][1] = v[7]; y[3][2] = v[11]; y[3][3] = v[15];
    dft4<DIR, sub4<0>(ZM)>(y[0][0], y[0][1], y[0][2], y[0][3]);
    dft4<DIR, sub4<1>(ZM)>(y[1][0], y[1][1], y[1][2], y[1][3]);
    dft4<DIR, sub4<2>(ZM)>(y[2][0], y[2][1], y[2][2], y[2][3]);
    dft4<DIR, sub4<3>(ZM)>(y[3][0], y[3][1], y[3][2], y[3][3]);
    const P c = P(ENS_C8), s = P(ENS_S8), r = P(ENS_R2);
    // twiddles w16^(n2 k1)
    y[1][1] = rotc<DIR>(y[1][1], c, s);
    y[1][2] = rotc<DIR>(y[1][2], r, r);
    y[1][3] = rotc<DIR>(y[1][3], s, c);
    y[2][1] = rotc<DIR>(y[2][1], r, r);
    y[2][2] = rot90<DIR>(y[2][2]);
    y[2][3] = rotc<DIR>(y[2][3], -r, r);
    y[3][1] = rotc<DIR>(y[3][1], s, c);
    y[3][2] = rotc<DIR>(y[3][2], -r, r);
    y[3][3] = rotc<DIR>(y[3][3], -c, -s);
#pragma unroll
    for (int k1 = 0; k1 < 4; k1++) {
        Cx<P> a0 = y[0][k1], a1 = y[1][k1], a2 = y[2][k1], a3 = y[3][k1];
        dft4<DIR>(a0, a1, a2, a3);
        v[k1] = a0; v[k1 + 4] = a1; v[k1 + 8] = a2; v[k1 + 12] = a3;
    }
}

template <int R, int DIR, unsigned ZM = 0u, typename P> __device__ __forceinline__ void dft(Cx<P> *v) {
    if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
    else if constexpr (R == 4) dft4<DIR, ZM>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<DIR, ZM>(v);
    else if constexpr (R == 16) dft16<DIR, ZM>(v);
    else static_assert(R == 2, "unsupported radix");
}

// Input slots m of a thread whose positions t + M m (every t < M) all lie
// strictly between K and N - K, i.e. hold truncated modes (zero) of an
// inverse transform's input: bit m of the mask.
__host__ __device__ constexpr unsigned truncated_slots(int N, int E, int K) {
    const int M = N / E;
    unsigned z = 0u;
    for (int m = 0; m < E && m < 32; m++)
        if (M * m > K && M * m + M - 1 < N - K) z |= 1u << m;
    return z;
}

// ---------------------------------------------------------------- stage plan
__host__ __device__ constexpr int stage_radix(int N, int E, int s) {
    int rem = N, r = 1;
    for (int i = 0; i <= s; i++) { r = rem < E ? rem : E; rem /= r; }
    return r;
}
__host__ __device__ constexpr int num_stages(int N, int E) {
    int rem = N, s = 0;
    while (rem > 1) { int r = rem < E ? rem : E; rem /= r; s++; }
    return s;
}
__host__ __device__ constexpr int stage_span(int N, int E, int s) {
    int p = 1;
    for (int i = 0; i < s; i++) p *= stage_radix(N, E, i);
    return p;
}

// Entries of the twiddle table a transform reads: 1 + the largest index
// m k N / (Ns r) over its stages (m < r, k < Ns).
__host__ __device__ constexpr int twiddle_span(int N, int E) {
    int mx = 0;
    for (int s = 1; s < num_stages(N, E); s++) {
        const int r = stage_radix(N, E, s), ns = stage_span(N, E, s);
        const int v = (r - 1) * (ns - 1) * (N / (ns * r));
        mx = v > mx ? v : mx;
    }
    return mx + 1;
}

template <int N, int E> struct Plan {
    static constexpr int M = N / E;                              // threads per line
    static constexpr int S = num_stages(N, E);
    static constexpr int RL = stage_radix(N, E, S - 1);          // last radix
    // output position of register slot `slot` of thread t after line_fft
    __device__ static __forceinline__ int out_pos(int t, int slot) {
        return t + M * (slot / RL) + (slot % RL) * (N / RL);
    }
    // input position of register slot m (before line_fft / after line_fft_T)
    __device__ static __forceinline__ int in_pos(int t, int m) { return t + M * m; }
};

// Twiddle w_N^idx for direction DIR from a table of exp(-2 pi i j / N).
template <int DIR, typename P> __device__ __forceinline__ Cx<P> twiddle(const Cx<P> *tw, int idx) {
    Cx<P> w = tw[idx];
    if constexpr (DIR > 0) w.im = -w.im;
    return w;
}

// Twiddles held in registers: for thread t, the factors of every stage s >= 1
// (butterflies b < E/r, m = 1..r-1), loaded once from the table; each
// transform of the thread then reads no twiddle from memory.
template <typename P, int N, int E> struct TwRegs {
    static constexpr int off(int s) {
        int o = 0;
        for (int i = 1; i < s; i++) { const int r = stage_radix(N, E, i); o += (E / r) * (r - 1); }
        return o;
    }
    static constexpr int CNT = off(num_stages(N, E));
    Cx<P> w[CNT > 0 ? CNT : 1];
    template <int s = 1> __device__ __forceinline__ void load(const Cx<P> *tw, int t) {
        if constexpr (s < num_stages(N, E)) {
            constexpr int R = stage_radix(N, E, s), NS = stage_span(N, E, s), M = N / E;
#pragma unroll
            for (int b = 0; b < E / R; b++) {
                const int k = (t + M * b) % NS;
#pragma unroll
                for (int m = 1; m < R; m++) w[off(s) + b * (R - 1) + m - 1] = tw[m * k * (N / (NS * R))];
            }
            load<s + 1>(tw, t);
        }
    }
    template <int DIR, int s> __device__ __forceinline__ Cx<P> get(int b, int m) const {
        constexpr int R = stage_radix(N, E, s);
        Cx<P> x = w[off(s) + b * (R - 1) + m - 1];
        if constexpr (DIR > 0) x.im = -x.im;
        return x;
    }
};
// twiddle m k N/(Ns r) of butterfly b, stage s, from a table or from registers
template <int DIR, int s, typename P>
__device__ __forceinline__ Cx<P> tw_at(const Cx<P> *tw, int b, int m, int idx) { return twiddle<DIR>(tw, idx); }
template <int DIR, int s, typename P, int N, int E>
__device__ __forceinline__ Cx<P> tw_at(const TwRegs<P, N, E> &tw, int b, int m, int idx) { return tw.template get<DIR, s>(b, m); }

template <typename P> using LdsT = typename V2<P>::T;

// Workgroup barrier for LDS exchanges: waits for this wave's LDS operations
// only.  A __syncthreads() fence would also wait for outstanding loads that
// write LDS directly (global_load_lds), which the pipelined passes keep in
// flight across the transforms.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
// Ordering of LDS accesses of one wave: the LDS executes a wave's operations
// in issue order, so lanes of one wave exchanging values through LDS need no
// hardware wait; this only keeps the compiler from moving LDS accesses
// across the point (it emits no instruction).
__device__ __forceinline__ void wave_fence() { asm volatile("" ::: "memory"); }
// Wait until this wave's LDS reads have returned (before memory they read
// is handed to a direct-to-LDS load, which is not ordered with them).
__device__ __forceinline__ void lds_wait() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Barrier between transform stages: __syncthreads() (SB = 0), lds_barrier()
// (SB = 1, for passes that keep direct-to-LDS loads in flight), or none but a
// compiler fence (SB = 2, for transforms whose lines belong to one wave).
template <int SB> __device__ __forceinline__ void stage_barrier() {
    if constexpr (SB == 2) wave_fence();
    else if constexpr (SB == 1) lds_barrier();
    else __syncthreads();
}

// LDS slot of (position p, line l) in the [position][line] layout of the
// exchanges between stages.  When a row of T values covers only half of the
// 32 banks (64 bytes: T = 8 complex FP32 or T = 4 complex FP64), the bank half
// is set by the parity of p, and in the radix-16 exchanges whose lanes all
// address positions 16 t + m of one parity an instruction would use half of
// the banks (two-way conflicts).  Exchanging the two rows of each even/odd
// pair in every other block of 16 positions (flipping bit 0 of p by bit 4)
// spreads those over both halves; positions t + 16 m, whose parity already
// varies across lanes, stay spread.  A bijection on positions: the
// transforms compute the same values.
template <typename P, int T> __device__ __forceinline__ int xslot(int p, int l) {
    if constexpr (T * (int)sizeof(LdsT<P>) == 64) return (p ^ ((p >> 4) & 1)) * T + l;
    else return p * T + l;
}

// Layouts of the exchanges: LDS slot of (position p, line l).
// RowLay: [position][line] with T lines, lines fastest (xslot).
template <typename P, int T> struct RowLay {
    __device__ static __forceinline__ int slot(int p, int l) { return xslot<P, T>(p, l); }
};
// WaveLay: one row of N slots per line (the lines of a wave are its own), the
// position XOR-ed within blocks of G = 128 bytes of complex values by its
// block index: lanes of a line at positions G t + m (stride G) and at
// positions t + G m (consecutive) both spread over all banks.
template <typename P, int N> struct WaveLay {
    static constexpr int G = 128 / (int)sizeof(LdsT<P>);
    __device__ static __forceinline__ int slot(int p, int l) { return l * N + (p ^ ((p / G) % G)); }
};

template <typename P> __device__ __forceinline__ void lds_put(LdsT<P> *lds, int i, Cx<P> v) {
    LdsT<P> x; x.x = v.re; x.y = v.im; lds[i] = x;
}
template <typename P> __device__ __forceinline__ Cx<P> lds_get(const LdsT<P> *lds, int i) {
    LdsT<P> x = lds[i]; return {x.x, x.y};
}

// One forward-flow stage s >= 1: gather from LDS, twiddle, butterfly.
template <typename P, int N, int E, int T, int DIR, int s, class LY, class TW>
__device__ __forceinline__ void stage_gather(Cx<P> *v, const LdsT<P> *lds, int l, int t, const TW &tw) {
    constexpr int R = stage_radix(N, E, s), NS = stage_span(N, E, s), M = N / E;
#pragma unroll
    for (int b = 0; b < E / R; b++) {
        const int j = t + M * b, k = j % NS;
#pragma unroll
        for (int m = 0; m < R; m++) {
            Cx<P> x = lds_get<P>(lds, LY::slot(j + m * (N / R), l));
            if (m > 0) x = cmul(x, tw_at<DIR, s>(tw, b, m, m * k * (N / (NS * R))));
            v[b * R + m] = x;
        }
        dft<R, DIR>(v + b * R);
    }
}

// Scatter the outputs of stage s to LDS.
template <typename P, int N, int E, int T, int s, class LY>
__device__ __forceinline__ void stage_scatter(const Cx<P> *v, LdsT<P> *lds, int l, int t) {
    constexpr int R = stage_radix(N, E, s), NS = stage_span(N, E, s), M = N / E;
#pragma unroll
    for (int b = 0; b < E / R; b++) {
        const int j = t + M * b, k = j % NS;
#pragma unroll
        for (int m = 0; m < R; m++) lds_put<P>(lds, LY::slot((j / NS) * NS * R + k + m * NS, l), v[b * R + m]);
    }
}

template <typename P, int N, int E, int T, int DIR, int s, int SB, class LY, class TW>
__device__ __forceinline__ void run_stages(Cx<P> *v, LdsT<P> *lds, int l, int t, const TW &tw) {
    if constexpr (s < num_stages(N, E)) {
        stage_barrier<SB>();
        stage_scatter<P, N, E, T, s - 1, LY>(v, lds, l, t);
        stage_barrier<SB>();
        stage_gather<P, N, E, T, DIR, s, LY>(v, lds, l, t, tw);
        run_stages<P, N, E, T, DIR, s + 1, SB, LY>(v, lds, l, t, tw);
    }
}

// Forward-flow transform.  All threads of the workgroup must call it (it
// contains barriers; with SB = 2 all lanes of the wave).  LDS: N*T elements
// of V2<P> (RowLay), or N per line of the wave (WaveLay).  ZM: input slots
// known to be zero (truncated_slots), skipped by the first stage's sums.
template <typename P, int N, int E, int T, int DIR, int SB = 0, class LY = RowLay<P, T>, unsigned ZM = 0u, class TW>
__device__ __forceinline__ void line_fft(Cx<P> *v, LdsT<P> *lds, int l, int t, const TW &tw) {
    static_assert(N % E == 0 && N >= E, "line length must be a multiple of E");
    dft<E, DIR, ZM>(v);                   // stage 0: span 1, no twiddles
    run_stages<P, N, E, T, DIR, 1, SB, LY>(v, lds, l, t, tw);
}

// ---- transposed flow (stages in reverse order, twiddles after the butterflies)
template <typename P, int N, int E, int T, int DIR, int s, class TW>
__device__ __forceinline__ void stageT_compute(Cx<P> *v, int t, const TW &tw) {
    constexpr int R = stage_radix(N, E, s), NS = stage_span(N, E, s), M = N / E;
#pragma unroll
    for (int b = 0; b < E / R; b++) {
        const int j = t + M * b, k = j % NS;
        dft<R, DIR>(v + b * R);
        if constexpr (NS > 1) {
#pragma unroll
            for (int m = 1; m < R; m++) v[b * R + m] = cmul(v[b * R + m], tw_at<DIR, s>(tw, b, m, m * k * (N / (NS * R))));
        }
    }
}
// after stage s (transposed) values belong at its input positions j + m N/R
template <typename P, int N, int E, int T, int s, class LY>
__device__ __forceinline__ void stageT_scatter(const Cx<P> *v, LdsT<P> *lds, int l, int t) {
    constexpr int R = stage_radix(N, E, s), M = N / E;
#pragma unroll
    for (int b = 0; b < E / R; b++) {
        const int j = t + M * b;
#pragma unroll
        for (int m = 0; m < R; m++) lds_put<P>(lds, LY::slot(j + m * (N / R), l), v[b * R + m]);
    }
}
// stage s (transposed) reads from its output positions
template <typename P, int N, int E, int T, int s, class LY>
__device__ __forceinline__ void stageT_gather(Cx<P> *v, const LdsT<P> *lds, int l, int t) {
    constexpr int R = stage_radix(N, E, s), NS = stage_span(N, E, s), M = N / E;
#pragma unroll
    for (int b = 0; b < E / R; b++) {
        const int j = t + M * b, k = j % NS;
#pragma unroll
        for (int m = 0; m < R; m++) v[b * R + m] = lds_get<P>(lds, LY::slot((j / NS) * NS * R + k + m * NS, l));
    }
}

template <typename P, int N, int E, int T, int DIR, int s, int SB, class LY, class TW>
__device__ __forceinline__ void run_stagesT(Cx<P> *v, LdsT<P> *lds, int l, int t, const TW &tw) {
    stageT_compute<P, N, E, T, DIR, s>(v, t, tw);
    if constexpr (s > 0) {
        stage_barrier<SB>();
        stageT_scatter<P, N, E, T, s, LY>(v, lds, l, t);
        stage_barrier<SB>();
        stageT_gather<P, N, E, T, s - 1, LY>(v, lds, l, t);
        run_stagesT<P, N, E, T, DIR, s - 1, SB, LY>(v, lds, l, t, tw);
    }
}

template <typename P, int N, int E, int T, int DIR, int SB = 0, class LY = RowLay<P, T>, class TW>
__device__ __forceinline__ void line_fft_T(Cx<P> *v, LdsT<P> *lds, int l, int t, const TW &tw) {
    run_stagesT<P, N, E, T, DIR, num_stages(N, E) - 1, SB, LY>(v, lds, l, t, tw);
}

}  // namespace ens
