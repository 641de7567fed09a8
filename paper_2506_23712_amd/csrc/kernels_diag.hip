// kernels_diag.hip -- spectral diagnostics of a member: the shell energy
// spectrum, and refinement of a member onto a finer grid.
#include "ens_diag.h"
#include "fft.hpp"
#include "gmem.hpp"

namespace ens {

// Shell of integer |m|^2 = m2: s - 1/2 <= |m| < s + 1/2, i.e.
// (2s - 1)^2 <= 4 m2 < (2s + 1)^2; the FP64 estimate is corrected by that test.
__device__ __forceinline__ int shell_of(long long m2) {
    int s = (int)floor(sqrt((double)m2) + 0.5);
    if (s > 0 && 4 * m2 < (long long)(2 * s - 1) * (2 * s - 1)) s--;
    else if (4 * m2 >= (long long)(2 * s + 1) * (2 * s + 1)) s++;
    return s;
}

// Rows of one z-mode plane iz, split over kDiagParts workgroups of 4 waves:
// wave v (0 .. 4 kDiagParts - 1 over the plane) takes rows iy = v, v + 4 kDiagParts, ...,
// RG rows at a time whose loads are issued together (indices clamped into the
// member so that every load is unconditional), a row in chunks of 64
// consecutive m_x, one per lane.  `f(mx, my, e)` receives each lane's mode
// numbers and energy e_m = (1/2)|u_hat_m|^2 of the full spectrum (weight 1 for
// m_x > 0: the mode and its mirror; 1/2 for m_x = 0); lanes past the row end
// get mx > K and e = 0.
template <typename P, int RG, class F>
__device__ __forceinline__ void plane_rows(const MemberDev &md, int iz, int v0, F &&f) {
    const int K = md.K, NY = 2 * K + 1, lane = threadIdx.x & 63;
    const long long zp = md.zp, S = (long long)NY * zp;     // state plane pitch, component stride
    const Fld<P> U[3] = {Fld<P>(md.uh, iz * zp), Fld<P>(md.uh, S + iz * zp), Fld<P>(md.uh, 2 * S + iz * zp)};
    constexpr int VS = 4 * kDiagParts;
    for (int iy0 = v0; iy0 < NY; iy0 += VS * RG) {
        for (int c0 = 0; c0 <= K; c0 += 64) {
            const int mx = c0 + lane, cx = mx <= K ? mx : K;
            Cx<P> v[RG][3];
#pragma unroll
            for (int r = 0; r < RG; r++) {
                const int iy = iy0 + VS * r, cy = iy < NY ? iy : NY - 1;
#pragma unroll
                for (int comp = 0; comp < 3; comp++) v[r][comp] = U[comp].ld((uint32_t)(cy * (K + 1) + cx));
            }
#pragma unroll
            for (int r = 0; r < RG; r++) {
                const int iy = iy0 + VS * r;
                if (iy >= NY) break;                 // wave-uniform
                const int my = iy <= K ? iy : iy - NY;
                double e = 0.0;
#pragma unroll
                for (int comp = 0; comp < 3; comp++)
                    e += (double)v[r][comp].re * (double)v[r][comp].re + (double)v[r][comp].im * (double)v[r][comp].im;
                e *= mx > 0 ? 1.0 : 0.5;
                f(mx, my, mx <= K ? e : 0.0);
            }
        }
    }
}

// Shell spectrum, first pass.  Along a row the shell index never decreases
// with m_x, so the lanes of one shell form one contiguous run: a segmented
// scan over the wave (keyed by shell) leaves each run's sum in its last lane,
// which adds it to the wave's own LDS bin of that shell (distinct shells, no
// two lanes on one bin).  The four waves' bins are summed in a fixed order into
// partials[s NB + b], b = iz kDiagParts + part, NB = (2K+1) kDiagParts (shell-major,
// so that the second pass reads each shell's partials contiguously).  Fixed
// order throughout: deterministic.
template <typename P, int RG>
__global__ void __launch_bounds__(256) k_spectrum_plane(const MemberDev *__restrict__ mp, int NS) {
    extern __shared__ double bins[];                 // [4][NS]
    const MemberDev &md = *mp;
    const int K = md.K, iz = blockIdx.x / kDiagParts, part = blockIdx.x % kDiagParts;
    const int mz = iz <= K ? iz : iz - (2 * K + 1);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double *my_bins = bins + w * NS;
    for (int i = threadIdx.x; i < 4 * NS; i += 256) bins[i] = 0.0;
    __syncthreads();
    plane_rows<P, RG>(md, iz, part * 4 + w, [&](int mx, int my, double e) {
        const long long m2 = (long long)mx * mx + (long long)my * my + (long long)mz * mz;
        const int sh = mx <= K ? shell_of(m2) : -1;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double eo = __shfl_up(e, off, 64);
            const int so = __shfl_up(sh, off, 64);
            if (lane >= off && so == sh) e += eo;
        }
        const int nx = __shfl_down(sh, 1, 64);
        if (sh >= 0 && (lane == 63 || nx != sh)) my_bins[sh] += e;
    });
    __syncthreads();
    const long long NB = (long long)(2 * K + 1) * kDiagParts;
    for (int s = threadIdx.x; s < NS; s += 256)
        md.partials[s * NB + blockIdx.x] = ((bins[s] + bins[NS + s]) + bins[2 * NS + s]) + bins[3 * NS + s];
}

// Second pass, one workgroup per shell s: out[s] = the sum of the shell's NB
// partials (thread t takes b = t, t + 256, ... in order, then a fixed tree);
// shells beyond the retained set are zero.
__global__ void __launch_bounds__(256) k_spectrum_sum(const MemberDev *__restrict__ mp, int NS,
                                                      double *__restrict__ out) {
    __shared__ double red[256];
    const MemberDev &md = *mp;
    const int s = blockIdx.x, NB = (2 * md.K + 1) * kDiagParts;
    double acc = 0.0;
    if (s < NS)
        for (int b = threadIdx.x; b < NB; b += 256) acc += md.partials[(long long)s * NB + b];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[s] = red[0];
}

hipError_t launch_spectrum(int prec, const MemberDev *mem, int K, int nshell, double *out, hipStream_t s) {
    const int NS = spectrum_shells(K);
    const size_t lds = 4 * (size_t)NS * sizeof(double);
    const unsigned nb = (unsigned)((2 * K + 1) * kDiagParts);
    if (prec == ENS_FP32) k_spectrum_plane<float, 8><<<nb, 256, lds, s>>>(mem, NS);
    else k_spectrum_plane<double, 4><<<nb, 256, lds, s>>>(mem, NS);
    k_spectrum_sum<<<nshell, 256, 0, s>>>(mem, NS, out);
    return hipGetLastError();
}

// Integral scales, first pass: e_m and e_m / |m| summed per workgroup in a
// fixed order into partials[2 b], partials[2 b + 1], b = iz kDiagParts + part.
template <typename P, int RG>
__global__ void __launch_bounds__(256) k_scales_plane(const MemberDev *__restrict__ mp) {
    __shared__ double red[2][256];
    const MemberDev &md = *mp;
    const int K = md.K, iz = blockIdx.x / kDiagParts, part = blockIdx.x % kDiagParts;
    const int mz = iz <= K ? iz : iz - (2 * K + 1);
    double ea = 0.0, ka = 0.0;
    plane_rows<P, RG>(md, iz, part * 4 + (int)(threadIdx.x >> 6), [&](int mx, int my, double e) {
        const long long m2 = (long long)mx * mx + (long long)my * my + (long long)mz * mz;
        ea += e;
        if (m2 > 0 && e != 0.0) ka += e / sqrt((double)m2);
    });
    red[0][threadIdx.x] = ea;
    red[1][threadIdx.x] = ka;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        md.partials[2 * blockIdx.x] = red[0][0];
        md.partials[2 * blockIdx.x + 1] = red[1][0];
    }
}

// Second pass (one workgroup): E, u' = sqrt(2E/3), L = (pi / (2 u'^2)) sum e_m / |k_m|
// with |k_m| = dk |m|, T = L / u'.
__global__ void __launch_bounds__(256) k_scales_final(const MemberDev *__restrict__ mp, double *__restrict__ out) {
    __shared__ double red[2][256];
    const MemberDev &md = *mp;
    const int np = (2 * md.K + 1) * kDiagParts;
    double ea = 0.0, ka = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) {
        ea += md.partials[2 * i];
        ka += md.partials[2 * i + 1];
    }
    red[0][threadIdx.x] = ea;
    red[1][threadIdx.x] = ka;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double E = red[0][0], up2 = 2.0 * E / 3.0, up = sqrt(up2);
        const double L = up2 > 0.0 ? 3.14159265358979323846 / (2.0 * up2) * red[1][0] / md.dk : 0.0;
        out[0] = E;
        out[1] = up;
        out[2] = L;
        out[3] = up > 0.0 ? L / up : 0.0;
    }
}

hipError_t launch_scales(int prec, const MemberDev *mem, int K, double *out, hipStream_t s) {
    const unsigned nb = (unsigned)((2 * K + 1) * kDiagParts);
    if (prec == ENS_FP32) k_scales_plane<float, 8><<<nb, 256, 0, s>>>(mem);
    else k_scales_plane<double, 4><<<nb, 256, 0, s>>>(mem);
    k_scales_final<<<1, 256, 0, s>>>(mem, out);
    return hipGetLastError();
}

// diag.E of a member whose field was replaced: the empty-band threshold of its
// next step is relative to the energy of the field it starts from.
__global__ void k_take_energy(const MemberDev *__restrict__ mp) {
    DevState *st = mp->st;
    st->diag.E = st->pad[0];
}

hipError_t launch_refresh_energy(int prec, const MemberDev *mem, DevState *st, int K, hipStream_t s) {
    hipError_t e = launch_scales(prec, mem, K, st->pad, s);
    if (e != hipSuccess) return e;
    k_take_energy<<<1, 1, 0, s>>>(mem);
    return hipGetLastError();
}

// dst storage entry (component, iz, plane offset) of the finer grid: the src
// value where the mode is retained by src, else zero (pad entries too); the RK
// register is cleared.  One thread per dst entry.
template <typename PS, typename PD>
__global__ void __launch_bounds__(256) k_refine(const MemberDev *__restrict__ sp, const MemberDev *__restrict__ dp) {
    const MemberDev &ms = *sp, &md = *dp;
    const int Ks = ms.K, Kd = md.K;
    const long long nzd = (long long)(2 * Kd + 1) * (Kd + 1), zpd = md.zp, Sd = (long long)(2 * Kd + 1) * zpd;
    const long long zps = ms.zp, Ss = (long long)(2 * Ks + 1) * zps;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= 3 * Sd) return;
    const int comp = (int)(i / Sd);
    const long long r = i - comp * Sd;
    const int iz = (int)(r / zpd);
    const long long rem = r - iz * zpd;
    LdsT<PD> v;
    v.x = PD(0);
    v.y = PD(0);
    if (rem < nzd) {
        const int iy = (int)(rem / (Kd + 1)), mx = (int)(rem % (Kd + 1));
        const int my = iy <= Kd ? iy : iy - (2 * Kd + 1), mz = iz <= Kd ? iz : iz - (2 * Kd + 1);
        if (mx <= Ks && my >= -Ks && my <= Ks && mz >= -Ks && mz <= Ks) {
            const int sy = my >= 0 ? my : my + 2 * Ks + 1, sz = mz >= 0 ? mz : mz + 2 * Ks + 1;
            const LdsT<PS> w = reinterpret_cast<const LdsT<PS> *>(ms.uh)[comp * Ss + (long long)sz * zps +
                                                                         (long long)sy * (Ks + 1) + mx];
            v.x = (PD)(double)w.x;
            v.y = (PD)(double)w.y;
        }
    }
    reinterpret_cast<LdsT<PD> *>(md.uh)[i] = v;
    LdsT<PD> z;
    z.x = PD(0);
    z.y = PD(0);
    reinterpret_cast<LdsT<PD> *>(md.q)[i] = z;
    if (i == 0) {
        *md.st = *ms.st;                    // time, step count, diagnostics, last E_f and dt
        md.st->umax_bits = 0ull;
    }
}

template <typename PS>
static hipError_t refine_to(int prec_dst, const MemberDev *src, const MemberDev *dst, long long total, hipStream_t s) {
    const unsigned nb = (unsigned)((total + 255) / 256);
    if (prec_dst == ENS_FP32) k_refine<PS, float><<<nb, 256, 0, s>>>(src, dst);
    else k_refine<PS, double><<<nb, 256, 0, s>>>(src, dst);
    return hipGetLastError();
}

hipError_t launch_refine(int prec_src, int prec_dst, const MemberDev *src, const MemberDev *dst, int n_dst,
                         hipStream_t s) {
    const long long total = 3 * make_geom(n_dst, prec_dst).S;
    return prec_src == ENS_FP32 ? refine_to<float>(prec_dst, src, dst, total, s)
                                : refine_to<double>(prec_dst, src, dst, total, s);
}

}  // namespace ens
