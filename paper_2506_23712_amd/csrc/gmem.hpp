// gmem.hpp -- global-memory access for the pass kernels.
//
// A field of a member buffer is addressed as a workgroup-uniform base pointer
// (kept in scalar registers) plus a 32-bit per-lane element offset, so loads
// and stores are `global_load/store ... v_off, s[base]` with no 64-bit address
// arithmetic per element.  Pointers are cast to the global address space so
// the compiler never falls back to flat instructions (those count against the
// LDS counter and would stall the LDS waits inside the transforms).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "fft.hpp"

#define ENS_GLOBAL __attribute__((address_space(1)))

namespace ens {

template <typename P> struct GV;
template <> struct GV<float> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct GV<double> { typedef double T __attribute__((ext_vector_type(2))); };

template <typename P> struct Fld {
    ENS_GLOBAL char *base;
    // field starting `off` complex elements into `buf`
    __device__ __forceinline__ Fld(const void *buf, long long off)
        : base((ENS_GLOBAL char *)buf + off * (long long)sizeof(Cx<P>)) {}
    __device__ __forceinline__ Cx<P> ld(uint32_t e) const {
        const typename GV<P>::T v = *(const ENS_GLOBAL typename GV<P>::T *)(base + e * (uint32_t)sizeof(Cx<P>));
        return {v.x, v.y};
    }
    __device__ __forceinline__ void st(uint32_t e, Cx<P> c) const {
        typename GV<P>::T v;
        v.x = c.re;
        v.y = c.im;
        *(ENS_GLOBAL typename GV<P>::T *)(base + e * (uint32_t)sizeof(Cx<P>)) = v;
    }
};

// XCD-aware workgroup placement.  Workgroups are handed to the 8 XCDs of the
// chip round-robin by linear id, and each XCD has its own L2.  Neighbouring
// tiles of a pass share cache lines at their edges, so the linear id is
// permuted such that XCD x processes one contiguous range of tiles: the
// neighbours of a tile then run on the same XCD at about the same time and the
// shared lines are fetched from HBM once.  Returns (tile, member).
__device__ __forceinline__ void xcd_tile(unsigned &tile, unsigned &member) {
    const unsigned gx = gridDim.x, G = gridDim.x * gridDim.y;
    const unsigned g = blockIdx.y * gx + blockIdx.x;
    const unsigned q = G >> 3, r = G & 7u, x = g & 7u;
    const unsigned gp = x * q + (x < r ? x : r) + (g >> 3);
    member = gp / gx;
    tile = gp - member * gx;
}

// s_waitcnt bounding only the vector-memory counter: wait until at most n
// vector-memory operations (loads, stores, direct-to-LDS loads) of this wave
// are outstanding; they complete in issue order.
template <int n> __device__ __forceinline__ void wait_vm() {
    static_assert(n >= 0 && n < 64, "vmcnt is a 6-bit counter");
    __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Direct-to-LDS copy of one tile of F fields into `dst` laid out [F][RV] in
// 16-byte vectors.  Field f's tile starts at byte b0 + f fstride (16-byte
// aligned; the tile is contiguous in HBM).  Each field is cut into
// ceil(RV/64) wave-sized chunks, the last one moved back to end at the
// field's last vector (re-copying a few vectors with identical data), so that
// every global_load_lds moves 64 consecutive vectors of one field: its global
// and LDS bases are wave-uniform (scalar registers) and the lane offset is
// lane * 16.  Every wave issues exactly dma_tile_ops<F, RV, NTH>() copies
// (surplus waves repeat the last chunk), so the vector-memory counter of every
// wave advances by the same known amount.
template <int F, int RV, int NTH>
__device__ __forceinline__ void dma_tile(void *dst, const char *b0, long long fstride) {
    constexpr int NCF = (RV + 63) / 64, NCH = F * NCF, NW = NTH / 64;
    static_assert(F >= 1 && RV >= 64 && NTH % 64 == 0, "tile too small for wave-wide copies");
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const unsigned lane16 = (threadIdx.x & 63u) * 16u;
#pragma unroll
    for (int j = 0; j < (NCH + NW - 1) / NW; j++) {
        int c = j * NW + wave;
        c = c < NCH ? c : NCH - 1;
        const int f = c / NCF, q = c - f * NCF;
        const int st = q * 64 < RV - 64 ? q * 64 : RV - 64;
        const ENS_GLOBAL char *src = (const ENS_GLOBAL char *)b0 + f * fstride + st * 16;
        __builtin_amdgcn_global_load_lds((const ENS_GLOBAL void *)(src + lane16),
                                         (__attribute__((address_space(3))) void *)((char *)dst + (f * RV + st) * 16), 16, 0, 0);
    }
}
// copies (or 16-byte stores in the same chunking) per wave for F fields of RV vectors
template <int F, int RV, int NTH> constexpr int dma_tile_ops() {
    return (F * ((RV + 63) / 64) + NTH / 64 - 1) / (NTH / 64);
}

}  // namespace ens
