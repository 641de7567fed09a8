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

}  // namespace ens
