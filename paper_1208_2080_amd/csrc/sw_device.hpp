// Device-side building blocks of the SW sweep for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_layout.hpp"

namespace swmi {

// ----------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products with the published multipliers, the key advanced by the
// two published Weyl increments between rounds.  The key is wave-uniform, so
// its schedule stays in scalar registers.
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // full 64-bit products: one v_mad_u64_u32 each on gfx950
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input xor in one instruction (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// The ten round keys of a wave-uniform key, held in vector registers.  Kernels
// short of scalar registers take the schedule from here; an identity DPP move
// keeps the compiler from folding the values back into scalar registers.
struct PhiloxKeys {
    uint32_t k0[10], k1[10];
};

__device__ __forceinline__ PhiloxKeys philox_keys_v(uint32_t k0, uint32_t k1)
{
    PhiloxKeys ks;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        ks.k0[round] = (uint32_t)__builtin_amdgcn_mov_dpp((int)(k0 + round * 0x9E3779B9u), 0xE4, 0xF, 0xF, false);
        ks.k1[round] = (uint32_t)__builtin_amdgcn_mov_dpp((int)(k1 + round * 0xBB67AE85u), 0xE4, 0xF, 0xF, false);
    }
    return ks;
}

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               const PhiloxKeys& ks)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, ks.k0[round], 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, ks.k1[round], 0x96);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
    }
    return {c0, c1, c2, c3};
}

// A 32-bit draw mapped onto one of q states: floor(w q / 2^32).
__device__ __forceinline__ uint32_t state_of_draw(uint32_t w, uint32_t q) { return __umulhi(w, q); }

// New state of the cluster whose root (smallest site index) is r in sweep t.
__device__ __forceinline__ uint32_t cluster_state(const LatDesc& d, uint32_t r, uint32_t t)
{
    return state_of_draw(philox4x32_10(r, 0u, t, 1u, d.key0, d.key1).x, d.q);
}

// XY lattices (Wolff's embedded clusters): the direction of sweep t, a uint32
// angle of which the top dir_bits are kept (Philox stream 3), and the
// reflection bit of the cluster whose root is r (stream 5, the top bit).
__device__ __forceinline__ uint32_t xy_direction(const LatDesc& d, uint32_t t)
{
    return philox4x32_10(0u, 0u, t, 3u, d.key0, d.key1).x & d.dir_keep;
}

__device__ __forceinline__ uint32_t xy_flip_bit(const LatDesc& d, uint32_t r, uint32_t t)
{
    return philox4x32_10(r, 0u, t, 5u, d.key0, d.key1).x >> 31;
}

// theta -> 2 phi + pi - theta: the reflection across the line perpendicular to
// the direction phi, exact in turn units.
__device__ __forceinline__ uint32_t xy_reflect(uint32_t a, uint32_t phi) { return 2u * phi + 0x80000000u - a; }

// -------------------------------------------------------------- division
// n / L for any 32-bit n by multiply-high (Granlund & Montgomery, PLDI'94,
// unsigned division by an invariant with a 33-bit multiplier).
__device__ __forceinline__ uint32_t div_L(const LatDesc& d, uint32_t n)
{
    if (d.log2L) return n >> d.log2L;
    const uint32_t t = __umulhi(d.magic, n);
    return (t + ((n - t) >> 1)) >> d.shift;
}

// ----------------------------------------------------------- wave helpers
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t popc64(uint64_t v) { return (uint32_t)__popcll(v); }

// ----------------------------------------------------------- global memory
// Pointers read from a descriptor have no known address space; accesses
// through them would compile to flat instructions, which also hold the LDS
// counter and so make every LDS wait cover outstanding global traffic.
// All global accesses go through these casts.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> glb(T* p)
{
    return (gptr<T>)p;
}

// ------------------------------------------------------- coherent access
// Labels are hooked by workgroups on different XCDs while the merge runs, so
// the hook is a device-coherent atomic.
__device__ __forceinline__ uint32_t min_coherent(gptr<uint32_t> p, uint32_t v)
{
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile index of workgroup b when n tiles are spread over the 8 XCDs: workgroups
// are dealt to XCDs round-robin, so XCD x gets a contiguous band of tiles and
// horizontally adjacent tiles run back to back on the same L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n)
{
    const uint32_t q8 = n >> 3, r8 = n & 7u;
    const uint32_t x = b & 7u, k = b >> 3;
    return (x < r8) ? x * (q8 + 1u) + k : r8 * (q8 + 1u) + (x - r8) * q8 + k;
}

}  // namespace swmi
