// Tile-level helpers shared by the sweep kernels of both models (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_device.hpp"

namespace swmi {

// Waves of a tile workgroup: every wave owns 16 rows of a 64- or 128-row tile
// (8 of a 32-row tile), one column per lane.
template <int TY>
constexpr uint32_t waves_of() { return TY == 128 ? 8u : 4u; }
template <int TY>
constexpr uint32_t threads_of() { return 64u * waves_of<TY>(); }

// Value of the neighbouring lane of the pair (lane ^ 1).
__device__ __forceinline__ uint32_t swap_pair(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
}

struct TileGeom {
    uint32_t tx, ty, x0, y0, w, h;
};

__device__ __forceinline__ TileGeom tile_geom(const LatDesc& d, uint32_t tile, uint32_t ty_rows)
{
    TileGeom g;
    // tiles per row: L / 64 for a power-of-two L >= 64 (a shift), else a division
    g.ty = d.log2L >= 6 ? tile >> (d.log2L - 6u) : tile / d.ntx;
    g.tx = tile - g.ty * d.ntx;
    g.x0 = g.tx * TX;
    g.y0 = g.ty * ty_rows;
    g.w = min(TX, d.L - g.x0);
    g.h = min(ty_rows, d.L - g.y0);
    return g;
}

// Which lattice (lat) and tile this workgroup (or wave) works on.  Without a
// map the work is the tiles of lattice 0, optionally spread over the XCDs so
// that each gets a contiguous band of tiles.  Mapped work (many lattices of
// uneven cost) keeps the hardware's round-robin dealing, which balances the
// XCDs better than bands do.
__device__ __forceinline__ bool pick(const LatDesc* descs, const WorkItem* map, uint32_t idx,
                                     bool spread, LatDesc& d, uint32_t& tile, uint32_t& lat)
{
    if (map) {
        const WorkItem it = map[idx];
        if (it.lat == INVALID) return false;
        d = descs[it.lat];
        tile = it.tile;
        lat = it.lat;
        return true;
    }
    lat = 0;
    d = descs[0];
    if (idx >= d.ntiles) return false;
    tile = spread ? xcd_tile(idx, d.ntiles) : idx;
    return true;
}

__device__ __forceinline__ void flag_error(uint32_t* err)
{
    __hip_atomic_fetch_or(glb(err), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Index of this wave in its workgroup as a wave-uniform (scalar) value, for
// kernels where work selected by it (descriptor loads) should stay scalar.
__device__ __forceinline__ uint32_t wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ void atomic_add_i64(int64_t* p, uint64_t v)
{
    __hip_atomic_fetch_add(glb(reinterpret_cast<unsigned long long*>(p)), (unsigned long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ phase clocks
// Profiling builds only (-DSW_PHASE_CLOCKS; the library is then built apart
// from the product one): each wave sums the shader-clock ticks it spends
// between consecutive marks, per phase, and its lane 0 adds the sums and a
// wave count to a per-kernel table of NCOPY rows of PHASES + 1 counters (rows
// picked by workgroup, to spread the atomics).  In every other build the marks
// compile to nothing.
constexpr uint32_t PHASES = 10;
#ifdef SW_PHASE_CLOCKS
struct PhaseClock {
    uint64_t last;
    uint32_t acc[PHASES];
    __device__ PhaseClock() : last(__builtin_amdgcn_s_memtime())
    {
        for (uint32_t i = 0; i < PHASES; ++i) acc[i] = 0;
    }
    __device__ void mark(uint32_t i)
    {
        const uint64_t now = __builtin_amdgcn_s_memtime();
        acc[i] += (uint32_t)(now - last);
        last = now;
    }
    __device__ void flush(unsigned long long* table)
    {
        if ((threadIdx.x & 63u) != 0) return;
        unsigned long long* row = table + (blockIdx.x % NCOPY) * (PHASES + 1);
        for (uint32_t i = 0; i < PHASES; ++i)
            if (acc[i]) atomicAdd(&row[i], (unsigned long long)acc[i]);
        atomicAdd(&row[PHASES], 1ull);
    }
};
#define SW_PHASE_START(pc) PhaseClock pc
#define SW_PHASE(pc, i) pc.mark(i)
#define SW_PHASE_FLUSH(pc, table) pc.flush(table)
#else
#define SW_PHASE_START(pc)
#define SW_PHASE(pc, i) ((void)0)
#define SW_PHASE_FLUSH(pc, table) ((void)0)
#endif

constexpr uint32_t LDS_CAP = 1u << 15;     // cap of union retries in LDS (> sites of a tile)

// ------------------------------------------------------- LDS union-find
// P holds, for every site of the tile (or of a whole lattice of at most
// 128 x 128 sites), an index below 2^15 (16 bits: a tile has at most 2^13
// sites, such a lattice 2^14) that is never larger than its own; roots point
// at themselves.  Entries only ever decrease (unions hook the larger root under
// the smaller one with a minimum; finds point nodes at their grandparents),
// so every walk that steps only to smaller indices ends.  A walk that stops at
// a node pointing to a larger index has met a corrupted forest and sets `bad`,
// which the kernel reports.  16-bit entries halve the forest's LDS, so more
// workgroups fit a CU; the minimum (there is no 16-bit LDS minimum) is a
// compare-and-swap on the entry's 32-bit word.
__device__ __forceinline__ uint32_t lds_ld(uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t lds_ld(uint16_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint16_t* p, uint32_t v)
{
    __hip_atomic_store(p, (uint16_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// min(P[i], v) into entry i; returns the entry's value before.
__device__ __forceinline__ uint32_t lds_min16(uint16_t* P, uint32_t i, uint32_t v, bool& bad)
{
    uint32_t* const w = reinterpret_cast<uint32_t*>(P) + (i >> 1);
    const uint32_t sh = (i & 1u) * 16u;
    uint32_t cur = lds_ld(w);
    for (uint32_t it = 0; it < LDS_CAP; ++it) {
        const uint32_t old = (cur >> sh) & 0xFFFFu;
        if (old <= v) return old;
        const uint32_t seen = atomicCAS(w, cur, (cur & ~(0xFFFFu << sh)) | (v << sh));
        if (seen == cur) return old;
        cur = seen;
    }
    bad = true;
    return v;
}

// Roots of a and b while unions may still run, both walked in the same loop
// so that their LDS round trips overlap, with path splitting: every visited
// node is pointed at its grandparent (a stored value is always an ancestor,
// so races with other finds and hooks are benign).
__device__ __forceinline__ void lds_find2(uint16_t* P, uint32_t& a, uint32_t& b, bool& bad)
{
    uint32_t pa = lds_ld(&P[a]), pb = lds_ld(&P[b]);
    while (pa < a || pb < b) {
        const bool sa = pa < a, sb = pb < b;
        const uint32_t ga = sa ? lds_ld(&P[pa]) : pa;
        const uint32_t gb = sb ? lds_ld(&P[pb]) : pb;
        if (sa) {
            lds_st(&P[a], ga);
            a = pa;
            pa = ga;
        }
        if (sb) {
            lds_st(&P[b], gb);
            b = pb;
            pb = gb;
        }
    }
    bad |= pa != a || pb != b;
}

__device__ void lds_union(uint16_t* P, uint32_t a, uint32_t b, bool& bad)
{
    for (uint32_t it = 0; it < LDS_CAP; ++it) {
        lds_find2(P, a, b, bad);
        if (a == b) return;
        const uint32_t hi = max(a, b), lo = min(a, b);
        const uint32_t old = lds_min16(P, hi, lo, bad);
        if (old == hi) return;
        // hi was hooked meanwhile: join its new parent with lo instead
        a = old;
        b = lo;
    }
    bad = true;
}

}  // namespace swmi
