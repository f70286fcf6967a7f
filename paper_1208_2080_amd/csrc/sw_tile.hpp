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

struct TileGeom {
    uint32_t tx, ty, x0, y0, w, h;
};

__device__ __forceinline__ TileGeom tile_geom(const LatDesc& d, uint32_t tile, uint32_t ty_rows)
{
    TileGeom g;
    g.ty = tile / d.ntx;
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

}  // namespace swmi
