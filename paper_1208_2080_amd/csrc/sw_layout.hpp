// Data layout of one lattice in device memory, shared by kernels and host runtime.
//
// Per lattice (site i = y*L + x, row-major; tiles of TX = 64 columns by TY
// rows, numbered row-major; a site's tile-local index is r*TX + c for row r,
// column c of its tile):
//   spins   uint8  [N]        Potts states; for an XY lattice uint32 [N]
//                             angles instead (unit: 2^-32 of a full turn)
//   labels  4N bytes:
//     tile labels  uint16 [N] at byte offset 2N, written by the labelling and
//                             read by the flip: per site, the tile-local index
//                             of a smaller site of its tile-local cluster (its
//                             union-find grandparent in the tile), or, for the
//                             cluster's smallest site (its tile-local root),
//                             ROOT16 | slot, slot the root's node in the tile's
//                             edge forest, NOSLOT if the cluster touches no
//                             tile edge
//     resolved     uint32 from byte 0: smallest site indices of the clusters,
//                             for label reads (at most N/2 sites at a time, so
//                             the tile labels stay intact); a lattice swept
//                             whole in LDS writes all N of them here instead
//   bonds   uint64 [tiles][2][TY]  tile-major bond words: tile t, plane p (0: +x,
//                             1: +y), row r; bit x = bond of site (x0 + x, y0 + r)
//   edges   uint32 [tiles][edge_words(TY)]  per-tile boundary record (below)
//   nodes   uint64 [tiles][nslot(TY)]  the edge forest: one node per tile-local
//                             cluster that touches a tile edge, numbered by its
//                             smallest site within the tile; a node's word is
//                             (smallest site index of its parent << 32) | parent
//                             node id, a root's parent being itself, so the
//                             forest's roots are the clusters' smallest sites
//   ring    int64  [slots][NCOPY][ring_stride(q)]  per-sweep sums: n_unsat,
//                             n_active, n_1..n_{q-1} (n_0 = N - the rest);
//                             an XY lattice's records are XY_WORDS long
//                             NCOPY partial copies, each on cache lines of its
//                             own, spread the workgroups' atomics
//   obs     int64  [slots][q + 1]  staging for reads: the NCOPY partial copies of
//                             the records being read, summed on the device
//   state   DevState          sweep counter and error flag
// TY = 32, 64 or 128.
#pragma once

#include <stdint.h>

namespace swmi {

constexpr uint32_t TX = 64;           // tile width: one wave, one column per lane
constexpr uint32_t NCOPY = 64;        // partial copies of each ring record
constexpr uint32_t NOSLOT = 0x7FFFu;       // root of a cluster inside its tile
constexpr uint32_t ROOT16 = 0x8000u;       // tile-local root's tag in 16-bit entries and tile labels
constexpr uint32_t INVALID = 0xFFFFFFFFu;
constexpr uint32_t WHOLE_LMAX = 128;       // largest L swept whole in one workgroup's LDS

// Boundary record of a tile with TY rows: 8 uint32 words, then uint16 slots
// (edge-forest nodes of the tile-local roots) of its edge sites:
//   words [0, 4)      right-edge crossing bonds, bit r = +x bond of (w-1, r)
//   words [4, 6)      bottom-edge crossing bonds, bit x = +y bond of (x, h-1)
//   words [6, 8)      unused
//   slots [0, TY)           right column, by row
//   slots [TY, 2TY)         left column, by row
//   slots [2TY, 2TY+TX)     bottom row, by column
//   slots [2TY+TX, 2TY+2TX) top row, by column
__host__ __device__ constexpr uint32_t edge_words(uint32_t ty) { return 8u + ty + TX; }

// Nodes of a tile's edge forest: at most one per edge site.
__host__ __device__ constexpr uint32_t nslot(uint32_t ty) { return 2u * TX + 2u * ty; }

// Words of a ring record: n_unsat, n_active, n_1..n_{q-1} (q + 1 sums), then
// the cluster-size sums of the sweep's clusters, sum |C|^2 and sum |C|^4 (the
// latter 128 bits: low word, high word), kept in partial copy 0 only.
__host__ __device__ constexpr uint32_t ring_words(uint32_t q) { return q + 4u; }
__host__ __device__ constexpr uint32_t cs_word(uint32_t q) { return q + 1u; }

// int64 words between partial copies of a ring record: the record and one
// more word (the whole-record flag below) rounded up to whole 256-byte blocks,
// so no two copies share a cache line.
__host__ __device__ constexpr uint32_t ring_stride(uint32_t q) { return (ring_words(q) + 1u + 31u) & ~31u; }

// Word ring_words(q) (XY_WORDS for an XY record) of partial copy 0 is the
// whole-record flag: nonzero when copy 0 holds the complete record (written by
// the workgroup that sweeps a whole lattice), so the other copies, which may
// hold stale sums of an older use of the slot, are not added.  Clearing a
// record clears the flag with it.

// Ring record of an XY lattice: n_active, then the sums over sites of
// cos(theta_i - theta_{i+x}), cos(theta_i - theta_{i+y}), sin of the same two
// differences, cos theta_i and sin theta_i, each term rounded to a multiple of
// 2^-30 (so the sums are exact integers, whatever the order of addition).
constexpr uint32_t XY_WORDS = 7;
constexpr uint32_t XY_STRIDE = (XY_WORDS + 1u + 31u) & ~31u;

struct DevState {
    uint32_t err;          // nonzero: a safety cap tripped
    uint32_t counter;      // sweeps done (plain lattice)
    uint32_t pad[62];
};

struct LatDesc {
    uint8_t* s;
    uint32_t* lab;         // resolved labels (base of the label region)
    uint16_t* tlab;        // tile labels (upper half of the label region)
    uint64_t* bonds;
    uint32_t* edges;
    uint64_t* nodes;       // edge forest, nslot(TY) words per tile
    uint64_t* csize;       // cluster sizes gathered at edge-forest roots (null: no cluster sums)
    int64_t* ring;
    int64_t* obs;          // staging of summed ring records (reads only)
    uint32_t* counter;     // sweeps done
    uint32_t* err;         // -> DevState::err
    uint32_t L, q, W;
    uint32_t ntx, nty, ntiles;
    uint32_t cap;          // ring capacity in sweeps (0 = no measurement)
    uint32_t thr_m1;       // threshold - 1 (bond active iff draw <= thr_m1 and thr_nz)
    uint32_t thr_nz;       // threshold != 0
    uint32_t key0, key1;
    uint32_t magic, shift; // division by L
    uint32_t log2L;        // log2 L when L is a power of two, else 0
    // XY lattices (null / zero for Potts)
    uint32_t* ang;         // angles, uint32 [N]
    double k2;             // 2K (may be +inf)
    uint32_t dir_keep;     // bits of the direction draw kept (the top dir_bits)
    uint32_t xy;           // 1: an XY lattice
};

// Block-to-work map entry of the batched form: lattice index and tile index.
struct WorkItem {
    uint32_t lat, tile;
};

}  // namespace swmi
