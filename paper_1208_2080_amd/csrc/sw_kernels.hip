// HIP kernels of one Swendsen-Wang sweep for gfx950, plus their launchers.
//
// One sweep is three launches over the tiles of the lattice (TX = 64 columns
// by TY rows; one workgroup per tile, four waves, eight for 128 rows; one
// column per lane):
//   k_bond_label  bonds (Sec. 2 step (1)) + tile-local cluster labelling
//                 + measurement of the configuration the bonds were drawn on
//   k_merge       joins tile-local clusters across tile edges (global union-find
//                 with atomicMin, larger root under smaller)
//   k_flip        every cluster takes the state drawn for its smallest site
//                 index (Sec. 2 step (3)); each site follows its in-tile
//                 pointers to a resolved tile-local root
// plus k_measure after the last sweep of a call, and small helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "sw_device.hpp"
#include "sw_kernels.hpp"

namespace swmi {

namespace {

// Every label points at a site index no larger than its own (roots at
// themselves).  Every pointer walk steps only to strictly smaller indices, so
// it ends even in a corrupted forest, and union retries carry caps; a forest
// that breaks the invariant sets the error flag instead of spinning.
constexpr uint32_t LDS_CAP = 1u << 15;     // cap of union retries in LDS (> sites of a tile)
constexpr uint32_t UNITE_CAP = 1u << 12;   // cap of union retries in the global forest
constexpr uint32_t SPW = TX + 4;           // LDS row stride of staged spins (bytes)

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

// Lane l's bit of a wave-uniform mask, as a lane predicate.
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Index of this wave in its workgroup as a wave-uniform (scalar) value, for
// kernels where work selected by it (descriptor loads) should stay scalar.
__device__ __forceinline__ uint32_t wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Sum over the wave of a per-lane value below 2^BITS, bit plane by bit plane
// (one ballot per plane: cheaper than 64 atomics on one LDS word).
template <int BITS>
__device__ __forceinline__ uint32_t wave_sum_small(uint32_t v)
{
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < BITS; ++k) s += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64((v >> k) & 1u)) << k;
    return s;
}

// Number of set bits of a wave-uniform mask below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Value of the neighbouring lane of the pair (lane ^ 1).
__device__ __forceinline__ uint32_t swap_pair(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
}

// ------------------------------------------------------- LDS union-find
// P holds, for every site of the tile (tile-local index), a label that is never
// larger than itself; roots point at themselves.  Entries only ever decrease
// (unions hook the larger root under the smaller one with atomicMin; finds
// point nodes at their grandparents), so every walk that steps only to
// smaller indices ends.  A walk that stops at a node pointing to a larger
// index has met a corrupted forest and sets `bad`, which the kernel reports.
__device__ __forceinline__ uint32_t lds_ld(uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x while unions may still run, with path splitting: every visited
// node is pointed at its grandparent (a stored value is always an ancestor,
// so races with other finds and hooks are benign).
__device__ __forceinline__ uint32_t lds_find(uint32_t* P, uint32_t x, bool& bad)
{
    uint32_t p = lds_ld(&P[x]);
    while (p < x) {
        const uint32_t gp = lds_ld(&P[p]);
        lds_st(&P[x], gp);
        x = p;
        p = gp;
    }
    bad |= p != x;
    return x;
}

// Root of x once the forest no longer changes (no writes).  The first two
// steps are taken without a branch (a root reads itself again), which covers
// most sites; only deeper chains enter the loop.
__device__ __forceinline__ uint32_t lds_root(const uint32_t* P, uint32_t x, bool& bad)
{
    uint32_t p = P[x];
    x = min(p, x);
    p = P[x];
    while (p < x) {
        x = p;
        p = P[x];
    }
    bad |= p != x;
    return x;
}

__device__ void lds_union(uint32_t* P, uint32_t a, uint32_t b, bool& bad)
{
    for (uint32_t it = 0; it < LDS_CAP; ++it) {
        a = lds_find(P, a, bad);
        b = lds_find(P, b, bad);
        if (a == b) return;
        const uint32_t hi = max(a, b), lo = min(a, b);
        const uint32_t old = __hip_atomic_fetch_min(&P[hi], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == hi) return;
        // hi was hooked meanwhile: join its new parent with lo instead
        a = old;
        b = lo;
    }
    bad = true;
}

// ---------------------------------------------------- global union-find
// The finds read through the caches.  A stale value is a parent the node had
// earlier, still a smaller index in the same cluster, so chases still end and
// only ever reach true ancestors or stale roots; the hook itself is a
// device-coherent atomicMin that returns the current parent, and a hook on a
// stale root retries from that value.  Hence the forest stays exact.  As in
// the LDS forest, walks step only to smaller indices (so they end and stay in
// bounds) and a stop at a larger index sets `bad`.

// Root of x with path splitting (every visited node is pointed at its
// grandparent; any stored value is an ancestor, so races are benign).
__device__ uint32_t g_find(gptr<uint32_t> lab, uint32_t x, bool& bad)
{
    uint32_t p = lab[x];
    while (p < x) {
        const uint32_t gp = lab[p];
        if (gp < p) lab[x] = gp;   // only a real shortcut is worth a store
        x = p;
        p = gp;
    }
    bad |= p != x;
    return x;
}

__device__ void g_unite(gptr<uint32_t> lab, uint64_t N, uint32_t a, uint32_t b, bool& bad)
{
    if (a >= N || b >= N) {
        bad = true;
        return;
    }
    for (uint32_t it = 0; it < UNITE_CAP; ++it) {
        a = g_find(lab, a, bad);
        b = g_find(lab, b, bad);
        if (a == b) return;
        const uint32_t hi = max(a, b), lo = min(a, b);
        const uint32_t old = min_coherent(lab + hi, lo);
        if (old == hi) return;
        // hi was hooked meanwhile: join its new parent with lo instead
        a = old;
        b = lo;
    }
    bad = true;
}

// Read-only root search once the forest is final (after the merge kernel).
__device__ uint32_t g_root(gptr<uint32_t> lab, uint32_t x, bool& bad)
{
    uint32_t p = lab[x];
    while (p < x) {
        x = p;
        p = lab[x];
    }
    bad |= p != x;
    return x;
}

// ------------------------------------------------------------ spin staging
// Spins of a tile and its halo in LDS: rows 0..h (row h is the row below the
// tile, periodic), columns 0..w-1 plus column w = the column right of the tile
// (periodic).  Row stride SPW bytes.
template <int TY>
__device__ __forceinline__ void stage_spins(uint8_t* sp, const LatDesc& d, const TileGeom& g, uint32_t tid)
{
    constexpr uint32_t NT = threads_of<TY>();
    const uint32_t L = d.L, w = g.w, h = g.h;
    const uint32_t yb = (g.y0 + h == L) ? 0u : g.y0 + h;          // row below the tile
    const uint32_t xh = (g.x0 + w == L) ? 0u : g.x0 + w;          // column right of the tile
    if ((L & 3u) == 0) {
        // rows start 4-byte aligned (w is then a multiple of 4): NT / 16 rows per pass
        const uint32_t c = tid & 15u, dw = w >> 2;
#pragma unroll
        for (uint32_t rr = 0; rr <= (uint32_t)TY; rr += NT / 16) {
            const uint32_t r = rr + (tid >> 4);
            if (r <= h && c < dw) {
                const uint32_t y = (r < h) ? g.y0 + r : yb;
                const uint32_t v = *reinterpret_cast<gptr<const uint32_t>>(glb(d.s) + (size_t)y * L + g.x0 + 4 * c);
                *reinterpret_cast<uint32_t*>(sp + r * SPW + 4 * c) = v;
            }
        }
    } else {
        const uint32_t c = tid & 63u;
#pragma unroll 4
        for (uint32_t rr = 0; rr <= (uint32_t)TY; rr += NT / 64) {
            const uint32_t r = rr + (tid >> 6);
            if (r <= h && c < w) {
                const uint32_t y = (r < h) ? g.y0 + r : yb;
                sp[r * SPW + c] = glb(d.s)[(size_t)y * L + g.x0 + c];
            }
        }
    }
    for (uint32_t r = tid; r <= h; r += NT) {
        const uint32_t y = (r < h) ? g.y0 + r : yb;
        sp[r * SPW + w] = glb(d.s)[(size_t)y * L + xh];
    }
}

// Per-lane state counters of the measurement for q <= 16: byte (c & 7) of word
// (c >> 3) counts this lane's sites in state c (at most 31 rows per lane).
// q <= 8 needs only the first word (count_state_byte).
__device__ __forceinline__ void count_state_byte(uint64_t (&w)[2], bool valid, uint32_t s)
{
    w[0] += (uint64_t)valid << (8u * (s & 7u));
}

__device__ __forceinline__ void count_state_bytes(uint64_t (&w)[2], bool valid, uint32_t s)
{
    const uint64_t one = (uint64_t)valid << (8u * (s & 7u));
    w[0] += (s < 8u) ? one : 0ull;
    w[1] += (s < 8u) ? 0ull : one;
}

// Wave totals of states 1..q-1 from the per-lane bytes, added into hist.
__device__ __forceinline__ void flush_state_bytes(const uint64_t (&w)[2], uint32_t* hist, uint32_t q, uint32_t lane)
{
    for (uint32_t c = 1; c < q; ++c) {
        const uint32_t n = wave_sum_small<5>((uint32_t)(w[c >> 3] >> (8u * (c & 7u))) & 0xFFu);
        if (lane == 0 && n) atomicAdd(&hist[c], n);
    }
}

// Sites of one row in each state c >= 1 for q > 16, straight into hist.
__device__ __forceinline__ void count_states(uint32_t* hist, bool valid, uint32_t s)
{
    if (valid && s) atomicAdd(&hist[s], 1u);
}

// Add a workgroup's measurement into a ring record (NCOPY partial copies).
__device__ __forceinline__ int64_t* ring_record(const LatDesc& d, uint32_t sweep, uint32_t copy)
{
    return d.ring + ((size_t)(sweep % d.cap) * NCOPY + copy) * ring_stride(d.q);   // cast at the access
}

__device__ __forceinline__ void atomic_add_i64(int64_t* p, uint64_t v)
{
    __hip_atomic_fetch_add(glb(reinterpret_cast<unsigned long long*>(p)), (unsigned long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Per-wave queue of pending unions (pairs of provisional labels, 16 bits
// each).  Row labelling never reads the union-find, so unions can wait and
// then run with every lane busy instead of one lane of a diverged wave.
// Union queue slots per wave (a two-row step queues at most 128); a little
// smaller for 128-row tiles so that three of their workgroups fit a CU's LDS.
template <int TY>
constexpr uint32_t qcap_of() { return TY == 128 ? 224u : 256u; }

struct UnionQueue {
    uint32_t* q;       // the wave's slots in LDS
    uint32_t* trash;   // an LDS word for lanes with nothing to store
    uint32_t n;        // wave-uniform fill
};

// Run the queued unions, one per lane.
__device__ __forceinline__ void drain(UnionQueue& uq, uint32_t* P, uint32_t lane, bool& bad)
{
    for (uint32_t j = lane; j < uq.n; j += 64) {
        const uint32_t e = lds_ld(&uq.q[j]);
        lds_union(P, e & 0xFFFFu, e >> 16, bad);
    }
    uq.n = 0;
}

// Queue the unions (a, b) of the lanes in `mask` where a != b (at most 64; the
// caller keeps at least 64 slots free).  The other lanes store to a scratch
// word instead of branching around the store.
__device__ __forceinline__ void enqueue(UnionQueue& uq, uint64_t mask, uint32_t a, uint32_t b)
{
    const uint64_t m = ballot(a != b) & mask;
    if (!m) return;
    lds_st(lane_in(m) ? &uq.q[uq.n + lanes_below(m)] : uq.trash, a | (b << 16));
    uq.n = __builtin_amdgcn_readfirstlane(uq.n + popc64(m));
}

// Provisional labels of one tile row, Hoshen-Kopelman style.  hx: +x bonds
// inside the tile; V: +y bonds from the row above (0 on a strip's first row);
// lp: this lane's label of the row above.  Every run of +x bonds takes one
// label: the label above one of its +y bonds, or, with none, its first site
// (a new root).  The runs are numbered by their first sites, and one LDS slot
// per run carries the choice to all its sites.  Any further +y bond into the
// run from a differently labelled site queues a union.  Every site's own
// union-find entry points at its label (itself for a new root), so the forest
// spans all sites and no separate array of provisional labels is kept.
__device__ __forceinline__ uint32_t row_labels(uint32_t* P, uint32_t* rl, UnionQueue& uq, uint32_t r, uint32_t x,
                                               uint64_t validm, uint64_t hx, uint64_t V, uint64_t hprev, uint32_t lp)
{
    const uint64_t C = hx << 1;                 // bit x: bond (x-1) -> x
    const uint64_t S = ~C & validm;             // first sites of runs
    const uint32_t ri = lanes_below(S >> 1);    // number of run starts in 1..x = run index of x
    const uint32_t fresh = r * TX + x;
    // lanes talk through the slots, so these accesses must not be folded away;
    // a run's first site offers itself and every +y bond offers the label
    // above, in one store: any offer may win (unions below cover the rest)
    const bool vb = lane_in(V);
    lds_st(lane_in(S | V) ? &rl[ri] : &rl[64], vb ? lp : fresh);
    const uint32_t lab = lds_ld(&rl[ri]);
    lds_st(&P[fresh], lab);   // columns outside the tile write entries no one reads
    // bonds x-1 and x from the same run above into the same run here add nothing
    const uint64_t R = V & (V << 1) & C & (hprev << 1);
    enqueue(uq, V & ~R, lp, lab);
    return lab;
}

}  // namespace

// ---------------------------------------------------------------------------
// Bonds + tile-local labels (+ measurement of the incoming configuration).
//
// Each wave owns a strip of TY/4 consecutive rows and labels it two rows at a
// time; strips are then stitched along their seams through the same LDS
// union-find, which always hangs the larger label under the smaller, so the
// final label of every tile-local cluster is its smallest site.
//
// Random words: with L even, one Philox call serves the pair of sites
// (2m, 2m+1) of one row; lane 2m draws for row r and lane 2m+1 for row r+1,
// and the two lanes swap the halves the other one needs.
//
// flags bit 0: also measure the configuration the bonds are drawn on (the
// result of the previous sweep, t - 1).
template <int TY>
__global__ __launch_bounds__(threads_of<TY>()) void k_bond_label(const LatDesc* descs, const WorkItem* map, uint32_t k,
                                                   uint32_t flags)
{
    constexpr uint32_t NW = waves_of<TY>(), NT = threads_of<TY>();
    constexpr uint32_t RPW = TY / NW;  // rows per wave (even)
    static_assert(RPW < 32, "per-lane measurement counters hold at most 31 rows");
    constexpr uint32_t QCAP = qcap_of<TY>();
    __shared__ uint32_t P[TY * TX];    // union-find over the tile's sites
    __shared__ __align__(16) uint8_t sp[(TY + 1) * SPW];
    __shared__ uint64_t rb[TY][2];     // per row: +x bond word, +y bond word
    // per wave: the label of every run of a row; once a wave has left its
    // strip, its row holds the labels of the strip's last row (the seam)
    __shared__ uint32_t RL[NW][65];    // [64]: scratch word of lanes with nothing to store
    __shared__ uint32_t UQT[NW];       // scratch words of the union queues
    uint32_t(*const seam)[65] = RL;
    __shared__ uint32_t UQ[NW][QCAP];  // per wave: pending unions
    __shared__ uint32_t hist[256];
    __shared__ uint32_t tot[2];

    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, blockIdx.x, true, d, tile, lat)) return;
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *glb(d.counter) + k;
    const bool meas = d.cap != 0;
    const bool meas_prev = meas && (flags & 1u);
    const uint32_t tid = threadIdx.x, wave = wave_id(), lane = tid & 63u;
    const uint32_t L = d.L, w = g.w, h = g.h, x0 = g.x0, y0 = g.y0;

    if (tid < 256) hist[tid] = 0;
    if (tid < 2) tot[tid] = 0;
    stage_spins<TY>(sp, d, g, tid);
    __syncthreads();

    const uint32_t x = lane;
    const bool vx = x < w;
    const uint64_t validm = (w == 64) ? ~0ull : ((1ull << w) - 1ull);
    const uint64_t cross = 1ull << (w - 1);   // the +x bond of column w-1 leaves the tile
    const uint32_t r0 = wave * RPW, r1 = min(h, r0 + RPW);
    const uint64_t bondm = d.thr_nz ? validm : 0ull;   // K = 0: no bond at all
    const bool even_L = (L & 1u) == 0;
    const bool q2 = d.q == 2;
    uint32_t* rl = RL[wave];
    UnionQueue uq{UQ[wave], &UQT[wave], 0u};
    // measurement: equal-spin pairs counted per wave (scalar), q = 2 spins
    // summed per lane (column), active bonds counted from the bond words
    uint32_t n_eq = 0, ones = 0;
    // q <= 16: each lane counts its sites in states 1..q-1 in the bytes of two
    // 64-bit words (at most 16 rows per lane, so no byte overflows)
    const bool q8 = !q2 && d.q <= 8, q16 = !q2 && d.q <= 16;
    uint64_t packed[2] = {0ull, 0ull};
    const uint32_t vbyte = vx ? 0xFFu : 0u;
    uint32_t lp = 0;
    const PhiloxKeys ks = philox_keys_v(d.key0, d.key1);
    bool bad = false;   // this lane met a corrupted forest
    uint64_t hprev = 0, vprev = 0;

    // The row loop, compiled twice: the q = 9..16 counters (two words per lane)
    // stay out of the common instantiation, whose code they would otherwise
    // perturb.
    auto strip_rows = [&](auto wide) {
        constexpr bool WIDE = decltype(wide)::value;
        for (uint32_t r = r0; r < r1; r += 2) {
            const bool two = r + 1 < r1;
            if (uq.n > QCAP - 128) drain(uq, P, lane, bad);
            const uint8_t* row = sp + r * SPW;
            const uint32_t s0 = row[x], s0r = row[x + 1];
            const uint32_t s1 = row[SPW + x], s1r = row[SPW + x + 1];
            const uint32_t s2 = two ? row[2 * SPW + x] : 0u;

            // Site indices in 32 bits: exact for every row of the lattice (N <= 2^32);
            // a draw for row r+1 past the last row wraps but is never used.
            const uint32_t base0 = (y0 + r) * L + x0;
            uint32_t wx0, wy0, wx1, wy1;
            if (even_L) {
                const bool odd = x & 1u;
                const uint32_t pair = ((odd ? base0 + L : base0) + (x & ~1u)) >> 1;
                const u32x4 q4 = philox4x32_10(pair, 0u, t, 0u, ks);
                const uint32_t recv0 = swap_pair(odd ? q4.x : q4.z);
                const uint32_t recv1 = swap_pair(odd ? q4.y : q4.w);
                wx0 = odd ? recv0 : q4.x;
                wy0 = odd ? recv1 : q4.y;
                wx1 = odd ? q4.z : recv0;
                wy1 = odd ? q4.w : recv1;
            } else {
                const uint32_t ga = base0 + x, gb = base0 + L + x;
                const u32x4 qa = philox4x32_10(ga >> 1, 0u, t, 0u, ks);
                const u32x4 qb = philox4x32_10(gb >> 1, 0u, t, 0u, ks);
                wx0 = (ga & 1u) ? qa.z : qa.x;
                wy0 = (ga & 1u) ? qa.w : qa.y;
                wx1 = (gb & 1u) ? qb.z : qb.x;
                wy1 = (gb & 1u) ? qb.w : qb.y;
            }
            // equal-spin masks and draw masks as wave ballots; a bond needs both
            const uint64_t EX0 = ballot(s0 == s0r) & validm, EY0 = ballot(s0 == s1) & validm;
            const uint64_t BX0 = EX0 & ballot(wx0 <= d.thr_m1) & bondm;
            const uint64_t BY0 = EY0 & ballot(wy0 <= d.thr_m1) & bondm;
            uint64_t EX1 = 0, EY1 = 0, BX1 = 0, BY1 = 0;
            if (two) {
                EX1 = ballot(s1 == s1r) & validm;
                EY1 = ballot(s1 == s2) & validm;
                BX1 = EX1 & ballot(wx1 <= d.thr_m1) & bondm;
                BY1 = EY1 & ballot(wy1 <= d.thr_m1) & bondm;
            }
            if (lane == 0) {
                rb[r][0] = BX0;
                rb[r][1] = BY0;
                if (two) {
                    rb[r + 1][0] = BX1;
                    rb[r + 1][1] = BY1;
                }
            }

            const uint64_t hx0 = BX0 & ~cross;
            const uint32_t lab0 = row_labels(P, rl, uq, r, x, validm, hx0, vprev, hprev, lp);
            lp = lab0;
            hprev = hx0;
            vprev = BY0;
            if (two) {
                const uint64_t hx1 = BX1 & ~cross;
                const uint32_t lab1 = row_labels(P, rl, uq, r + 1, x, validm, hx1, vprev, hprev, lp);
                lp = lab1;
                hprev = hx1;
                vprev = BY1;
            }

            if (meas_prev) {
                n_eq += popc64(EX0) + popc64(EY0) + popc64(EX1) + popc64(EY1);   // EX1, EY1 are 0 without row r+1
                if (q2) ones += (s0 & vbyte) + (s1 & (two ? vbyte : 0u));
                else if (q8) {
                    // (lanes outside the tile add nothing; their bytes may be stale)
                    count_state_byte(packed, vx, s0);
                    count_state_byte(packed, vx && two, s1);
                } else if (WIDE) {
                    count_state_bytes(packed, vx, s0 & 15u);
                    count_state_bytes(packed, vx && two, s1 & 15u);
                } else {
                    count_states(hist, vx, s0);
                    if (two) count_states(hist, vx, s1);
                }
            }
        }
    };
    if (q16 && !q8) strip_rows(std::true_type{});
    else strip_rows(std::false_type{});
    seam[wave][lane] = lp;
    if (meas_prev) {
        // every site of the strip owns two bonds
        if (lane == 0 && r0 < r1) atomicAdd(&tot[0], 2u * w * (r1 - r0) - n_eq);
        if (q2) {
            const uint32_t n1 = wave_sum_small<6>(ones);   // a lane counts at most TY / 4 <= 32 rows
            if (lane == 0 && n1) atomicAdd(&hist[1], n1);
        }
        if (q16) flush_state_bytes(packed, hist, d.q, lane);
    }
    __syncthreads();

    // Seams: +y bonds from the last row of the strip above into this strip.
    if (wave > 0 && r0 < h) {
        const uint32_t ru = r0 - 1;
        const uint64_t V = rb[ru][1];
        const uint64_t hu = rb[ru][0] & ~cross, hc = rb[r0][0] & ~cross;
        const uint64_t R = V & (V << 1) & (hc << 1) & (hu << 1);
        const uint32_t up = seam[wave - 1][lane];
        // the site's entry is its label or, after path halving, an ancestor of it
        const uint32_t first_prov = lds_ld(&P[r0 * TX + x]);
        if (uq.n > QCAP - 64) drain(uq, P, lane, bad);
        enqueue(uq, V & ~R, up, first_prov);
    }
    drain(uq, P, lane, bad);

    // Tile record: bond words (tile-major), crossing-bond masks.
    gptr<uint32_t> rec = glb(d.edges) + (size_t)tile * edge_words(TY);
    gptr<uint64_t> bw = glb(d.bonds) + (size_t)tile * 2 * TY;
    for (uint32_t j0 = 0; j0 < 2 * TY; j0 += NT) {
        const uint32_t j = j0 + tid, r = j % TY;
        const uint64_t word = (j < 2 * TY && r < h) ? rb[r][j / TY] : 0ull;
        if (j < 2 * TY && r < h) bw[j] = word;
        if (meas) {
            const uint32_t n = wave_sum_small<7>(popc64(word));   // active bonds
            if (lane == 0 && n) atomicAdd(&tot[1], n);
        }
    }
    if (wave == 0) {
        for (uint32_t j = 0; j < TY; j += 64) {
            const uint32_t r = j + lane;
            const bool bit = r < h && ((rb[r][0] >> (w - 1)) & 1ull);
            const uint64_t m = ballot(bit);
            if (lane == 0) {
                rec[j / 32] = (uint32_t)m;
                rec[j / 32 + 1] = (uint32_t)(m >> 32);
            }
        }
        if (lane == 0) {
            if (TY < 128) {
                rec[2] = 0;
                rec[3] = 0;
            }
            const uint64_t b = rb[h - 1][1];
            rec[4] = (uint32_t)b;
            rec[5] = (uint32_t)(b >> 32);
        }
    }
    __syncthreads();

    // Labels out: every site gets its union-find grandparent as a global site
    // index (a smaller site of its tile-local cluster, or itself for the
    // tile-local root); the flip follows these pointers inside the tile.  Entries of
    // columns outside the tile are never stored (full-width tiles, the common
    // case, need no mask at all).
    // a site index fits 32 bits (N <= 2^32) and y, L fit 24 bits
    auto global_index = [&](uint32_t la) { return __umul24(y0 + la / TX, L) + x0 + la % TX; };
    auto parents_out = [&](auto full) {
        constexpr bool FULL = decltype(full)::value;
        const bool vs = FULL || vx;
        for (uint32_t r = r0; r < r1; ++r) {
            // the grandparent: one more read here saves the flip a longer walk
            const uint32_t ga = global_index(P[P[r * TX + x]]);
            const gptr<uint32_t> lrow = glb(d.lab) + (size_t)(y0 + r) * L + x0;
            if (vs) lrow[x] = ga;
        }
    };
    if (w == TX && r1 - r0 == RPW) {
        // a full strip: all parent reads first, then all grandparent reads, so
        // the LDS round trips overlap; the stores go out from the strip's
        // (wave-uniform) base with 32-bit per-lane offsets
        uint32_t p[RPW];
#pragma unroll
        for (uint32_t k = 0; k < RPW; ++k) p[k] = P[(r0 + k) * TX + x];
#pragma unroll
        for (uint32_t k = 0; k < RPW; ++k) p[k] = P[p[k]];
        const gptr<char> strip = (gptr<char>)(glb(d.lab) + (size_t)(y0 + r0) * L + x0);
#pragma unroll
        for (uint32_t k = 0; k < RPW; ++k) *(gptr<uint32_t>)(strip + (k * L + x) * 4u) = global_index(p[k]);
    } else if (w == TX) {
        parents_out(std::true_type{});
    } else {
        parents_out(std::false_type{});
    }
    // The tile's edges for the merge carry tile-local roots: lane i walks the
    // left and right sites of strip row i; the first and last strips walk the
    // top and bottom rows.
    if (r0 < r1 && lane < r1 - r0) {
        const uint32_t r = r0 + lane;
        rec[8 + r] = global_index(lds_root(P, r * TX + w - 1, bad));
        rec[8 + TY + r] = global_index(lds_root(P, r * TX, bad));
    }
    if (r0 == 0 && r0 < r1 && vx) rec[8 + 2 * TY + TX + x] = global_index(lds_root(P, x, bad));   // top row
    if (r1 == h && r0 < r1 && vx) rec[8 + 2 * TY + x] = global_index(lds_root(P, (h - 1) * TX + x, bad));   // bottom
    if (bad) flag_error(d.err);

    if (meas) {
        const uint32_t copy = blockIdx.x % NCOPY;
        if (tid == 0) atomic_add_i64(&ring_record(d, t, copy)[1], tot[1]);
        if (meas_prev) {
            int64_t* rp = ring_record(d, t - 1, copy);
            if (tid == 0) atomic_add_i64(&rp[0], tot[0]);
            if (tid >= 1 && tid < d.q && hist[tid]) atomic_add_i64(&rp[1 + tid], hist[tid]);
        }
    }
}

// ---------------------------------------------------------------------------
// Join tile-local clusters across tile edges.  One wave per tile handles the
// crossing bonds of its right and bottom edges (periodic neighbours).
template <int TY>
__global__ __launch_bounds__(256) void k_merge(const LatDesc* descs, const WorkItem* map, uint32_t nitems)
{
    const uint32_t wave = wave_id(), lane = threadIdx.x & 63u;
    const uint32_t idx = blockIdx.x * 4 + wave;
    if (idx >= nitems) return;
    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, idx, false, d, tile, lat)) return;
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t EW = edge_words(TY);
    const uint64_t N = (uint64_t)d.L * d.L;
    const uint32_t t_right = g.ty * d.ntx + ((g.tx + 1 == d.ntx) ? 0u : g.tx + 1);
    const uint32_t t_below = ((g.ty + 1 == d.nty) ? 0u : g.ty + 1) * d.ntx + g.tx;
    const gptr<uint32_t> rec = glb(d.edges) + (size_t)tile * EW;
    const gptr<uint32_t> recR = glb(d.edges) + (size_t)t_right * EW;
    const gptr<uint32_t> recB = glb(d.edges) + (size_t)t_below * EW;

    bool bad = false;
    // Right edge: row r joins (w-1, r) here with (0, r) of the right neighbour.
    uint32_t pa = INVALID, pb = INVALID;
    for (uint32_t j = 0; j < TY; j += 64) {
        const uint32_t r = j + lane;
        const bool bit = r < g.h && ((rec[r >> 5] >> (r & 31u)) & 1u);
        uint32_t a = INVALID, b = INVALID;
        if (bit) {
            a = rec[8 + r];
            b = recR[8 + TY + r];
        }
        uint32_t ua = __shfl_up(a, 1), ub = __shfl_up(b, 1);
        if (lane == 0) {
            ua = pa;
            ub = pb;
        }
        pa = __shfl(a, 63);
        pb = __shfl(b, 63);
        // consecutive crossing bonds between the same two clusters: join once
        if (bit && !(ua == a && ub == b)) g_unite(glb(d.lab), N, a, b, bad);
    }
    // Bottom edge: column x joins (x, h-1) here with (x, 0) of the tile below.
    {
        const uint32_t x = lane;
        const bool bit = x < g.w && ((rec[4 + (x >> 5)] >> (x & 31u)) & 1u);
        uint32_t a = INVALID, b = INVALID;
        if (bit) {
            a = rec[8 + 2 * TY + x];
            b = recB[8 + 2 * TY + TX + x];
        }
        uint32_t ua = __shfl_up(a, 1), ub = __shfl_up(b, 1);
        if (lane == 0) {
            ua = INVALID;
            ub = INVALID;
        }
        if (bit && !(ua == a && ub == b)) g_unite(glb(d.lab), N, a, b, bad);
    }
    if (bad) flag_error(d.err);
}

// ---------------------------------------------------------------------------
// Flip: every site takes the state drawn for the smallest site index of its
// cluster.  Inside the tile the labels form a forest whose terminals are the
// sites that are global roots or whose parent lies outside the tile; only the
// terminals search the global forest (halving the paths they walk) and draw a
// state, in compacted lanes.  Wave w owns rows w, w+4, w+8, ... (lane =
// column); its labels are all loaded first, and its terminals go to a list of
// its own.
template <int TY>
__global__ __launch_bounds__(threads_of<TY>()) void k_flip(const LatDesc* descs, const WorkItem* map, uint32_t k)
{
    constexpr uint32_t NW = waves_of<TY>(), NT = threads_of<TY>();
    constexpr uint32_t PER = TY / NW;  // rows per wave
    __shared__ uint32_t E[TY * TX];
    __shared__ uint16_t list[NW][PER * TX + 64];   // + a scratch slot per lane

    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, blockIdx.x, true, d, tile, lat)) return;
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *glb(d.counter) + k;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    const uint32_t L = d.L, w = g.w, h = g.h, x0 = g.x0, y0 = g.y0;
    const uint32_t col = lane;
    uint16_t* my_list = list[wave];
    const gptr<uint32_t> lab = glb(d.lab);
    bool bad = false;

    // Full tiles (the common case) need no masks for columns or rows outside;
    // a power-of-two L divides by a shift.
    // The tile's entries are addressed from a wave-uniform base with 32-bit
    // per-lane byte offsets (a tile spans fewer than 2^32 / 4 sites of the
    // arrays), which keeps 64-bit address arithmetic out of the vector units.
    const uint32_t site0 = wave * L + col;         // this lane's first site, from the tile origin
    const uint32_t wave_step = NW * L;             // sites between a wave's consecutive rows
    const gptr<const char> lab_tile = (gptr<const char>)(glb(d.lab) + (size_t)y0 * L + x0);
    const gptr<char> s_tile = (gptr<char>)(glb(d.s) + (size_t)y0 * L + x0);

    auto body = [&](auto full, auto pow2) {
        constexpr bool FULL = decltype(full)::value;
        constexpr bool POW2 = decltype(pow2)::value;
        const bool vcol = FULL || col < w;
        uint32_t v[PER];
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t r = wave + NW * j;
            const uint32_t byte_off = (site0 + j * wave_step) * 4u;
            v[j] = (vcol && (FULL || r < h)) ? *(gptr<const uint32_t>)(lab_tile + byte_off) : 0u;
        }

        // row j of this wave: tile index li0 + j NW TX, site index gi0 + j wave_step
        // (site indices fit 32 bits, N <= 2^32; rows and L fit 24 bits)
        const uint32_t li0 = wave * TX + col;
        const uint32_t gi0 = __umul24(y0 + wave, L) + x0 + col;
        uint32_t nterm = 0;   // wave-uniform
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t r = wave + NW * j;
            if (!FULL && r >= h) continue;
            const uint32_t li = li0 + j * NW * TX;
            const uint32_t gi = gi0 + j * wave_step;
            const uint32_t vv = v[j];
            bool term;
            uint32_t local;
            if (FULL && POW2) {
                // power-of-two L, aligned full tile: the label is inside iff it
                // agrees with the site's own index outside the in-tile bits
                const uint32_t inner = ((uint32_t)(TY - 1) << d.log2L) | (TX - 1u);
                term = vv == gi || ((vv ^ gi) & ~inner) != 0u;
                local = (((vv >> d.log2L) & (TY - 1u)) * TX) | (vv & (TX - 1u));
            } else {
                // tile coordinates of the label (meaningless, and rejected, outside the tile)
                const uint32_t vy = POW2 ? vv >> d.log2L : div_L(d, vv);
                const uint32_t dy = vy - y0, dx = (POW2 ? (vv & (L - 1u)) : vv - __umul24(vy, L)) - x0;
                term = vcol && (vv == gi || dy >= (FULL ? TY : h) || dx >= (FULL ? TX : w));
                local = dy * TX + dx;
            }
            const uint64_t m = ballot(term);
            const bool is_term = lane_in(m);
            if (vcol) E[li] = is_term ? vv : local;
            // terminals append to the list, the other lanes write their scratch slot
            const uint32_t at_list = nterm + lanes_below(m), at_scratch = PER * TX + lane;
            my_list[is_term ? at_list : at_scratch] = (uint16_t)li;
            nterm = __builtin_amdgcn_readfirstlane(nterm + popc64(m));
        }

        // a wave resolves the terminals it found (all its own entries of E),
        // 64 at a time; lanes past the end work on a copy they do not store
        for (uint32_t j0 = 0; j0 < nterm; j0 += 64) {
            const uint32_t j = j0 + lane;
            const bool act = j < nterm;
            const uint32_t li = my_list[act ? j : 0];
            const uint32_t vv = E[li];
            const uint32_t gi = __umul24(y0 + li / TX, L) + x0 + li % TX;
            uint32_t root = vv;
            if (act && vv < gi) root = g_find(lab, vv, bad);
            bad |= act && vv > gi;
            const uint32_t st = TERM | cluster_state(d, root, t);
            if (act) E[li] = st;
        }
        __syncthreads();

        // Every site follows in-tile pointers (each to a smaller tile index, so
        // the walk ends) to a resolved entry; the new spins are stored at the end.
        uint32_t e[PER];
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t r = wave + NW * j;
            e[j] = TERM;
            if (vcol && (FULL || r < h)) {
                uint32_t cur = li0 + j * NW * TX, x = E[cur];
                while (!(x & TERM) && x < cur) {
                    cur = x;
                    x = E[cur];
                }
                bad |= !(x & TERM);
                e[j] = x;
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t r = wave + NW * j;
            if (vcol && (FULL || r < h)) *(gptr<uint8_t>)(s_tile + (site0 + j * wave_step)) = (uint8_t)e[j];
        }
    };
    if (w == TX && h == TY) {
        if (d.log2L) body(std::true_type{}, std::true_type{});
        else body(std::true_type{}, std::false_type{});
    } else {
        body(std::false_type{}, std::false_type{});
    }
    if (bad) flag_error(d.err);

    // The ring record of the next sweep starts from zero.
    if (d.cap && tile == 0) {
        const uint32_t words = NCOPY * ring_stride(d.q);
        gptr<int64_t> rec = glb(d.ring) + (size_t)((t + 1) % d.cap) * words;
        for (uint32_t i = tid; i < words; i += NT) rec[i] = 0;
    }
}

// ---------------------------------------------------------------------------
// Measurement of the current configuration into the ring record of sweep
// counter + k (used after the last sweep of a call).
template <int TY>
__global__ __launch_bounds__(threads_of<TY>()) void k_measure(const LatDesc* descs, const WorkItem* map, uint32_t k,
                                                const uint32_t* n_each)
{
    constexpr uint32_t RPW = TY / waves_of<TY>();
    __shared__ __align__(16) uint8_t sp[(TY + 1) * SPW];
    __shared__ uint32_t hist[256];
    __shared__ uint32_t tot;
    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, blockIdx.x, true, d, tile, lat)) return;
    if (d.cap == 0) return;
    if (n_each) {
        const uint32_t nl = n_each[lat];
        if (nl == 0) return;
        k = nl - 1;
    }
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *glb(d.counter) + k;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    const uint32_t w = g.w, h = g.h;
    if (tid < 256) hist[tid] = 0;
    if (tid == 0) tot = 0;
    stage_spins<TY>(sp, d, g, tid);
    __syncthreads();
    const uint32_t x = lane;
    const bool vx = x < w;
    const uint64_t validm = (w == 64) ? ~0ull : ((1ull << w) - 1ull);
    const uint32_t r0 = wave * RPW, r1 = min(h, r0 + RPW);
    static_assert(RPW < 32, "per-lane counters hold at most 31 rows");
    // unequal pairs counted per wave in a scalar; for q <= 16 the states
    // 1..q-1 in per-lane bytes (as in k_bond_label), other q through the
    // shared histogram
    const bool q8 = d.q <= 8, q16 = d.q <= 16;
    uint32_t n_unsat = 0;
    uint64_t packed[2] = {0ull, 0ull};
    for (uint32_t r = r0; r < r1; ++r) {
        const uint8_t* row = sp + r * SPW;
        const uint32_t s = row[x], sr = row[x + 1], sd = row[SPW + x];
        n_unsat += popc64(ballot(s != sr) & validm) + popc64(ballot(s != sd) & validm);
        if (q8) count_state_byte(packed, vx, s);
        else if (q16) count_state_bytes(packed, vx, s & 15u);
        else count_states(hist, vx, s);
    }
    if (lane == 0) atomicAdd(&tot, n_unsat);
    if (q16) flush_state_bytes(packed, hist, d.q, lane);
    __syncthreads();
    int64_t* rp = ring_record(d, t, blockIdx.x % NCOPY);
    if (tid == 0) atomic_add_i64(&rp[0], tot);
    if (tid >= 1 && tid < d.q && hist[tid]) atomic_add_i64(&rp[1 + tid], hist[tid]);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init(const LatDesc* descs, uint32_t lat, uint32_t random_start)
{
    const LatDesc d = descs[lat];
    const size_t N = (size_t)d.L * d.L;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        glb(d.s)[i] = random_start
                     ? (uint8_t)state_of_draw(philox4x32_10((uint32_t)i, 0u, 0u, 2u, d.key0, d.key1).x, d.q)
                     : (uint8_t)0;
    }
}

// Labels of the last sweep resolved to the smallest site index of each cluster.
__global__ __launch_bounds__(256) void k_resolve(const LatDesc* descs, uint32_t lat)
{
    const LatDesc d = descs[lat];
    const size_t N = (size_t)d.L * d.L;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t v = glb(d.lab)[i];
        bool bad = v > i;
        if (!bad) glb(d.lab)[i] = g_root(glb(d.lab), v, bad);
        if (bad) flag_error(d.err);
    }
}

// One thread per (record, word): the sum of the word over the record's NCOPY
// partial copies.
__global__ __launch_bounds__(256) void k_ring_sum(const int64_t* ring, int64_t* out, uint32_t slots, uint32_t slot0,
                                                  uint32_t n, uint32_t q)
{
    const uint32_t W = q + 1;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * W) return;
    const uint32_t rec = i / W, w = i - rec * W;
    const uint32_t slot = (uint32_t)(((uint64_t)slot0 + rec) % slots);
    const size_t R = ring_stride(q);
    const gptr<const int64_t> base = glb(ring) + (size_t)slot * NCOPY * R + w;
    int64_t sum = 0;
#pragma unroll 8
    for (uint32_t c = 0; c < NCOPY; ++c) sum += base[(size_t)c * R];
    glb(out)[i] = sum;
}

// Advance sweep counters: lattice i by n (or by n_each[i] when given).
__global__ void k_bump(const LatDesc* descs, uint32_t count, const uint32_t* n_each, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const uint32_t add = n_each ? n_each[i] : n;
        if (add) *glb(descs[i].counter) += add;
    }
}

// Set-up of a lattice whose descriptor and state live in caller-independent
// scratch (the no-allocation entry point): descriptor copied in, error flag
// cleared, sweep counter set, ring records zeroed.  A plain kernel rather than
// copies and fills, so the whole call can be captured in a graph.
__global__ __launch_bounds__(256) void k_static_setup(LatDesc d, LatDesc* d_out, DevState* st, uint32_t counter,
                                                      int64_t* ring, uint32_t ring_words)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *d_out = d;
        st->err = 0;
        st->counter = counter;
    }
    for (uint32_t j = i; j < ring_words; j += gridDim.x * blockDim.x) glb(ring)[j] = 0;
}

// One finished ring record as an observable row [n_unsat, n_active, n_0, ...,
// n_{q-1}] (n_0 = N minus the other counts), summed over its NCOPY partial
// copies; optionally the error flag into *status.  One workgroup of 256.
__global__ __launch_bounds__(256) void k_emit_row(const int64_t* ring, uint32_t slots, uint32_t slot, uint32_t q,
                                                  uint64_t N, int64_t* row, const uint32_t* err, uint32_t* status)
{
    __shared__ int64_t word[256];
    const uint32_t w = threadIdx.x;
    if (row) {
        const size_t R = ring_stride(q);
        int64_t sum = 0;
        if (w <= q) {
            const gptr<const int64_t> base = glb(ring) + (size_t)(slot % slots) * NCOPY * R + w;
            for (uint32_t c = 0; c < NCOPY; ++c) sum += base[(size_t)c * R];
        }
        word[w] = sum;
        __syncthreads();
        if (w == 0) {
            int64_t rest = 0;
            for (uint32_t c = 1; c < q; ++c) rest += word[1 + c];
            glb(row)[0] = word[0];
            glb(row)[1] = word[1];
            glb(row)[2] = (int64_t)N - rest;
        } else if (w < q) {
            glb(row)[2 + w] = word[1 + w];
        }
    }
    if (status && w == 0) *glb(status) = *glb(err);
}

// ---------------------------------------------------------------- launchers
namespace {
uint32_t init_grid(size_t N)
{
    const size_t b = (N + 255) / 256;
    return (uint32_t)(b < 65536 ? (b ? b : 1) : 65536);
}
}  // namespace

// BLOCK(T): threads per workgroup of the kernel instantiated for T rows.
#define SWMI_TY_DISPATCH_B(TYV, KERNEL, GRID, BLOCK, ...)                                                    \
    switch (TYV) {                                                                                         \
    case 32: hipLaunchKernelGGL(KERNEL<32>, dim3(GRID), dim3(BLOCK(32)), 0, w.stream, __VA_ARGS__); break;    \
    case 64: hipLaunchKernelGGL(KERNEL<64>, dim3(GRID), dim3(BLOCK(64)), 0, w.stream, __VA_ARGS__); break;    \
    case 128: hipLaunchKernelGGL(KERNEL<128>, dim3(GRID), dim3(BLOCK(128)), 0, w.stream, __VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                                                                  \
    }
#define SWMI_TILE_BLOCK(T) threads_of<T>()
#define SWMI_FOUR_WAVES(T) 256
#define SWMI_TY_DISPATCH(TYV, KERNEL, GRID, ...) SWMI_TY_DISPATCH_B(TYV, KERNEL, GRID, SWMI_TILE_BLOCK, __VA_ARGS__)

hipError_t launch_bond_label(const Work& w, uint32_t k, uint32_t flags)
{
    if (w.nitems == 0) return hipSuccess;
    SWMI_TY_DISPATCH(w.ty, k_bond_label, w.nitems, w.descs, w.map, k, flags);
    return hipGetLastError();
}

hipError_t launch_merge(const Work& w)
{
    if (w.nitems == 0) return hipSuccess;
    SWMI_TY_DISPATCH_B(w.ty, k_merge, (w.nitems + 3) / 4, SWMI_FOUR_WAVES, w.descs, w.map, w.nitems);
    return hipGetLastError();
}

hipError_t launch_flip(const Work& w, uint32_t k)
{
    if (w.nitems == 0) return hipSuccess;
    SWMI_TY_DISPATCH(w.ty, k_flip, w.nitems, w.descs, w.map, k);
    return hipGetLastError();
}

hipError_t launch_measure(const Work& w, uint32_t k)
{
    if (w.nitems == 0) return hipSuccess;
    SWMI_TY_DISPATCH(w.ty, k_measure, w.nitems, w.descs, w.map, k, (const uint32_t*)nullptr);
    return hipGetLastError();
}

hipError_t launch_measure_each(const Work& w, const uint32_t* n_each)
{
    if (w.nitems == 0) return hipSuccess;
    if (!w.map) return hipErrorInvalidValue;
    SWMI_TY_DISPATCH(w.ty, k_measure, w.nitems, w.descs, w.map, 0u, n_each);
    return hipGetLastError();
}

hipError_t launch_init(const LatDesc* descs, uint32_t lat, size_t N, uint32_t random_start, hipStream_t s)
{
    hipLaunchKernelGGL(k_init, dim3(init_grid(N)), dim3(256), 0, s, descs, lat, random_start);
    return hipGetLastError();
}

hipError_t launch_resolve(const LatDesc* descs, uint32_t lat, size_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_resolve, dim3(init_grid(N)), dim3(256), 0, s, descs, lat);
    return hipGetLastError();
}

hipError_t launch_ring_sum(const int64_t* ring, int64_t* out, uint32_t slots, uint32_t slot0, uint32_t n, uint32_t q,
                           hipStream_t s)
{
    const uint64_t total = (uint64_t)n * (q + 1);
    if (total == 0) return hipSuccess;
    if (total > 0xFFFFFFFFull || slot0 >= slots || n >= slots) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ring_sum, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, ring, out, slots, slot0, n, q);
    return hipGetLastError();
}

hipError_t launch_static_setup(const LatDesc& d, LatDesc* d_out, DevState* st, uint32_t counter, int64_t* ring,
                               uint32_t ring_words, hipStream_t s)
{
    const uint32_t grid = std::max(1u, std::min(1024u, (ring_words + 255) / 256));
    hipLaunchKernelGGL(k_static_setup, dim3(grid), dim3(256), 0, s, d, d_out, st, counter, ring, ring_words);
    return hipGetLastError();
}

hipError_t launch_emit_row(const int64_t* ring, uint32_t slots, uint32_t slot, uint32_t q, uint64_t N, int64_t* row,
                           const uint32_t* err, uint32_t* status, hipStream_t s)
{
    if (q < 2 || q > 255 || slots == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_emit_row, dim3(1), dim3(256), 0, s, ring, slots, slot, q, N, row, err, status);
    return hipGetLastError();
}

hipError_t launch_bump(const LatDesc* descs, uint32_t count, const uint32_t* n_each, uint32_t n, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bump, dim3((count + 255) / 256), dim3(256), 0, s, descs, count, n_each, n);
    return hipGetLastError();
}

}  // namespace swmi
