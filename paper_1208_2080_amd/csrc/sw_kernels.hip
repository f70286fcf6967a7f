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
#include "sw_tile.hpp"

namespace swmi {

namespace {

// Every label points at a site index no larger than its own (roots at
// themselves).  Every pointer walk steps only to strictly smaller indices, so
// it ends even in a corrupted forest, and union retries carry caps; a forest
// that breaks the invariant sets the error flag instead of spinning.
constexpr uint32_t UNITE_CAP = 1u << 12;   // cap of union retries in the global forest
constexpr uint32_t SPW = TX + 4;           // LDS row stride of staged spins (bytes)

// Lane l's bit of a wave-uniform mask, as a lane predicate.
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Sum over the wave of a per-lane value (all 64 lanes active), in vector
// instructions only: pairs and quads by quad permutes, rows of 16 by half-row
// and row mirrors, then the rows' sums broadcast into row 3 (row_bcast:15 into
// rows 1 and 3, row_bcast:31 into rows 2 and 3), so lane 63 holds the total.
// Where the scalar unit is the busier one this beats a ballot per bit plane.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);            // quad_perm [1,0,3,2]
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);            // quad_perm [2,3,0,1]
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);           // row_half_mirror
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);           // row_mirror
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);     // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);     // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Number of set bits of a wave-uniform mask below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ------------------------------------------------------ edge forest (global)
// One node per tile-local cluster that touches a tile edge.  A node's word is
// (key << 32) | parent: parent is a node id, key the smallest site index of the
// parent (a root is its own parent, its key its own smallest site).  Words only
// ever decrease, and ordering words orders keys, so hooking the root with the
// larger word under the one with the smaller (a 64-bit atomicMin) leaves every
// cluster's root at its smallest site.
//
// The finds read through the caches.  A stale word is one the node had
// earlier, still pointing at an ancestor, so chases still end and only ever
// reach true ancestors or stale roots; the hook itself is a device-coherent
// atomicMin that returns the current word, and a hook on a stale root retries
// from that value.  Every step goes to a strictly smaller key, so walks end
// even in a corrupted forest; a step that does not (or leaves the node array)
// sets `bad` and stops.
__device__ __forceinline__ uint32_t node_of(uint64_t w) { return (uint32_t)w; }
__device__ __forceinline__ uint32_t key_of(uint64_t w) { return (uint32_t)(w >> 32); }

__device__ __forceinline__ uint64_t min_coherent64(gptr<uint64_t> p, uint64_t v)
{
    return __hip_atomic_fetch_min(reinterpret_cast<gptr<unsigned long long>>(p), (unsigned long long)v,
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root word of node x whose word w was loaded already (x < n), with path
// splitting (every visited node is pointed at its grandparent when that is a
// real shortcut; any stored word is an ancestor's, so races are benign).
// n: nodes in the array.
__device__ uint64_t n_find_from(gptr<uint64_t> nodes, uint32_t n, uint32_t x, uint64_t w, bool& bad)
{
    for (uint32_t it = 0; it < UNITE_CAP; ++it) {
        const uint32_t p = node_of(w);
        if (p == x) return w;
        if (p >= n) break;
        const uint64_t wp = nodes[p];
        if (key_of(wp) >= key_of(w) && node_of(wp) != p) break;   // keys must fall
        if (wp < w) nodes[x] = wp;
        x = p;
        w = wp;
    }
    bad = true;
    return w;
}

// Read-only root search once the forest is final.
__device__ uint64_t n_root(gptr<const uint64_t> nodes, uint32_t n, uint32_t x, bool& bad)
{
    if (x >= n) {
        bad = true;
        return 0;
    }
    uint64_t w = nodes[x];
    for (uint32_t it = 0; it < UNITE_CAP; ++it) {
        const uint32_t p = node_of(w);
        if (p == x) return w;
        if (p >= n) break;
        const uint64_t wp = nodes[p];
        if (key_of(wp) >= key_of(w) && node_of(wp) != p) break;
        x = p;
        w = wp;
    }
    bad = true;
    return w;
}

// One step of a find (path splitting): from node x with word w to its parent.
// Returns false (and sets bad) if the forest is corrupted.
__device__ __forceinline__ bool n_step(gptr<uint64_t> nodes, uint32_t n, uint32_t& x, uint64_t& w, uint64_t wp,
                                       bool& bad)
{
    const uint32_t p = node_of(w);
    if (key_of(wp) >= key_of(w) && node_of(wp) != p) {   // keys must fall
        bad = true;
        return false;
    }
    if (wp < w) nodes[x] = wp;
    x = p;
    w = wp;
    return true;
}

// Roots of M nodes x[m] (words w[m] already loaded; only the chains whose bit
// is set in `live` are walked), one level of every unfinished chain per step so
// that the loads of all chains overlap.
template <int M>
__device__ void n_find_m(gptr<uint64_t> nodes, uint32_t n, uint32_t (&x)[M], uint64_t (&w)[M], uint32_t live,
                         bool& bad)
{
    for (uint32_t it = 0; it < UNITE_CAP; ++it) {
        bool done = true;
        uint64_t wp[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const bool walk = ((live >> m) & 1u) && node_of(w[m]) != x[m];
            if (walk && node_of(w[m]) >= n) {
                bad = true;
                return;
            }
            wp[m] = walk ? nodes[node_of(w[m])] : w[m];
            done &= !walk;
        }
        if (done) return;
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (((live >> m) & 1u) && node_of(w[m]) != x[m] && !n_step(nodes, n, x[m], w[m], wp[m], bad)) return;
    }
    bad = true;
}

// Every word in the forest, (key << 32) | p, is also the word node p holds
// while it is a root (a node's key is its own).  So a hook can name two roots
// by their words alone: hook(a, b) hangs the node of the larger word under the
// smaller with one atomicMin.  If that node was no longer a root, the atomic
// returns its current word, whose node is the parent it had meanwhile gained
// (and a smaller word stored by the atomic dropped that link), so the hook goes
// on with that word and the smaller one: no reload and no new walk, one round
// trip per attempt.  The larger word falls at every attempt, so the loop ends.
// Two hooks of one lane run in step so that their atomics overlap.
__device__ void n_hook2(gptr<uint64_t> nodes, uint32_t n, uint64_t (&a)[2], uint64_t (&b)[2], bool& bad)
{
    for (uint32_t it = 0; it < UNITE_CAP; ++it) {
        bool done = true;
        uint64_t old[2], hi[2], lo[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            hi[m] = max(a[m], b[m]);
            lo[m] = min(a[m], b[m]);
            const bool act = hi[m] != lo[m];
            if (act && node_of(hi[m]) >= n) {
                bad = true;
                return;
            }
            old[m] = act ? min_coherent64(nodes + node_of(hi[m]), lo[m]) : hi[m];
        }
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            a[m] = old[m] == hi[m] ? lo[m] : old[m];
            b[m] = lo[m];
            done &= old[m] == hi[m];
        }
        if (done) return;
    }
    bad = true;
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
        const uint32_t n = wave_sum((uint32_t)(w[c >> 3] >> (8u * (c & 7u))) & 0xFFu);
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
__device__ __forceinline__ void drain(UnionQueue& uq, uint16_t* P, uint32_t lane, bool& bad)
{
    for (uint32_t j = lane; j < uq.n; j += 64) {
        const uint32_t e = lds_ld(&uq.q[j]);
        lds_union(P, e & 0xFFFFu, e >> 16, bad);
    }
    uq.n = 0;
}

// Queue the unions (a, b) of the lanes in `mask` where a != b (at most 64; the
// caller keeps at least 64 slots free).  The other lanes store to a scratch
// word instead of branching around the store (no branch on the scalar unit).
__device__ __forceinline__ void enqueue(UnionQueue& uq, uint64_t mask, uint32_t a, uint32_t b)
{
    const uint64_t m = ballot(a != b) & mask;
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
__device__ __forceinline__ uint32_t row_labels(uint16_t* P, uint32_t* rl, UnionQueue& uq, uint32_t r, uint32_t x,
                                               uint64_t validm, uint64_t hx, uint64_t V, uint64_t hprev, uint32_t lp)
{
    const uint64_t C = hx << 1;                 // bit x: bond (x-1) -> x
    const uint64_t S = ~C & validm;             // first sites of runs (site 0 always is one)
    // run index of x = run starts in 0..x, less one: counted from an initial
    // value of (x starts a run) - 1, with no scalar shift of S
    const uint32_t ri = __builtin_amdgcn_mbcnt_hi((uint32_t)(S >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)S, (uint32_t)lane_in(S) - 1u));
    const uint32_t fresh = r * TX + x;
    // lanes talk through the slots, so these accesses must not be folded away;
    // a run's first site offers itself and every +y bond offers the label
    // above, in one store: any offer may win (unions below cover the rest)
    const bool vb = lane_in(V);
    lds_st(lane_in(S | V) ? &rl[ri] : &rl[64], vb ? lp : fresh);
    const uint32_t lab = lds_ld(&rl[ri]);
    lds_st(&P[fresh], lab);   // columns outside the tile write entries no one reads
    // bonds x-1 and x from the same run above into the same run here add nothing
    const uint64_t R = (V & C) & ((V & hprev) << 1);
    enqueue(uq, V & ~R, lp, lab);
    return lab;
}

}  // namespace

#ifdef SW_PHASE_CLOCKS
// Phase-clock tables of the profiling build: [kernel][NCOPY][PHASES + 1], the
// kernels being the bond-and-label kernel (Potts), the merge, the flip
// (Potts), the labelling of preset bonds and the flip that reflects (XY).
constexpr uint32_t PHASE_KERNELS = 5;
static __device__ unsigned long long g_phase_table[PHASE_KERNELS * NCOPY * (PHASES + 1)];
__device__ __forceinline__ unsigned long long* phase_table(uint32_t kernel)
{
    return g_phase_table + (size_t)kernel * NCOPY * (PHASES + 1);
}

// Profiling builds only (C linkage, so the namespace does not matter): the
// phase-clock tables summed over their rows into
// host [PHASE_KERNELS][PHASES + 1] (ticks per phase, then waves), and cleared
// when `clear` is nonzero.  Synchronises the device.
extern "C" int sw_phase_clocks(unsigned long long* host, int clear)
{
    static unsigned long long t[PHASE_KERNELS * NCOPY * (PHASES + 1)];
    if (hipDeviceSynchronize() != hipSuccess) return -1;
    if (hipMemcpyFromSymbol(t, HIP_SYMBOL(g_phase_table), sizeof(t)) != hipSuccess) return -1;
    for (uint32_t k = 0; k < PHASE_KERNELS; ++k)
        for (uint32_t i = 0; i <= PHASES; ++i) {
            unsigned long long sum = 0;
            for (uint32_t c = 0; c < NCOPY; ++c) sum += t[(k * NCOPY + c) * (PHASES + 1) + i];
            host[k * (PHASES + 1) + i] = sum;
        }
    if (clear) {
        for (auto& v : t) v = 0;
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_phase_table), t, sizeof(t)) != hipSuccess) return -1;
    }
    return 0;
}
#endif

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
// PRESET: the bonds are already in the bond plane (drawn by the XY model's own
// kernel); the kernel then only labels, and measures nothing.
template <int TY, bool PRESET = false>
__global__ __launch_bounds__(threads_of<TY>()) __attribute__((amdgpu_waves_per_eu(8))) void k_bond_label(const LatDesc* descs, const WorkItem* map, uint32_t k,
                                                   uint32_t flags)
{
    constexpr uint32_t NW = waves_of<TY>(), NT = threads_of<TY>();
    constexpr uint32_t RPW = TY / NW;  // rows per wave (even)
    static_assert(RPW < 32, "per-lane measurement counters hold at most 31 rows");
    constexpr uint32_t QCAP = qcap_of<TY>();
    __shared__ __align__(16) uint16_t P[TY * TX];   // union-find over the tile's sites
    __shared__ __align__(16) uint8_t sp[(TY + 1) * SPW];
    __shared__ uint64_t rb[TY][2];     // per row: +x bond word, +y bond word
    // per wave: the label of every run of a row; once a wave has left its
    // strip, its row holds the labels of the strip's last row (the seam)
    __shared__ uint32_t RL[NW][65];    // [64]: scratch word of lanes with nothing to store
    __shared__ uint32_t UQT[NW];       // scratch words of the union queues
    uint32_t(*const seam)[65] = RL;
    __shared__ uint32_t UQ[NW][QCAP];  // per wave: pending unions
    __shared__ uint32_t hist[256];
    __shared__ uint32_t tot[3];        // unequal pairs, active bonds, edge-forest nodes

    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, blockIdx.x, true, d, tile, lat)) return;
    SW_PHASE_START(pc);
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *glb(d.counter) + k;
    const bool meas = !PRESET && d.cap != 0;
    const bool meas_prev = meas && (flags & 1u);
    const uint32_t tid = threadIdx.x, wave = wave_id(), lane = tid & 63u;
    const uint32_t L = d.L, w = g.w, h = g.h, x0 = g.x0, y0 = g.y0;

    if (tid < 256) hist[tid] = 0;
    if (tid < 3) tot[tid] = 0;
    if constexpr (PRESET) {
        const gptr<uint64_t> bin = glb(d.bonds) + (size_t)tile * 2 * TY;
        for (uint32_t j = tid; j < 2 * TY; j += NT) {
            const uint32_t r = j % TY;
            rb[r][j / TY] = r < h ? bin[j] : 0ull;
        }
    } else {
        stage_spins<TY>(sp, d, g, tid);
    }
    __syncthreads();
    SW_PHASE(pc, 0);   // staging

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
    // measurement: equal-spin pairs and q = 2 spins counted per lane (column;
    // vector adds keep the work off the scalar unit), active bonds counted from
    // the bond words
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

    // The row loop, compiled three times: the q = 9..16 counters (two words per
    // lane) stay out of the common instantiations, whose code they would
    // otherwise perturb; FAST is a full strip of a full-width tile of a lattice
    // of even L, q <= 8 and K > 0: no lane or row masks, always two rows, one
    // Philox path, the measurement counted without branches (used only when
    // measuring) and the bond words gathered into lanes, one row per lane, and
    // stored once per strip.  That keeps the scalar unit's share of the loop
    // small (it is the busier of the two issue units here).
    auto strip_rows = [&](auto wide, auto fast) {
        constexpr bool WIDE = decltype(wide)::value;
        constexpr bool FAST = decltype(fast)::value;
        const uint64_t vm = FAST ? ~0ull : validm, bm = FAST ? ~0ull : bondm;
        uint32_t bxl = 0, bxh = 0, byl = 0, byh = 0;   // FAST: lane k holds row r0 + k's bond words
#pragma unroll 1
        for (uint32_t r = r0; r < r1; r += 2) {
            const bool two = FAST || r + 1 < r1;
            if (uq.n > QCAP - 128) drain(uq, P, lane, bad);
            const uint8_t* row = sp + r * SPW;
            const uint32_t s0 = row[x], s0r = row[x + 1];
            const uint32_t s1 = row[SPW + x], s1r = row[SPW + x + 1];
            const uint32_t s2 = two ? row[2 * SPW + x] : 0u;

            // Site indices in 32 bits: exact for every row of the lattice (N <= 2^32);
            // a draw for row r+1 past the last row wraps but is never used.
            const uint32_t base0 = (y0 + r) * L + x0;
            uint32_t wx0, wy0, wx1, wy1;
            if (FAST || even_L) {
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
            const uint64_t EX0 = ballot(s0 == s0r) & vm, EY0 = ballot(s0 == s1) & vm;
            const uint64_t BX0 = EX0 & ballot(wx0 <= d.thr_m1) & bm;
            const uint64_t BY0 = EY0 & ballot(wy0 <= d.thr_m1) & bm;
            uint64_t EX1 = 0, EY1 = 0, BX1 = 0, BY1 = 0;
            if (two) {
                EX1 = ballot(s1 == s1r) & vm;
                EY1 = ballot(s1 == s2) & vm;
                BX1 = EX1 & ballot(wx1 <= d.thr_m1) & bm;
                BY1 = EY1 & ballot(wy1 <= d.thr_m1) & bm;
            }
            if constexpr (FAST) {
                // vector selects only (no scalar work): lane k takes row r0 + k
                const uint32_t k = r - r0;
                const bool at0 = lane == k, at1 = lane == k + 1;
                bxl = at0 ? (uint32_t)BX0 : at1 ? (uint32_t)BX1 : bxl;
                bxh = at0 ? (uint32_t)(BX0 >> 32) : at1 ? (uint32_t)(BX1 >> 32) : bxh;
                byl = at0 ? (uint32_t)BY0 : at1 ? (uint32_t)BY1 : byl;
                byh = at0 ? (uint32_t)(BY0 >> 32) : at1 ? (uint32_t)(BY1 >> 32) : byh;
            } else if (lane == 0) {
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

            if (FAST) {
                n_eq += (uint32_t)lane_in(EX0) + (uint32_t)lane_in(EY0) + (uint32_t)lane_in(EX1) +
                        (uint32_t)lane_in(EY1);
                count_state_byte(packed, true, s0);
                count_state_byte(packed, true, s1);
            } else if (meas_prev) {
                // this lane's equal pairs (EX1, EY1 are 0 without row r+1)
                n_eq += (uint32_t)lane_in(EX0) + (uint32_t)lane_in(EY0) + (uint32_t)lane_in(EX1) +
                        (uint32_t)lane_in(EY1);
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
        if constexpr (FAST) {
            if (lane < RPW) {
                rb[r0 + lane][0] = ((uint64_t)bxh << 32) | bxl;
                rb[r0 + lane][1] = ((uint64_t)byh << 32) | byl;
            }
        }
    };
    // the same row labelling over bond words that are already in LDS
    auto preset_rows = [&]() {
        for (uint32_t r = r0; r < r1; ++r) {
            if (uq.n > QCAP - 64) drain(uq, P, lane, bad);
            const uint64_t hx = rb[r][0] & ~cross;
            lp = row_labels(P, rl, uq, r, x, validm, hx, vprev, hprev, lp);
            hprev = hx;
            vprev = rb[r][1];
        }
    };
    const bool fast = w == TX && r1 - r0 == RPW && even_L && d.thr_nz && d.q <= 8;
    if constexpr (PRESET) preset_rows();
    else if (q16 && !q8) strip_rows(std::true_type{}, std::false_type{});
    else if (fast) strip_rows(std::false_type{}, std::true_type{});
    else strip_rows(std::false_type{}, std::false_type{});
    SW_PHASE(pc, 1);   // rows: draws, ballots, row labels, queue drains, counting
    seam[wave][lane] = lp;
    if (meas_prev) {
        // every site of the strip owns two bonds
        const uint32_t eq = wave_sum(n_eq);
        if (lane == 0 && r0 < r1) atomicAdd(&tot[0], 2u * w * (r1 - r0) - eq);
        if (q2 && !fast) {
            const uint32_t n1 = wave_sum(ones);
            if (lane == 0 && n1) atomicAdd(&hist[1], n1);
        }
        if (q16 || fast) flush_state_bytes(packed, hist, d.q, lane);   // (fast: q <= 8, one word)
    }
    SW_PHASE(pc, 2);   // measurement sums of the strip
    __syncthreads();
    SW_PHASE(pc, 3);   // barrier

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
    SW_PHASE(pc, 4);   // seams and the last drain

    // Tile record: bond words (tile-major), crossing-bond masks.
    gptr<uint32_t> rec = glb(d.edges) + (size_t)tile * edge_words(TY);
    gptr<uint64_t> bw = glb(d.bonds) + (size_t)tile * 2 * TY;
    for (uint32_t j0 = 0; j0 < 2 * TY; j0 += NT) {
        const uint32_t j = j0 + tid, r = j % TY;
        const uint64_t word = (j < 2 * TY && r < h) ? rb[r][j / TY] : 0ull;
        if (!PRESET && j < 2 * TY && r < h) bw[j] = word;
        if (meas) {
            const uint32_t n = wave_sum(popc64(word));   // active bonds
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
    SW_PHASE(pc, 5);   // bond words out, edge record, barrier

    // Edge sites find their tile-local roots (lane i takes the left and right
    // sites of strip row i; the first and last strips the top and bottom rows).
    // The first lane to reach a root claims it as a node of the tile's edge
    // forest: it takes the next slot (in no particular order: a node's word
    // carries its key), writes the node's word (a root of its own, keyed by its
    // site index) and tags the root's LDS entry ROOT16 | slot, which the labels
    // and the edge record copy.  Walks stop at tagged entries (all walks end
    // before the first claim).
    // a site index fits 32 bits (N <= 2^32) and y, L fit 24 bits
    auto global_index = [&](uint32_t la) { return __umul24(y0 + la / TX, L) + x0 + la % TX; };
    const uint32_t node0 = tile * nslot(TY);
    auto edge_root = [&](uint32_t li) {
        uint32_t p = lds_ld(&P[li]);
        while (!(p & ROOT16) && p < li) {
            li = p;
            p = lds_ld(&P[li]);
        }
        bad |= !(p & ROOT16) && p != li;
        return li;
    };
    // A claim of root r sets the ROOT16 bit of its entry with one LDS atomic
    // OR on the entry's 32-bit word: the lane that finds the bit clear is the
    // first and wins; an entry tagged already keeps its value (a slot stored
    // by another winner is never overwritten).  The four claims of a lane go
    // out together, then the wave's winners take consecutive slots with one
    // LDS atomic and tag their roots ROOT16 | slot.
    auto claim = [&](bool want, uint32_t r) {
        if (!want) return false;
        const uint32_t sh = (r & 1u) * 16u;
        const uint32_t old = atomicOr(reinterpret_cast<uint32_t*>(P) + (r >> 1), ROOT16 << sh);
        return ((old >> sh) & 0xFFFFu) == r;
    };
    const bool side = r0 < r1 && lane < r1 - r0;
    const bool top = r0 == 0 && r0 < r1 && vx;
    const bool bottom = r1 == h && r0 < r1 && vx;
    const uint32_t rs = r0 + lane;
    const uint32_t rootR = side ? edge_root(rs * TX + w - 1) : 0u;
    const uint32_t rootL = side ? edge_root(rs * TX) : 0u;
    const uint32_t rootT = top ? edge_root(x) : 0u;
    const uint32_t rootB = bottom ? edge_root((h - 1) * TX + x) : 0u;
    const bool wR = claim(side, rootR), wL = claim(side, rootL), wT = claim(top, rootT), wB = claim(bottom, rootB);
    {
        const uint64_t mR = ballot(wR), mL = ballot(wL), mT = ballot(wT), mB = ballot(wB);
        const uint32_t nR = popc64(mR), nL = popc64(mL), nT = popc64(mT), n_won = nR + nL + nT + popc64(mB);
        uint32_t base = 0;
        if (lane == 0 && n_won) base = atomicAdd(&tot[2], n_won);
        base = __builtin_amdgcn_readfirstlane(base);
        auto assign = [&](bool won, uint32_t r, uint32_t slot) {
            if (!won) return;
            glb(d.nodes)[node0 + slot] = ((uint64_t)global_index(r) << 32) | (node0 + slot);
            lds_st(&P[r], ROOT16 | slot);
        };
        assign(wR, rootR, base + lanes_below(mR));
        assign(wL, rootL, base + nR + lanes_below(mL));
        assign(wT, rootT, base + nR + nL + lanes_below(mT));
        assign(wB, rootB, base + nR + nL + nT + lanes_below(mB));
    }
    __syncthreads();
    SW_PHASE(pc, 6);   // edge roots, node claims, barrier
    if (tid == 0) rec[6] = tot[2];   // nodes of the tile

    // Tile labels out (16 bits), per site: the tile-local index of its
    // union-find grandparent (a smaller site of its tile-local cluster; the
    // flip follows these pointers inside the tile), or, for a tile-local root,
    // ROOT16 | its slot (NOSLOT if its cluster touches no tile edge).  A grandparent that is a
    // node is not copied (its entry carries a slot, not an index): the parent
    // is.  (The grandparent read is masked into the tile: a tagged entry's
    // slot, or an unused column's entry, reads some entry that is not used.)
    // Entries of columns outside the tile are never stored (full-width tiles,
    // the common case, need no mask at all).
    auto label_of = [&](uint32_t li, uint32_t p, uint32_t gp) {
        return (p & ROOT16) ? p : (p == li) ? (ROOT16 | NOSLOT) : (gp & ROOT16) ? p : gp;
    };
    auto labels_out = [&](auto full) {
        constexpr bool FULL = decltype(full)::value;
        const bool vs = FULL || vx;
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t li = r * TX + x, p = P[li];
            const uint32_t out = label_of(li, p, P[p & (TY * TX - 1u)]);
            const gptr<uint16_t> lrow = glb(d.tlab) + (size_t)(y0 + r) * L + x0;
            if (vs) lrow[x] = (uint16_t)out;
        }
    };
    if (w == TX && r1 - r0 == RPW) {
        // a full strip: all parent reads first, then all grandparent reads, so
        // the LDS round trips overlap; each row is stored from its own
        // wave-uniform (scalar) base, the lane's column as the only vector part
        uint32_t p[RPW], gp[RPW];
#pragma unroll
        for (uint32_t k = 0; k < RPW; ++k) p[k] = P[(r0 + k) * TX + x];   // (16-bit entries)
#pragma unroll
        for (uint32_t k = 0; k < RPW; ++k) gp[k] = P[p[k] & (TY * TX - 1u)];
        gptr<uint16_t> out = glb(d.tlab) + (size_t)(y0 + r0) * L + x0 + x;   // this lane's site, row by row
#pragma unroll
        for (uint32_t k = 0; k < RPW; ++k, out += L) *out = (uint16_t)label_of((r0 + k) * TX + x, p[k], gp[k]);
    } else if (w == TX) {
        labels_out(std::true_type{});
    } else {
        labels_out(std::false_type{});
    }
    SW_PHASE(pc, 7);   // tile labels out
    // The edge record's slots, for the merge.
    const gptr<uint16_t> slots = (gptr<uint16_t>)(rec + 8);
    if (side) {
        slots[rs] = P[rootR] & ~ROOT16;
        slots[TY + rs] = P[rootL] & ~ROOT16;
    }
    if (top) slots[2 * TY + TX + x] = P[rootT] & ~ROOT16;
    if (bottom) slots[2 * TY + x] = P[rootB] & ~ROOT16;
    if (bad) flag_error(d.err);

    // the workgroup's sums into the ring, by wave 0 alone (the slot's modulo is
    // scalar work the other waves need not repeat)
    if (meas && wave == 0) {
        const uint32_t copy = blockIdx.x % NCOPY;
        const uint32_t slot = t % d.cap, prev = slot ? slot - 1u : d.cap - 1u;
        int64_t* const rc = d.ring + ((size_t)slot * NCOPY + copy) * ring_stride(d.q);
        if (lane == 0) atomic_add_i64(&rc[1], tot[1]);
        if (meas_prev) {
            int64_t* const rp = d.ring + ((size_t)prev * NCOPY + copy) * ring_stride(d.q);
            if (lane == 0) atomic_add_i64(&rp[0], tot[0]);
            for (uint32_t c = lane; c < d.q; c += 64)
                if (c >= 1 && hist[c]) atomic_add_i64(&rp[1 + c], hist[c]);
        }
    }
    SW_PHASE(pc, 8);   // slots, ring sums
    SW_PHASE_FLUSH(pc, phase_table(PRESET ? 3u : 0u));
}

// ---------------------------------------------------------------------------
// Join tile-local clusters across tile edges.  One wave per tile handles the
// crossing bonds of its right and bottom edges (periodic neighbours): each
// joins the edge-forest nodes of the two sites' tile-local roots.
template <int TY>
__global__ __launch_bounds__(256) void k_merge(const LatDesc* descs, const WorkItem* map, uint32_t nitems)
{
    const uint32_t wave = wave_id(), lane = threadIdx.x & 63u;
    const uint32_t idx = blockIdx.x * 4 + wave;
    if (idx >= nitems) return;
    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, idx, false, d, tile, lat)) return;
    SW_PHASE_START(pc);
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t EW = edge_words(TY), NS = nslot(TY);
    const uint32_t n = d.ntiles * NS;
    const uint32_t t_right = g.ty * d.ntx + ((g.tx + 1 == d.ntx) ? 0u : g.tx + 1);
    const uint32_t t_below = ((g.ty + 1 == d.nty) ? 0u : g.ty + 1) * d.ntx + g.tx;
    const gptr<uint32_t> rec = glb(d.edges) + (size_t)tile * EW;
    const gptr<const uint16_t> sl = (gptr<const uint16_t>)(rec + 8);
    const gptr<const uint16_t> slR = (gptr<const uint16_t>)(glb(d.edges) + (size_t)t_right * EW + 8);
    const gptr<const uint16_t> slB = (gptr<const uint16_t>)(glb(d.edges) + (size_t)t_below * EW + 8);
    const gptr<uint64_t> nodes = glb(d.nodes);

    // Lane l takes the crossing bond of row l of the right edge (row l of the
    // right neighbour's left column) and of column l of the bottom edge
    // (column l of the top row of the tile below); consecutive crossing bonds
    // between the same two clusters are joined once.  The nodes' words are all
    // loaded before the first union, so their round trips overlap.
    bool bad = false;
    uint32_t pa = INVALID, pb = INVALID;
    for (uint32_t j = 0; j < TY; j += 64) {
        const uint32_t r = j + lane, x = lane;
        // the crossing bits and the slots at both ends of every edge site are
        // loaded together (all inside the records; slots of sites without a
        // crossing bond are not used)
        const uint32_t wr = rec[r >> 5], wb = rec[4 + (x >> 5)];
        const uint32_t sa1 = sl[r], sb1 = slR[TY + r];
        const uint32_t sa2 = sl[2 * TY + x], sb2 = slB[2 * TY + TX + x];
        const bool right = r < g.h && ((wr >> (r & 31u)) & 1u);
        const bool below = j == 0 && x < g.w && ((wb >> (x & 31u)) & 1u);
        SW_PHASE(pc, 0);   // edge record and slots
        uint32_t a1 = INVALID, b1 = INVALID, a2 = INVALID, b2 = INVALID;
        if (right) {
            a1 = tile * NS + sa1;
            b1 = t_right * NS + sb1;
        }
        if (below) {
            a2 = tile * NS + sa2;
            b2 = t_below * NS + sb2;
        }
        uint32_t ua = __shfl_up(a1, 1), ub = __shfl_up(b1, 1);
        uint32_t va = __shfl_up(a2, 1), vb = __shfl_up(b2, 1);
        if (lane == 0) {
            ua = pa;
            ub = pb;
            va = INVALID;
            vb = INVALID;
        }
        pa = __shfl(a1, 63);
        pb = __shfl(b1, 63);
        const bool u1 = right && !(ua == a1 && ub == b1) && a1 < n && b1 < n;
        const bool u2 = below && !(va == a2 && vb == b2) && a2 < n && b2 < n;
        bad |= (right && !(a1 < n && b1 < n)) || (below && !(a2 < n && b2 < n));
        // both unions' four walks in step, then both hooks
        uint32_t xs[4] = {a1, b1, a2, b2};
        uint64_t ws[4] = {u1 ? nodes[a1] : 0ull, u1 ? nodes[b1] : 0ull, u2 ? nodes[a2] : 0ull, u2 ? nodes[b2] : 0ull};
        n_find_m<4>(nodes, n, xs, ws, (u1 ? 3u : 0u) | (u2 ? 12u : 0u), bad);
        SW_PHASE(pc, 1);   // node words, walks to the roots
        if (bad) break;
        uint64_t ha[2] = {ws[0], ws[2]}, hb[2] = {ws[1], ws[3]};
        n_hook2(nodes, n, ha, hb, bad);
        SW_PHASE(pc, 2);   // hooks
    }
    if (bad) flag_error(d.err);
    SW_PHASE_FLUSH(pc, phase_table(1u));
}

// ---------------------------------------------------------------------------
// Flip: every site takes the state drawn for the smallest site index of its
// cluster.  Inside the tile the labels form a forest of tile-local indices
// whose terminals are the tile-local roots.  The tile's edge-forest nodes are
// loaded together at the start (node j by lane j / NW of wave j % NW) and
// search their roots (halving the paths they walk); then each wave draws, in
// compacted lanes, the states of its nodes (keyed by their roots) and of the
// roots of clusters inside the tile it found (keyed by their own sites).
// Wave w owns rows w, w+4, w+8, ... (lane = column); its labels are all
// loaded first.  LDS entries are 16 bits (so more workgroups fit a CU): a
// tile-local index, ROOT16 | slot for a node, ROOT16 | RES16 | state for a
// resolved root inside the tile.
// XY: the draw per cluster is a reflection bit instead of a state, and each
// site of a reflected cluster has its angle reflected across the line
// perpendicular to the sweep's direction (the others are not touched).
template <int TY, bool XY = false>
__global__ __launch_bounds__(threads_of<TY>()) __attribute__((amdgpu_waves_per_eu(8))) void k_flip(
    const LatDesc* descs, const WorkItem* map, uint32_t k)
{
    constexpr uint32_t NW = waves_of<TY>(), NT = threads_of<TY>();
    constexpr uint32_t PER = TY / NW;       // rows per wave
    constexpr uint32_t RES16 = 0x4000u;     // a resolved root inside the tile
    constexpr uint32_t NKN = 512;           // node table (>= nslot(TY), a power of two)
    constexpr uint32_t NODE_ENTRY = 0x8000u;   // a list entry that names a node
    static_assert(nslot(TY) <= NKN && nslot(TY) <= NT && nslot(TY) < RES16, "one thread per node");
    __shared__ uint16_t E[TY * TX];
    __shared__ uint16_t list[NW][PER * TX + 64 + 64];   // roots inside the tile, nodes, a scratch slot per lane
    __shared__ uint32_t NK[NKN];            // per node: its root's key, then its state

    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, blockIdx.x, true, d, tile, lat)) return;
    SW_PHASE_START(pc);
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *glb(d.counter) + k;
    const uint32_t tid = threadIdx.x, wave = wave_id(), lane = tid & 63u;
    const uint32_t L = d.L, w = g.w, h = g.h, x0 = g.x0, y0 = g.y0;
    const uint32_t col = lane;
    uint16_t* my_list = list[wave];
    const uint32_t NS = nslot(TY), n_nodes = d.ntiles * NS, node0 = tile * NS;
    const gptr<uint64_t> nodes = glb(d.nodes);
    bool bad = false;

    // The tile's entries are addressed from one wave-uniform base with 32-bit
    // per-lane offsets (a tile spans fewer than 2^32 / 4 sites of the arrays):
    // one vector add per row, where a scalar base per row would cost the busier
    // scalar unit two 64-bit adds.  Row j of this wave is row wave + NW j.
    const uint32_t site0 = wave * L + col;         // this lane's first site, from the tile origin
    const uint32_t wave_step = NW * L;             // sites between a wave's consecutive rows
    const gptr<const char> lab_tile = (gptr<const char>)(glb(d.tlab) + (size_t)y0 * L + x0);
    const gptr<char> s_tile = (gptr<char>)(glb(d.s) + (size_t)y0 * L + x0);
    const uint32_t n_used = min(glb(d.edges)[(size_t)tile * edge_words(TY) + 6], NS);
    // XY: the sweep's direction (wave-uniform)
    const uint32_t phi = XY ? __builtin_amdgcn_readfirstlane(xy_direction(d, t)) : 0u;

    // Full tiles (the common case) need no masks for columns or rows outside.
    auto body = [&](auto full) {
        constexpr bool FULL = decltype(full)::value;
        const bool vcol = FULL || col < w;
        uint32_t v[PER];
        gptr<const uint16_t> lab_p = (gptr<const uint16_t>)lab_tile + site0;
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t r = wave + NW * j;
            v[j] = (vcol && (FULL || r < h)) ? (uint32_t)*lab_p : 0u;
            lab_p += wave_step;
        }
        const uint32_t nj = lane * NW + wave;   // this lane's node
        const bool is_node = nj < n_used;
        const uint64_t nw = is_node ? nodes[node0 + nj] : 0ull;

        // row j of this wave: tile index li0 + j NW TX.  The labels go to E.  A
        // pointer to a larger site is found by the walk below.
        const uint32_t li0 = wave * TX + col;
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t r = wave + NW * j;
            if (!FULL && r >= h) continue;
            if (vcol) E[li0 + j * NW * TX] = (uint16_t)v[j];
        }
        SW_PHASE(pc, 0);   // labels in
        // The roots (tagged ROOT16), one ballot per row: a cluster inside the
        // tile joins this wave's list, a node's slot must name a node of the
        // tile (labels outside the tile are 0).  Lanes with nothing to list store
        // to their scratch slot instead of branching around the store.
        uint32_t nterm = 0;   // wave-uniform
        uint32_t badv = 0;
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t r = wave + NW * j;
            if (!FULL && r >= h) continue;
            const uint64_t m = ballot(v[j] == (ROOT16 | NOSLOT));
            badv |= (v[j] - (ROOT16 + n_used)) < (NOSLOT - n_used) ? 1u : 0u;
            my_list[lane_in(m) ? nterm + lanes_below(m) : PER * TX + 64 + lane] = (uint16_t)(li0 + j * NW * TX);
            nterm += popc64(m);
        }
        bad |= badv != 0;
        SW_PHASE(pc, 1);   // roots inside the tile listed
        // this wave's nodes find their roots' keys and join the list
        if (is_node) NK[nj] = key_of(n_find_from(nodes, n_nodes, node0 + nj, nw, bad));
        {
            const uint64_t m = ballot(is_node);
            if (is_node) my_list[nterm + lanes_below(m)] = (uint16_t)(NODE_ENTRY | nj);
            nterm += popc64(m);
        }
        SW_PHASE(pc, 2);   // node roots found

        // the states, 64 list entries at a time; lanes past the end work on a
        // copy they do not store
        for (uint32_t j0 = 0; j0 < nterm; j0 += 64) {
            const uint32_t j = j0 + lane;
            const bool act = j < nterm;
            const uint32_t e = my_list[act ? j : 0];
            const bool node = (e & NODE_ENTRY) != 0u;
            const uint32_t idx = e & ~NODE_ENTRY;
            const uint32_t key = node ? NK[idx & (NKN - 1u)] : __umul24(y0 + idx / TX, L) + x0 + idx % TX;
            const uint32_t st = XY ? xy_flip_bit(d, key, t) : cluster_state(d, key, t);
            if (act && node) NK[idx & (NKN - 1u)] = st;
            if (act && !node) E[idx & (TY * TX - 1u)] = ROOT16 | RES16 | st;
        }
        SW_PHASE(pc, 3);   // states drawn
        __syncthreads();
        SW_PHASE(pc, 4);   // barrier

        // Every site follows in-tile pointers (each to a smaller tile index, so
        // the walk ends) to a root: resolved inside the tile, or a node whose
        // state is in the table; the new spins are stored at the end.
        // (A root's entry, ROOT16 and up, is larger than every tile index, so
        // `x < cur` alone continues the walk.)
        auto walk = [&](uint32_t j) -> uint32_t {
            uint32_t cur = li0 + j * NW * TX, x = E[cur];
            while (x < cur) {
                cur = x;
                x = E[cur];
            }
            bad |= !(x & ROOT16);
            return (x & RES16) ? x : NK[x & (NKN - 1u)];
        };
        if constexpr (XY) {
            // one bit per row (reflect or not) keeps the loop's registers few
            uint32_t bits = 0;
#pragma unroll
            for (uint32_t j = 0; j < PER; ++j) {
                const uint32_t r = wave + NW * j;
                if (vcol && (FULL || r < h)) bits |= (walk(j) & 1u) << j;
            }
            SW_PHASE(pc, 5);   // walks
            // the reflected sites' angles in batches of eight: all loads of a
            // batch in flight together, then its stores
            const gptr<char> a_tile = (gptr<char>)(glb(d.ang) + (size_t)y0 * L + x0);
            constexpr uint32_t B = PER < 8 ? PER : 8;
#pragma unroll 1
            for (uint32_t j0 = 0; j0 < PER; j0 += B) {
                uint32_t av[B];
#pragma unroll
                for (uint32_t j = 0; j < B; ++j)
                    av[j] = ((bits >> (j0 + j)) & 1u) ? *(gptr<const uint32_t>)(a_tile + (site0 + (j0 + j) * wave_step) * 4u) : 0u;
#pragma unroll
                for (uint32_t j = 0; j < B; ++j)
                    if ((bits >> (j0 + j)) & 1u)
                        *(gptr<uint32_t>)(a_tile + (site0 + (j0 + j) * wave_step) * 4u) = xy_reflect(av[j], phi);
            }
        } else {
            uint32_t e[PER];
#pragma unroll
            for (uint32_t j = 0; j < PER; ++j) {
                const uint32_t r = wave + NW * j;
                e[j] = (vcol && (FULL || r < h)) ? walk(j) : 0u;
            }
            SW_PHASE(pc, 5);   // walks
            gptr<uint8_t> s_p = (gptr<uint8_t>)s_tile + site0;
#pragma unroll
            for (uint32_t j = 0; j < PER; ++j) {
                const uint32_t r = wave + NW * j;
                if (vcol && (FULL || r < h)) *s_p = (uint8_t)e[j];
                s_p += wave_step;
            }
        }
    };
    if (w == TX && h == TY) body(std::true_type{});
    else body(std::false_type{});
    SW_PHASE(pc, 6);   // spins out (Potts) or reflections (XY)
    if (bad) flag_error(d.err);
    SW_PHASE_FLUSH(pc, phase_table(XY ? 4u : 2u));

    // The ring record of the next sweep starts from zero.
    if (d.cap && tile == 0) {
        const uint32_t words = NCOPY * (XY ? XY_STRIDE : ring_stride(d.q));
        gptr<int64_t> rec = glb(d.ring) + (size_t)((t + 1) % d.cap) * words;
        for (uint32_t i = tid; i < words; i += NT) rec[i] = 0;
    }
}

// ---------------------------------------------------------------------------
// Cluster-size sums of a sweep's clusters, for the improved estimators of the
// moments of the magnetisation (given the clusters, the mean of |M|^2 over the
// clusters' independent uniform states is sum |C|^2, and that of |M|^4 a
// combination of (sum |C|^2)^2 and sum |C|^4).  After the flip the labels and
// the edge forest still describe the sweep's clusters.  k_csize: one workgroup
// per tile counts the sites of each tile-local cluster in LDS; a cluster
// inside the tile adds |C|^2 and |C|^4 at once, the others add their count to
// their edge-forest root.  k_croot: every edge-forest root adds the square and
// fourth power of its gathered size and clears it.  |C| <= 2^30, so |C|^2 fits
// 64 bits and the sums of |C|^4 take 128 (two words, carried by hand).

// v added to the 128-bit number (lo, hi), atomically.
template <class P>
__device__ __forceinline__ void add_u128(P lo, P hi, unsigned __int128 v, int scope)
{
    const uint64_t vl = (uint64_t)v, vh = (uint64_t)(v >> 64);
    if (!vl && !vh) return;
    uint64_t old = 0;
    if (scope == __HIP_MEMORY_SCOPE_AGENT)
        old = __hip_atomic_fetch_add(lo, (unsigned long long)vl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        old = __hip_atomic_fetch_add(lo, (unsigned long long)vl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const uint64_t up = vh + ((old + vl) < old ? 1u : 0u);
    if (!up) return;
    if (scope == __HIP_MEMORY_SCOPE_AGENT)
        __hip_atomic_fetch_add(hi, (unsigned long long)up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        __hip_atomic_fetch_add(hi, (unsigned long long)up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The workgroup's sums (in LDS) into ring record t, partial copy 0.
__device__ __forceinline__ void cs_flush(const LatDesc& d, uint32_t t, unsigned long long* sums, uint32_t tid)
{
    if (tid != 0 || !d.cap) return;
    const gptr<unsigned long long> rec =
        (gptr<unsigned long long>)(glb(d.ring) + (size_t)(t % d.cap) * NCOPY * ring_stride(d.q) + cs_word(d.q));
    if (sums[0]) __hip_atomic_fetch_add(rec, sums[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    add_u128(rec + 1, rec + 2, ((unsigned __int128)sums[2] << 64) | sums[1], __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void cs_add(unsigned long long* sums, uint64_t c)
{
    const uint64_t c2 = c * c;
    __hip_atomic_fetch_add(&sums[0], (unsigned long long)c2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    add_u128(&sums[1], &sums[2], (unsigned __int128)c2 * c2, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int TY>
__global__ __launch_bounds__(threads_of<TY>()) void k_csize(const LatDesc* descs, const WorkItem* map, uint32_t k)
{
    constexpr uint32_t NT = threads_of<TY>();
    __shared__ uint16_t E[TY * TX];
    __shared__ uint32_t C[TY * TX];
    __shared__ unsigned long long sums[3];
    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, blockIdx.x, true, d, tile, lat)) return;
    if (!d.csize) return;
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *glb(d.counter) + k;
    const uint32_t tid = threadIdx.x;
    const uint32_t NS = nslot(TY), n_nodes = d.ntiles * NS, node0 = tile * NS;
    const gptr<const uint16_t> lab = glb(d.tlab);
    bool bad = false;
    if (tid < 3) sums[tid] = 0;
    for (uint32_t li = tid; li < TY * TX; li += NT) {
        const uint32_t r = li / TX, c = li % TX;
        E[li] = (r < g.h && c < g.w) ? lab[(size_t)(g.y0 + r) * d.L + g.x0 + c] : (ROOT16 | NOSLOT);
        C[li] = 0;
    }
    __syncthreads();
    for (uint32_t li = tid; li < TY * TX; li += NT) {
        if (li / TX >= g.h || li % TX >= g.w) continue;
        uint32_t cur = li, x = E[cur];
        while (!(x & ROOT16) && x < cur) {
            cur = x;
            x = E[cur];
        }
        if (!(x & ROOT16)) {
            bad = true;
            continue;
        }
        atomicAdd(&C[cur], 1u);
    }
    __syncthreads();
    for (uint32_t li = tid; li < TY * TX; li += NT) {
        const uint32_t x = E[li], c = C[li];
        if (!(x & ROOT16) || !c) continue;
        const uint32_t slot = x & 0x7FFFu;
        if (slot == NOSLOT) {
            cs_add(sums, c);
        } else {
            const uint64_t rw = n_root(glb(d.nodes), n_nodes, node0 + slot, bad);
            if (!bad)
                __hip_atomic_fetch_add((gptr<unsigned long long>)(glb(d.csize) + node_of(rw)), (unsigned long long)c,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    cs_flush(d, t, sums, tid);
    if (bad) flag_error(d.err);
}

template <int TY>
__global__ __launch_bounds__(threads_of<TY>()) void k_croot(const LatDesc* descs, const WorkItem* map, uint32_t k)
{
    constexpr uint32_t NT = threads_of<TY>();
    __shared__ unsigned long long sums[3];
    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, blockIdx.x, true, d, tile, lat)) return;
    if (!d.csize) return;
    const uint32_t t = *glb(d.counter) + k;
    const uint32_t tid = threadIdx.x;
    const uint32_t NS = nslot(TY), node0 = tile * NS;
    const uint32_t n_used = min(glb(d.edges)[(size_t)tile * edge_words(TY) + 6], NS);
    if (tid < 3) sums[tid] = 0;
    __syncthreads();
    for (uint32_t s = tid; s < n_used; s += NT) {
        const uint32_t node = node0 + s;
        if (node_of(glb(d.nodes)[node]) != node) continue;   // not a root
        const uint64_t c = glb(d.csize)[node];
        glb(d.csize)[node] = 0;
        if (c) cs_add(sums, c);
    }
    __syncthreads();
    cs_flush(d, t, sums, tid);
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

// The last sweep's labels of rows [ya, yb) resolved to the smallest site index
// of each cluster, written from the base of the label region (row ya first):
// one workgroup per tile walks its sites' pointers in LDS to their tile-local
// roots and those, if they are nodes, to the edge forest's roots.  The tile
// labels (upper half of the region) are only read, so that (yb - ya) L <= N/2
// keeps the output clear of them.
template <int TY>
__global__ __launch_bounds__(threads_of<TY>()) void k_resolve(const LatDesc* descs, uint32_t lat, uint32_t ya,
                                                              uint32_t yb)
{
    constexpr uint32_t NT = threads_of<TY>();
    __shared__ uint16_t E[TY * TX];
    const LatDesc d = descs[lat];
    const uint32_t tile = blockIdx.x;
    if (tile >= d.ntiles) return;
    const TileGeom g = tile_geom(d, tile, TY);
    if (g.y0 >= yb || g.y0 + g.h <= ya) return;
    const uint32_t NS = nslot(TY), n_nodes = d.ntiles * NS, node0 = tile * NS;
    const gptr<const uint16_t> lab = glb(d.tlab);
    const gptr<uint32_t> out = glb(d.lab);
    bool bad = false;
    for (uint32_t li = threadIdx.x; li < TY * TX; li += NT) {
        const uint32_t r = li / TX, c = li % TX;
        E[li] = (r < g.h && c < g.w) ? lab[(size_t)(g.y0 + r) * d.L + g.x0 + c] : (ROOT16 | NOSLOT);
    }
    __syncthreads();
    for (uint32_t li = threadIdx.x; li < TY * TX; li += NT) {
        const uint32_t r = li / TX, c = li % TX, y = g.y0 + r;
        if (r >= g.h || c >= g.w || y < ya || y >= yb) continue;
        uint32_t cur = li, v = E[cur];
        while (!(v & ROOT16) && v < cur) {
            cur = v;
            v = E[cur];
        }
        uint32_t root = INVALID;
        if (!(v & ROOT16)) {
            bad = true;
        } else if ((v & ~ROOT16) == NOSLOT) {
            root = (g.y0 + cur / TX) * d.L + g.x0 + cur % TX;
        } else {
            root = key_of(n_root(glb(d.nodes), n_nodes, node0 + (v & ~ROOT16), bad));
        }
        out[(size_t)(y - ya) * d.L + g.x0 + c] = root;
    }
    if (bad) flag_error(d.err);
}

// One thread per (record, word): the sum of the word over the record's NCOPY
// partial copies.
__global__ __launch_bounds__(256) void k_ring_sum(const int64_t* ring, int64_t* out, uint32_t slots, uint32_t slot0,
                                                  uint32_t n, uint32_t W, uint32_t stride)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * W) return;
    const uint32_t rec = i / W, w = i - rec * W;
    const uint32_t slot = (uint32_t)(((uint64_t)slot0 + rec) % slots);
    const size_t R = stride;
    const gptr<const int64_t> copy0 = glb(ring) + (size_t)slot * NCOPY * R;
    const gptr<const int64_t> base = copy0 + w;
    int64_t sum = 0;
    if (copy0[W] != 0) {
        sum = base[0];   // the whole record is in copy 0
    } else {
#pragma unroll 8
        for (uint32_t c = 0; c < NCOPY; ++c) sum += base[(size_t)c * R];
    }
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

hipError_t launch_label_preset(const Work& w)
{
    if (w.nitems == 0) return hipSuccess;
    switch (w.ty) {
    case 32: hipLaunchKernelGGL((k_bond_label<32, true>), dim3(w.nitems), dim3(threads_of<32>()), 0, w.stream, w.descs, w.map, 0u, 0u); break;
    case 64: hipLaunchKernelGGL((k_bond_label<64, true>), dim3(w.nitems), dim3(threads_of<64>()), 0, w.stream, w.descs, w.map, 0u, 0u); break;
    case 128: hipLaunchKernelGGL((k_bond_label<128, true>), dim3(w.nitems), dim3(threads_of<128>()), 0, w.stream, w.descs, w.map, 0u, 0u); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_flip_xy(const Work& w, uint32_t k)
{
    if (w.nitems == 0) return hipSuccess;
    switch (w.ty) {
    case 32: hipLaunchKernelGGL((k_flip<32, true>), dim3(w.nitems), dim3(threads_of<32>()), 0, w.stream, w.descs, w.map, k); break;
    case 64: hipLaunchKernelGGL((k_flip<64, true>), dim3(w.nitems), dim3(threads_of<64>()), 0, w.stream, w.descs, w.map, k); break;
    case 128: hipLaunchKernelGGL((k_flip<128, true>), dim3(w.nitems), dim3(threads_of<128>()), 0, w.stream, w.descs, w.map, k); break;
    default: return hipErrorInvalidValue;
    }
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

hipError_t launch_cluster_sums(const Work& w, uint32_t k)
{
    if (w.nitems == 0) return hipSuccess;
    SWMI_TY_DISPATCH(w.ty, k_csize, w.nitems, w.descs, w.map, k);
    SWMI_TY_DISPATCH(w.ty, k_croot, w.nitems, w.descs, w.map, k);
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

hipError_t launch_resolve(const LatDesc* descs, uint32_t lat, uint32_t ntiles, uint32_t ty, uint32_t ya, uint32_t yb,
                          hipStream_t s)
{
    switch (ty) {
    case 32: hipLaunchKernelGGL(k_resolve<32>, dim3(ntiles), dim3(threads_of<32>()), 0, s, descs, lat, ya, yb); break;
    case 64: hipLaunchKernelGGL(k_resolve<64>, dim3(ntiles), dim3(threads_of<64>()), 0, s, descs, lat, ya, yb); break;
    case 128:
        hipLaunchKernelGGL(k_resolve<128>, dim3(ntiles), dim3(threads_of<128>()), 0, s, descs, lat, ya, yb);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ring_sum(const int64_t* ring, int64_t* out, uint32_t slots, uint32_t slot0, uint32_t n,
                           uint32_t words, uint32_t stride, hipStream_t s)
{
    const uint64_t total = (uint64_t)n * words;
    if (total == 0) return hipSuccess;
    if (total > 0xFFFFFFFFull || slot0 >= slots || n >= slots || words > stride) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ring_sum, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, ring, out, slots, slot0, n,
                       words, stride);
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
