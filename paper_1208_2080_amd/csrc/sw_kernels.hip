// HIP kernels of one Swendsen-Wang sweep for gfx950, plus their launchers.
//
// One sweep is three launches over the tiles of the lattice (TX = 128 columns
// by TY rows, one 256-thread workgroup per tile):
//   k_bond_label  bonds (Sec. 2 step (1)) + tile-local cluster labelling in LDS
//                 + measurement of the configuration the bonds were drawn on
//   k_merge       joins tile-local clusters across tile edges (global union-find
//                 with atomicMin, larger root under smaller)
//   k_flip        every cluster takes the state drawn for its smallest site
//                 index (Sec. 2 step (3)); each site copies it from its
//                 tile-local root
// plus k_measure after the last sweep of a call, and small helpers.
#include <hip/hip_runtime.h>

#include "sw_device.hpp"
#include "sw_kernels.hpp"

namespace swmi {

namespace {

// Every label points at a site index no larger than its own (roots at
// themselves), so every pointer chase strictly decreases and ends.  The loops
// still check that invariant and carry step caps, so a corrupted forest sets
// the error flag instead of spinning.
constexpr uint32_t LDS_CAP = 1u << 15;     // > sites of the largest tile
constexpr uint32_t FIND_CAP = 1u << 20;    // safety cap of global pointer chases
constexpr uint32_t UNITE_CAP = 1u << 12;   // safety cap of union retries

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

// Which lattice and tile this workgroup (or wave) works on.  Without a map the
// work is the tiles of lattice 0, optionally spread over XCDs.
__device__ __forceinline__ bool pick(const LatDesc* descs, const WorkItem* map, uint32_t idx,
                                     bool spread, LatDesc& d, uint32_t& tile)
{
    if (map) {
        const WorkItem it = map[idx];
        if (it.lat == INVALID) return false;
        d = descs[it.lat];
        tile = it.tile;
        return true;
    }
    d = descs[0];
    if (idx >= d.ntiles) return false;
    tile = spread ? xcd_tile(idx, d.ntiles) : idx;
    return true;
}

__device__ __forceinline__ void flag_error(uint32_t* err) { atomicOr(err, 1u); }

// ------------------------------------------------------- LDS union-find
// P holds, for every site of the tile, a tile-local index that is never larger
// than the site's own; roots point at themselves.  Finds halve paths with
// plain stores (a stored value is always an ancestor, so races are benign);
// unions hook the larger root under the smaller one with atomicMin and retry
// from the old value when the hooked node was no longer a root.
__device__ __forceinline__ uint32_t lds_ld(uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ uint32_t lds_find(uint32_t* P, uint32_t x, uint32_t* err)
{
    for (uint32_t it = 0; it < LDS_CAP; ++it) {
        const uint32_t p = lds_ld(&P[x]);
        if (p == x) return x;
        const uint32_t gp = lds_ld(&P[p]);
        if (p > x || gp > p) break;
        if (gp == p) return p;
        lds_st(&P[x], gp);
        x = gp;
    }
    flag_error(err);
    return x;
}

__device__ void lds_union(uint32_t* P, uint32_t a, uint32_t b, uint32_t* err)
{
    for (uint32_t it = 0; it < LDS_CAP; ++it) {
        a = lds_find(P, a, err);
        b = lds_find(P, b, err);
        if (a == b) return;
        if (a < b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        const uint32_t old = __hip_atomic_fetch_min(&P[a], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == a) return;
        a = old;
    }
    flag_error(err);
}

// ---------------------------------------------------- global union-find
__device__ uint32_t g_find(uint32_t* lab, uint32_t x, uint32_t* err)
{
    for (uint32_t it = 0; it < FIND_CAP; ++it) {
        const uint32_t p = ld_coherent(&lab[x]);
        if (p == x) return x;
        if (p > x) break;
        const uint32_t gp = ld_coherent(&lab[p]);
        if (gp == p) return p;
        if (gp > p) break;
        st_coherent(&lab[x], gp);
        x = gp;
    }
    flag_error(err);
    return x;
}

__device__ void g_unite(uint32_t* lab, uint64_t N, uint32_t a, uint32_t b, uint32_t* err)
{
    if (a >= N || b >= N) {
        flag_error(err);
        return;
    }
    for (uint32_t it = 0; it < UNITE_CAP; ++it) {
        a = g_find(lab, a, err);
        b = g_find(lab, b, err);
        if (a == b) return;
        if (a < b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        const uint32_t old = min_coherent(&lab[a], b);
        if (old == a) return;
        a = old;
    }
    flag_error(err);
}

// Read-only root search once the forest is final (after the merge kernel).
__device__ uint32_t g_root(const uint32_t* lab, uint32_t x, uint32_t* err)
{
    for (uint32_t it = 0; it < FIND_CAP; ++it) {
        const uint32_t p = lab[x];
        if (p == x) return x;
        if (p > x) break;
        x = p;
    }
    flag_error(err);
    return x;
}

// ------------------------------------------------------------ row access
// Lane l holds sites x0+2l and x0+2l+1 of a row (a = even offset, b = odd).
struct RowSpins {
    uint32_t a, b, halo;
};

__device__ __forceinline__ RowSpins load_row(const uint8_t* s, size_t base, uint32_t x0, uint32_t xa,
                                             bool va, bool vb, uint32_t xh)
{
    RowSpins r;
    r.a = va ? s[base + x0 + xa] : 0u;
    r.b = vb ? s[base + x0 + xa + 1] : 0u;
    r.halo = s[base + xh];
    return r;
}

// Count, for the measurement, the sites of this row in each state c >= 1.
__device__ __forceinline__ void count_states(uint32_t* hist, uint32_t q, uint32_t lane, bool va, bool vb,
                                             uint32_t sa, uint32_t sb)
{
    if (q <= 16) {
        for (uint32_t c = 1; c < q; ++c) {
            const uint32_t n = popc64(ballot(va && sa == c)) + popc64(ballot(vb && sb == c));
            if (lane == 0 && n) atomicAdd(&hist[c], n);
        }
    } else {
        if (va && sa) atomicAdd(&hist[sa], 1u);
        if (vb && sb) atomicAdd(&hist[sb], 1u);
    }
}

// Add a workgroup's measurement into a ring record (NCOPY partial copies).
__device__ __forceinline__ int64_t* ring_record(const LatDesc& d, uint32_t sweep, uint32_t copy)
{
    return d.ring + ((size_t)(sweep % d.cap) * NCOPY + copy) * (d.q + 1);
}

__device__ __forceinline__ void atomic_add_i64(int64_t* p, uint64_t v)
{
    atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}

}  // namespace

// ---------------------------------------------------------------------------
// Bonds + tile-local labels (+ measurement of the incoming configuration).
// flags bit 0: also measure the configuration the bonds are drawn on (it is
// the result of the previous sweep, t - 1).
template <int TY>
__global__ __launch_bounds__(256) void k_bond_label(const LatDesc* descs, const WorkItem* map, uint32_t k,
                                                   uint32_t flags)
{
    constexpr uint32_t RPW = TY / 4;   // rows per wave
    __shared__ uint32_t P[TY * TX];
    __shared__ uint64_t rb[TY][4];     // per row: +x bonds (2 words), +y bonds (2 words)
    __shared__ uint32_t hist[256];
    __shared__ uint32_t tot[2];

    LatDesc d;
    uint32_t tile;
    if (!pick(descs, map, blockIdx.x, true, d, tile)) return;
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *d.counter + k;
    const bool meas = d.cap != 0;
    const bool meas_prev = meas && (flags & 1u);
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    const uint32_t L = d.L, w = g.w, h = g.h, x0 = g.x0, y0 = g.y0;

    hist[tid] = 0;
    if (tid < 2) tot[tid] = 0;
    __syncthreads();

    const uint32_t xa = 2 * lane, xb = xa + 1;
    const bool va = xa < w, vb = xb < w;
    const uint32_t xh = (x0 + w == L) ? 0u : x0 + w;   // right halo column
    const uint32_t r0 = wave * RPW, r1 = min(h, r0 + RPW);
    uint32_t n_unsat = 0, n_active = 0;

    if (r0 < r1) {
        uint32_t y = y0 + r0;
        size_t base = (size_t)y * L;
        RowSpins cur = load_row(d.s, base, x0, xa, va, vb, xh);
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t yn = (r + 1 < h) ? y + 1 : ((y0 + h == L) ? 0u : y0 + h);
            const size_t nbase = (size_t)yn * L;
            const RowSpins nxt = load_row(d.s, nbase, x0, xa, va, vb, xh);

            const uint32_t s_next = __shfl_down(cur.a, 1);
            const uint32_t right_a = vb ? cur.b : cur.halo;
            const uint32_t right_b = (xb + 1 < w) ? s_next : cur.halo;

            // Philox words: one call covers the pair (2m, 2m+1) of site indices.
            const uint32_t site_a = (uint32_t)(base + x0 + xa);
            uint32_t wxa, wya, wxb, wyb;
            if (((base + x0) & 1u) == 0) {
                const u32x4 r4 = philox4x32_10(site_a >> 1, 0u, t, 0u, d.key0, d.key1);
                wxa = r4.x; wya = r4.y; wxb = r4.z; wyb = r4.w;
            } else {
                const u32x4 p4 = philox4x32_10(site_a >> 1, 0u, t, 0u, d.key0, d.key1);
                const u32x4 n4 = philox4x32_10((site_a >> 1) + 1u, 0u, t, 0u, d.key0, d.key1);
                wxa = p4.z; wya = p4.w; wxb = n4.x; wyb = n4.y;
            }
            const bool exa = cur.a == right_a, eya = cur.a == nxt.a;
            const bool exb = cur.b == right_b, eyb = cur.b == nxt.b;
            const bool on = d.thr_nz != 0;
            const bool bxa = va && exa && on && wxa <= d.thr_m1;
            const bool bya = va && eya && on && wya <= d.thr_m1;
            const bool bxb = vb && exb && on && wxb <= d.thr_m1;
            const bool byb = vb && eyb && on && wyb <= d.thr_m1;
            uint64_t bx0, bx1, by0, by1;
            interleave_row(ballot(bxa), ballot(bxb), bx0, bx1);
            interleave_row(ballot(bya), ballot(byb), by0, by1);
            if (lane == 0) {
                rb[r][0] = bx0; rb[r][1] = bx1; rb[r][2] = by0; rb[r][3] = by1;
                uint64_t* px = d.bonds + (size_t)y * d.W + 2 * g.tx;
                uint64_t* py = d.bonds + ((size_t)L + y) * d.W + 2 * g.tx;
                px[0] = bx0;
                py[0] = by0;
                if (w > 64) {
                    px[1] = bx1;
                    py[1] = by1;
                }
            }

            // Runs of +x bonds inside the tile: each site starts out labelled by
            // the first site of its run (the crossing bond at w-1 is left out).
            uint64_t hx0 = bx0, hx1 = bx1;
            if (w <= 64) hx0 &= ~(1ull << (w - 1));
            else hx1 &= ~(1ull << (w - 65));
            const uint64_t S0 = ~(hx0 << 1);
            const uint64_t S1 = ~((hx1 << 1) | (hx0 >> 63));
            uint32_t st_a;
            bool link_ab;
            if (xa < 64) {
                st_a = msb64(S0 & upto(xa));
                link_ab = (hx0 >> xa) & 1ull;
            } else {
                const uint64_t m = S1 & upto(xa - 64);
                st_a = m ? 64u + msb64(m) : msb64(S0);
                link_ab = (hx1 >> (xa - 64)) & 1ull;
            }
            const uint32_t st_b = link_ab ? st_a : xb;
            P[r * TX + xa] = r * TX + st_a;
            P[r * TX + xb] = r * TX + st_b;

            if (meas) {
                n_active += popc64(bx0) + popc64(bx1) + popc64(by0) + popc64(by1);
                if (meas_prev) {
                    n_unsat += popc64(ballot(va && !exa)) + popc64(ballot(va && !eya)) +
                               popc64(ballot(vb && !exb)) + popc64(ballot(vb && !eyb));
                    count_states(hist, d.q, lane, va, vb, cur.a, cur.b);
                }
            }
            cur = nxt;
            base = nbase;
            y = yn;
        }
    }
    if (meas && lane == 0) {
        atomicAdd(&tot[0], n_unsat);
        atomicAdd(&tot[1], n_active);
    }
    __syncthreads();

    // Tile edge record: crossing-bond masks.
    uint32_t* rec = d.edges + (size_t)tile * edge_words(TY);
    if (wave == 0) {
        for (uint32_t j = 0; j < TY; j += 64) {
            const uint32_t r = j + lane;
            bool bit = false;
            if (r < h) bit = (w <= 64) ? ((rb[r][0] >> (w - 1)) & 1ull) : ((rb[r][1] >> (w - 65)) & 1ull);
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
            const uint64_t b0 = rb[h - 1][2], b1 = rb[h - 1][3];
            rec[4] = (uint32_t)b0;
            rec[5] = (uint32_t)(b0 >> 32);
            rec[6] = (uint32_t)b1;
            rec[7] = (uint32_t)(b1 >> 32);
        }
    }

    // Vertical links between consecutive rows of the tile, skipping those that
    // join two runs already joined one column to the left.
    for (uint32_t r = r0; r < r1 && r + 1 < h; ++r) {
        uint64_t vy0 = rb[r][2], vy1 = rb[r][3];
        uint64_t h0 = rb[r][0], h1 = rb[r][1], n0 = rb[r + 1][0], n1 = rb[r + 1][1];
        if (w <= 64) {
            h0 &= ~(1ull << (w - 1));
            n0 &= ~(1ull << (w - 1));
        } else {
            h1 &= ~(1ull << (w - 65));
            n1 &= ~(1ull << (w - 65));
        }
        const uint64_t red0 = (vy0 << 1) & (h0 << 1) & (n0 << 1);
        const uint64_t red1 = ((vy1 << 1) | (vy0 >> 63)) & ((h1 << 1) | (h0 >> 63)) & ((n1 << 1) | (n0 >> 63));
        const uint64_t u0 = vy0 & ~red0, u1 = vy1 & ~red1;
        const uint64_t word = (xa < 64) ? u0 : u1;
        const uint32_t sh = xa & 63u;
        if ((word >> sh) & 1ull) lds_union(P, r * TX + xa, (r + 1) * TX + xa, d.err);
        if ((word >> (sh + 1)) & 1ull) lds_union(P, r * TX + xb, (r + 1) * TX + xb, d.err);
    }
    __syncthreads();

    // Final tile-local labels as global site indices.
    for (uint32_t r = r0; r < r1; ++r) {
        const size_t row = (size_t)(y0 + r) * L + x0;
        const uint32_t la = lds_find(P, r * TX + xa, d.err);
        const uint32_t lb = lds_find(P, r * TX + xb, d.err);
        const uint32_t ga = (uint32_t)((size_t)(y0 + (la >> 7)) * L + x0 + (la & 127u));
        const uint32_t gb = (uint32_t)((size_t)(y0 + (lb >> 7)) * L + x0 + (lb & 127u));
        if (va) d.lab[row + xa] = ga;
        if (vb) d.lab[row + xb] = gb;
        if (va && xa == w - 1) rec[8 + r] = ga;
        if (vb && xb == w - 1) rec[8 + r] = gb;
        if (lane == 0) rec[8 + TY + r] = ga;
        if (r == h - 1) {
            if (va) rec[8 + 2 * TY + xa] = ga;
            if (vb) rec[8 + 2 * TY + xb] = gb;
        }
        if (r == 0) {
            if (va) rec[8 + 2 * TY + TX + xa] = ga;
            if (vb) rec[8 + 2 * TY + TX + xb] = gb;
        }
    }

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
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t idx = blockIdx.x * 4 + wave;
    if (idx >= nitems) return;
    LatDesc d;
    uint32_t tile;
    if (!pick(descs, map, idx, false, d, tile)) return;
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t EW = edge_words(TY);
    const uint32_t t_right = g.ty * d.ntx + ((g.tx + 1 == d.ntx) ? 0u : g.tx + 1);
    const uint32_t t_below = ((g.ty + 1 == d.nty) ? 0u : g.ty + 1) * d.ntx + g.tx;
    const uint32_t* rec = d.edges + (size_t)tile * EW;
    const uint32_t* recR = d.edges + (size_t)t_right * EW;
    const uint32_t* recB = d.edges + (size_t)t_below * EW;

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
        if (bit && !(ua == a && ub == b)) g_unite(d.lab, (uint64_t)d.L * d.L, a, b, d.err);
    }
    // Bottom edge: column x joins (x, h-1) here with (x, 0) of the tile below.
    pa = INVALID;
    pb = INVALID;
    for (uint32_t j = 0; j < TX; j += 64) {
        const uint32_t x = j + lane;
        const bool bit = x < g.w && ((rec[4 + (x >> 5)] >> (x & 31u)) & 1u);
        uint32_t a = INVALID, b = INVALID;
        if (bit) {
            a = rec[8 + 2 * TY + x];
            b = recB[8 + 2 * TY + TX + x];
        }
        uint32_t ua = __shfl_up(a, 1), ub = __shfl_up(b, 1);
        if (lane == 0) {
            ua = pa;
            ub = pb;
        }
        pa = __shfl(a, 63);
        pb = __shfl(b, 63);
        if (bit && !(ua == a && ub == b)) g_unite(d.lab, (uint64_t)d.L * d.L, a, b, d.err);
    }
}

// ---------------------------------------------------------------------------
// Flip: every site takes the state drawn for the smallest site index of its
// cluster.  Inside the tile the labels form a forest whose terminals are the
// sites that are global roots or whose parent lies outside the tile; only the
// terminals search the global forest and draw a state, in compacted lanes.
template <int TY>
__global__ __launch_bounds__(256) void k_flip(const LatDesc* descs, const WorkItem* map, uint32_t k)
{
    constexpr uint32_t RPW = TY / 4;
    __shared__ uint32_t E[TY * TX];
    __shared__ uint16_t list[TY * TX];
    __shared__ uint32_t nlist;

    LatDesc d;
    uint32_t tile;
    if (!pick(descs, map, blockIdx.x, true, d, tile)) return;
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *d.counter + k;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    const uint32_t L = d.L, w = g.w, h = g.h, x0 = g.x0, y0 = g.y0;
    const uint32_t xa = 2 * lane, xb = xa + 1;
    const bool va = xa < w, vb = xb < w;
    const uint32_t r0 = wave * RPW, r1 = min(h, r0 + RPW);

    if (tid == 0) nlist = 0;
    __syncthreads();

    for (uint32_t r = r0; r < r1; ++r) {
        const size_t row = (size_t)(y0 + r) * L + x0;
#pragma unroll
        for (uint32_t part = 0; part < 2; ++part) {
            const uint32_t x = part ? xb : xa;
            const bool valid = part ? vb : va;
            const uint32_t li = r * TX + x;
            bool term = false;
            if (valid) {
                const uint32_t gi = (uint32_t)(row + x);
                const uint32_t v = d.lab[gi];
                term = true;
                if (v != gi) {
                    const uint32_t vy = div_L(d, v);
                    const uint32_t dy = vy - y0, dx = (v - vy * L) - x0;
                    if (dy < h && dx < w) {
                        E[li] = dy * TX + dx;
                        term = false;
                    }
                }
                if (term) E[li] = v;
            }
            const uint64_t m = ballot(term);
            if (m) {
                uint32_t at = 0;
                if (lane == 0) at = atomicAdd(&nlist, popc64(m));
                at = __shfl(at, 0);
                if (term) list[at + popc64(m & ((1ull << lane) - 1ull))] = (uint16_t)li;
            }
        }
    }
    __syncthreads();

    const uint32_t n = nlist;
    for (uint32_t j = tid; j < n; j += 256) {
        const uint32_t li = list[j];
        const uint32_t v = E[li];
        const uint32_t gi = (uint32_t)((size_t)(y0 + li / TX) * L + x0 + li % TX);
        uint32_t root = v;
        if (v != gi) {
            if (v < gi) root = g_root(d.lab, v, d.err);
            else flag_error(d.err);
        }
        E[li] = TERM | cluster_state(d, root, t);
    }
    __syncthreads();

    for (uint32_t r = r0; r < r1; ++r) {
        const size_t row = (size_t)(y0 + r) * L + x0;
        uint32_t ea = va ? E[r * TX + xa] : TERM;
        uint32_t eb = vb ? E[r * TX + xb] : TERM;
        // in-tile pointers strictly decrease, so these chases end
        for (uint32_t it = 0; it < LDS_CAP && !(ea & TERM); ++it) ea = E[ea];
        for (uint32_t it = 0; it < LDS_CAP && !(eb & TERM); ++it) eb = E[eb];
        if (!(ea & eb & TERM)) flag_error(d.err);
        if (va) d.s[row + xa] = (uint8_t)ea;
        if (vb) d.s[row + xb] = (uint8_t)eb;
    }

    // The ring record of the next sweep starts from zero.
    if (d.cap && tile == 0) {
        int64_t* rec = d.ring + (size_t)((t + 1) % d.cap) * NCOPY * (d.q + 1);
        for (uint32_t i = tid; i < NCOPY * (d.q + 1); i += 256) rec[i] = 0;
    }
}

// ---------------------------------------------------------------------------
// Measurement of the current configuration into the ring record of sweep
// counter + k (used after the last sweep of a call).
template <int TY>
__global__ __launch_bounds__(256) void k_measure(const LatDesc* descs, const WorkItem* map, uint32_t k,
                                                const uint32_t* n_each)
{
    constexpr uint32_t RPW = TY / 4;
    __shared__ uint32_t hist[256];
    __shared__ uint32_t tot;
    LatDesc d;
    uint32_t tile;
    if (!pick(descs, map, blockIdx.x, true, d, tile)) return;
    if (d.cap == 0) return;
    if (n_each) {
        const uint32_t nl = n_each[map[blockIdx.x].lat];
        if (nl == 0) return;
        k = nl - 1;
    }
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *d.counter + k;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    const uint32_t L = d.L, w = g.w, h = g.h, x0 = g.x0, y0 = g.y0;
    hist[tid] = 0;
    if (tid == 0) tot = 0;
    __syncthreads();
    const uint32_t xa = 2 * lane, xb = xa + 1;
    const bool va = xa < w, vb = xb < w;
    const uint32_t xh = (x0 + w == L) ? 0u : x0 + w;
    const uint32_t r0 = wave * RPW, r1 = min(h, r0 + RPW);
    uint32_t n_unsat = 0;
    if (r0 < r1) {
        uint32_t y = y0 + r0;
        size_t base = (size_t)y * L;
        RowSpins cur = load_row(d.s, base, x0, xa, va, vb, xh);
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t yn = (r + 1 < h) ? y + 1 : ((y0 + h == L) ? 0u : y0 + h);
            const size_t nbase = (size_t)yn * L;
            const RowSpins nxt = load_row(d.s, nbase, x0, xa, va, vb, xh);
            const uint32_t s_next = __shfl_down(cur.a, 1);
            const uint32_t right_a = vb ? cur.b : cur.halo;
            const uint32_t right_b = (xb + 1 < w) ? s_next : cur.halo;
            n_unsat += popc64(ballot(va && cur.a != right_a)) + popc64(ballot(va && cur.a != nxt.a)) +
                       popc64(ballot(vb && cur.b != right_b)) + popc64(ballot(vb && cur.b != nxt.b));
            count_states(hist, d.q, lane, va, vb, cur.a, cur.b);
            cur = nxt;
            base = nbase;
            y = yn;
        }
    }
    if (lane == 0) atomicAdd(&tot, n_unsat);
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
        d.s[i] = random_start
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
        const uint32_t v = d.lab[i];
        if (v <= i) d.lab[i] = g_root(d.lab, v, d.err);
        else flag_error(d.err);
    }
}

// Advance sweep counters: lattice i by n (or by n_each[i] when given).
__global__ void k_bump(const LatDesc* descs, uint32_t count, const uint32_t* n_each, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const uint32_t add = n_each ? n_each[i] : n;
        if (add) *descs[i].counter += add;
    }
}

// ---------------------------------------------------------------- launchers
namespace {
uint32_t init_grid(size_t N)
{
    const size_t b = (N + 255) / 256;
    return (uint32_t)(b < 65536 ? (b ? b : 1) : 65536);
}
}  // namespace

#define SWMI_TY_DISPATCH(TYV, KERNEL, GRID, ...)                                                  \
    switch (TYV) {                                                                                \
    case 32: hipLaunchKernelGGL(KERNEL<32>, dim3(GRID), dim3(256), 0, w.stream, __VA_ARGS__); break;  \
    case 64: hipLaunchKernelGGL(KERNEL<64>, dim3(GRID), dim3(256), 0, w.stream, __VA_ARGS__); break;  \
    case 128: hipLaunchKernelGGL(KERNEL<128>, dim3(GRID), dim3(256), 0, w.stream, __VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                                                         \
    }

hipError_t launch_bond_label(const Work& w, uint32_t k, uint32_t flags)
{
    if (w.nitems == 0) return hipSuccess;
    SWMI_TY_DISPATCH(w.ty, k_bond_label, w.nitems, w.descs, w.map, k, flags);
    return hipGetLastError();
}

hipError_t launch_merge(const Work& w)
{
    if (w.nitems == 0) return hipSuccess;
    SWMI_TY_DISPATCH(w.ty, k_merge, (w.nitems + 3) / 4, w.descs, w.map, w.nitems);
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

hipError_t launch_bump(const LatDesc* descs, uint32_t count, const uint32_t* n_each, uint32_t n, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bump, dim3((count + 255) / 256), dim3(256), 0, s, descs, count, n_each, n);
    return hipGetLastError();
}

}  // namespace swmi
