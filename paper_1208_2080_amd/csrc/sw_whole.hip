// Small lattices swept whole in one workgroup's LDS, many sweeps per launch.
//
// A lattice of at most 128 x 128 sites fits a workgroup's LDS with its spins,
// bonds and union-find; one launch then runs any number of sweeps without
// touching global memory between them (no per-sweep launches, which is what
// bounds the tile kernels at these sizes).  Each sweep takes the three steps of
// Sec. 2 with the same random streams and the same cluster keys as the tile
// kernels, so results are bit-identical to them (and to the oracle):
//   (1) bonds: one Philox call per site pair (counter (i >> 1, 0, t, 0), the
//       pair's words 2b, 2b + 1 for site parity b) against the threshold;
//       with L even a lane pair draws for two rows at once (lane 2m the pair
//       of row y, lane 2m + 1 that of row y + 1, halves swapped), as in the
//       tile kernels, so each call is made once;
//   (2) labels: every wave takes whole rows; within a row (64 columns at a
//       time) a site points at the first site of its run of +x bonds (a
//       ballot, no atomics), then union-find joins the runs along the +y
//       bonds (one bond per pair of runs), across 64-column chunks and across
//       the periodic edges, the larger root hooked under the smaller, so each
//       cluster's root is its smallest site;
//   (3) every root draws its cluster's state (counter (root, 0, t, 1)), the
//       roots gathered into a per-wave list and drawn 64 at a time, and every
//       site copies its root's;
// then the measurement of the new configuration into the ring record of the
// sweep (written whole into copy 0, with the whole-record flag).  After the
// last sweep: the spins go back to global memory, and on request the labels
// (smallest site indices) and the tile-major bond words of that sweep.
#include <hip/hip_runtime.h>

#include "sw_device.hpp"
#include "sw_kernels.hpp"
#include "sw_tile.hpp"

namespace swmi {

namespace {

template <int LMAX>
constexpr uint32_t whole_threads() { return LMAX <= 64 ? 512u : 1024u; }

// The states of the wave's lanes counted into hist (LDS): one pass per
// distinct state present in the wave.
__device__ __forceinline__ void count_wave_states(uint32_t* hist, bool valid, uint32_t s)
{
    uint64_t left = ballot(valid);
    while (left) {
        const uint32_t first = (uint32_t)__builtin_ctzll(left);
        const uint32_t c = __builtin_amdgcn_readlane(s, first);
        const uint64_t same = ballot(valid && s == c);
        if ((threadIdx.x & 63u) == 0) atomicAdd(&hist[c], (uint32_t)__popcll(same));
        left &= ~same;
    }
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o);
    return v;
}

// Sweeps counter + k0 .. counter + k0 + n - 1.  flags bit 0: write the labels
// and bond words of the last sweep; bit 1: leave the sweep counter (the caller
// advances it), else set it past the last sweep.  ty: tile height of the
// lattice's bond-word layout.
template <int LMAX>
__global__ __launch_bounds__(whole_threads<LMAX>()) void k_whole(const LatDesc* descs, const uint32_t* list,
                                                                  uint32_t k0, uint32_t n_uniform,
                                                                  const uint32_t* n_each, uint32_t flags, uint32_t ty)
{
    constexpr uint32_t NT = whole_threads<LMAX>();
    constexpr uint32_t NMAX = LMAX * LMAX;
    __shared__ uint8_t s[NMAX];
    __shared__ uint8_t bnd[NMAX];                     // bit 0: +x bond, bit 1: +y bond
    __shared__ __align__(16) uint16_t P[NMAX];
    __shared__ uint32_t hist[256];
    __shared__ uint32_t tot[2];                       // n_unsat, n_active
    constexpr uint32_t QCAP = 256;                    // per wave: queued unions (two 16-bit sites each)
    __shared__ uint32_t UQ[NT / 64][QCAP];

    const uint32_t lat = list ? list[blockIdx.x] : blockIdx.x;
    const LatDesc d = descs[lat];
    const uint32_t n = n_each ? n_each[lat] : n_uniform;
    if (n == 0) return;
    constexpr uint32_t NW = NT / 64;
    const uint32_t L = d.L, N = L * L, q = d.q;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    if (L > LMAX) {   // (the host sorts lattices by size; never taken)
        if (tid == 0) flag_error(d.err);
        return;
    }
    const uint32_t t0 = *glb(d.counter) + k0;
    const bool meas = d.cap != 0;
    bool bad = false;

    auto right = [&](uint32_t i, uint32_t x) { return (x + 1 == L) ? i - x : i + 1; };
    auto down = [&](uint32_t i, uint32_t x, uint32_t y) { return (y + 1 == L) ? x : i + L; };

    for (uint32_t i = tid; i < N; i += NT) s[i] = glb(d.s)[i];
    __syncthreads();

    for (uint32_t k = 0; k < n; ++k) {
        const uint32_t t = t0 + k;
        if (tid < 256) hist[tid] = 0;
        if (tid < 2) tot[tid] = 0;
        // (1) bonds, row by row (64 columns per pass, one column per lane), each
        // site's two draws from its pair's Philox call; each site points at the
        // first site of its run
        uint32_t active = 0;
        {
        auto bond_row = [&](uint32_t y, uint32_t x0, uint32_t wx, uint32_t wy) {
            const uint32_t x = x0 + lane, i = y * L + x;
            const bool v = x < L;
            bool bx = false, by = false;
            if (v) {
                const uint32_t si = s[i];
                bx = d.thr_nz && si == s[right(i, x)] && wx <= d.thr_m1;
                by = d.thr_nz && si == s[down(i, x, y)] && wy <= d.thr_m1;
                bnd[i] = (uint8_t)((bx ? 1u : 0u) | (by ? 2u : 0u));
            }
            active += (uint32_t)bx + (uint32_t)by;
            const uint64_t validm = ballot(v);
            const uint64_t C = (ballot(bx) << 1) & validm;   // bit x: bond (x-1) -> x inside the pass
            const uint64_t S = ~C & validm;                  // first sites of runs
            const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
            if (v) P[i] = (uint16_t)(y * L + x0 + 63u - (uint32_t)__builtin_clzll(S & upto));
        };
        if ((L & 1u) == 0) {
            // wave w takes the row pairs (2w, 2w + 1), (2w + 2 NW, ...), ...; a
            // pass's valid lanes come in whole pairs (L and 64 are even)
            const bool odd = lane & 1u;
            for (uint32_t y = 2 * wave; y < L; y += 2 * NW) {
                for (uint32_t x0 = 0; x0 < L; x0 += TX) {
                    const uint32_t pair = ((odd ? (y + 1) * L : y * L) + x0 + (lane & ~1u)) >> 1;
                    const u32x4 q4 = philox4x32_10(pair, 0u, t, 0u, d.key0, d.key1);
                    const uint32_t recv0 = swap_pair(odd ? q4.x : q4.z);
                    const uint32_t recv1 = swap_pair(odd ? q4.y : q4.w);
                    bond_row(y, x0, odd ? recv0 : q4.x, odd ? recv1 : q4.y);
                    bond_row(y + 1, x0, odd ? q4.z : recv0, odd ? q4.w : recv1);
                }
            }
        } else {
            // wave w takes rows w, w + NW, ...; each lane its own site's call
            for (uint32_t y = wave; y < L; y += NW) {
                for (uint32_t x0 = 0; x0 < L; x0 += TX) {
                    const uint32_t i = y * L + x0 + lane;
                    const u32x4 w = philox4x32_10(i >> 1, 0u, t, 0u, d.key0, d.key1);
                    bond_row(y, x0, (i & 1u) ? w.z : w.x, (i & 1u) ? w.w : w.y);
                }
            }
        }
        }
        __syncthreads();
        // (2) unions, queued per wave and run 64 at a time with every lane busy
        // (the cost of a union is a few dependent LDS round trips, so batches
        // matter more than counts): the +x bonds leaving a 64-column pass
        // (into the next pass or across the periodic edge) and the +y bonds
        // between runs (one per pair of runs: a bond whose left neighbour joins
        // the same two runs adds nothing); each wave takes a strip of rows, and
        // the +y bonds out of a strip's last row are joined after a barrier
        uint32_t qn = 0;   // wave-uniform
        auto drain = [&]() {
            for (uint32_t j0 = 0; j0 < qn; j0 += 64) {
                const uint32_t j = j0 + lane;
                if (j < qn) {
                    const uint32_t e = UQ[wave][j];
                    lds_union(P, e & 0xFFFFu, e >> 16, bad);
                }
            }
            qn = 0;
        };
        auto push = [&](uint64_t m, uint32_t a, uint32_t b) {
            const uint32_t at = qn + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            if ((m >> lane) & 1ull) UQ[wave][at] = a | (b << 16);
            qn += (uint32_t)__popcll(m);
            if (qn > QCAP - 64) drain();
        };
        auto vertical = [&](uint32_t y, uint32_t x0) {
            const uint32_t yd = (y + 1 == L) ? 0u : y + 1;
            const uint32_t x = x0 + lane, i = y * L + x;
            const bool v = x < L;
            const uint32_t b = v ? bnd[i] : 0u, bd = v ? bnd[yd * L + x] : 0u;
            const uint64_t validm = ballot(v);
            const uint64_t V = ballot(b & 2u);
            const uint64_t Cu = (ballot(b & 1u) << 1) & validm, Cd = (ballot(bd & 1u) << 1) & validm;
            const uint64_t R = V & (V << 1) & Cu & Cd;
            push(V & ~R, i, yd * L + x);
        };
        const uint32_t rps = (L + NW - 1) / NW;   // rows of a wave's strip
        const uint32_t y_lo = min(L, wave * rps), y_hi = min(L, y_lo + rps);
        for (uint32_t y = y_lo; y < y_hi; ++y) {
            for (uint32_t x0 = 0; x0 < L; x0 += TX) {
                const uint32_t x = x0 + lane, i = y * L + x;
                const bool out = x < L && (bnd[i] & 1u) && (lane == 63 || x + 1 == L);
                push(ballot(out), i, x < L ? right(i, x) : 0u);
            }
            if (y + 1 < y_hi)
                for (uint32_t x0 = 0; x0 < L; x0 += TX) vertical(y, x0);
        }
        drain();
        __syncthreads();
        if (y_lo < y_hi)
            for (uint32_t x0 = 0; x0 < L; x0 += TX) vertical(y_hi - 1, x0);
        drain();
        __syncthreads();
        // every entry straight to its root: the forest is final, so a site walks
        // to its root reading only and stores it; a walk passing a stored entry
        // meets the same root (entries only ever point at ancestors)
        for (uint32_t i = tid; i < N; i += NT) {
            uint32_t r = i, p = lds_ld(&P[r]);
            for (uint32_t it = 0; p < r && it < LDS_CAP; ++it) {
                r = p;
                p = lds_ld(&P[r]);
            }
            bad |= p != r;
            lds_st(&P[i], r);
        }
        __syncthreads();
        // (3) roots draw their clusters' states, gathered into the wave's queue
        // (free after the unions) and drawn 64 at a time, then every site takes
        // its root's
        {
            uint32_t nr = 0;   // wave-uniform
            auto draw = [&]() {
                for (uint32_t j0 = 0; j0 < nr; j0 += 64) {
                    const uint32_t j = j0 + lane;
                    if (j < nr) {
                        const uint32_t r = UQ[wave][j];
                        s[r] = (uint8_t)state_of_draw(philox4x32_10(r, 0u, t, 1u, d.key0, d.key1).x, q);
                    }
                }
                nr = 0;
            };
            for (uint32_t i0 = 0; i0 < N; i0 += NT) {
                const uint32_t i = i0 + tid;
                const bool root = i < N && P[i] == i;
                const uint64_t m = ballot(root);
                if (root) UQ[wave][nr + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = i;
                nr += (uint32_t)__popcll(m);
                if (nr > QCAP - 64) draw();
            }
            draw();
        }
        __syncthreads();
        for (uint32_t i = tid; i < N; i += NT) {
            const uint32_t r = P[i];
            if (r != i) s[i] = s[r];
        }
        __syncthreads();
        if (meas) {
            // the new configuration: unequal nearest-neighbour pairs, states
            uint32_t unsat = 0;
            for (uint32_t i0 = 0; i0 < N; i0 += NT) {   // every lane of a wave takes part in the counting
                const uint32_t i = i0 + tid;
                const bool v = i < N;
                uint32_t si = 0;
                if (v) {
                    const uint32_t y = div_L(d, i), x = i - y * L;
                    si = s[i];
                    unsat += (uint32_t)(si != s[right(i, x)]) + (uint32_t)(si != s[down(i, x, y)]);
                }
                count_wave_states(hist, v, si);
            }
            const uint32_t us = wave_sum_u32(unsat), ac = wave_sum_u32(active);
            if ((tid & 63u) == 0) {
                atomicAdd(&tot[0], us);
                atomicAdd(&tot[1], ac);
            }
            __syncthreads();
            // the whole record into copy 0, flagged as whole
            const gptr<int64_t> rec = glb(d.ring) + (size_t)(t % d.cap) * NCOPY * ring_stride(q);
            if (tid == 0) {
                rec[0] = tot[0];
                rec[1] = tot[1];
                rec[ring_words(q)] = 1;
            }
            if (tid >= 1 && tid < q) rec[1 + tid] = hist[tid];
            __syncthreads();
        }
    }

    // back to global memory: spins, and on request the last sweep's labels and bonds
    for (uint32_t i = tid; i < N; i += NT) glb(d.s)[i] = s[i];
    if (flags & 1u) {
        for (uint32_t i = tid; i < N; i += NT) glb(d.lab)[i] = P[i];
        // bond words, tile-major (tile, plane, row), one ballot per row, plane
        // and 64-column tile; wave w takes rows w, w + NT/64, ...
        for (uint32_t y = wave; y < L; y += NT / 64) {
            for (uint32_t x0 = 0; x0 < L; x0 += TX) {
                const uint32_t x = x0 + lane;
                const uint32_t b = x < L ? bnd[y * L + x] : 0u;
                const uint64_t bx = ballot(b & 1u), by = ballot(b & 2u);
                const size_t tile = (size_t)(y / ty) * d.ntx + x0 / TX;
                const uint32_t r = y % ty;
                if (lane == 0) {
                    glb(d.bonds)[(tile * 2 + 0) * ty + r] = bx;
                    glb(d.bonds)[(tile * 2 + 1) * ty + r] = by;
                }
            }
        }
    }
    // the record after the last one starts from zero (the tile kernels add into it)
    if (meas) {
        const uint32_t words = NCOPY * ring_stride(q);
        const gptr<int64_t> rec = glb(d.ring) + (size_t)((t0 + n) % d.cap) * words;
        for (uint32_t i = tid; i < words; i += NT) rec[i] = 0;
    }
    if (bad) flag_error(d.err);
    __syncthreads();
    if (tid == 0 && !(flags & 2u)) *glb(d.counter) = t0 + n;
}

}  // namespace

hipError_t launch_whole(const LatDesc* descs, const uint32_t* list, uint32_t count, uint32_t lmax, uint32_t k0,
                        uint32_t n_uniform, const uint32_t* n_each, uint32_t flags, uint32_t ty, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    if (lmax <= 64)
        hipLaunchKernelGGL(k_whole<64>, dim3(count), dim3(whole_threads<64>()), 0, s, descs, list, k0, n_uniform,
                           n_each, flags, ty);
    else if (lmax <= WHOLE_LMAX)
        hipLaunchKernelGGL(k_whole<128>, dim3(count), dim3(whole_threads<128>()), 0, s, descs, list, k0, n_uniform,
                           n_each, flags, ty);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace swmi
