// The classical XY model swept by the same SW multi-cluster machinery, with
// Wolff's embedded clusters (the extension named in Sec. 5 of the paper): a
// random direction r = (cos phi, sin phi) per sweep, the projections
// c_i = cos(theta_i - phi), a bond between neighbours with c_i c_j > 0 active
// with probability 1 - exp(-2K c_i c_j), and every cluster reflected across
// the line perpendicular to r with probability 1/2.
//
// Only the bond step and the measurement are the model's own (this file);
// the labelling runs the Potts labeller over the bond words written here, the
// cross-tile merge is shared unchanged, and the flip is the Potts flip's
// per-cluster walk with a reflection bit in place of a new state.
//
// Angles are uint32 fractions of a full turn (unit 2^-32).  The bond test and
// the observables need sin and cos; both take off the nearest quarter turn in
// integer arithmetic (exact) and evaluate the rest, at most an eighth of a
// turn, in FP64 by Taylor polynomials, then rotate by the quarter turns.
#include <hip/hip_runtime.h>

#include "sw_device.hpp"
#include "sw_kernels.hpp"
#include "sw_tile.hpp"

namespace swmi {

namespace {

constexpr double PI_2_31 = 3.14159265358979323846264338327950288 / 2147483648.0;   // pi / 2^31

// sin and cos of the angle a (a fraction a / 2^32 of a turn).  With k the
// nearest quarter turn and d = a - k 2^30 in [-2^29, 2^29), x = d pi / 2^31
// lies in [-pi/4, pi/4); the Taylor series of sin to x^17 and of cos to x^18
// leave out less than 1e-19 there.
__device__ __forceinline__ void sincos_turn(uint32_t a, double& s, double& c)
{
    const uint32_t k = ((a + 0x20000000u) >> 30) & 3u;
    const int32_t d = (int32_t)(a - (k << 30));
    const double x = (double)d * PI_2_31;
    const double x2 = x * x;
    // sin x = x + x^3 (-1/3! + x^2 (1/5! - ...)), cos x = 1 + x^2 (-1/2! + x^2 (1/4! - ...))
    double ps = 1.0 / 355687428096000.0;           // 1/17!
    ps = fma(ps, x2, -1.0 / 1307674368000.0);      // 1/15!
    ps = fma(ps, x2, 1.0 / 6227020800.0);          // 1/13!
    ps = fma(ps, x2, -1.0 / 39916800.0);           // 1/11!
    ps = fma(ps, x2, 1.0 / 362880.0);              // 1/9!
    ps = fma(ps, x2, -1.0 / 5040.0);               // 1/7!
    ps = fma(ps, x2, 1.0 / 120.0);                 // 1/5!
    ps = fma(ps, x2, -1.0 / 6.0);                  // 1/3!
    const double sx = fma(x * x2, ps, x);
    double pc = 1.0 / 6402373705728000.0;          // 1/18!
    pc = fma(pc, x2, -1.0 / 20922789888000.0);     // 1/16!
    pc = fma(pc, x2, 1.0 / 87178291200.0);         // 1/14!
    pc = fma(pc, x2, -1.0 / 479001600.0);          // 1/12!
    pc = fma(pc, x2, 1.0 / 3628800.0);             // 1/10!
    pc = fma(pc, x2, -1.0 / 40320.0);              // 1/8!
    pc = fma(pc, x2, 1.0 / 720.0);                 // 1/6!
    pc = fma(pc, x2, -1.0 / 24.0);                 // 1/4!
    pc = fma(pc, x2, 0.5);                         // the 1/2! term, subtracted below
    const double cx = fma(-x2, pc, 1.0);
    // rotate by k quarter turns
    const bool odd = k & 1u;
    const double ss = odd ? cx : sx, cc = odd ? sx : cx;
    s = (k >= 2u) ? -ss : ss;
    c = (k == 1u || k == 2u) ? -cc : cc;
}

// A term of an observable sum: v rounded to a multiple of 2^-30 (to nearest,
// ties to even), in those units.
__device__ __forceinline__ long long fx30(double v) { return __double2ll_rn(v * 1073741824.0); }

__device__ __forceinline__ uint64_t shfl_down1(uint64_t v)
{
    const uint32_t lo = (uint32_t)__shfl_down((int)(uint32_t)v, 1), hi = (uint32_t)__shfl_down((int)(uint32_t)(v >> 32), 1);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ long long wave_sum_i64(long long v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o), hi = (uint32_t)__shfl_xor((int)(uint32_t)((uint64_t)v >> 32), o);
        v += (long long)(((uint64_t)hi << 32) | lo);
    }
    return v;
}

__device__ __forceinline__ int64_t* xy_record(const LatDesc& d, uint32_t sweep, uint32_t copy)
{
    return d.ring + ((size_t)(sweep % d.cap) * NCOPY + copy) * XY_STRIDE;
}

// ---------------------------------------------------------------------------
// Bonds of sweep t = counter + k, and/or the measurement of a configuration.
//
// flags bit 0: also measure the incoming configuration (the result of sweep
// t - 1) into record t - 1; bit 1: only measure the current configuration
// into record t (no bonds; k = 0xFFFFFFFF names the last sweep done).
//
// One workgroup per tile, one column per lane, each wave a strip of rows.  A
// site's +x and +y bonds use one Philox call (counter (i, 0, t, 4)): words
// 0, 1 make the 53-bit uniform of the +x bond, words 2, 3 that of the +y bond.
// The projection of the site below is the next row's own, and that of the
// site to the right the right-hand lane's, so each site evaluates one
// projection; the column right of the tile is evaluated once per tile.  The
// bond words go to the tile-major bond plane the labeller reads.
template <int TY>
__global__ __launch_bounds__(threads_of<TY>()) void k_xy_bonds(const LatDesc* descs, const WorkItem* map, uint32_t k,
                                                               uint32_t flags)
{
    constexpr uint32_t NW = waves_of<TY>();
    constexpr uint32_t RPW = TY / NW;
    __shared__ unsigned long long acc[XY_WORDS];   // n_active, Ex, Ey, Ix, Iy, Mx, My
    __shared__ double cedge[TY];                   // projections of the column right of the tile
    __shared__ uint32_t aedge[TY];                 // its angles

    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, blockIdx.x, true, d, tile, lat)) return;
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *glb(d.counter) + k;
    const bool only_measure = (flags & 2u) != 0;
    const bool meas = d.cap != 0 && (flags & 3u) != 0;
    const uint32_t tid = threadIdx.x, wave = wave_id(), lane = tid & 63u;
    const uint32_t L = d.L, w = g.w, h = g.h, x0 = g.x0, y0 = g.y0;
    const uint32_t phi = xy_direction(d, t);
    const gptr<uint32_t> ang = glb(d.ang);
    const uint32_t xe = (x0 + w == L) ? 0u : x0 + w;   // the column right of the tile

    if (tid < XY_WORDS) acc[tid] = 0ull;
    if (tid < h) {
        const uint32_t ae = ang[(y0 + tid) * L + xe];
        double s, c;
        sincos_turn(ae - phi, s, c);
        aedge[tid] = ae;
        cedge[tid] = c;
    }
    __syncthreads();

    const bool vx = lane < w;
    const bool edge = lane == w - 1;
    const uint32_t x = x0 + (vx ? lane : 0u);
    const uint32_t r0 = wave * RPW, r1 = min(h, r0 + RPW);
    const uint64_t validm = (w == 64) ? ~0ull : ((1ull << w) - 1ull);
    const double k2 = d.k2;
    const PhiloxKeys ks = philox_keys_v(d.key0, d.key1);
    const gptr<uint64_t> bw = glb(d.bonds) + (size_t)tile * 2 * TY;
    uint32_t n_active = 0;   // wave-uniform
    long long ex = 0, ey = 0, ix = 0, iy = 0, mx = 0, my = 0;

    if (r0 < r1) {
        uint32_t a = ang[(y0 + r0) * L + x];
        double cp;
        {
            double s;
            sincos_turn(a - phi, s, cp);
        }
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t y = y0 + r, yd = (y + 1 == L) ? 0u : y + 1;
            const uint32_t i = y * L + x;   // site indices fit 32 bits (N <= 2^32)
            const uint32_t ad = ang[yd * L + x];
            const uint32_t a_right = (uint32_t)__shfl_down((int)a, 1);
            const uint32_t ar = edge ? aedge[r] : a_right;
            double cd;
            {
                double s;
                sincos_turn(ad - phi, s, cd);
            }
            if (!only_measure) {
                const double c_right = __longlong_as_double((long long)shfl_down1((uint64_t)__double_as_longlong(cp)));
                const double cr = edge ? cedge[r] : c_right;
                const u32x4 q = philox4x32_10(i, 0u, t, 4u, ks);
                const double ux = (double)((((uint64_t)q.x) << 21) | (q.y >> 11)) * 0x1p-53;
                const double uy = (double)((((uint64_t)q.z) << 21) | (q.w >> 11)) * 0x1p-53;
                const double kc = k2 * cp;
                bool bx = false, by = false;
                if (vx && cp * cr > 0.0) bx = ux < -expm1(-kc * cr);
                if (vx && cp * cd > 0.0) by = uy < -expm1(-kc * cd);
                const uint64_t BX = ballot(bx) & validm, BY = ballot(by) & validm;
                if (lane == 0) {
                    bw[r] = BX;
                    bw[TY + r] = BY;
                }
                n_active += popc64(BX) + popc64(BY);
            }
            if (meas && vx) {
                double sx, cx, sy, cy, st, ct;
                sincos_turn(a - ar, sx, cx);
                sincos_turn(a - ad, sy, cy);
                sincos_turn(a, st, ct);
                ex += fx30(cx);
                ey += fx30(cy);
                ix += fx30(sx);
                iy += fx30(sy);
                mx += fx30(ct);
                my += fx30(st);
            }
            a = ad;
            cp = cd;
        }
    }

    if (meas) {
        const long long v[6] = {ex, ey, ix, iy, mx, my};
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const long long sum = wave_sum_i64(v[j]);
            if (lane == 0 && sum) atomicAdd(&acc[1 + j], (unsigned long long)sum);
        }
    }
    if (!only_measure && lane == 0 && n_active) atomicAdd(&acc[0], (unsigned long long)n_active);
    __syncthreads();
    if (d.cap) {
        const uint32_t copy = blockIdx.x % NCOPY;
        if (!only_measure && tid == 0 && acc[0]) atomic_add_i64(&xy_record(d, t, copy)[0], acc[0]);
        if (meas && tid >= 1 && tid < XY_WORDS && acc[tid])
            atomic_add_i64(&xy_record(d, only_measure ? t : t - 1, copy)[tid], acc[tid]);
    }
}

// Initial angles: Philox counter (i, 0, 0, 6), word 0, or all zero.
__global__ __launch_bounds__(256) void k_xy_init(const LatDesc* descs, uint32_t random_start)
{
    const LatDesc d = descs[0];
    const size_t N = (size_t)d.L * d.L;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256)
        glb(d.ang)[i] = random_start ? philox4x32_10((uint32_t)i, 0u, 0u, 6u, d.key0, d.key1).x : 0u;
}

}  // namespace

hipError_t launch_xy_bonds(const Work& w, uint32_t k, uint32_t flags)
{
    if (w.nitems == 0) return hipSuccess;
    switch (w.ty) {
    case 32: hipLaunchKernelGGL(k_xy_bonds<32>, dim3(w.nitems), dim3(threads_of<32>()), 0, w.stream, w.descs, w.map, k, flags); break;
    case 64: hipLaunchKernelGGL(k_xy_bonds<64>, dim3(w.nitems), dim3(threads_of<64>()), 0, w.stream, w.descs, w.map, k, flags); break;
    case 128: hipLaunchKernelGGL(k_xy_bonds<128>, dim3(w.nitems), dim3(threads_of<128>()), 0, w.stream, w.descs, w.map, k, flags); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_xy_init(const LatDesc* descs, size_t N, uint32_t random_start, hipStream_t s)
{
    const size_t b = (N + 255) / 256;
    const uint32_t grid = (uint32_t)(b < 65536 ? (b ? b : 1) : 65536);
    hipLaunchKernelGGL(k_xy_init, dim3(grid), dim3(256), 0, s, descs, random_start);
    return hipGetLastError();
}

}  // namespace swmi
