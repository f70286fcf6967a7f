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
// Angles are uint32 fractions of a full turn (unit 2^-32).  sin and cos of an
// angle take off its nearest quarter turn in integer arithmetic (exact) and
// evaluate the rest, at most an eighth of a turn, in FP64 by Taylor
// polynomials, then rotate by the quarter turns; a site's projection on the
// direction and the cos and sin of its bonds' angle differences follow from
// products of those values.  The bond test is the FP64 rule u < -expm1(-y),
// with an FP32 estimate deciding whenever u is far from the threshold.
#include <hip/hip_runtime.h>

#include "sw_device.hpp"
#include "sw_kernels.hpp"
#include "sw_tile.hpp"

namespace swmi {

namespace {

constexpr double PI_2_31 = 3.14159265358979323846264338327950288 / 2147483648.0;   // pi / 2^31

// a * b + k rounded once, for a constant k, as the three-operand FP64 fused
// multiply-add (left to itself the compiler copies k into the destination of
// the two-operand multiply-accumulate first, one more instruction per step).
__device__ __forceinline__ double fma_k(double a, double b, double k)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

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
    ps = fma_k(ps, x2, -1.0 / 1307674368000.0);      // 1/15!
    ps = fma_k(ps, x2, 1.0 / 6227020800.0);          // 1/13!
    ps = fma_k(ps, x2, -1.0 / 39916800.0);           // 1/11!
    ps = fma_k(ps, x2, 1.0 / 362880.0);              // 1/9!
    ps = fma_k(ps, x2, -1.0 / 5040.0);               // 1/7!
    ps = fma_k(ps, x2, 1.0 / 120.0);                 // 1/5!
    ps = fma_k(ps, x2, -1.0 / 6.0);                  // 1/3!
    const double sx = fma(x * x2, ps, x);
    double pc = 1.0 / 6402373705728000.0;          // 1/18!
    pc = fma_k(pc, x2, -1.0 / 20922789888000.0);     // 1/16!
    pc = fma_k(pc, x2, 1.0 / 87178291200.0);         // 1/14!
    pc = fma_k(pc, x2, -1.0 / 479001600.0);          // 1/12!
    pc = fma_k(pc, x2, 1.0 / 3628800.0);             // 1/10!
    pc = fma_k(pc, x2, -1.0 / 40320.0);              // 1/8!
    pc = fma_k(pc, x2, 1.0 / 720.0);                 // 1/6!
    pc = fma_k(pc, x2, -1.0 / 24.0);                 // 1/4!
    pc = fma_k(pc, x2, 0.5);                         // the 1/2! term, subtracted below
    const double cx = fma(-x2, pc, 1.0);
    // rotate by k quarter turns
    const bool odd = k & 1u;
    const double ss = odd ? cx : sx, cc = odd ? sx : cx;
    s = (k >= 2u) ? -ss : ss;
    c = (k == 1u || k == 2u) ? -cc : cc;
}

// A term of an observable sum: v (|v| <= 1) rounded to a multiple of 2^-30
// (to nearest, ties to even), in those units, as an integer-valued double: a
// lane adds one term per row of its strip (at most TY, |sum| <= 2^37 < 2^53),
// so its sums are exact in FP64 and become int64 unchanged.
__device__ __forceinline__ double fx30(double v) { return rint(v * 1073741824.0); }

// The projection cos(theta - phi) = cos theta cos phi + sin theta sin phi,
// rounded product by product (no fused multiply-add): for a spin exactly a
// quarter turn from phi the two products are equal and opposite (the quarter
// turn only permutes and negates the polynomial values), so it is exactly 0.
__device__ __forceinline__ double projection(double s, double c, double sphi, double cphi)
{
    return __dadd_rn(__dmul_rn(c, cphi), __dmul_rn(s, sphi));
}

// u < 1 - exp(-y), y >= 0 (may be +inf), decided as in FP64: an FP32
// estimate of 1 - e^{-y} is within a few 1e-7 of the FP64 value, so when u is
// farther than BOND_MARGIN from it the estimate decides, else FP64 expm1 does.
constexpr double BOND_MARGIN = 1.0 / 4096.0;

__device__ __forceinline__ bool bond_test(double u, double y)
{
    const double pf = (double)(1.0f - __expf(-(float)y));
    if (u < pf - BOND_MARGIN) return true;
    if (u >= pf + BOND_MARGIN) return false;
    return u < -expm1(-y);
}

template <class T>
__device__ __forceinline__ T shfl_down1(T v)
{
    static_assert(sizeof(T) == 8, "64-bit values");
    uint64_t b;
    __builtin_memcpy(&b, &v, 8);
    const uint32_t lo = (uint32_t)__shfl_down((int)(uint32_t)b, 1), hi = (uint32_t)__shfl_down((int)(uint32_t)(b >> 32), 1);
    b = ((uint64_t)hi << 32) | lo;
    T out;
    __builtin_memcpy(&out, &b, 8);
    return out;
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
// One workgroup per tile, one column per lane, each wave a strip of rows.
// Every site evaluates sin and cos of its own angle once; its projection, the
// pair terms cos and sin(theta_i - theta_j) of its +x and +y bonds and its
// magnetisation terms are products of those with the direction's and the
// neighbours' (the right-hand lane's, the next row's; the column right of the
// tile is evaluated once per tile).  A site's +x and +y bonds use one Philox
// call (counter (i, 0, t, 4)): words 0, 1 make the 53-bit uniform of the +x
// bond, words 2, 3 that of the +y bond.  The bond words go to the tile-major
// bond plane the labeller reads.
template <int TY>
__global__ __launch_bounds__(threads_of<TY>()) __attribute__((amdgpu_waves_per_eu(4))) void k_xy_bonds(const LatDesc* descs, const WorkItem* map, uint32_t k,
                                                               uint32_t flags)
{
    constexpr uint32_t NW = waves_of<TY>();
    constexpr uint32_t RPW = TY / NW;
    __shared__ unsigned long long acc[XY_WORDS];   // n_active, Ex, Ey, Ix, Iy, Mx, My
    __shared__ double sedge[TY], cedge[TY];        // sin, cos of the column right of the tile

    LatDesc d;
    uint32_t tile, lat;
    if (!pick(descs, map, blockIdx.x, true, d, tile, lat)) return;
    const TileGeom g = tile_geom(d, tile, TY);
    const uint32_t t = *glb(d.counter) + k;
    const bool only_measure = (flags & 2u) != 0;
    const bool meas = d.cap != 0 && (flags & 3u) != 0;
    const uint32_t tid = threadIdx.x, wave = wave_id(), lane = tid & 63u;
    const uint32_t L = d.L, w = g.w, h = g.h, x0 = g.x0, y0 = g.y0;
    const gptr<uint32_t> ang = glb(d.ang);
    const uint32_t xe = (x0 + w == L) ? 0u : x0 + w;   // the column right of the tile

    if (tid < XY_WORDS) acc[tid] = 0ull;
    if (tid < h) {
        double se, ce;
        sincos_turn(ang[(y0 + tid) * L + xe], se, ce);
        sedge[tid] = se;
        cedge[tid] = ce;
    }
    __syncthreads();

    double sphi, cphi;
    sincos_turn(xy_direction(d, t), sphi, cphi);
    const bool vx = lane < w;
    const bool edge = lane == w - 1;
    const uint32_t x = x0 + (vx ? lane : 0u);
    const uint32_t r0 = wave * RPW, r1 = min(h, r0 + RPW);
    const uint64_t validm = (w == 64) ? ~0ull : ((1ull << w) - 1ull);
    const double k2 = d.k2;
    const PhiloxKeys ks = philox_keys_v(d.key0, d.key1);
    const gptr<uint64_t> bw = glb(d.bonds) + (size_t)tile * 2 * TY;
    uint32_t n_active = 0;   // wave-uniform
    double ex = 0, ey = 0, ix = 0, iy = 0, mx = 0, my = 0;

    if (r0 < r1) {
        // tile row rr of this column (row h is the first row of the tile below,
        // or row 0 of the lattice)
        auto row_angle = [&](uint32_t rr) { return ang[((y0 + rr == L) ? 0u : y0 + rr) * L + x]; };
        double si, ci;
        sincos_turn(row_angle(r0), si, ci);
        // the rows below are loaded two iterations ahead of their use
        uint32_t a1 = row_angle(r0 + 1), a2 = (r0 + 2 <= r1) ? row_angle(r0 + 2) : 0u;
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t y = y0 + r;
            const uint32_t i = y * L + x;   // site indices fit 32 bits (N <= 2^32)
            const uint32_t ad = a1;
            a1 = a2;
            if (r + 3 <= r1) a2 = row_angle(r + 3);
            double sd, cd;
            sincos_turn(ad, sd, cd);
            const double s_right = shfl_down1(si), c_right = shfl_down1(ci);
            const double sr = edge ? sedge[r] : s_right, cr = edge ? cedge[r] : c_right;
            if (!only_measure) {
                const double pi_ = projection(si, ci, sphi, cphi);
                const double pr = projection(sr, cr, sphi, cphi);
                const double pd = projection(sd, cd, sphi, cphi);
                const u32x4 q = philox4x32_10(i, 0u, t, 4u, ks);
                const double ux = (double)((((uint64_t)q.x) << 21) | (q.y >> 11)) * 0x1p-53;
                const double uy = (double)((((uint64_t)q.z) << 21) | (q.w >> 11)) * 0x1p-53;
                const double kc = k2 * pi_;
                const bool bx = vx && pi_ * pr > 0.0 && bond_test(ux, kc * pr);
                const bool by = vx && pi_ * pd > 0.0 && bond_test(uy, kc * pd);
                const uint64_t BX = ballot(bx) & validm, BY = ballot(by) & validm;
                if (lane == 0) {
                    bw[r] = BX;
                    bw[TY + r] = BY;
                }
                n_active += popc64(BX) + popc64(BY);
            }
            if (meas && vx) {
                // cos and sin of theta_i - theta_j from the two sites' sin and cos
                ex += fx30(fma(ci, cr, si * sr));
                ix += fx30(fma(si, cr, -(ci * sr)));
                ey += fx30(fma(ci, cd, si * sd));
                iy += fx30(fma(si, cd, -(ci * sd)));
                mx += fx30(ci);
                my += fx30(si);
            }
            si = sd;
            ci = cd;
        }
    }

    if (meas) {
        const long long v[6] = {(long long)ex, (long long)ey, (long long)ix, (long long)iy, (long long)mx,
                                (long long)my};
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
