/*
 * CPU oracle for the Swendsen-Wang (SW) multi-cluster update of the 2D
 * classical XY model on an L x L periodic square lattice, with Wolff's
 * embedded clusters (the extension named in Sec. 5 of Komura & Okabe; the
 * embedding is Wolff, Phys. Rev. Lett. 62 (1989) 361).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct; only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or constant generator with the HIP library.
 *
 * The model: H = -J sum_<ij> cos(theta_i - theta_j), K = J / k_B T.
 * One sweep, in the order of the method:
 *   (0) draw a direction r = (cos phi, sin phi);
 *   (1) project every spin on r, c_i = cos(theta_i - phi); a bond <ij> is
 *       active with probability 1 - exp(-2 K c_i c_j) when c_i c_j > 0 (the
 *       spins lie on the same side of the line perpendicular to r), never
 *       otherwise -- the SW bond rule of the Ising model that the projections
 *       embed, whose couplings are K |c_i| |c_j|;
 *   (2) label the clusters of active bonds (the same Hoshen-Kopelman labelling
 *       as the Potts oracle: the root is the smallest site index);
 *   (3) reflect every spin of a cluster across the line perpendicular to r,
 *       theta -> 2 phi + pi - theta, with probability 1/2 per cluster.
 *
 * Readings (the paper names the extension only; these are fixed once here and
 * implemented independently by the GPU path from the same written rules):
 *   - an angle is a uint32 a, theta = 2 pi a / 2^32; differences of angles are
 *     exact integers mod 2^32; the reflection is exact: a' = 2 a_phi + 2^31 - a
 *     (mod 2^32);
 *   - sin and cos of an angle a: its nearest quarter turn k is taken off in
 *     integer arithmetic, the rest d = a - k 2^30 (an int32 in [-2^29, 2^29),
 *     at most an eighth of a turn) becomes radians by one FP64 multiplication
 *     by pi / 2^31, and sin, cos of that (C library) are rotated by k quarter
 *     turns; so a spin exactly a quarter turn from the direction projects to
 *     zero, and no bond reaches it;
 *   - dir_bits in 1..32: a_phi keeps its top dir_bits bits (the others zero),
 *     so phi is a multiple of 2 pi / 2^dir_bits; 32 is the continuous model;
 *     a cold start with dir_bits = 1 or 2 stays on {0, pi} (the Ising model at
 *     coupling K), dir_bits = b >= 2 on the 2^(b-1)-state clock model;
 *   - bond test in FP64: u < -expm1(-((2K) c_i) c_j), evaluated by the site
 *     that owns the bond (i = (x, y), j = (x+1, y) or (x, y+1)), with c_i c_j > 0
 *     required first; K = +inf makes every such bond active;
 *   - random numbers: Philox4x32-10 under key (seed lo, seed hi), counters
 *       direction of sweep t:           (0, 0, t, 3), word 0;
 *       bond uniforms of site i, sweep t: (i lo, i hi, t, 4): words 0, 1 for
 *         the +x bond, words 2, 3 for the +y bond, u = ((w_a << 21) |
 *         (w_b >> 11)) 2^-53, a 53-bit uniform in [0, 1);
 *       reflection bit of cluster root r: (r lo, r hi, t, 5), top bit of word 0;
 *       random initial angle of site i:  (i lo, i hi, 0, 6), word 0;
 *   - observables of a configuration, each term rounded to a multiple of 2^-30
 *     (round to nearest even) and summed exactly in int64:
 *       Ex = sum_i cos(theta_i - theta_{i+x}),  Ey likewise along +y,
 *       Ix = sum_i sin(theta_i - theta_{i+x}),  Iy likewise,
 *       Mx = sum_i cos theta_i,                 My = sum_i sin theta_i;
 *     the energy is -J (Ex + Ey), the magnetisation (Mx, My), and Ex, Ix (Ey,
 *     Iy) give the helicity modulus along x (y).
 */
#include "xy_oracle.h"

#include <math.h>
#include <stdlib.h>

#include "sw_oracle.h"

/* pi rounded to the nearest double (the same value as the usual M_PI) */
static const double XY_PI = 3.14159265358979323846264338327950288;

static void xy_draw(uint64_t seed, uint64_t index, uint32_t sweep, uint32_t stream, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), sweep, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox(ctr, key, out);
}

uint32_t or_xy_direction(uint64_t seed, uint32_t sweep, uint32_t dir_bits)
{
    uint32_t w[4];
    xy_draw(seed, 0, sweep, 3u, w);
    if (dir_bits >= 32) return w[0];
    uint32_t keep = dir_bits == 0 ? 0u : ~(0xFFFFFFFFu >> dir_bits);
    return w[0] & keep;
}

uint32_t or_xy_initangle(uint64_t seed, uint64_t site)
{
    uint32_t w[4];
    xy_draw(seed, site, 0u, 6u, w);
    return w[0];
}

double or_xy_uniform(uint64_t seed, uint32_t sweep, uint64_t site, uint32_t dir)
{
    uint32_t w[4];
    xy_draw(seed, site, sweep, 4u, w);
    uint32_t hi = w[2 * (dir & 1u)], lo = w[2 * (dir & 1u) + 1];
    uint64_t m = ((uint64_t)hi << 21) | (lo >> 11);
    return ldexp((double)m, -53);
}

uint32_t or_xy_flipbit(uint64_t seed, uint32_t sweep, uint64_t root)
{
    uint32_t w[4];
    xy_draw(seed, root, sweep, 5u, w);
    return w[0] >> 31;
}

/* sin and cos of the angle of a (see the readings above). */
void or_xy_sincos(uint32_t a, double* s, double* c)
{
    uint32_t k = ((a + 0x20000000u) >> 30) & 3u;   /* nearest quarter turn */
    int32_t d = (int32_t)(a - (k << 30));            /* in [-2^29, 2^29) */
    double x = (double)d * ldexp(XY_PI, -31);
    double sx = sin(x), cx = cos(x);
    switch (k) {
    case 0: *s = sx; *c = cx; break;
    case 1: *s = cx; *c = -sx; break;
    case 2: *s = -sx; *c = -cx; break;
    default: *s = -cx; *c = sx; break;
    }
}

double or_xy_projection(uint32_t a, uint32_t phi)
{
    double s, c;
    or_xy_sincos(a - phi, &s, &c);
    return c;
}

uint32_t or_xy_reflect(uint32_t a, uint32_t phi)
{
    return 2u * phi + 0x80000000u - a;
}

int or_xy_init(uint32_t L, uint64_t seed, int random_start, uint32_t* a)
{
    if (L < 2 || !a) return -1;
    uint64_t N = (uint64_t)L * L;
    for (uint64_t i = 0; i < N; ++i) a[i] = random_start ? or_xy_initangle(seed, i) : 0u;
    return 0;
}

static int64_t fx(double v)
{
    return (int64_t)nearbyint(ldexp(v, 30));
}

void or_xy_observe(uint32_t L, const uint32_t* a, int64_t* obs)
{
    int64_t ex = 0, ey = 0, ix = 0, iy = 0, mx = 0, my = 0;
    for (uint32_t y = 0; y < L; ++y) {
        uint32_t yd = (y + 1 == L) ? 0 : y + 1;
        for (uint32_t x = 0; x < L; ++x) {
            uint32_t xr = (x + 1 == L) ? 0 : x + 1;
            uint32_t ai = a[(uint64_t)y * L + x];
            double sx, cx, sy, cy, st, ct;
            or_xy_sincos(ai - a[(uint64_t)y * L + xr], &sx, &cx);
            or_xy_sincos(ai - a[(uint64_t)yd * L + x], &sy, &cy);
            or_xy_sincos(ai, &st, &ct);
            ex += fx(cx);
            ey += fx(cy);
            ix += fx(sx);
            iy += fx(sy);
            mx += fx(ct);
            my += fx(st);
        }
    }
    obs[0] = 0;
    obs[1] = ex;
    obs[2] = ey;
    obs[3] = ix;
    obs[4] = iy;
    obs[5] = mx;
    obs[6] = my;
}

/* FP64 observables of one configuration straight from the angles:
 * out[0] = energy per site, -(sum over bonds of cos) / N;
 * out[1] = squared magnetisation per site, |sum_i s_i|^2 / N^2;
 * out[2] = the configuration's helicity-modulus estimator in units of J,
 *          averaged over x and y: [(Ex + Ey) / 2 - K (Ix^2 + Iy^2) / 2] / N
 *          (its mean over configurations is the helicity modulus). */
void or_xy_derived(uint32_t L, double K, const uint32_t* a, double* out)
{
    double N = (double)L * (double)L;
    double ex = 0, ey = 0, ix = 0, iy = 0, mx = 0, my = 0;
    for (uint32_t y = 0; y < L; ++y) {
        uint32_t yd = (y + 1 == L) ? 0 : y + 1;
        for (uint32_t x = 0; x < L; ++x) {
            uint32_t xr = (x + 1 == L) ? 0 : x + 1;
            uint32_t ai = a[(uint64_t)y * L + x];
            double sx, cx, sy, cy, st, ct;
            or_xy_sincos(ai - a[(uint64_t)y * L + xr], &sx, &cx);
            or_xy_sincos(ai - a[(uint64_t)yd * L + x], &sy, &cy);
            or_xy_sincos(ai, &st, &ct);
            ex += cx;
            ey += cy;
            ix += sx;
            iy += sy;
            mx += ct;
            my += st;
        }
    }
    out[0] = -(ex + ey) / N;
    out[1] = (mx * mx + my * my) / (N * N);
    out[2] = (0.5 * (ex + ey) - K * 0.5 * (ix * ix + iy * iy)) / N;
}

/* Steps (0) and (1): the sweep's direction, the projections, the bonds. */
int or_xy_bonds(uint32_t L, double K, uint64_t seed, uint32_t sweep, uint32_t dir_bits, const uint32_t* a,
                uint8_t* bx, uint8_t* by)
{
    if (L < 2 || !a || !bx || !by || isnan(K) || K < 0.0 || dir_bits < 1 || dir_bits > 32) return -1;
    uint32_t phi = or_xy_direction(seed, sweep, dir_bits);
    double k2 = 2.0 * K;
    for (uint32_t y = 0; y < L; ++y) {
        uint32_t yd = (y + 1 == L) ? 0 : y + 1;
        for (uint32_t x = 0; x < L; ++x) {
            uint32_t xr = (x + 1 == L) ? 0 : x + 1;
            uint64_t i = (uint64_t)y * L + x;
            double ci = or_xy_projection(a[i], phi);
            double cr = or_xy_projection(a[(uint64_t)y * L + xr], phi);
            double cd = or_xy_projection(a[(uint64_t)yd * L + x], phi);
            double ux = or_xy_uniform(seed, sweep, i, 0);
            double uy = or_xy_uniform(seed, sweep, i, 1);
            bx[i] = (ci * cr > 0.0) && (ux < -expm1(-(k2 * ci) * cr));
            by[i] = (ci * cd > 0.0) && (uy < -expm1(-(k2 * ci) * cd));
        }
    }
    return 0;
}

/* Step (3): every cluster whose root draws a set bit is reflected; then the
 * observables of the new configuration (obs may be NULL). */
int or_xy_flip(uint32_t L, uint64_t seed, uint32_t sweep, uint32_t dir_bits, uint32_t* a, const uint8_t* bx,
               const uint8_t* by, const uint32_t* label, int64_t* obs)
{
    if (L < 2 || !a || !bx || !by || !label || dir_bits < 1 || dir_bits > 32) return -1;
    uint64_t N = (uint64_t)L * L;
    uint32_t phi = or_xy_direction(seed, sweep, dir_bits);
    for (uint64_t i = 0; i < N; ++i)
        if (or_xy_flipbit(seed, sweep, label[i])) a[i] = or_xy_reflect(a[i], phi);
    if (obs) {
        or_xy_observe(L, a, obs);
        int64_t active = 0;
        for (uint64_t i = 0; i < N; ++i) active += bx[i] + by[i];
        obs[0] = active;
    }
    return 0;
}

int or_xy_sweep(uint32_t L, double K, uint64_t seed, uint32_t sweep, uint32_t dir_bits, uint32_t* a,
                uint8_t* bx, uint8_t* by, uint32_t* label, int64_t* obs)
{
    if (or_xy_bonds(L, K, seed, sweep, dir_bits, a, bx, by) != 0) return -1;   /* (0), (1) */
    or_label(L, bx, by, label);                                                 /* (2) */
    return or_xy_flip(L, seed, sweep, dir_bits, a, bx, by, label, obs);         /* (3) */
}

int or_xy_run(uint32_t L, double K, uint64_t seed, uint32_t first_sweep, uint32_t n_sweeps, uint32_t dir_bits,
              uint32_t* a, int64_t* obs_out)
{
    if (L < 2 || !a) return -1;
    uint64_t N = (uint64_t)L * L;
    uint8_t* bx = (uint8_t*)malloc(N);
    uint8_t* by = (uint8_t*)malloc(N);
    uint32_t* label = (uint32_t*)malloc(N * sizeof(uint32_t));
    int rc = 0;
    if (!bx || !by || !label) rc = -2;
    for (uint32_t k = 0; rc == 0 && k < n_sweeps; ++k)
        rc = or_xy_sweep(L, K, seed, first_sweep + k, dir_bits, a, bx, by, label,
                         obs_out ? obs_out + (uint64_t)k * OR_XY_OBS_WORDS : NULL);
    free(bx);
    free(by);
    free(label);
    return rc;
}
