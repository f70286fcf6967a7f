/*
 * The classical XY model on the same Swendsen-Wang machinery: C ABI.
 *
 * Sec. 5 of Komura & Okabe (the paper whose Potts sweep sw.h implements)
 * names the extension of the multi-cluster sweep to continuous spins through
 * Wolff's embedded clusters (Phys. Rev. Lett. 62 (1989) 361).  One sweep:
 *   (0) a random direction r = (cos phi, sin phi);
 *   (1) projections c_i = cos(theta_i - phi); a bond between nearest
 *       neighbours with c_i c_j > 0 is active with probability
 *       1 - exp(-2 K c_i c_j), never otherwise (the SW bond rule of the Ising
 *       model embedded in the projections, couplings K |c_i| |c_j|);
 *   (2) the clusters of active bonds (the same labelling as the Potts sweep);
 *   (3) every cluster is reflected across the line perpendicular to r,
 *       theta -> 2 phi + pi - theta, with probability 1/2.
 * H = -J sum_<ij> cos(theta_i - theta_j), K = J / k_B T, periodic L x L.
 *
 * An XY lattice is an sw_lattice created by sw_xy_init.  These calls of sw.h
 * work on it unchanged: sw_sweep, sw_sweep_profiled, sw_sweeps_done,
 * sw_measure, sw_measure_after, sw_read_labels, sw_read_bonds,
 * sw_label_equivalence, sw_destroy.  sw_read_spins, sw_read_spins_after,
 * sw_load_spins and sw_cluster_sums return SW_EINVAL for it (it has angles,
 * not states), and sw_group_sweep does not take it.
 *
 * Angles: uint32, theta = 2 pi a / 2^32 (a fraction of a full turn), so the
 * reflection a' = 2 a_phi + 2^31 - a (mod 2^32) is exact.  sin and cos take
 * off the nearest quarter turn exactly and evaluate the rest in FP64.
 *
 * Random numbers: Philox4x32-10 under key (seed lo, seed hi), counters
 *   direction of sweep t:             (0, 0, t, 3), word 0, top dir_bits kept;
 *   bond uniforms of site i, sweep t:  (i, 0, t, 4): words 0, 1 (+x bond) and
 *                                      2, 3 (+y bond), u = ((w_a << 21) |
 *                                      (w_b >> 11)) 2^-53; bond iff
 *                                      c_i c_j > 0 and
 *                                      u < -expm1(-((2K) c_i) c_j) in FP64;
 *   reflection bit of cluster root r:  (r, 0, t, 5), top bit of word 0;
 *   random initial angle of site i:    (i, 0, 0, 6), word 0.
 * A run is a function of (L, K, dir_bits, seed, init) only.
 *
 * Observable rows (sw_measure): int64 [n_active, Ex, Ey, Ix, Iy, Mx, My] per
 * sweep, with Ex = sum_i cos(theta_i - theta_{i+x}), Ey the same along y, Ix,
 * Iy the sums of sin of the same differences, Mx = sum_i cos theta_i, My =
 * sum_i sin theta_i, each term rounded to a multiple of 2^-30 (to nearest,
 * ties to even) and the sums in those units -- exact integers, independent
 * of the order of summation.
 */
#ifndef SW_XY_H
#define SW_XY_H

#include <stddef.h>
#include <stdint.h>

#include "sw.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SW_XY_OBS_WORDS 7

typedef struct sw_xy_params {
    uint32_t L;            /* linear size, 2..65536 */
    uint32_t dir_bits;     /* 1..32: the direction keeps the top dir_bits bits of
                              its draw, so phi is a multiple of 2 pi / 2^dir_bits;
                              32 is the XY model; with a cold start, 1 and 2 keep
                              the angles on {0, pi} (the Ising model at coupling
                              K) and b >= 2 on the 2^(b-1)-state clock model */
    double K;              /* J / k_B T >= 0; +inf allowed */
    uint64_t seed;         /* Philox key */
    uint32_t init;         /* 0 = cold start (all angles 0), 1 = random start */
    uint32_t obs_capacity; /* sweeps of observables kept in the device ring
                              (0 = none, else >= 2) */
    uint32_t tile_rows;    /* labelling tile height: 0 (default), 32, 64 or 128 */
    uint32_t reserved;     /* must be 0 */
} sw_xy_params;

/* Device workspace bytes an XY lattice needs (0 if the parameters are
 * invalid): 4 bytes of angles and 4 of labels per site, the bond words, the
 * per-tile edge records and edge forest, and the ring. */
size_t sw_xy_workspace_bytes(const sw_xy_params* p);

/* Create an XY lattice in dev_ws (device memory, 256-byte aligned, at least
 * sw_xy_workspace_bytes; owned by the caller, which keeps it alive and
 * untouched until sw_destroy) bound to hip_stream; angles cold or random per
 * p->init.  Synchronises the stream.  SW_EINVAL / SW_ESPACE on bad
 * parameters or a small workspace. */
int sw_xy_init(const sw_xy_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, sw_lattice** out);

/* Copy the L*L angles (row-major uint32) to host memory; synchronises. */
int sw_xy_read_angles(sw_lattice* h, uint32_t* host_out);

/* Overwrite the angles with L*L host values and set the sweep counter to
 * `sweep` (checkpoint resume: the run continues exactly as if it had reached
 * this state itself); clears the observable ring.  Synchronises. */
int sw_xy_load_angles(sw_lattice* h, const uint32_t* host_in, uint32_t sweep);

/* FP64 quantities of one observable row of an L x L lattice at coupling K:
 * out[0] = energy per site, -(Ex + Ey) / N (units of J);
 * out[1] = squared magnetisation per site, (Mx^2 + My^2) / N^2;
 * out[2] = the configuration's helicity-modulus estimator in units of J,
 *          [(Ex + Ey) / 2 - K (Ix^2 + Iy^2) / 2] / N (its mean over
 *          configurations is the helicity modulus, averaged over x and y).
 * SW_EINVAL if a sum exceeds N in magnitude. */
int sw_xy_derived(uint32_t L, double K, const int64_t* row, double* out);

#ifdef __cplusplus
}
#endif

#endif
