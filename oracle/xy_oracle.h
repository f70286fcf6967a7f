/*
 * CPU oracle for the Swendsen-Wang sweep of the 2D classical XY model with
 * Wolff's embedded clusters.  TEST INFRASTRUCTURE ONLY: used by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark, never by the library.
 *
 * Conventions: site index i = y*L + x; an angle is a uint32 a, the angle
 * theta = 2 pi a / 2^32 (a fraction of a full turn in 32-bit fixed point);
 * bonds and labels as in sw_oracle.h.  Observable rows are int64
 * [n_active, Ex, Ey, Ix, Iy, Mx, My], the last six fixed-point sums (one unit =
 * 2^-30) defined in xy_oracle.c.
 */
#ifndef XY_ORACLE_H
#define XY_ORACLE_H

#include <stdint.h>

#define OR_XY_OBS_WORDS 7

#ifdef __cplusplus
extern "C" {
#endif

uint32_t or_xy_direction(uint64_t seed, uint32_t sweep, uint32_t dir_bits);
uint32_t or_xy_initangle(uint64_t seed, uint64_t site);
double or_xy_uniform(uint64_t seed, uint32_t sweep, uint64_t site, uint32_t dir);
uint32_t or_xy_flipbit(uint64_t seed, uint32_t sweep, uint64_t root);
void or_xy_sincos(uint32_t a, double* s, double* c);
double or_xy_projection(uint32_t a, uint32_t phi);
uint32_t or_xy_reflect(uint32_t a, uint32_t phi);
int or_xy_init(uint32_t L, uint64_t seed, int random_start, uint32_t* a);
void or_xy_observe(uint32_t L, const uint32_t* a, int64_t* obs);
void or_xy_derived(uint32_t L, double K, const uint32_t* a, double* out);
int or_xy_bonds(uint32_t L, double K, uint64_t seed, uint32_t sweep, uint32_t dir_bits, const uint32_t* a,
                uint8_t* bx, uint8_t* by);
int or_xy_flip(uint32_t L, uint64_t seed, uint32_t sweep, uint32_t dir_bits, uint32_t* a, const uint8_t* bx,
               const uint8_t* by, const uint32_t* label, int64_t* obs);
int or_xy_sweep(uint32_t L, double K, uint64_t seed, uint32_t sweep, uint32_t dir_bits, uint32_t* a,
                uint8_t* bx, uint8_t* by, uint32_t* label, int64_t* obs);
int or_xy_run(uint32_t L, double K, uint64_t seed, uint32_t first_sweep, uint32_t n_sweeps, uint32_t dir_bits,
              uint32_t* a, int64_t* obs_out);

#ifdef __cplusplus
}
#endif

#endif
