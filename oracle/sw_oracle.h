/*
 * CPU oracle for the Swendsen-Wang sweep of the 2D q-state Potts model.
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the library.
 *
 * Conventions: site index i = y*L + x (row-major); spins 0..q-1 as uint8;
 * bonds as one byte per site and direction (bx[i]: bond i -> (x+1, y),
 * by[i]: bond i -> (x, y+1), both periodic); labels are uint32 site indices.
 * obs rows are int64 [n_unsat, n_active, n_0, ..., n_{q-1}].
 */
#ifndef SW_ORACLE_H
#define SW_ORACLE_H

#include <stdint.h>

#define OR_BAD_THRESHOLD ((uint64_t)-1)

#ifdef __cplusplus
extern "C" {
#endif

void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint64_t or_threshold(double K);
uint32_t or_state_of_draw(uint32_t w, uint32_t q);
uint32_t or_newspin(uint64_t seed, uint32_t sweep, uint64_t root, uint32_t q);
uint32_t or_initspin(uint64_t seed, uint64_t site, uint32_t q);
void or_bond_draws(uint64_t seed, uint32_t sweep, uint64_t site, uint32_t* wx, uint32_t* wy);
int or_init(uint32_t L, uint32_t q, uint64_t seed, int random_start, uint8_t* s);
void or_observe(uint32_t L, uint32_t q, const uint8_t* s, int64_t* obs);
void or_derived(uint32_t L, uint32_t q, const uint8_t* s, double* out);
void or_label(uint32_t L, const uint8_t* bx, const uint8_t* by, uint32_t* label);
int or_bonds(uint32_t L, double K, uint64_t seed, uint32_t sweep, const uint8_t* s, uint8_t* bx, uint8_t* by);
int or_flip(uint32_t L, uint32_t q, uint64_t seed, uint32_t sweep, uint8_t* s, const uint8_t* bx,
            const uint8_t* by, const uint32_t* label, int64_t* obs);
int or_sweep(uint32_t L, uint32_t q, double K, uint64_t seed, uint32_t sweep,
             uint8_t* s, uint8_t* bx, uint8_t* by, uint32_t* label, int64_t* obs);
int or_run(uint32_t L, uint32_t q, double K, uint64_t seed, uint32_t first_sweep,
           uint32_t n_sweeps, uint8_t* s, int64_t* obs_out);

#ifdef __cplusplus
}
#endif

#endif
