/*
 * CPU oracle for the Swendsen-Wang (SW) multi-cluster update of the 2D q-state
 * Potts model on an L x L periodic square lattice.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant generator with the HIP library.
 *
 * What it computes (Komura & Okabe, "Multi-GPU-based Swendsen-Wang
 * multi-cluster algorithm for the simulation of two-dimensional q-state Potts
 * model"):
 *   - the Hamiltonian of Sec. 2, Eq. (1): H = -J sum_<ij> (delta(S_i,S_j) - 1),
 *     nearest neighbours, periodic boundaries; the energy in units of J is the
 *     number of nearest-neighbour bonds whose spins differ (n_unsat);
 *   - the three SW steps listed in Sec. 2: (1) activate bonds, (2) label the
 *     clusters of active bonds, (3) give every cluster a uniformly random new
 *     state out of q;
 *   - step (2) with the Hoshen-Kopelman idea of Sec. 2: the proper label of a
 *     cluster is its smallest label, found by following label[label].
 *
 * Readings where the paper is silent (all fixed once, shared with the GPU path
 * only as a written specification):
 *   - bond probability p = 1 - exp(-K), K = J / k_B T, bonds only between
 *     equal spins (standard SW for Eq. (1)); integer test w < floor(2^32 p);
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11) replaces the paper's
 *     linear congruential generator (Sec. 3, last paragraph).  Keying:
 *       key = (seed mod 2^32, seed >> 32)
 *       bond draws of site i in sweep t: counter (pair lo, pair hi, t, 0),
 *         pair = i >> 1; site parity b = i & 1 takes word 2b for the +x bond
 *         and word 2b+1 for the +y bond;
 *       new-spin draw of cluster root r in sweep t: counter (r lo, r hi, t, 1),
 *         word 0;
 *       random initial spin of site i: counter (i lo, i hi, 0, 2), word 0;
 *   - a draw w maps to a state by floor(w * q / 2^32);
 *   - spins are 0..q-1 (the paper's S_i - 1); each site owns its bonds to
 *     (x+1, y) and (x, y+1), both periodic, so there are 2N bonds (for L = 2
 *     two distinct bonds join the same pair and both count);
 *   - the cluster root is the minimum site index i = y*L + x of the cluster,
 *     which is the paper's "smallest label" when labels are site indices.
 */
#include "sw_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- Philox */

/* Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw (SC'11):
 * ten rounds of two 32x32->64 multiplications and xors, the key bumped by the
 * two Weyl constants between rounds. */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint64_t index, uint32_t sweep, uint32_t stream,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), sweep, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox(ctr, key, out);
}

/* ---------------------------------------------------------- small pieces */

uint64_t or_threshold(double K)
{
    if (isnan(K) || K < 0.0) return OR_BAD_THRESHOLD;
    if (isinf(K)) return (uint64_t)1 << 32;
    double p = -expm1(-K);            /* bond probability 1 - e^{-K} */
    return (uint64_t)floor(ldexp(p, 32));
}

uint32_t or_state_of_draw(uint32_t w, uint32_t q)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)q) >> 32);
}

uint32_t or_newspin(uint64_t seed, uint32_t sweep, uint64_t root, uint32_t q)
{
    uint32_t w[4];
    draw(seed, root, sweep, 1u, w);
    return or_state_of_draw(w[0], q);
}

uint32_t or_initspin(uint64_t seed, uint64_t site, uint32_t q)
{
    uint32_t w[4];
    draw(seed, site, 0u, 2u, w);
    return or_state_of_draw(w[0], q);
}

void or_bond_draws(uint64_t seed, uint32_t sweep, uint64_t site,
                   uint32_t* wx, uint32_t* wy)
{
    uint32_t w[4];
    draw(seed, site >> 1, sweep, 0u, w);
    unsigned b = (unsigned)(site & 1u);
    *wx = w[2 * b];
    *wy = w[2 * b + 1];
}

int or_init(uint32_t L, uint32_t q, uint64_t seed, int random_start, uint8_t* s)
{
    if (L < 2 || q < 2 || q > 255 || !s) return -1;
    uint64_t N = (uint64_t)L * L;
    for (uint64_t i = 0; i < N; ++i)
        s[i] = random_start ? (uint8_t)or_initspin(seed, i, q) : 0;
    return 0;
}

/* ------------------------------------------------------------ observables */

void or_observe(uint32_t L, uint32_t q, const uint8_t* s, int64_t* obs)
{
    uint64_t N = (uint64_t)L * L;
    int64_t unsat = 0;
    for (uint32_t c = 0; c < q; ++c) obs[2 + c] = 0;
    for (uint32_t y = 0; y < L; ++y) {
        uint32_t yd = (y + 1 == L) ? 0 : y + 1;
        for (uint32_t x = 0; x < L; ++x) {
            uint32_t xr = (x + 1 == L) ? 0 : x + 1;
            uint8_t si = s[(uint64_t)y * L + x];
            unsat += (si != s[(uint64_t)y * L + xr]);
            unsat += (si != s[(uint64_t)yd * L + x]);
            obs[2 + si] += 1;
        }
    }
    (void)N;
    obs[0] = unsat;
}

/* Derived observables of one configuration in FP64, straight from the spins
 * (Sec. 4 measures the energy and the magnetisation; these are the readings of
 * them): out[0] = energy per site, the number of unequal nearest-neighbour
 * pairs of Eq. (1) over N; out[1] = Potts order parameter
 * (q * max_c f_c - 1) / (q - 1), f_c the fraction of sites in state c;
 * out[2] = Ising magnetisation sum_i (1 - 2 s_i) for q = 2 (0 otherwise). */
void or_derived(uint32_t L, uint32_t q, const uint8_t* s, double* out)
{
    double N = (double)L * (double)L;
    double e = 0.0, mag = 0.0;
    double* frac = (double*)calloc(q, sizeof(double));
    if (!frac) {
        out[0] = out[1] = out[2] = NAN;
        return;
    }
    for (uint32_t y = 0; y < L; ++y) {
        uint32_t yd = (y + 1 == L) ? 0 : y + 1;
        for (uint32_t x = 0; x < L; ++x) {
            uint32_t xr = (x + 1 == L) ? 0 : x + 1;
            uint8_t si = s[(uint64_t)y * L + x];
            if (si != s[(uint64_t)y * L + xr]) e += 1.0;
            if (si != s[(uint64_t)yd * L + x]) e += 1.0;
            frac[si] += 1.0;
            mag += (si == 0) ? 1.0 : -1.0;
        }
    }
    double fmax = 0.0;
    for (uint32_t c = 0; c < q; ++c)
        if (frac[c] > fmax) fmax = frac[c];
    free(frac);
    out[0] = e / N;
    out[1] = ((double)q * (fmax / N) - 1.0) / (double)(q - 1);
    out[2] = (q == 2) ? mag : 0.0;
}

/* ------------------------------------------------- Hoshen-Kopelman labels */

/* Proper label: follow label[label] until it points at itself (Sec. 2), then
 * point every visited entry straight at it. */
static uint32_t find_root(uint32_t* label, uint32_t i)
{
    uint32_t r = i;
    while (label[r] != r) r = label[r];
    while (label[i] != r) {
        uint32_t next = label[i];
        label[i] = r;
        i = next;
    }
    return r;
}

/* Two clusters meet: the larger proper label is pointed at the smaller one, so
 * the proper label of every cluster stays its smallest label. */
static void join(uint32_t* label, uint32_t a, uint32_t b)
{
    uint32_t ra = find_root(label, a), rb = find_root(label, b);
    if (ra == rb) return;
    if (ra < rb) label[rb] = ra;
    else label[ra] = rb;
}

void or_label(uint32_t L, const uint8_t* bx, const uint8_t* by, uint32_t* label)
{
    uint64_t N = (uint64_t)L * L;
    /* raster scan: a site starts its own label (its index), then it is joined
     * with the already visited left and upper neighbours it is bonded to */
    for (uint32_t y = 0; y < L; ++y) {
        for (uint32_t x = 0; x < L; ++x) {
            uint32_t i = (uint32_t)((uint64_t)y * L + x);
            label[i] = i;
            if (x > 0 && bx[i - 1]) join(label, i - 1, i);
            if (y > 0 && by[i - L]) join(label, i - L, i);
        }
    }
    /* periodic boundaries: the bonds that wrap around the torus */
    for (uint32_t y = 0; y < L; ++y) {
        uint32_t i = (uint32_t)((uint64_t)y * L + (L - 1));
        if (bx[i]) join(label, i, (uint32_t)((uint64_t)y * L));
    }
    for (uint32_t x = 0; x < L; ++x) {
        uint32_t i = (uint32_t)((uint64_t)(L - 1) * L + x);
        if (by[i]) join(label, i, x);
    }
    for (uint64_t i = 0; i < N; ++i) label[i] = find_root(label, (uint32_t)i);
}

/* ------------------------------------------------------------- one sweep */

/* Step (1) of Sec. 2: bond activation on equal-spin bonds with probability p. */
int or_bonds(uint32_t L, double K, uint64_t seed, uint32_t sweep, const uint8_t* s, uint8_t* bx, uint8_t* by)
{
    if (L < 2 || !s || !bx || !by) return -1;
    uint64_t thr = or_threshold(K);
    if (thr == OR_BAD_THRESHOLD) return -1;
    for (uint32_t y = 0; y < L; ++y) {
        uint32_t yd = (y + 1 == L) ? 0 : y + 1;
        for (uint32_t x = 0; x < L; ++x) {
            uint32_t xr = (x + 1 == L) ? 0 : x + 1;
            uint64_t i = (uint64_t)y * L + x;
            uint32_t wx, wy;
            or_bond_draws(seed, sweep, i, &wx, &wy);
            bx[i] = (s[i] == s[(uint64_t)y * L + xr]) && ((uint64_t)wx < thr);
            by[i] = (s[i] == s[(uint64_t)yd * L + x]) && ((uint64_t)wy < thr);
        }
    }
    return 0;
}

/* Step (3) of Sec. 2: every cluster takes the new state drawn for its root;
 * then the observables of the new configuration (obs may be NULL). */
int or_flip(uint32_t L, uint32_t q, uint64_t seed, uint32_t sweep, uint8_t* s, const uint8_t* bx,
            const uint8_t* by, const uint32_t* label, int64_t* obs)
{
    if (L < 2 || q < 2 || q > 255 || !s || !bx || !by || !label) return -1;
    uint64_t N = (uint64_t)L * L;
    for (uint64_t i = 0; i < N; ++i)
        s[i] = (uint8_t)or_newspin(seed, sweep, label[i], q);
    if (obs) {
        or_observe(L, q, s, obs);
        int64_t active = 0;
        for (uint64_t i = 0; i < N; ++i) active += bx[i] + by[i];
        obs[1] = active;
    }
    return 0;
}

int or_sweep(uint32_t L, uint32_t q, double K, uint64_t seed, uint32_t sweep,
             uint8_t* s, uint8_t* bx, uint8_t* by, uint32_t* label, int64_t* obs)
{
    if (L < 2 || q < 2 || q > 255 || !s || !bx || !by || !label) return -1;
    if (or_bonds(L, K, seed, sweep, s, bx, by) != 0) return -1;   /* step (1) */
    or_label(L, bx, by, label);                                   /* step (2): root = smallest site index */
    return or_flip(L, q, seed, sweep, s, bx, by, label, obs);     /* step (3) */
}

int or_run(uint32_t L, uint32_t q, double K, uint64_t seed, uint32_t first_sweep,
           uint32_t n_sweeps, uint8_t* s, int64_t* obs_out)
{
    if (L < 2 || q < 2 || q > 255 || !s) return -1;
    uint64_t N = (uint64_t)L * L;
    uint8_t* bx = (uint8_t*)malloc(N);
    uint8_t* by = (uint8_t*)malloc(N);
    uint32_t* label = (uint32_t*)malloc(N * sizeof(uint32_t));
    int rc = 0;
    if (!bx || !by || !label) rc = -2;
    for (uint32_t k = 0; rc == 0 && k < n_sweeps; ++k)
        rc = or_sweep(L, q, K, seed, first_sweep + k, s, bx, by, label,
                      obs_out ? obs_out + (uint64_t)k * (2 + q) : NULL);
    free(bx);
    free(by);
    free(label);
    return rc;
}
