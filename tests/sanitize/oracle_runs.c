/* Runs of the CPU oracles (Potts and XY) for a sanitized build: reads one run
 * per line from stdin and prints its final state and observable rows, so a
 * test can compare them with the same runs of the ordinary build.
 *   potts L q K seed random_start first_sweep n_sweeps
 *   xy    L K seed random_start first_sweep n_sweeps dir_bits
 * Output per run: the run line, then the state (one value per site) and the
 * observable rows, as decimal integers separated by spaces. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sw_oracle.h"
#include "xy_oracle.h"

int main(void)
{
    char kind[16];
    while (scanf("%15s", kind) == 1) {
        unsigned L, q = 0, first, n, bits = 0;
        int rs;
        double K;
        unsigned long long seed;
        if (strcmp(kind, "potts") == 0) {
            if (scanf("%u %u %lf %llu %d %u %u", &L, &q, &K, &seed, &rs, &first, &n) != 7) return 2;
        } else if (strcmp(kind, "xy") == 0) {
            if (scanf("%u %lf %llu %d %u %u %u", &L, &K, &seed, &rs, &first, &n, &bits) != 7) return 2;
        } else {
            return 2;
        }
        const size_t N = (size_t)L * L;
        const size_t words = (size_t)n * (q ? 2 + q : OR_XY_OBS_WORDS);
        long long* obs = malloc(words * sizeof *obs);
        int rc;
        printf("%s\n", kind);
        if (q) {
            unsigned char* s = malloc(N);
            rc = or_init(L, q, seed, rs, s) || or_run(L, q, K, seed, first, n, s, (int64_t*)obs);
            for (size_t i = 0; i < N; ++i) printf("%u ", s[i]);
            free(s);
        } else {
            unsigned* a = malloc(N * sizeof *a);
            rc = or_xy_init(L, seed, rs, a) || or_xy_run(L, K, seed, first, n, bits, a, (int64_t*)obs);
            for (size_t i = 0; i < N; ++i) printf("%u ", a[i]);
            free(a);
        }
        printf("\n");
        for (size_t i = 0; i < words; ++i) printf("%lld ", obs[i]);
        printf("\nrc %d\n", rc);
        free(obs);
    }
    return 0;
}
