/* Drives the oracle (oracle/sa_oracle.c) through every entry point on small fixtures, for a build
 * with the address and undefined-behaviour sanitizers.  Prints "ok". */
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/sa_oracle.h"

static int failures = 0;
static void expect(int c, const char *what) {
    if (!c) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

int main(void) {
    /* E = 2 z0^2 - 3 z0 z1 + z1 z2^3 + 5 z0 - 4 z2 + (z1 z2 repeated, cancelling) */
    const int64_t ptr[] = {0, 2, 4, 8, 9, 10, 12, 14};
    const int32_t fac[] = {0, 0, 0, 1, 1, 2, 2, 2, 0, 2, 1, 2, 2, 1};
    const int64_t coef[] = {2, -3, 1, 5, -4, 7, -7};
    const int32_t lo[] = {-3, 0, -2}, hi[] = {4, 5, 2};
    sao_poly *p = NULL;
    expect(sao_poly_build(3, 7, ptr, fac, coef, lo, hi, &p) == SAO_OK, "build");
    expect(sao_poly_n_terms(p) == 5, "merged terms");
    double beta[12], ti, tf;
    expect(sao_schedule(p, 12, beta, &ti, &tf) == SAO_OK, "schedule");
    int32_t z[3 * 5];
    int64_t e[5];
    uint64_t h[5 * 12];
    for (int rule = 0; rule < 4; ++rule) {
        for (int cache = 0; cache < 2; ++cache) {
            expect(sao_anneal_reads(p, rule, beta, 12, 0, 12, 5, NULL, 9, 1, -1.0, cache, 2, NULL, z, e, h) == SAO_OK,
                   "anneal");
            for (int r = 0; r < 5; ++r) {
                int64_t E;
                sao_energy(p, z + 3 * r, &E);
                expect(E == e[r], "tracked energy");
                expect(h[r * 12 + 11] == sao_state_hash(3, z + 3 * r), "last hash is the final state's");
            }
        }
        sao_step_info info;
        expect(sao_explain_step(p, rule, z, 1, 4, 2, beta[4], 0.5, 9, 1, &info) == SAO_OK, "explain");
        int32_t v[64];
        expect(sao_single_step(p, rule, z, 2, 3, 0.2, 0.5, 64, 11, 0, v) == SAO_OK, "single step");
    }
    int64_t d;
    expect(sao_delta(p, z, 0, lo[0], &d) == SAO_OK, "delta");
    sao_poly_free(p);
    /* the int64 bound at 2^62: 4 * (2^30)^2 is rejected */
    const int64_t ptr2[] = {0, 2};
    const int32_t fac2[] = {0, 0};
    const int64_t coef2[] = {4};
    const int32_t lo2[] = {-(1 << 30)}, hi2[] = {(1 << 30) - 2};
    expect(sao_poly_build(1, 1, ptr2, fac2, coef2, lo2, hi2, &p) == SAO_ERANGE, "bound");
    if (failures) return 1;
    printf("ok\n");
    return 0;
}
