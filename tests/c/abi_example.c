/* The library driven from C alone: a noisy D2Q9 lattice with a thermal
 * start, 200 steps with a correlator sample every 10 (graph-replayed
 * periods), the FP64 sums read back, the conservation sums, and the
 * velocity-set tables of D3Q15.  Prints one line:
 *   t nsamples checksum(sums) sum(rho - rho0) D Q
 * With "--invalid" it only checks that a rejected creation returns NULL
 * with a message (no device needed). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "flb.h"
#include "flb_dq.h"

int main(int argc, char **argv)
{
    const double tau[9] = {1, 1, 1, 0.8, 0.8, 1.0, 1, 1, 1};
    const double u0[2] = {0.05, 0.0};
    if (argc > 1 && strcmp(argv[1], "--invalid") == 0) {
        const double bad_tau[9] = {1, 1, 1, 0.4, 0.8, 1.0, 1, 1, 1};
        flb_t *h = flb_create(48, 40, bad_tau, 1e-4, 1.0, u0, 7);
        if (h) {
            flb_destroy(h);
            return 1;
        }
        printf("rejected: %s\n", flb_last_error());
        return 0;
    }
    const int nx = 48, ny = 40;
    flb_t *h = flb_create(nx, ny, tau, 1e-4, 1.0, u0, 7);
    if (!h) {
        fprintf(stderr, "create: %s\n", flb_last_error());
        return 1;
    }
    if (flb_thermalize(h) != FLB_OK || flb_run(h, 200, 10) != FLB_OK) {
        fprintf(stderr, "run: %s\n", flb_last_error());
        return 1;
    }
    const size_t n = (size_t)flb_num_kinds(h) * ny * (nx / 2 + 1);
    double *acc = malloc(n * sizeof *acc);
    int64_t ns = 0;
    double cons[5];
    if (!acc || flb_read_correlators(h, 0, acc, n, &ns) != FLB_OK ||
        flb_conservation(h, 0, cons) != FLB_OK) {
        fprintf(stderr, "read: %s\n", flb_last_error());
        return 1;
    }
    double sum = 0.0;
    for (size_t i = 0; i < n; ++i) sum += acc[i];
    int32_t D = 0, Q = 0, v[3 * FLB_DQ_MAXQ];
    double w[FLB_DQ_MAXQ], m[FLB_DQ_MAXQ * FLB_DQ_MAXQ];
    if (flb_dq_tables(FLB_DQ_D3Q15, &D, &Q, v, w, m) != FLB_OK) {
        fprintf(stderr, "tables: %s\n", flb_last_error());
        return 1;
    }
    printf("%lld %lld %.17g %.17g %d %d\n", (long long)flb_get_step(h), (long long)ns, sum,
           cons[0], (int)D, (int)Q);
    free(acc);
    flb_destroy(h);
    return 0;
}
