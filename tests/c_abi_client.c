/* A C client of libhubga (no Python, no torch): the library allocates its own
 * workspace and works on the null stream.  Reads an instance from a binary
 * file, evaluates hub sets, solves, round-trips the GA state, exercises the
 * error paths, and prints the results for the calling test to check.
 *   usage: c_abi_client <instance.bin> <generations>
 * instance.bin: int32 n, int32 p, int32 count, then C (n*n f64), W (n*n f64),
 * hubs (count*p int32). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hubga.h"

static int check(ga_status s, const ga_ctx *ctx, const char *what)
{
    if (s != GA_OK) {
        fprintf(stderr, "%s: %s (%s)\n", what, ga_status_str(s), ga_last_error(ctx));
        return 1;
    }
    return 0;
}

int main(int argc, char **argv)
{
    if (argc < 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int hdr[3];
    if (fread(hdr, sizeof(int), 3, f) != 3) return 2;
    const int n = hdr[0], p = hdr[1], count = hdr[2];
    const int gens = atoi(argv[2]);
    double *C = malloc(sizeof(double) * (size_t)n * n), *W = malloc(sizeof(double) * (size_t)n * n);
    int *hubs = malloc(sizeof(int) * (size_t)count * p);
    if (fread(C, sizeof(double), (size_t)n * n, f) != (size_t)n * n) return 2;
    if (fread(W, sizeof(double), (size_t)n * n, f) != (size_t)n * n) return 2;
    if (fread(hubs, sizeof(int), (size_t)count * p, f) != (size_t)count * p) return 2;
    fclose(f);

    ga_params q;
    ga_params_default(&q, n, p);
    q.chi = 3.0;
    q.alpha = 0.75;
    q.delta = 2.0;
    q.population = 64;
    q.island_size = 16;
    q.n1 = 5;
    q.seed = 11;
    q.precision = GA_PREC_SPLIT_BF16;
    q.kernel = GA_KERN_BATCHED;
    printf("workspace_bytes %zu\n", ga_workspace_bytes(&q, GA_DT_F64, GA_DT_F64));

    ga_ctx *ctx = NULL;
    /* invalid first: p > n */
    ga_params bad = q;
    bad.p = n + 1;
    printf("invalid_init %s\n", ga_status_str(ga_init(&bad, C, GA_DT_F64, W, GA_DT_F64, NULL, 0, NULL, &ctx)));
    if (check(ga_init(&q, C, GA_DT_F64, W, GA_DT_F64, NULL, 0, NULL, &ctx), NULL, "ga_init")) return 1;

    double *cost = malloc(sizeof(double) * count), *eps = malloc(sizeof(double) * count);
    if (check(ga_evaluate(ctx, hubs, count, cost, NULL, NULL, eps), ctx, "ga_evaluate")) return 1;
    for (int s = 0; s < count; ++s) printf("cost %d %.17g %.17g\n", s, cost[s], eps[s]);

    int dup[2] = {0, 0};
    int *badh = malloc(sizeof(int) * p);
    for (int k = 0; k < p; ++k) badh[k] = k;
    badh[p - 1] = badh[0];
    (void)dup;
    printf("invalid_eval %s\n", ga_status_str(ga_evaluate(ctx, badh, 1, cost, NULL, NULL, NULL)));

    /* solve in two halves across a state round trip into a second context */
    if (check(ga_step(ctx, gens / 2), ctx, "ga_step")) return 1;
    size_t bytes = 0;
    if (check(ga_get_state(ctx, NULL, &bytes), ctx, "state size")) return 1;
    void *blob = malloc(bytes);
    if (check(ga_get_state(ctx, blob, &bytes), ctx, "ga_get_state")) return 1;
    ga_ctx *ctx2 = NULL;
    if (check(ga_init(&q, C, GA_DT_F64, W, GA_DT_F64, NULL, 0, NULL, &ctx2), NULL, "ga_init 2")) return 1;
    if (check(ga_set_state(ctx2, blob, bytes), ctx2, "ga_set_state")) return 1;
    int *best = malloc(sizeof(int) * p), *alloc = malloc(sizeof(int) * n);
    double bc = 0.0;
    if (check(ga_solve(ctx2, gens - gens / 2, best, alloc, &bc), ctx2, "ga_solve")) return 1;
    printf("best_cost %.17g\n", bc);
    printf("best_hubs");
    for (int k = 0; k < p; ++k) printf(" %d", best[k]);
    printf("\n");
    int64_t st[4];
    if (check(ga_stats(ctx2, st), ctx2, "ga_stats")) return 1;
    printf("stats %lld %lld %lld %lld\n", (long long)st[0], (long long)st[1], (long long)st[2], (long long)st[3]);
    printf("wrong_state %s\n", ga_status_str(ga_set_state(ctx2, blob, bytes - 8)));
    ga_free(ctx);
    ga_free(ctx2);
    free(C);
    free(W);
    free(hubs);
    free(cost);
    free(eps);
    free(blob);
    free(best);
    free(alloc);
    free(badh);
    return 0;
}
