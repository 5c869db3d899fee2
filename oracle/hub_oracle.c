/*
 * hub_oracle.c -- plain FP64 CPU oracle for the USApHMP parallel genetic
 * algorithm of Benaini, Berrajaa, Boukachour and Oudani, "Solving the
 * Uncapacitated Single Allocation p-Hub Median Problem on GPU"
 * (arXiv 1704.06258).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Arithmetic rules (the "canonical order" every exact GPU kernel reproduces):
 *   - every floating-point operation is a separately rounded IEEE binary64
 *     operation (built with -ffp-contract=off, SSE2 doubles, no FMA);
 *   - every accumulator starts at +0.0 and sums in ascending index order.
 *
 * Cost of one allocation a (a[i] = hub node of node i), eq. (1) of Sec. 3
 * with every inter-hub flow routed directly hub->hub (the per-path cost
 * chi*C_ik + alpha*C_kl + delta*C_jl of Sec. 6.2):
 *   O_i = sum_j W_ij            D_j = sum_i W_ij            c_i = C[i][a_i]
 *   Cc  = sum_i O_i*c_i         Dd  = sum_i D_i*c_i
 *   t_j = sum_i W_ij*C[a_i][a_j]                  T = sum_j t_j
 *   f   = ((chi*Cc) + (alpha*T)) + (delta*Dd),    cost = f*scale
 * scale is 1 (raw cost), 1/sum(W) (CAB-style fitness) or 1e-3 (AP/Urand-style
 * fitness), Sec. 4.3.
 *
 * Multi-hop routing (the "_routed" entry points): in the MIP of Sec. 3 the
 * variables Y_kl^i exist for every arc (k, l) and eq. (4) only conserves flow,
 * so for fixed hubs and allocation the cheapest routing of the flow from hub
 * a_i to hub a_j follows a shortest path of the network with arc costs C
 * (Sec. 3: with the hubs fixed the problem is solved by a shortest-path
 * algorithm).  The transfer term then reads C* = the all-pairs shortest-path
 * distances of C instead of C:  t_j = sum_i W_ij*C*[a_i][a_j].  Collection
 * and distribution keep the direct arcs C_ik of eq. (1).  C* is computed by
 * Floyd-Warshall in binary64 (intermediate node k ascending, then i, then j
 * ascending; a path through k replaces the entry only when strictly shorter).
 * With a metric C, C* = C up to rounding.
 *
 * The GA (Sec. 4 and 5) is a heuristic, so this file follows its steps in the
 * paper's order: perturbation of the island ancestor (Sec. 4.1 and 5),
 * single-point crossover of thread pairs, hub<->spoke swap mutation,
 * correction to exactly p hubs (Sec. 4.2), nearest-hub allocation and Eval
 * (Sec. 5), island argmin with ancestor update (Sec. 5) and the global argmin
 * of the outer loop (Sec. 5).  Random draws come from Philox4x64-10 (Salmon,
 * Moraes, Dror, Shaw, SC'11), written here from that paper's definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ RNG -- */

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL /* golden ratio */
#define PHILOX_W1 0xBB67AE8584CAA73BULL /* sqrt(3) - 1 */

/* Philox4x64 with 10 rounds: each round multiplies words 0 and 2 by the two
 * round multipliers, crosses the halves and xors in the round key; the key is
 * bumped by the Weyl constants between rounds. */
void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        u128 p0 = (u128)PHILOX_M0 * x0;
        u128 p1 = (u128)PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Uniform index in [0, M): floor(w * M / 2^64). */
uint64_t oracle_mulhi(uint64_t w, uint64_t m) { return (uint64_t)(((u128)w * m) >> 64); }

#define GA_KEY_DOMAIN 0x4741ULL

/* The four words drawn for (generation g, index idx, operator op, repeat t). */
void oracle_ga_draw(uint64_t seed, uint64_t g, uint64_t idx, uint64_t op, uint64_t t, uint64_t out[4])
{
    uint64_t ctr[4] = {g, idx, op, t};
    uint64_t key[2] = {seed, GA_KEY_DOMAIN};
    oracle_philox4x64_10(ctr, key, out);
}

/* ---------------------------------------------------------- cost, Sec. 3 -- */

/* O_i (row sums) and D_j (column sums), ascending order. */
void oracle_flows(int n, const double *W, double *O, double *D)
{
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc = acc + W[(size_t)i * n + j];
        O[i] = acc;
    }
    for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i) acc = acc + W[(size_t)i * n + j];
        D[j] = acc;
    }
}

/* Cost of an arbitrary allocation a (node ids), canonical order above.
 * parts (may be NULL) receives {Cc, T, Dd}.  Returns cost = f*scale. */
static double cost_with_flows(int n, const double *C, const double *Ctr, const double *W, const double *O,
                              const double *D, const int *a, double chi, double alpha, double delta, double scale,
                              double *parts)
{
    double Cc = 0.0, Dd = 0.0, T = 0.0;
    for (int i = 0; i < n; ++i) {
        double ci = C[(size_t)i * n + a[i]];
        Cc = Cc + O[i] * ci;
    }
    for (int i = 0; i < n; ++i) {
        double ci = C[(size_t)i * n + a[i]];
        Dd = Dd + D[i] * ci;
    }
    for (int j = 0; j < n; ++j) {
        double tj = 0.0;
        for (int i = 0; i < n; ++i) tj = tj + W[(size_t)i * n + j] * Ctr[(size_t)a[i] * n + a[j]];
        T = T + tj;
    }
    double f = ((chi * Cc) + (alpha * T)) + (delta * Dd);
    if (parts) {
        parts[0] = Cc;
        parts[1] = T;
        parts[2] = Dd;
    }
    return f * scale;
}

/* Transfer matrix Ctr (NULL: C itself, direct hub-to-hub routing). */
double oracle_cost_alloc_routed(int n, const double *C, const double *Ctr, const double *W, const int *a, double chi,
                                double alpha, double delta, double scale, double *parts)
{
    double *O = (double *)malloc(sizeof(double) * (size_t)n);
    double *D = (double *)malloc(sizeof(double) * (size_t)n);
    oracle_flows(n, W, O, D);
    double f = cost_with_flows(n, C, Ctr ? Ctr : C, W, O, D, a, chi, alpha, delta, scale, parts);
    free(O);
    free(D);
    return f;
}

double oracle_cost_alloc(int n, const double *C, const double *W, const int *a, double chi, double alpha,
                         double delta, double scale, double *parts)
{
    return oracle_cost_alloc_routed(n, C, NULL, W, a, chi, alpha, delta, scale, parts);
}

/* All-pairs shortest-path distances of C (Floyd-Warshall, binary64): out
 * starts as C; for k ascending, every (i, j) in ascending order takes
 * out[i][k] + out[k][j] when that is strictly smaller. */
void oracle_shortest_paths(int n, const double *C, double *out)
{
    memcpy(out, C, sizeof(double) * (size_t)n * n);
    for (int k = 0; k < n; ++k)
        for (int i = 0; i < n; ++i) {
            const double dik = out[(size_t)i * n + k];
            for (int j = 0; j < n; ++j) {
                const double via = dik + out[(size_t)k * n + j];
                if (via < out[(size_t)i * n + j]) out[(size_t)i * n + j] = via;
            }
        }
}

/* Hub-to-hub flow matrix F[k][l] = sum_i sum_j [k(i)=k][k(j)=l] W_ij, with
 * k(i) the hub position of node i (diagnostic; ascending i then j). */
void oracle_flow_matrix(int n, int p, const double *W, const int *kpos, double *F)
{
    for (int k = 0; k < p * p; ++k) F[k] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            size_t kl = (size_t)kpos[i] * p + kpos[j];
            F[kl] = F[kl] + W[(size_t)i * n + j];
        }
}

/* ------------------------------------------------- allocation, Sec. 4.1 -- */

/* Nearest-hub allocation for a sorted hub list h[0..p): each node goes to the
 * hub with the smallest C[i][h_k] (scan k ascending, strict <, so ties go to
 * the smaller hub id); every hub is allocated to itself.  a[i] = hub node id,
 * kpos[i] = its position in h (either may be NULL). */
void oracle_allocate(int n, int p, const double *C, const int *h, int *a, int *kpos)
{
    for (int i = 0; i < n; ++i) {
        int best = 0;
        double bd = C[(size_t)i * n + h[0]];
        for (int k = 1; k < p; ++k) {
            double d = C[(size_t)i * n + h[k]];
            if (d < bd) {
                bd = d;
                best = k;
            }
        }
        for (int k = 0; k < p; ++k)
            if (h[k] == i) best = k;
        if (a) a[i] = h[best];
        if (kpos) kpos[i] = best;
    }
}

/* Middle nodes: d_i = sum_j C_ij; the p nodes with the smallest d_i (ties to
 * the smaller i), returned sorted ascending. */
void oracle_middle_nodes(int n, int p, const double *C, int *hubs)
{
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    char *taken = (char *)calloc((size_t)n, 1);
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc = acc + C[(size_t)i * n + j];
        d[i] = acc;
    }
    for (int k = 0; k < p; ++k) {
        int best = -1;
        for (int i = 0; i < n; ++i) {
            if (taken[i]) continue;
            if (best < 0 || d[i] < d[best]) best = i;
        }
        taken[best] = 1;
    }
    int c = 0;
    for (int i = 0; i < n; ++i)
        if (taken[i]) hubs[c++] = i;
    free(d);
    free(taken);
}

/* ------------------------------------------- sorted hub-list operations -- */

/* r-th (0-based) node that is not in the sorted list x[0..cnt). */
static int nth_spoke(const int *x, int cnt, int r)
{
    int v = r;
    for (int k = 0; k < cnt; ++k) {
        if (x[k] <= v)
            v++;
        else
            break;
    }
    return v;
}

static void remove_at(int *x, int *cnt, int pos)
{
    for (int k = pos; k + 1 < *cnt; ++k) x[k] = x[k + 1];
    (*cnt)--;
}

static void insert_sorted(int *x, int *cnt, int v)
{
    int k = *cnt;
    while (k > 0 && x[k - 1] > v) {
        x[k] = x[k - 1];
        k--;
    }
    x[k] = v;
    (*cnt)++;
}

/* Hub<->spoke swap: remove the hub at position pos_draw over cnt, add the
 * spoke of rank rank_draw over n-cnt (spokes ranked before the removal). */
static void swap_move(int n, int *x, int *cnt, uint64_t w_pos, uint64_t w_rank)
{
    int pos = (int)oracle_mulhi(w_pos, (uint64_t)*cnt);
    int v = nth_spoke(x, *cnt, (int)oracle_mulhi(w_rank, (uint64_t)(n - *cnt)));
    remove_at(x, cnt, pos);
    insert_sorted(x, cnt, v);
}

/* Operators with their draws passed in, exported for unit tests. */
void oracle_op_swap(int n, int *x, int *cnt, uint64_t w_pos, uint64_t w_rank)
{
    if (*cnt > 0 && *cnt < n) swap_move(n, x, cnt, w_pos, w_rank);
}

/* Single-point crossover at cut c in [1, n-1]: out = {h in xa : h < c} u
 * {h in xb : h >= c}; returns the hub count of out. */
int oracle_op_crossover(const int *xa, int ca, const int *xb, int cb, int cut, int *out)
{
    int c = 0;
    for (int k = 0; k < ca; ++k)
        if (xa[k] < cut) out[c++] = xa[k];
    for (int k = 0; k < cb; ++k)
        if (xb[k] >= cut) out[c++] = xb[k];
    return c;
}

/* Correction to exactly p hubs; draws[t] is the word used by fix t.  Returns
 * the number of draws used. */
int oracle_op_correct(int n, int p, int *x, int *cnt, const uint64_t *draws)
{
    int t = 0;
    while (*cnt > p) {
        remove_at(x, cnt, (int)oracle_mulhi(draws[t], (uint64_t)*cnt));
        t++;
    }
    while (*cnt < p) {
        insert_sorted(x, cnt, nth_spoke(x, *cnt, (int)oracle_mulhi(draws[t], (uint64_t)(n - *cnt))));
        t++;
    }
    return t;
}

/* --------------------------------------------------------- GA, Sec. 4-5 -- */

typedef struct {
    int n, p, S, m, n1, elitist;
    double chi, alpha, delta, scale;
    uint64_t seed;
} ga_cfg;

/* Child s of generation g, built from the ancestor of its island. */
static void make_child(const ga_cfg *cf, const double *C, const int *anc, uint64_t g, int s, int *child, int *scratch)
{
    (void)C;
    const int n = cf->n, p = cf->p;
    const int q = s / 2;
    const int r = s / cf->m;
    int *pa = scratch, *pb = scratch + p, *cx = scratch + 2 * p;
    int ca = p, cb = p;
    uint64_t w[4];
    /* perturbation of the island ancestor, one per parent (op 0) */
    memcpy(pa, anc + (size_t)r * p, sizeof(int) * (size_t)p);
    memcpy(pb, anc + (size_t)r * p, sizeof(int) * (size_t)p);
    if (p < n) {
        oracle_ga_draw(cf->seed, g, (uint64_t)(2 * q), 0, 0, w);
        swap_move(n, pa, &ca, w[0], w[1]);
        oracle_ga_draw(cf->seed, g, (uint64_t)(2 * q + 1), 0, 0, w);
        swap_move(n, pb, &cb, w[0], w[1]);
    }
    /* crossover of the pair (op 1, one cut per pair) */
    oracle_ga_draw(cf->seed, g, (uint64_t)q, 1, 0, w);
    int cut = 1 + (int)oracle_mulhi(w[0], (uint64_t)(n - 1));
    int cnt = (s % 2 == 0) ? oracle_op_crossover(pa, ca, pb, cb, cut, cx) : oracle_op_crossover(pb, cb, pa, ca, cut, cx);
    /* mutation (op 2) */
    oracle_ga_draw(cf->seed, g, (uint64_t)s, 2, 0, w);
    if (cnt > 0 && cnt < n) swap_move(n, cx, &cnt, w[0], w[1]);
    /* correction (op 3, one draw per fix) */
    uint64_t t = 0;
    while (cnt > p) {
        oracle_ga_draw(cf->seed, g, (uint64_t)s, 3, t, w);
        remove_at(cx, &cnt, (int)oracle_mulhi(w[0], (uint64_t)cnt));
        t++;
    }
    while (cnt < p) {
        oracle_ga_draw(cf->seed, g, (uint64_t)s, 3, t, w);
        insert_sorted(cx, &cnt, nth_spoke(cx, cnt, (int)oracle_mulhi(w[0], (uint64_t)(n - cnt))));
        t++;
    }
    memcpy(child, cx, sizeof(int) * (size_t)p);
}

static int cfg_ok(const ga_cfg *cf)
{
    return cf->n >= 1 && cf->p >= 1 && cf->p <= cf->n && cf->m >= 2 && cf->m % 2 == 0 && cf->S >= cf->m &&
           cf->S % cf->m == 0 && cf->n1 >= 1;
}

/* All S children of generation g (exported so the GPU operators can be
 * compared child by child). */
int oracle_ga_children(int n, int p, int S, int m, uint64_t seed, uint64_t g, const int *anc, int *children)
{
    ga_cfg cf = {n, p, S, m, 1, 1, 0, 0, 0, 1, seed};
    if (!cfg_ok(&cf)) return 1;
#pragma omp parallel
    {
        int *scratch = (int *)malloc(sizeof(int) * (size_t)(4 * p + 4));
#pragma omp for schedule(static)
        for (int s = 0; s < S; ++s) make_child(&cf, NULL, anc, g, s, children + (size_t)s * p, scratch);
        free(scratch);
    }
    return 0;
}

static void sort_ints(int *x, int c)
{
    for (int i = 1; i < c; ++i) {
        int v = x[i], k = i;
        while (k > 0 && x[k - 1] > v) {
            x[k] = x[k - 1];
            k--;
        }
        x[k] = v;
    }
}

/* Batch evaluation of hub sets (any order; sorted here).  cost[s] is the
 * scaled cost; parts (3 per set) and alloc (n per set) may be NULL.  Returns
 * 0, or 1 when a hub set is invalid (out of range or repeated). */
int oracle_evaluate_routed(int n, int p, const double *C, const double *Ctr, const double *W, int count,
                           const int *hubs, double chi, double alpha, double delta, double scale, double *cost,
                           double *parts, int *alloc)
{
    if (!Ctr) Ctr = C;
    double *O = (double *)malloc(sizeof(double) * (size_t)n);
    double *D = (double *)malloc(sizeof(double) * (size_t)n);
    oracle_flows(n, W, O, D);
    int bad = 0;
#pragma omp parallel
    {
        int *h = (int *)malloc(sizeof(int) * (size_t)p);
        int *a = (int *)malloc(sizeof(int) * (size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int s = 0; s < count; ++s) {
            memcpy(h, hubs + (size_t)s * p, sizeof(int) * (size_t)p);
            sort_ints(h, p);
            int ok = h[0] >= 0 && h[p - 1] < n;
            for (int k = 1; k < p; ++k)
                if (h[k] == h[k - 1]) ok = 0;
            if (!ok) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            oracle_allocate(n, p, C, h, a, NULL);
            cost[s] = cost_with_flows(n, C, Ctr, W, O, D, a, chi, alpha, delta, scale,
                                      parts ? parts + (size_t)3 * s : NULL);
            if (alloc) memcpy(alloc + (size_t)s * n, a, sizeof(int) * (size_t)n);
        }
        free(h);
        free(a);
    }
    free(O);
    free(D);
    return bad;
}

int oracle_evaluate(int n, int p, const double *C, const double *W, int count, const int *hubs, double chi,
                    double alpha, double delta, double scale, double *cost, double *parts, int *alloc)
{
    return oracle_evaluate_routed(n, p, C, NULL, W, count, hubs, chi, alpha, delta, scale, cost, parts, alloc);
}

/* GA state, caller-owned arrays:
 *   anc[R*p] ancestors (sorted), anc_cost[R], anc_parts[3R],
 *   best[p], best_cost[1], best_parts[3], gen[1] (generation counter g).
 * oracle_ga_init sets every ancestor to the middle-node solution P0. */
int oracle_ga_init_routed(int n, int p, const double *C, const double *Ctr, const double *W, int S, int m, double chi,
                          double alpha, double delta, double scale, int *anc, double *anc_cost, double *anc_parts,
                          int *best, double *best_cost, double *best_parts, int64_t *gen)
{
    if (n < 1 || p < 1 || p > n || m < 2 || m % 2 || S < m || S % m) return 1;
    int R = S / m;
    int *h = (int *)malloc(sizeof(int) * (size_t)p);
    int *a = (int *)malloc(sizeof(int) * (size_t)n);
    double parts[3];
    oracle_middle_nodes(n, p, C, h);
    oracle_allocate(n, p, C, h, a, NULL);
    double f = oracle_cost_alloc_routed(n, C, Ctr, W, a, chi, alpha, delta, scale, parts);
    for (int r = 0; r < R; ++r) {
        memcpy(anc + (size_t)r * p, h, sizeof(int) * (size_t)p);
        anc_cost[r] = f;
        memcpy(anc_parts + (size_t)3 * r, parts, sizeof(parts));
    }
    memcpy(best, h, sizeof(int) * (size_t)p);
    *best_cost = f;
    memcpy(best_parts, parts, sizeof(parts));
    *gen = 0;
    free(h);
    free(a);
    return 0;
}

/* Run `generations` generations from the given state.  trace (may be NULL)
 * receives best_cost after each generation. */
int oracle_ga_run_routed(int n, int p, const double *C, const double *Ctr, const double *W, int S, int m, int n1,
                         int elitist, double chi, double alpha, double delta, double scale, uint64_t seed,
                         int generations, int *anc, double *anc_cost, double *anc_parts, int *best,
                         double *best_cost, double *best_parts, int64_t *gen, double *trace)
{
    ga_cfg cf = {n, p, S, m, n1, elitist, chi, alpha, delta, scale, seed};
    if (!cfg_ok(&cf)) return 1;
    const int R = S / m;
    int *children = (int *)malloc(sizeof(int) * (size_t)S * p);
    double *cost = (double *)malloc(sizeof(double) * (size_t)S);
    double *parts = (double *)malloc(sizeof(double) * (size_t)3 * S);
    for (int it = 0; it < generations; ++it) {
        uint64_t g = (uint64_t)*gen;
        oracle_ga_children(n, p, S, m, seed, g, anc, children);
        oracle_evaluate_routed(n, p, C, Ctr, W, S, children, chi, alpha, delta, scale, cost, parts, NULL);
        /* island selection: argmin over the island's m children */
        for (int r = 0; r < R; ++r) {
            int js = r * m;
            for (int j = r * m + 1; j < (r + 1) * m; ++j)
                if (cost[j] < cost[js]) js = j;
            if (!elitist || cost[js] < anc_cost[r]) {
                memcpy(anc + (size_t)r * p, children + (size_t)js * p, sizeof(int) * (size_t)p);
                anc_cost[r] = cost[js];
                memcpy(anc_parts + (size_t)3 * r, parts + (size_t)3 * js, sizeof(double) * 3);
            }
        }
        /* outer loop: the best island ancestor becomes every ancestor */
        if ((g + 1) % (uint64_t)n1 == 0) {
            int rs = 0;
            for (int r = 1; r < R; ++r)
                if (anc_cost[r] < anc_cost[rs]) rs = r;
            for (int r = 0; r < R; ++r) {
                if (r == rs) continue;
                memcpy(anc + (size_t)r * p, anc + (size_t)rs * p, sizeof(int) * (size_t)p);
                anc_cost[r] = anc_cost[rs];
                memcpy(anc_parts + (size_t)3 * r, anc_parts + (size_t)3 * rs, sizeof(double) * 3);
            }
        }
        /* best so far */
        int rb = 0;
        for (int r = 1; r < R; ++r)
            if (anc_cost[r] < anc_cost[rb]) rb = r;
        if (anc_cost[rb] < *best_cost) {
            memcpy(best, anc + (size_t)rb * p, sizeof(int) * (size_t)p);
            *best_cost = anc_cost[rb];
            memcpy(best_parts, anc_parts + (size_t)3 * rb, sizeof(double) * 3);
        }
        *gen = (int64_t)(g + 1);
        if (trace) trace[it] = *best_cost;
    }
    free(children);
    free(cost);
    free(parts);
    return 0;
}

int oracle_ga_init(int n, int p, const double *C, const double *W, int S, int m, double chi, double alpha,
                   double delta, double scale, int *anc, double *anc_cost, double *anc_parts, int *best,
                   double *best_cost, double *best_parts, int64_t *gen)
{
    return oracle_ga_init_routed(n, p, C, NULL, W, S, m, chi, alpha, delta, scale, anc, anc_cost, anc_parts, best,
                                 best_cost, best_parts, gen);
}

int oracle_ga_run(int n, int p, const double *C, const double *W, int S, int m, int n1, int elitist, double chi,
                  double alpha, double delta, double scale, uint64_t seed, int generations, int *anc,
                  double *anc_cost, double *anc_parts, int *best, double *best_cost, double *best_parts,
                  int64_t *gen, double *trace)
{
    return oracle_ga_run_routed(n, p, C, NULL, W, S, m, n1, elitist, chi, alpha, delta, scale, seed, generations,
                                anc, anc_cost, anc_parts, best, best_cost, best_parts, gen, trace);
}
