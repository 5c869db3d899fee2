/*
 * hubga.h -- C ABI of libhubga.so, the MI355X (gfx950) engine for the parallel
 * genetic algorithm of Benaini, Berrajaa, Boukachour and Oudani, "Solving the
 * Uncapacitated Single Allocation p-Hub Median Problem on GPU" (arXiv
 * 1704.06258).
 *
 * Problem (Sec. 3): n nodes with unit costs C (n x n) and flows W (n x n);
 * open exactly p hubs, allocate every node to one hub (each hub to itself)
 * and minimise objective (1).  With inter-hub flow routed directly hub->hub,
 * i.e. the per-path cost chi*C_ik + alpha*C_kl + delta*C_jl of Sec. 6.2, the
 * cost of an allocation a (a_i = hub node of node i) is
 *     f = chi*sum_i O_i*C[i][a_i] + alpha*sum_i sum_j W_ij*C[a_i][a_j]
 *       + delta*sum_i D_i*C[i][a_i],     O_i = sum_j W_ij,  D_j = sum_i W_ij,
 * reported as cost = f*scale (Sec. 4.3: scale 1/sum(W) for CAB-style fitness,
 * 1e-3 for AP/Urand-style fitness, 1 for the raw objective).  The
 * transfer leg of a flow whose ends share a hub k costs alpha*C[k][k], which
 * is zero for a distance matrix.
 *
 * Individuals are hub sets; their allocation is nearest-hub (Sec. 4.1 and 5):
 * a_i = the hub h minimising C[i][h], ties to the smaller hub id, every hub
 * allocated to itself.
 *
 * Conventions for every entry point:
 *   - matrices are n x n row-major, element (i, j) at [i*n + j];
 *   - host pointers are plain CPU memory owned by the caller; the library
 *     copies what it needs before returning and never keeps them;
 *   - "d_" pointers are device memory owned by the caller, accessed in order
 *     on the context's stream;
 *   - every call returns a ga_status and never throws; invalid arguments are
 *     rejected before any device work (GA_ERR_INVALID, message in
 *     ga_last_error); a HIP failure returns GA_ERR_DEVICE and poisons the
 *     context, after which every call except ga_last_error / ga_free returns
 *     GA_ERR_STATE;
 *   - a context is not thread-safe; distinct contexts are independent.
 */
#ifndef HUBGA_H
#define HUBGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ga_ctx ga_ctx;

typedef enum {
    GA_OK = 0,
    GA_ERR_INVALID = 1, /* bad argument; nothing was done */
    GA_ERR_OOM = 2,     /* workspace too small or device allocation failed */
    GA_ERR_DEVICE = 3,  /* HIP error; the context is poisoned */
    GA_ERR_STATE = 4    /* call on a poisoned context, or a state blob that does not fit */
} ga_status;

typedef enum { GA_DT_F64 = 0, GA_DT_F32 = 1 } ga_dtype;

/* Arithmetic of the fitness evaluation.
 *   GA_PREC_FP64       exact: every cost is bit-identical to the binary64
 *                      evaluation in the canonical order (ascending sums:
 *                      O_i and D_j; Cc = sum_i O_i*c_i, Dd = sum_i D_i*c_i;
 *                      t_j = sum_i W_ij*C[a_i][a_j], T = sum_j t_j;
 *                      f = ((chi*Cc) + (alpha*T)) + (delta*Dd); no FMA).
 *   GA_PREC_FP32       FP32 flow sums, FP64 final reduction.
 *   GA_PREC_SPLIT_BF16 W split into bf16 hi + lo parts, the flow product
 *                      W * [A_1 ... A_S] (A_s the one-hot n x p allocation
 *                      matrix of individual s) on bf16 matrix cores with FP32
 *                      accumulation, FP64 epilogue and reduction.
 *   GA_PREC_SPLIT3_BF16 the same with W split into three bf16 parts
 *                      (hi, mid, lo: each the round-to-nearest-even of what
 *                      the previous parts leave), |W - hi - mid - lo| <=
 *                      2^-24 W against 2^-16 W for two parts, for 1.5x the
 *                      matrix-core work; register-staged tile configurations
 *                      (0, 2, 3 and 5) only.
 * In the approximate modes every returned cost carries a rigorous relative
 * error bound (ga_evaluate's eps_out) and GA selection is certified: any
 * individual whose interval could change a decision is re-evaluated exactly,
 * so GA trajectories are identical in all modes. */
typedef enum { GA_PREC_FP64 = 0, GA_PREC_FP32 = 1, GA_PREC_SPLIT_BF16 = 2, GA_PREC_SPLIT3_BF16 = 3 } ga_precision;

/* GA_KERN_PLAIN: one workgroup per individual (FP64 or FP32).
 * GA_KERN_BATCHED: the whole population in one launch -- with SPLIT_BF16 the
 * one-hot matrix-core product; with FP32 a vector kernel in which a workgroup
 * applies each W element it loads to a group of individuals, gathering their
 * hub-to-hub distances from LDS (n^2 multiply-adds per individual whatever p
 * is; the same error bound as FP32 + PLAIN). */
typedef enum { GA_KERN_PLAIN = 0, GA_KERN_BATCHED = 1 } ga_kernel;

typedef struct {
    int32_t n;            /* nodes, 1 <= n <= 8192 */
    int32_t p;            /* hubs, 1 <= p <= min(n, 64) */
    double chi;           /* collection factor, finite and >= 0 */
    double alpha;         /* inter-hub (transfer) factor, finite and >= 0 */
    double delta;         /* distribution factor, finite and >= 0 */
    double scale;         /* cost = f*scale, finite and > 0 */
    uint64_t seed;        /* Philox key word of the GA */
    int32_t population;   /* S: individuals per generation (and per evaluation batch) */
    int32_t island_size;  /* m: individuals per island, even, divides S; R = S/m islands */
    int32_t n1;           /* generations per outer step (global argmin every n1), >= 1 */
    int32_t elitist;      /* 1: an island ancestor is replaced only by a strictly better child */
    int32_t precision;    /* ga_precision */
    int32_t kernel;       /* ga_kernel: PLAIN with FP64/FP32, BATCHED with FP32/SPLIT_BF16/SPLIT3_BF16 */
    int32_t c_symmetric;  /* 1: C == C^T (checked by ga_init); 0: a transposed copy is kept */
    int32_t multihop;     /* 0: inter-hub flow goes directly hub -> hub (C[h_k][h_l]);
                           * 1: along shortest paths of the network (eq. (4) of Sec. 3 lets
                           *    flow use every arc): the transfer term reads the all-pairs
                           *    shortest-path distances C* of C (Floyd-Warshall in binary64
                           *    at ga_init, O(n^3)), collection and distribution keep C.
                           *    Differs from 0 only when C breaks the triangle inequality
                           *    (the PlanetLab setting of Sec. 6.1). */
} ga_params;

/* Fill p with defaults for n nodes and p hubs: chi=3, alpha=0.75, delta=2,
 * scale=1, seed=1, population 64, island 64, n1=10, elitist, FP64 plain,
 * c_symmetric=0, multihop=0. */
void ga_params_default(ga_params *p, int32_t n, int32_t hubs);

/* Device workspace bytes ga_init needs for these parameters and dtypes; 0 if
 * the parameters are invalid.  Lets a caller admit work against an HBM budget
 * before allocating anything. */
size_t ga_workspace_bytes(const ga_params *params, ga_dtype c_dtype, ga_dtype w_dtype);

/* Create a context (Sec. 5, host steps: build the ancestor, copy the data to
 * GPU global memory).  C and W are host arrays (n x n, dtypes as given; all
 * entries finite and >= 0).  d_workspace / ws_bytes: caller-owned device
 * memory of at least ga_workspace_bytes bytes that must outlive the context,
 * or NULL/0 to let the library allocate (and free in ga_free).  hip_stream is
 * a hipStream_t (NULL = the null stream) on which all device work is ordered.
 * On return the instance is resident, the ancestor P0 (the p middle nodes,
 * smallest sum_j C_ij with ties to the smaller index, Sec. 4.1) has been
 * evaluated exactly, every island ancestor is P0 and the generation is 0.
 * Synchronous. */
ga_status ga_init(const ga_params *params, const void *C, ga_dtype c_dtype, const void *W, ga_dtype w_dtype,
                  void *d_workspace, size_t ws_bytes, void *hip_stream, ga_ctx **out);

/* Allocation-free variant of ga_init, for callers that cannot allocate device
 * memory (harnesses that forbid hipMalloc, serving loops that must not
 * allocate): the same context as ga_init, built on a static workspace that
 * the library holds per device from module load until the process ends
 * (32 MiB), on the current device.
 * Allocates nothing: no hipMalloc, hipFree or allocating library call (C and
 * W are copied from the caller's host arrays as in ga_init).
 *   - GA_ERR_INVALID when ga_workspace_bytes(params, ...) exceeds the static
 *     workspace (use ga_init), or for the arguments ga_init rejects;
 *   - GA_ERR_STATE while another context created by ga_init_static on the
 *     same device is live: the device's one array holds that context's data
 *     until ga_free releases it.  Contexts on different devices are
 *     independent.  Nothing else shares the array.
 * The array keeps the last context's contents; ga_init_static initialises
 * every value the context reads before reading it, as ga_init does on a
 * caller's uninitialised workspace.  Synchronous. */
ga_status ga_init_static(const ga_params *params, const void *C, ga_dtype c_dtype, const void *W, ga_dtype w_dtype,
                         void *hip_stream, ga_ctx **out);

/* Evaluate `count` hub sets (host int32, count x p, any order, distinct ids in
 * [0, n)) with the context's precision and kernel (objective (1), Sec. 3 and
 * Sec. 4.3).  Outputs (host, caller-owned; any may be NULL except cost_out):
 *   cost_out[count]      scaled cost;
 *   parts_out[3*count]   {Cc, T, Dd} per set (collection, transfer,
 *                        distribution sums before the factors);
 *   alloc_out[count*n]   hub node id of every node (the S array of Sec. 4.1);
 *   eps_out[count]       relative error bound of cost_out (0 in FP64 mode).
 * Batches larger than the population are processed in chunks.  Synchronous. */
ga_status ga_evaluate(ga_ctx *ctx, const int32_t *hubs, int32_t count, double *cost_out, double *parts_out,
                      int32_t *alloc_out, double *eps_out);

/* Device-pointer variant, ordered on the context's stream (returns after
 * enqueueing).  d_hubs: count x p int32, each row sorted ascending, distinct,
 * in [0, n) (ids outside [0, n) are clamped, never dereferenced; 1 <= count <= population).
 * d_kidx (may be NULL): count x n uint16, hub position of each node's hub.
 * d_cost: count doubles (scaled cost). */
ga_status ga_evaluate_dev(ga_ctx *ctx, const int32_t *d_hubs, int32_t count, uint16_t *d_kidx, double *d_cost);

/* Exhaustive search of the nearest-hub solution space (the optimum the GA's
 * results are compared with in Sec. 6.2, Tables 1 and 3, restricted to the
 * allocation rule of Sec. 4.1 and 5): the hub sets of lexicographic ranks
 * [first, first + count) among all C(n, p) p-subsets of the nodes (rank 0 =
 * {0, 1, ..., p-1}; count = -1: through the last) are evaluated with the
 * context's precision and kernels, in chunks of the population size, and the
 * set of smallest exact cost is returned (ties to the lower rank).  In the
 * approximate modes every set whose error interval could hold the minimum is
 * re-evaluated exactly in binary64 (canonical order), so the result is the
 * exact argmin.  Outputs (host, caller-owned, any may be NULL):
 *   hubs_out[p], cost_out (exact scaled cost), parts_out[3] {Cc, T, Dd},
 *   rank_out (its rank);
 *   costs_all[count], eps_all[count]: every set's cost as evaluated and its
 *   relative error bound, in rank order (these copies wait per chunk);
 *   rechecks_out: sets re-evaluated exactly.
 * GA_ERR_INVALID when C(n, p) >= 2^62 or the range is empty or outside
 * [0, C(n, p)).  Overwrites the population buffers (ga_population) but not
 * the GA state.  Synchronous. */
ga_status ga_enumerate(ga_ctx *ctx, int64_t first, int64_t count, int32_t *hubs_out, double *cost_out,
                       double *parts_out, int64_t *rank_out, double *costs_all, double *eps_all,
                       int64_t *rechecks_out);

/* Advance the GA by `generations` generations (Sec. 4.2 and 5): per island,
 * every child is a perturbation of the island ancestor, crossed with its pair
 * partner, mutated, corrected to p hubs, allocated to nearest hubs and
 * evaluated; the island's best child replaces the ancestor (if strictly
 * better when elitist); every n1 generations the best ancestor replaces all
 * ancestors.  Random draws are Philox4x64-10 with key (seed, 0x4741) and
 * counter (g, index, operator, repeat).  Enqueued on the stream; returns
 * without waiting. */
ga_status ga_step(ga_ctx *ctx, int32_t generations);

/* Best solution so far (waits for queued work): hub node ids (p, sorted),
 * allocation (n hub node ids), exact scaled cost, {Cc, T, Dd}, and the number
 * of generations run.  Any output may be NULL. */
ga_status ga_best(ga_ctx *ctx, int32_t *hubs_out, int32_t *alloc_out, double *cost_out, double *parts_out,
                  int64_t *generation_out);

/* ga_step(generations) then ga_best (Sec. 5, host step 5: read the solution). */
ga_status ga_solve(ga_ctx *ctx, int32_t generations, int32_t *hubs_out, int32_t *alloc_out, double *cost_out);

/* Last generation's children (host, population x p) and their costs as
 * evaluated in the context's precision (population doubles); waits. */
ga_status ga_population(ga_ctx *ctx, int32_t *hubs_out, double *cost_out);

/* Island ancestors (host, R x p) and their exact costs (R); waits. */
ga_status ga_ancestors(ga_ctx *ctx, int32_t *hubs_out, double *cost_out);

/* Serialised GA state (generation, ancestors with exact costs and parts, best
 * so far).  ga_get_state with buf == NULL stores the size in *bytes.  A state
 * restored into a context with the same n, p, population, island size and
 * seed continues exactly as the original would have. */
ga_status ga_get_state(ga_ctx *ctx, void *buf, size_t *bytes);
ga_status ga_set_state(ga_ctx *ctx, const void *buf, size_t bytes);

/* Counters since ga_init: stats[0] generations, [1] exact re-evaluations of
 * selection candidates, [2] islands whose decision needed one, [3] fitness
 * evaluations.  Waits. */
ga_status ga_stats(ga_ctx *ctx, int64_t stats[4]);

/* Kernel timing with HIP events recorded on the context's stream around every
 * launch of the dominant evaluation kernel (the batched matrix-core kernel,
 * or the plain per-individual kernel).  enable=1 resets and starts, 0 stops.
 * ga_profile_read waits and returns the summed milliseconds and launches. */
ga_status ga_profile_enable(ga_ctx *ctx, int32_t enable);
ga_status ga_profile_read(ga_ctx *ctx, double *ms_total, int64_t *launches);

/* Move the context to another stream (hipStream_t, non-null or NULL): work
 * already queued on the old stream stays ordered before everything issued
 * afterwards on the new one (an event, no host wait).  The context must not
 * be in a batch whose stream differs from the new one when the batch steps. */
ga_status ga_set_stream(ga_ctx *ctx, void *hip_stream);

/* Tile configurations of the batched matrix-core kernel, for autotuning:
 * ga_tile_config_count() configurations, numbered from 0; ga_tile_config_info
 * gives rows and columns of W x [A_1..A_S] per workgroup tile and the K depth
 * staged per step.  ga_set_tile_config selects one for the context's later
 * batched evaluations (results agree to the returned error bounds in every
 * configuration; the default is 0).  Pipelined configurations (the K tiles
 * staged through an LDS ring: 6 and above) are the ones batches take. */
int32_t ga_tile_config_count(void);
ga_status ga_tile_config_info(int32_t config, int32_t *rows, int32_t *cols, int32_t *ktile);
ga_status ga_set_tile_config(ga_ctx *ctx, int32_t config);

/* Folded evaluation of the inter-hub term T of objective (1) (Sec. 3, each
 * node allocated to one hub a(i)): when C is symmetric,
 * sum_{i,j} W_ij C[a(i)][a(j)] equals the same sum over the folded matrix
 * W_ij + W_ji (j > i), W_ii (j = i), 0 (j < i).  The pipelined configurations
 * with a K depth of 64 then multiply only the K tiles on and above each row
 * tile's diagonal block, about half the matrix-core work; results keep their
 * error bounds (W >= 0, so the folded entries carry the same relative split
 * error).  *folded is set to 1 when the context's current tile configuration
 * does this (split-bf16 precision, c_symmetric set, a K-64 pipelined
 * configuration, at least 3 hubs), else 0.  GA_ERR_INVALID for a NULL
 * argument. */
ga_status ga_evaluation_folded(ga_ctx *ctx, int32_t *folded);

/* Batches: several contexts advanced together, generation by generation (the
 * islands of every context run the steps of ga_step).  Split-bf16 contexts
 * whose hub count the tile configuration takes (p >= 3 for the default one)
 * are grouped: each step of their generation (operators, allocation, the
 * matrix-core product, cost assembly, selection, exact re-evaluation, island
 * decisions) is one launch over all of them, its grid the concatenation of
 * the contexts' own grids.  The six launches are captured once as a HIP graph
 * whose kernels read the composition from the batch's device table; it is
 * replayed for every composition that fits its grids and captured anew, with
 * room to grow, when one does not (at most 256 grouped contexts).  The grouped
 * generation then costs one graph launch.  Other contexts replay their own generation graph
 * on side streams beside the grouped launches.  tile_config must be a
 * pipelined configuration (see ga_tile_config_info).  Every context must use
 * the batch's (non-null) stream (ga_set_stream moves one there) and must not
 * be stepped on its own while it is in the batch.  ga_batch_set replaces the
 * batch's contexts without waiting for queued generations: the new job tables
 * are copied in stream order from pinned staging; it fails with
 * GA_ERR_INVALID for a NULL or repeated context or one on another stream, and
 * GA_ERR_STATE for a poisoned one.  ga_batch_step enqueues `generations`
 * generations and returns without waiting.  Results are those of stepping each
 * context alone.  A context's generation counter, best and state are read
 * with the usual per-context calls.  The batch does not own its contexts;
 * ga_batch_free waits for the batch's stream and frees only the batch. */
typedef struct ga_batch ga_batch;
ga_status ga_batch_create(void *hip_stream, int32_t tile_config, ga_batch **out);
ga_status ga_batch_set(ga_batch *batch, ga_ctx *const *ctxs, int32_t count);
ga_status ga_batch_step(ga_batch *batch, int32_t generations);
void ga_batch_free(ga_batch *batch);

const char *ga_status_str(ga_status s);
const char *ga_last_error(const ga_ctx *ctx);   /* also valid for ctx == NULL (last init error) */
void ga_free(ga_ctx *ctx);                        /* waits for queued work; NULL is a no-op */

#ifdef __cplusplus
}
#endif
#endif /* HUBGA_H */
