// Per-individual fitness evaluation, one workgroup per individual (the
// "plain" kernels; Eval of Sec. 4.3 and Sec. 5, objective (1) of Sec. 3).
//
// k_eval_exact: binary64 in the canonical order, bit-identical to a
//   sequential evaluation: lane j accumulates t_j = sum_i W_ij*C[a_i][a_j]
//   over ascending i (coalesced W rows), then T, Cc and Dd are summed in
//   ascending order by one lane from LDS; no FMA contraction anywhere.
//   Also used to re-evaluate selection candidates exactly.
// k_eval_fp32: FP32 per-column sums with FMA, FP64 tree reduction of the
//   columns; Cc and Dd come from the allocation kernel.  Returns a rigorous
//   relative error bound with every cost.
#include "kernels.hpp"
#include "select_dev.hpp"

#include <algorithm>

namespace hubga {

// LDS carve-up of the exact kernel: Ch (p*p doubles), buf (n doubles),
// kid (n uint16), h (p ints).
__host__ __device__ inline size_t exact_smem_bytes(int n, int p)
{
    return (size_t)p * p * 8 + (size_t)n * 8 + (((size_t)n * 2 + 15) / 16) * 16 + (size_t)kMaxP * 4;
}

// Sequential ascending sum of buf[0..n) by the calling lane.
__device__ inline double seq_sum(const double *buf, int n)
{
#pragma clang fp contract(off)
    double acc = 0.0;
    int i = 0;
    for (; i + 4 <= n; i += 4) {
        double a = buf[i], b = buf[i + 1], c = buf[i + 2], d = buf[i + 3];
        acc = acc + a;
        acc = acc + b;
        acc = acc + c;
        acc = acc + d;
    }
    for (; i < n; ++i) acc = acc + buf[i];
    return acc;
}

template <typename CT, typename WT>
__device__ void eval_exact_body(const int32_t *__restrict__ hg, const uint16_t *__restrict__ krow, int n, int p,
                                const CT *__restrict__ C, const WT *__restrict__ W, const double *__restrict__ O,
                                const double *__restrict__ D, double chi, double alpha, double delta, double scale,
                                double *cost_out, double *parts_out, char *smem)
{
#pragma clang fp contract(off)
    double *Ch = (double *)smem;
    double *buf = Ch + (size_t)p * p;
    uint16_t *kid = (uint16_t *)(buf + n);
    int *h = (int *)(smem + exact_smem_bytes(n, p) - (size_t)kMaxP * 4);
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid < p) h[tid] = hg[tid];
    for (int i = tid; i < n; i += nt) kid[i] = krow[i];
    __syncthreads();
    for (int e = tid; e < p * p; e += nt) Ch[e] = (double)C[(size_t)h[e / p] * n + h[e % p]];
    __syncthreads();
    // t_j = sum over ascending i of W_ij * C[a_i][a_j], four columns per lane at a time
    for (int j0 = tid; j0 < n; j0 += 4 * nt) {
        int js[4], kj[4];
        double acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            js[q] = j0 + q * nt;
            kj[q] = js[q] < n ? kid[js[q]] : 0;
            acc[q] = 0.0;
        }
        // rows in groups of 8: 32 loads in flight per lane, then the adds in
        // ascending row order (absent columns read 0 and are discarded)
        int jc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) jc[q] = js[q] < n ? js[q] : 0;
        int i = 0;
        for (; i + 8 <= n; i += 8) {
            double w[8][4];
            int ki[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const WT *wr = W + (size_t)(i + u) * n;
                ki[u] = kid[i + u];
#pragma unroll
                for (int q = 0; q < 4; ++q) w[u][q] = (double)wr[jc[q]];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double *chr = Ch + (size_t)ki[u] * p;
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = acc[q] + w[u][q] * chr[kj[q]];
            }
        }
        for (; i < n; ++i) {
            const WT *wr = W + (size_t)i * n;
            const double *chr = Ch + (size_t)kid[i] * p;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = acc[q] + (double)wr[jc[q]] * chr[kj[q]];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (js[q] < n) buf[js[q]] = acc[q];
    }
    __syncthreads();
    double T = 0.0, Cc = 0.0, Dd = 0.0;
    if (tid == 0) T = seq_sum(buf, n);
    __syncthreads();
    for (int i = tid; i < n; i += nt) buf[i] = O[i] * (double)C[(size_t)i * n + h[kid[i]]];
    __syncthreads();
    if (tid == 0) Cc = seq_sum(buf, n);
    __syncthreads();
    for (int i = tid; i < n; i += nt) buf[i] = D[i] * (double)C[(size_t)i * n + h[kid[i]]];
    __syncthreads();
    if (tid == 0) {
        Dd = seq_sum(buf, n);
        double f = ((chi * Cc) + (alpha * T)) + (delta * Dd);
        *cost_out = f * scale;
        if (parts_out) {
            parts_out[0] = Cc;
            parts_out[1] = T;
            parts_out[2] = Dd;
        }
    }
}

template <typename CT, typename WT>
__global__ __launch_bounds__(256) void k_eval_exact(const int32_t *__restrict__ hubs,
                                                    const uint16_t *__restrict__ kidx, int count, int n, int n_pad,
                                                    int p, const CT *__restrict__ C, const WT *__restrict__ W,
                                                    const double *__restrict__ O, const double *__restrict__ D,
                                                    double chi, double alpha, double delta, double scale,
                                                    double *__restrict__ cost, double *__restrict__ parts,
                                                    double *__restrict__ eps)
{
    extern __shared__ __align__(16) char smem[];
    const int s = blockIdx.x;
    if (s >= count) return;
    eval_exact_body<CT, WT>(hubs + (size_t)s * p, kidx + (size_t)s * n_pad, n, p, C, W, O, D, chi, alpha, delta,
                            scale, cost + s, parts + 3 * (size_t)s, smem);
    if (threadIdx.x == 0 && eps) eps[s] = 0.0;
}

// Column-parallel exact evaluation of selection candidates.
//
// The last workgroup of the selection kernel lists candidate slots in island
// order, up to `tot` in all; the rest form an extra list.
//
// k_canon_cols loops over (slot, 32-column chunk) items: 128-row tiles of W
// are staged through LDS (loads issued two tiles ahead), every lane of the
// workgroup forms products W_ij * C[a_i][a_j] for the tile -- the same binary64
// products as the sequential definition -- and one lane per column adds them
// in ascending row order into t_j.  k_canon_sums then sums T, Cc and Dd in
// ascending order and evaluates the extra candidates whole (one workgroup
// each); k_select2 decides every island on exact costs.
constexpr int kCanonCols = 32;
constexpr int kCanonRows = 128;

__host__ __device__ inline size_t canon_cols_smem(int n, int p)
{
    return (size_t)p * p * 8 + (size_t)kCanonRows * kCanonCols * 8 + (((size_t)n * 2 + 15) / 16) * 16;
}

// One item (candidate slot, 32-column chunk) of the column sums (LDS:
// canon_cols_smem); every lane of the workgroup takes part.
template <typename CT, typename WT>
__device__ __forceinline__ void canon_cols_item(const int32_t *__restrict__ hubs, const uint16_t *__restrict__ kidx,
                                                const int32_t *__restrict__ cand, const int32_t *__restrict__ slot_r,
                                                const int32_t *__restrict__ slot_c, int m, int n, int n_pad, int p,
                                                const CT *__restrict__ C, const WT *__restrict__ W,
                                                double *__restrict__ tbuf, char *smem, int item)
{
#pragma clang fp contract(off)
    double *Ch = (double *)smem;
    double *tile = Ch + (size_t)p * p;                        // products [row][col]
    uint16_t *kid = (uint16_t *)(tile + kCanonRows * kCanonCols);
    __shared__ int h[kMaxP];
    const int tid = threadIdx.x;
    const int nchunks = (n + kCanonCols - 1) / kCanonCols;
    constexpr int PER = kCanonRows * kCanonCols / 256;   // tile elements per thread
    const int nb = (n + kCanonRows - 1) / kCanonRows;
    const int slot = item / nchunks, chunk = item % nchunks;
    const int r = slot_r[slot], c = slot_c[slot];
    const int s = cand[(size_t)r * m + c];
    const int j0 = chunk * kCanonCols;
    const int32_t *hg = hubs + (size_t)s * p;
    __syncthreads();   // previous item done with LDS
    if (tid < p) h[tid] = hg[tid];
    const uint16_t *krow = kidx + (size_t)s * n_pad;
    for (int i = tid; i < n; i += 256) kid[i] = krow[i];
    __syncthreads();
    for (int e = tid; e < p * p; e += 256) Ch[e] = (double)C[(size_t)h[e / p] * n + h[e % p]];
    // this thread's tile elements: column e % 32 (fixed), rows e / 32
    const int col = tid % kCanonCols, j = j0 + col;
    const bool jin = j < n;
    WT reg0[PER], reg1[PER];
    auto load = [&](int b, WT *dst) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = b * kCanonRows + (tid + q * 256) / kCanonCols;
            dst[q] = (i < n && jin) ? W[(size_t)i * n + j] : (WT)0;
        }
    };
    const bool owner = tid < kCanonCols && jin;
    double acc = 0.0;
    load(0, reg0);
    if (nb > 1) load(1, reg1);
    __syncthreads();   // Ch and kid ready
    const int kj = jin ? kid[j] : 0;
    auto step = [&](int b, WT *rg) {
        const int i0 = b * kCanonRows;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * 256, i = i0 + e / kCanonCols;
            tile[e] = i < n ? (double)rg[q] * Ch[(size_t)kid[i] * p + kj] : 0.0;
        }
        __syncthreads();
        if (b + 2 < nb) load(b + 2, rg);
        if (owner) {
            const int rows = n - i0 < kCanonRows ? n - i0 : kCanonRows;
            if (rows == kCanonRows) {
                // reads of the next 16 rows in flight while the current 16 are added
                double cur[16], nxt[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) cur[u] = tile[u * kCanonCols + tid];
#pragma unroll
                for (int c = 0; c < kCanonRows / 16; ++c) {
                    if (c + 1 < kCanonRows / 16) {
#pragma unroll
                        for (int u = 0; u < 16; ++u) nxt[u] = tile[((c + 1) * 16 + u) * kCanonCols + tid];
                    }
#pragma unroll
                    for (int u = 0; u < 16; ++u) acc = acc + cur[u];
#pragma unroll
                    for (int u = 0; u < 16; ++u) cur[u] = nxt[u];
                }
            } else {
                for (int ii = 0; ii < rows; ++ii) acc = acc + tile[ii * kCanonCols + tid];
            }
        }
        __syncthreads();
    };
    for (int b = 0; b < nb; b += 2) {
        step(b, reg0);
        if (b + 1 < nb) step(b + 1, reg1);
    }
    if (owner) tbuf[(size_t)slot * n + j] = acc;
}

__host__ __device__ inline int canon_cols_chunks(int n) { return (n + kCanonCols - 1) / kCanonCols; }

// Workgroup blk of nblk persistent ones of a context (LDS: canon_cols_smem).
template <typename CT, typename WT>
__device__ __forceinline__ void canon_cols_body(const int32_t *__restrict__ hubs, const uint16_t *__restrict__ kidx,
                                                const int32_t *__restrict__ cand, const int32_t *__restrict__ slot_r,
                                                const int32_t *__restrict__ slot_c,
                                                const int32_t *__restrict__ total, int m, int n, int n_pad, int p,
                                                const CT *__restrict__ C, const WT *__restrict__ W,
                                                double *__restrict__ tbuf, char *smem, int blk, int nblk)
{
    const int items = *total * canon_cols_chunks(n);
    for (int item = blk; item < items; item += nblk)
        canon_cols_item<CT, WT>(hubs, kidx, cand, slot_r, slot_c, m, n, n_pad, p, C, W, tbuf, smem, item);
}

// LDS of the candidate sums: three n-vectors when they fit (T, Cc and Dd are
// then summed by three lanes at once), else two (Dd after T and Cc).
__host__ __device__ inline bool sums_three(int n) { return (size_t)24 * n <= 96 * 1024; }
__host__ __device__ inline size_t canon_sums_smem(int n, int p)
{
    const size_t vec = (size_t)(sums_three(n) ? 24 : 16) * n;
    const size_t ex = exact_smem_bytes(n, p);
    return vec > ex ? vec : ex;
}

// One item of the candidate sums (LDS: canon_sums_smem): item < total is a
// slot with its column sums in tbuf, the others are extra candidates
// evaluated whole.
template <typename CT, typename WT>
__device__ __forceinline__ void canon_sums_item(const SelState &S, const int32_t *__restrict__ kidx,
                                                const int32_t *__restrict__ slot_r, const int32_t *__restrict__ slot_c,
                                                int tot, const int32_t *__restrict__ extra_r,
                                                const int32_t *__restrict__ extra_c, int n, int n_pad,
                                                const CT *__restrict__ C, const WT *__restrict__ W,
                                                const double *__restrict__ O, const double *__restrict__ D,
                                                const double *__restrict__ tbuf, double chi, double alpha,
                                                double delta, double scale, double *__restrict__ cand_cost,
                                                double *__restrict__ cand_parts, char *smem, int item)
{
#pragma clang fp contract(off)
    double *bufA = (double *)smem, *bufB = bufA + n;
    __shared__ int h[kMaxP];
    __shared__ double sh_cc, sh_dd;
    const int tid = threadIdx.x;
    const int p = S.p, m = S.m;
    const uint16_t *kid16 = (const uint16_t *)kidx;
    if (item < tot) {
        const int slot = item;
        const int r = slot_r[slot], c = slot_c[slot];
        const int s = S.cand[(size_t)r * m + c];
        __syncthreads();
        if (tid < p) h[tid] = S.children[(size_t)s * p + tid];
        const uint16_t *krow = kid16 + (size_t)s * n_pad;
        const double *t = tbuf + (size_t)slot * n;
        __syncthreads();
        const bool three = sums_three(n);
        double *bufC = three ? bufB + n : bufA;
        for (int i = tid; i < n; i += 256) {
            const double ci = (double)C[(size_t)i * n + h[krow[i]]];
            bufA[i] = t[i];
            bufB[i] = O[i] * ci;
            if (three) bufC[i] = D[i] * ci;
        }
        __syncthreads();
        double T = 0.0, Dd = 0.0;
        if (tid == 0) T = seq_sum(bufA, n);   // three chains in three waves
        if (tid == 64) sh_cc = seq_sum(bufB, n);
        if (three && tid == 128) sh_dd = seq_sum(bufC, n);
        __syncthreads();
        if (!three) {
            for (int i = tid; i < n; i += 256) bufA[i] = D[i] * (double)C[(size_t)i * n + h[krow[i]]];
            __syncthreads();
            if (tid == 0) Dd = seq_sum(bufA, n);
        } else {
            Dd = sh_dd;
        }
        if (tid == 0) {
            const double Cc = sh_cc;
            const size_t o = (size_t)r * m + c;
            cand_cost[o] = (((chi * Cc) + (alpha * T)) + (delta * Dd)) * scale;
            cand_parts[3 * o + 0] = Cc;
            cand_parts[3 * o + 1] = T;
            cand_parts[3 * o + 2] = Dd;
        }
    } else {   // a candidate beyond the slots: evaluated whole
        const int e = item - tot;
        const int r = extra_r[e], c = extra_c[e];
        const int s = S.cand[(size_t)r * m + c];
        __syncthreads();
        const size_t o = (size_t)r * m + c;
        eval_exact_body<CT, WT>(S.children + (size_t)s * p, kid16 + (size_t)s * n_pad, n, p, C, W, O, D, chi,
                                alpha, delta, scale, cand_cost + o, cand_parts + 3 * o, smem);
    }
}

// Workgroup blk of nblk of a context (LDS: canon_sums_smem).
template <typename CT, typename WT>
__device__ __forceinline__ void canon_sums_body(const SelState &S, const int32_t *__restrict__ kidx,
                                                const int32_t *__restrict__ slot_r, const int32_t *__restrict__ slot_c,
                                                const int32_t *__restrict__ total,
                                                const int32_t *__restrict__ extra_r,
                                                const int32_t *__restrict__ extra_c,
                                                const int32_t *__restrict__ nextra, int n, int n_pad,
                                                const CT *__restrict__ C, const WT *__restrict__ W,
                                                const double *__restrict__ O, const double *__restrict__ D,
                                                const double *__restrict__ tbuf, double chi, double alpha,
                                                double delta, double scale, double *__restrict__ cand_cost,
                                                double *__restrict__ cand_parts, char *smem, int blk, int nblk)
{
    const int tot = *total, items = tot + *nextra;
    for (int item = blk; item < items; item += nblk)
        canon_sums_item<CT, WT>(S, kidx, slot_r, slot_c, tot, extra_r, extra_c, n, n_pad, C, W, O, D, tbuf, chi,
                                alpha, delta, scale, cand_cost, cand_parts, smem, item);
}

// Island decisions on exact costs, one workgroup per island; the last
// workgroup ends the generation (global step, best so far, g + 1).
__device__ __forceinline__ void select2_body(const SelState &S, int *__restrict__ sync, int blk, int nblk)
{
    select_island_exact(S, blk);
    if (!last_block(sync, nblk)) return;
    global_step(S);
}

template <typename CT, typename WT>
__global__ __launch_bounds__(256) void k_canon_cols(const int32_t *__restrict__ hubs,
                                                    const uint16_t *__restrict__ kidx,
                                                    const int32_t *__restrict__ cand, const int32_t *__restrict__ slot_r,
                                                    const int32_t *__restrict__ slot_c,
                                                    const int32_t *__restrict__ total, int m, int n, int n_pad, int p,
                                                    const CT *__restrict__ C, const WT *__restrict__ W,
                                                    double *__restrict__ tbuf)
{
    extern __shared__ __align__(16) char smem[];
    canon_cols_body<CT, WT>(hubs, kidx, cand, slot_r, slot_c, total, m, n, n_pad, p, C, W, tbuf, smem, blockIdx.x,
                            gridDim.x);
}

template <typename CT, typename WT>
__global__ __launch_bounds__(256) void k_canon_sums(SelState S, const int32_t *__restrict__ kidx,
                                                    const int32_t *__restrict__ slot_r,
                                                    const int32_t *__restrict__ slot_c,
                                                    const int32_t *__restrict__ total,
                                                    const int32_t *__restrict__ extra_r,
                                                    const int32_t *__restrict__ extra_c,
                                                    const int32_t *__restrict__ nextra, int n, int n_pad,
                                                    const CT *__restrict__ C, const WT *__restrict__ W,
                                                    const double *__restrict__ O, const double *__restrict__ D,
                                                    const double *__restrict__ tbuf, double chi, double alpha,
                                                    double delta, double scale, double *__restrict__ cand_cost,
                                                    double *__restrict__ cand_parts)
{
    extern __shared__ __align__(16) char smem[];
    canon_sums_body<CT, WT>(S, kidx, slot_r, slot_c, total, extra_r, extra_c, nextra, n, n_pad, C, W, O, D, tbuf,
                            chi, alpha, delta, scale, cand_cost, cand_parts, smem, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_select2(SelState S, int *__restrict__ sync)
{
    select2_body(S, sync, blockIdx.x, gridDim.x);
}

// Grouped re-evaluation and decisions (split-bf16 generations of several
// contexts).  The column sums and candidate sums draw from one pool: the
// items of all contexts, concatenated in context order, shared by every
// workgroup of the launch, so a context with many candidates does not wait on
// a fixed share of workgroups.

// Exclusive prefix of one count per context (njobs <= kMaxPoolJobs, block of
// 256 lanes): pre[j] = items of contexts before j, pre[njobs] = all items.
template <typename F>
__device__ inline int pool_prefix(int njobs, F count, int *pre)
{
    const int tid = threadIdx.x;
    int v = tid < njobs ? count(tid) : 0;
    pre[tid + 1] = v;
    if (tid == 0) pre[0] = 0;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {   // inclusive scan of pre[1..256]
        const int add = tid >= off ? pre[tid + 1 - off] : 0;
        __syncthreads();
        pre[tid + 1] += add;
        __syncthreads();
    }
    return pre[njobs];
}

__device__ inline int pool_job(const int *pre, int njobs, int g)   // last j with pre[j] <= g
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename CT, typename WT>
__device__ __forceinline__ void cols_item(const TickJob &J, char *smem, int item)
{
    const DevPtrs &P = J.P;
    const Dims &d = J.d;
    canon_cols_item<CT, WT>(P.hubs, P.kidx, P.cand, P.slot_r, P.slot_c, d.m, d.n, d.n_pad, d.p, (const CT *)P.C,
                            (const WT *)P.W, P.tbuf, smem, item);
}

__global__ __launch_bounds__(256) void k_canon_cols_group(const TickJob *__restrict__ jobs, int njobs)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int pre[kMaxPoolJobs + 1];
    const int items =
        pool_prefix(njobs, [&](int j) { return *jobs[j].P.total * canon_cols_chunks(jobs[j].d.n); }, pre);
    for (int g = blockIdx.x; g < items; g += gridDim.x) {
        const int j = pool_job(pre, njobs, g);
        const TickJob &J = jobs[j];
        const int item = g - pre[j];
        if (J.d.c_f32) {
            if (J.d.w_f32) cols_item<float, float>(J, smem, item);
            else cols_item<float, double>(J, smem, item);
        } else {
            if (J.d.w_f32) cols_item<double, float>(J, smem, item);
            else cols_item<double, double>(J, smem, item);
        }
    }
}

template <typename CT, typename WT>
__device__ __forceinline__ void sums_item(const TickJob &J, char *smem, int tot, int item)
{
    const DevPtrs &P = J.P;
    const Dims &d = J.d;
    const SelState S = make_sel_state(P, d);
    canon_sums_item<CT, WT>(S, (const int32_t *)P.kidx, P.slot_r, P.slot_c, tot, P.extra_r, P.extra_c, d.n, d.n_pad,
                            (const CT *)P.C, (const WT *)P.W, P.O, P.D, P.tbuf, d.chi, d.alpha, d.delta, d.scale,
                            P.cand_cost, P.cand_parts, smem, item);
}

__global__ __launch_bounds__(256) void k_canon_sums_group(const TickJob *__restrict__ jobs, int njobs)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int pre[kMaxPoolJobs + 1];
    const int items = pool_prefix(njobs, [&](int j) { return *jobs[j].P.total + *jobs[j].P.nextra; }, pre);
    for (int g = blockIdx.x; g < items; g += gridDim.x) {
        const int j = pool_job(pre, njobs, g);
        const TickJob &J = jobs[j];
        const int item = g - pre[j], tot = *J.P.total;
        if (J.d.c_f32) {
            if (J.d.w_f32) sums_item<float, float>(J, smem, tot, item);
            else sums_item<float, double>(J, smem, tot, item);
        } else {
            if (J.d.w_f32) sums_item<double, float>(J, smem, tot, item);
            else sums_item<double, double>(J, smem, tot, item);
        }
    }
}

__global__ __launch_bounds__(256) void k_select2_group(const TickJob *__restrict__ jobs, int njobs)
{
    const TickJob &J = jobs[tick_job(jobs, njobs, kTickSel2, blockIdx.x)];
    const SelState S = make_sel_state(J.P, J.d);
    select2_body(S, J.P.sync + 1, blockIdx.x - J.start[kTickSel2], J.blocks[kTickSel2]);
}

// ------------------------------------------------------------- FP32 --

template <typename CT>
__global__ __launch_bounds__(256) void k_eval_fp32(const int32_t *__restrict__ hubs, const uint16_t *__restrict__ kidx,
                                                   int count, int n, int n_pad, int p, const CT *__restrict__ Ct,
                                                   const float *__restrict__ W, double chi, double alpha,
                                                   double delta, double scale, double eps_bound,
                                                   double *__restrict__ cost, double *__restrict__ parts,
                                                   double *__restrict__ eps)
{
#pragma clang fp contract(off)
    extern __shared__ __align__(16) char smem[];
    float *Ch = (float *)smem;                            // p*p
    uint16_t *kid = (uint16_t *)(Ch + (size_t)kMaxP * kMaxP);   // n
    __shared__ double red[256];
    __shared__ int h[kMaxP];
    const int s = blockIdx.x;
    if (s >= count) return;
    const int tid = threadIdx.x, nt = blockDim.x;
    const uint16_t *krow = kidx + (size_t)s * n_pad;
    if (tid < p) h[tid] = hubs[(size_t)s * p + tid];
    for (int i = tid; i < n; i += nt) kid[i] = krow[i];
    __syncthreads();
    for (int e = tid; e < p * p; e += nt) Ch[e] = (float)Ct[(size_t)h[e % p] * n + h[e / p]];
    __syncthreads();
    double tsum = 0.0;
    for (int j0 = tid; j0 < n; j0 += 4 * nt) {
        int js[4], kj[4];
        float acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            js[q] = j0 + q * nt;
            kj[q] = js[q] < n ? kid[js[q]] : 0;
            acc[q] = 0.0f;
        }
        const bool full = js[3] < n;
        for (int i = 0; i < n; ++i) {
            const float *wr = W + (size_t)i * n;
            const float *chr = Ch + (size_t)kid[i] * p;
            if (full) {
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = __builtin_fmaf(wr[js[q]], chr[kj[q]], acc[q]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (js[q] < n) acc[q] = __builtin_fmaf(wr[js[q]], chr[kj[q]], acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (js[q] < n) tsum = tsum + (double)acc[q];
    }
    red[tid] = tsum;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] = red[tid] + red[tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        double T = red[0];
        double Cc = parts[3 * (size_t)s], Dd = parts[3 * (size_t)s + 2];
        parts[3 * (size_t)s + 1] = T;
        cost[s] = (((chi * Cc) + (alpha * T)) + (delta * Dd)) * scale;
        if (eps) eps[s] = eps_bound;
    }
}

// ------------------------------------------------------------ launchers --

static int eval_block(int n) { return n >= 512 ? 256 : (n >= 128 ? 128 : 64); }

template <typename CT, typename WT>
static hipError_t exact_launch(const DevPtrs &P, const Dims &d, const int32_t *hubs, const uint16_t *kidx, int count,
                               double *cost, double *parts, double *eps, hipStream_t st)
{
    size_t sm = exact_smem_bytes(d.n, d.p);
    k_eval_exact<CT, WT><<<count, eval_block(d.n), sm, st>>>(hubs, kidx, count, d.n, d.n_pad, d.p, (const CT *)P.C,
                                                             (const WT *)P.W, P.O, P.D, d.chi, d.alpha, d.delta,
                                                             d.scale, cost, parts, eps);
    return hipGetLastError();
}

hipError_t launch_eval_exact(const DevPtrs &P, const Dims &d, const int32_t *hubs, const uint16_t *kidx, int count,
                             double *cost, double *parts, double *eps, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (d.c_f32 && d.w_f32) return exact_launch<float, float>(P, d, hubs, kidx, count, cost, parts, eps, st);
    if (d.c_f32) return exact_launch<float, double>(P, d, hubs, kidx, count, cost, parts, eps, st);
    if (d.w_f32) return exact_launch<double, float>(P, d, hubs, kidx, count, cost, parts, eps, st);
    return exact_launch<double, double>(P, d, hubs, kidx, count, cost, parts, eps, st);
}

template <typename CT, typename WT>
static hipError_t recheck_launch(const DevPtrs &P, const Dims &d, const SelState &S, hipStream_t st)
{
    hipError_t e;
    const size_t smA = canon_cols_smem(d.n, d.p);
    k_canon_cols<CT, WT><<<512, 256, smA, st>>>(P.hubs, P.kidx, P.cand, P.slot_r, P.slot_c, P.total, d.m, d.n,
                                                d.n_pad, d.p, (const CT *)P.C, (const WT *)P.W, P.tbuf);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t smB = canon_sums_smem(d.n, d.p);
    k_canon_sums<CT, WT><<<256, 256, smB, st>>>(S, (const int32_t *)P.kidx, P.slot_r, P.slot_c, P.total, P.extra_r,
                                                P.extra_c, P.nextra, d.n, d.n_pad, (const CT *)P.C, (const WT *)P.W,
                                                P.O, P.D, P.tbuf, d.chi, d.alpha, d.delta, d.scale, P.cand_cost,
                                                P.cand_parts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_select2<<<d.R, 256, 0, st>>>(S, P.sync + 1);
    return hipGetLastError();
}

hipError_t launch_recheck(const DevPtrs &P, const Dims &d, const SelState &S, hipStream_t st)
{
    if (d.c_f32 && d.w_f32) return recheck_launch<float, float>(P, d, S, st);
    if (d.c_f32) return recheck_launch<float, double>(P, d, S, st);
    if (d.w_f32) return recheck_launch<double, float>(P, d, S, st);
    return recheck_launch<double, double>(P, d, S, st);
}

// The exact cost of the single solution in best (P0 of Sec. 4.1), column
// parallel: one workgroup per 32-column chunk, then the sums in one workgroup;
// the result is the sequential definition, bit for bit.  cand, slot_r and
// slot_c are unused before the first generation; their first entries become
// the one-slot index of best.
__global__ void k_p0_index(int32_t *__restrict__ cand, int32_t *__restrict__ slot_r, int32_t *__restrict__ slot_c)
{
    if (threadIdx.x == 0) cand[0] = slot_r[0] = slot_c[0] = 0;
}

template <typename CT, typename WT>
__global__ __launch_bounds__(256) void k_p0_cols(DevPtrs P, Dims d)
{
    extern __shared__ __align__(16) char smem[];
    canon_cols_item<CT, WT>(P.best, P.kidx_one, P.cand, P.slot_r, P.slot_c, 1, d.n, d.n_pad, d.p, (const CT *)P.C,
                            (const WT *)P.W, P.tbuf, smem, blockIdx.x);
}

template <typename CT, typename WT>
__global__ __launch_bounds__(256) void k_p0_sums(DevPtrs P, Dims d)
{
    extern __shared__ __align__(16) char smem[];
    SelState S = make_sel_state(P, d);
    S.children = P.best;
    S.m = 1;
    canon_sums_item<CT, WT>(S, (const int32_t *)P.kidx_one, P.slot_r, P.slot_c, 1, P.extra_r, P.extra_c, d.n, d.n_pad,
                            (const CT *)P.C, (const WT *)P.W, P.O, P.D, P.tbuf, d.chi, d.alpha, d.delta, d.scale,
                            P.best_cost, P.best_cost + 1, smem, 0);
}

template <typename CT, typename WT>
static hipError_t p0_launch(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    hipError_t e;
    k_p0_index<<<1, 64, 0, st>>>(P.cand, P.slot_r, P.slot_c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_p0_cols<CT, WT><<<canon_cols_chunks(d.n), 256, canon_cols_smem(d.n, d.p), st>>>(P, d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_p0_sums<CT, WT><<<1, 256, canon_sums_smem(d.n, d.p), st>>>(P, d);
    return hipGetLastError();
}

hipError_t launch_p0_exact(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    if (d.c_f32 && d.w_f32) return p0_launch<float, float>(P, d, st);
    if (d.c_f32) return p0_launch<float, double>(P, d, st);
    if (d.w_f32) return p0_launch<double, float>(P, d, st);
    return p0_launch<double, double>(P, d, st);
}

size_t recheck_lds_cols(int n, int p) { return canon_cols_smem(n, p); }
size_t recheck_lds_sums(int n, int p) { return canon_sums_smem(n, p); }

hipError_t launch_recheck_group(const TickJob *jobs, int njobs, const int *blocks, size_t lds_cols, size_t lds_sums,
                                hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    hipError_t e;
    if (njobs > kMaxPoolJobs) return hipErrorInvalidValue;
    k_canon_cols_group<<<kPoolColsBlocks, 256, lds_cols, st>>>(jobs, njobs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_canon_sums_group<<<kPoolSumsBlocks, 256, lds_sums, st>>>(jobs, njobs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_select2_group<<<blocks[kTickSel2], 256, 0, st>>>(jobs, njobs);
    return hipGetLastError();
}

double fp32_eps_bound(int n)
{
    return gamma_k(n + 2.0, kU32) + gamma_k(2.0 * n + 16.0, kU64);
}

hipError_t launch_eval_fp32(const DevPtrs &P, const Dims &d, const int32_t *hubs, const uint16_t *kidx, int count,
                            hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const float *W = d.w_f32 ? (const float *)P.W : P.W32;
    size_t sm = (size_t)kMaxP * kMaxP * 4 + (size_t)d.n * 2 + 16;
    double eb = fp32_eps_bound(d.n);
    if (d.c_f32) {
        k_eval_fp32<float><<<count, eval_block(d.n), sm, st>>>(hubs, kidx, count, d.n, d.n_pad, d.p,
                                                                (const float *)P.Ct, W, d.chi, d.alpha, d.delta,
                                                                d.scale, eb, P.cost, P.parts, P.eps);
    } else {
        k_eval_fp32<double><<<count, eval_block(d.n), sm, st>>>(hubs, kidx, count, d.n, d.n_pad, d.p,
                                                                 (const double *)P.Ct, W, d.chi, d.alpha, d.delta,
                                                                 d.scale, eb, P.cost, P.parts, P.eps);
    }
    return hipGetLastError();
}

// Raise the dynamic-LDS cap of every kernel here that may need more than the
// default, once per process (never during graph capture).
static size_t g_group_lds_cap[2] = {0, 0};   // dynamic LDS limits of the grouped re-evaluation kernels

size_t recheck_group_lds_cap(int which) { return g_group_lds_cap[which ? 1 : 0]; }

hipError_t prepare_plain_kernels(int max_lds)
{
    const void *fns[] = {(const void *)k_eval_exact<double, double>, (const void *)k_eval_exact<double, float>,
                         (const void *)k_eval_exact<float, double>,  (const void *)k_eval_exact<float, float>,
                         (const void *)k_canon_cols<double, double>, (const void *)k_canon_cols<double, float>,
                         (const void *)k_canon_cols<float, double>,  (const void *)k_canon_cols<float, float>,
                         (const void *)k_canon_sums<double, double>, (const void *)k_canon_sums<double, float>,
                         (const void *)k_canon_sums<float, double>,  (const void *)k_canon_sums<float, float>,
                         (const void *)k_eval_fp32<double>,          (const void *)k_eval_fp32<float>,
                         (const void *)k_canon_cols_group,           (const void *)k_canon_sums_group,
                         (const void *)k_p0_cols<double, double>,    (const void *)k_p0_cols<double, float>,
                         (const void *)k_p0_cols<float, double>,     (const void *)k_p0_cols<float, float>,
                         (const void *)k_p0_sums<double, double>,    (const void *)k_p0_sums<double, float>,
                         (const void *)k_p0_sums<float, double>,     (const void *)k_p0_sums<float, float>};
    for (const void *f : fns) {
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, f);
        if (e != hipSuccess) return e;
        const int dyn = max_lds - (int)fa.sharedSizeBytes;   // the cap excludes the kernel's static LDS
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        if (e != hipSuccess) return e;
        if (f == (const void *)k_canon_cols_group) g_group_lds_cap[0] = (size_t)dyn;
        if (f == (const void *)k_canon_sums_group) g_group_lds_cap[1] = (size_t)dyn;
    }
    return hipSuccess;
}

}  // namespace hubga
