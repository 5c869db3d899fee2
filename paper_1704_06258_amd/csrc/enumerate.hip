// Exhaustive search of the nearest-hub solution space: every p-subset of the
// n nodes, in lexicographic order, evaluated with the context's kernels
// (allocation, batched product or plain evaluation, cost assembly), keeping
// the exact minimum.  The paper compares its GA with optimal solutions
// (Sec. 6.2, Tables 1 and 3); over hub sets with nearest-hub allocation
// (the space the GA searches, Sec. 4.1 and 5) that optimum is this argmin.
//
// Per chunk of at most S sets:
//   k_enum_unrank  rank -> hub set (lexicographic unranking, one lane per set);
//   evaluation     the context's own kernels, unchanged;
//   k_enum_screen  exact modes: chunk argmin merged into the running best;
//                  approximate modes: every set whose interval
//                  [f~(1 - e), f~(1 + e)] could hold the minimum (its lower
//                  end at most the smallest upper end and the running exact
//                  best) is listed, in ascending rank;
//   k_enum_exact   the listed sets re-evaluated in binary64, canonical order;
//   k_enum_merge   their exact argmin merged into the running best.
// Ties go to the lower rank: a set replaces the running best only when
// strictly cheaper, and within a chunk the lower rank wins.
#include "kernels.hpp"
#include "exact_dev.hpp"
#include "select_dev.hpp"

namespace hubga {

// The rank-th p-subset of {0..n-1} in lexicographic order (rank < C(n, p)).
// Position k takes the smallest c whose block of subsets -- those that
// continue the prefix with c, C(n-1-c, p-1-k) of them -- holds the rank.
// binom[m*(p+1) + j] = C(m, j), saturated at 2^63 (the rank is below 2^62).
__global__ __launch_bounds__(256) void k_enum_unrank(int64_t first, int count, int n, int p,
                                                     const uint64_t *__restrict__ binom, int32_t *__restrict__ hubs)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    uint64_t r = (uint64_t)(first + s);
    int32_t *out = hubs + (size_t)s * p;
    int c = 0;
    for (int k = 0; k < p; ++k) {
        const int j = p - 1 - k;
        while (c < n - 1 - j) {   // the last feasible value needs no test
            const uint64_t blk = binom[(size_t)(n - 1 - c) * (p + 1) + j];
            if (r < blk) break;
            r -= blk;
            ++c;
        }
        out[k] = c;
        ++c;
    }
}

__global__ void k_enum_init(EnumState *st)
{
    if (threadIdx.x == 0) {
        st->best_cost = __builtin_inf();
        for (int q = 0; q < 3; ++q) st->best_parts[q] = 0.0;
        st->best_rank = -1;
        st->rechecks = 0;
        st->cand_count = 0;
    }
}

// Running best <- set s of the chunk (cost, parts, hubs, rank) if strictly
// cheaper.  One workgroup; every lane calls it with the same arguments.
__device__ inline void enum_take(EnumState *st, int32_t *best_hubs, const int32_t *hubs, int p, int64_t first, int s,
                                 double v, const double *parts)
{
    const bool take = s >= 0 && v < st->best_cost;
    __syncthreads();
    if (take) {
        for (int k = threadIdx.x; k < p; k += blockDim.x) best_hubs[k] = hubs[(size_t)s * p + k];
        if (threadIdx.x == 0) {
            st->best_cost = v;
            for (int q = 0; q < 3; ++q) st->best_parts[q] = parts[q];
            st->best_rank = first + s;
        }
    }
    __syncthreads();
}

// One workgroup of 1024 lanes.
__global__ __launch_bounds__(1024) void k_enum_screen(const double *__restrict__ cost,
                                                      const double *__restrict__ eps,
                                                      const double *__restrict__ parts,
                                                      const int32_t *__restrict__ hubs, int count, int p,
                                                      int64_t first, int exact, EnumState *st,
                                                      int32_t *__restrict__ best_hubs, int32_t *__restrict__ cand)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    if (exact) {
        double v;
        const int s = block_argmin(count, [&](int i) { return cost[i]; }, &v);
        enum_take(st, best_hubs, hubs, p, first, s, v, parts + 3 * (size_t)(s < 0 ? 0 : s));
        if (tid == 0) st->cand_count = 0;
        return;
    }
    // smallest upper end, with the running exact best
    double ub_min;
    (void)block_argmin(count, [&](int i) { return cost[i] * (1.0 + (2.0 * eps[i] + 8.881784197001252e-16)); },
                       &ub_min);
    const double U = fmin(ub_min, st->best_cost);
    // list every set whose lower end is <= U, in ascending order
    __shared__ int wave_cnt[16];
    __shared__ int base;
    if (tid == 0) base = 0;
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, nw = nt >> 6;
    for (int i0 = 0; i0 < count; i0 += nt) {
        const int i = i0 + tid;
        bool c = false;
        if (i < count) c = cost[i] * (1.0 - (2.0 * eps[i] + 8.881784197001252e-16)) <= U;
        const unsigned long long m = __ballot(c);
        if (lane == 0) wave_cnt[wave] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += wave_cnt[w];
        if (c) cand[off + __popcll(m & ((1ull << lane) - 1ull))] = i;
        __syncthreads();
        if (tid == 0)
            for (int w = 0; w < nw; ++w) base += wave_cnt[w];
        __syncthreads();
    }
    if (tid == 0) {
        st->cand_count = base;
        st->rechecks += base;
    }
}

// Listed sets in binary64, canonical order: a fixed grid, each workgroup
// taking every gridDim.x-th entry of the list.
template <typename CT, typename WT>
__global__ __launch_bounds__(256) void k_enum_exact(const int32_t *__restrict__ hubs, const uint16_t *__restrict__ kidx,
                                                    const int32_t *__restrict__ cand, const EnumState *st, int n,
                                                    int n_pad, int p, const CT *__restrict__ C,
                                                    const double *__restrict__ Ctr, const WT *__restrict__ W,
                                                    const double *__restrict__ O,
                                                    const double *__restrict__ D, double chi, double alpha,
                                                    double delta, double scale, double *__restrict__ cand_cost,
                                                    double *__restrict__ cand_parts)
{
    extern __shared__ __align__(16) char smem[];
    const int cnt = st->cand_count;
    for (int c = blockIdx.x; c < cnt; c += gridDim.x) {
        const int s = cand[c];
        eval_exact_body<CT, WT>(hubs + (size_t)s * p, kidx + (size_t)s * n_pad, n, p, C, Ctr, W, O, D, chi, alpha,
                                delta, scale, cand_cost + c, cand_parts + 3 * (size_t)c, smem);
        __syncthreads();   // the LDS is reused by the next entry
    }
}

// Exact argmin of the listed sets (the list ascends in rank, so the lower
// entry of a tie is the lower rank) merged into the running best.
__global__ __launch_bounds__(256) void k_enum_merge(const int32_t *__restrict__ hubs, const int32_t *__restrict__ cand,
                                                    const double *__restrict__ cand_cost,
                                                    const double *__restrict__ cand_parts, int p, int64_t first,
                                                    EnumState *st, int32_t *__restrict__ best_hubs)
{
    const int cnt = st->cand_count;
    double v;
    const int c = block_argmin(cnt, [&](int i) { return cand_cost[i]; }, &v);
    enum_take(st, best_hubs, hubs, p, first, c < 0 ? -1 : cand[c], v, cand_parts + 3 * (size_t)(c < 0 ? 0 : c));
}

// ------------------------------------------------------------ launchers --

static constexpr int kEnumExactBlocks = 256;

template <typename CT, typename WT>
static hipError_t enum_exact_launch(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    k_enum_exact<CT, WT><<<kEnumExactBlocks, 256, exact_smem_bytes(d.n, d.p), st>>>(
        P.hubs, P.kidx, P.cand, P.enum_state, d.n, d.n_pad, d.p, (const CT *)P.C, P.Ctr, (const WT *)P.W, P.O, P.D,
        d.chi,
        d.alpha, d.delta, d.scale, P.cand_cost, P.cand_parts);
    return hipGetLastError();
}

hipError_t launch_enum_init(const DevPtrs &P, hipStream_t st)
{
    k_enum_init<<<1, 64, 0, st>>>(P.enum_state);
    return hipGetLastError();
}

hipError_t launch_enum_unrank(const DevPtrs &P, const Dims &d, int64_t first, int count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    k_enum_unrank<<<(count + 255) / 256, 256, 0, st>>>(first, count, d.n, d.p, P.binom, P.hubs);
    return hipGetLastError();
}

// Screening, exact re-evaluation of the listed sets and the merge, for a
// chunk of `count` evaluated sets of ranks [first, first + count).
hipError_t launch_enum_select(const DevPtrs &P, const Dims &d, int64_t first, int count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int exact = d.prec == kFP64;
    k_enum_screen<<<1, 1024, 0, st>>>(P.cost, P.eps, P.parts, P.hubs, count, d.p, first, exact, P.enum_state,
                                      P.enum_best, P.cand);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || exact) return e;
    if (d.c_f32 && d.w_f32) e = enum_exact_launch<float, float>(P, d, st);
    else if (d.c_f32) e = enum_exact_launch<float, double>(P, d, st);
    else if (d.w_f32) e = enum_exact_launch<double, float>(P, d, st);
    else e = enum_exact_launch<double, double>(P, d, st);
    if (e != hipSuccess) return e;
    k_enum_merge<<<1, 256, 0, st>>>(P.hubs, P.cand, P.cand_cost, P.cand_parts, d.p, first, P.enum_state, P.enum_best);
    return hipGetLastError();
}

hipError_t prepare_enum_kernels(int max_lds)
{
    const void *fns[] = {(const void *)k_enum_exact<double, double>, (const void *)k_enum_exact<double, float>,
                         (const void *)k_enum_exact<float, double>, (const void *)k_enum_exact<float, float>};
    for (const void *f : fns) {
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, f);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds - (int)fa.sharedSizeBytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hubga
