// Selection (Sec. 5): each island's best child (argmin, ties to the lowest
// child index) replaces the island ancestor -- only when strictly better in
// elitist mode -- and every n1 generations the best ancestor (ties to the
// lowest island) replaces all ancestors.  Ancestor costs are always exact.
//
// With approximate costs f~ (FP32 or split-bf16) every child carries a
// rigorous bound |f~ - f| <= eps f, hence f in [lb, ub] = f~(1 -+ eps').
// Stage 1 keeps as candidates the children whose interval could hold the
// island minimum (lb <= min ub) and could beat the ancestor (lb < f_anc);
// their exact costs are recomputed (k_recheck) and the
// decision is taken on exact values, so it is the one exact arithmetic takes.
// The last workgroup of k_select1 lists the candidates for re-evaluation (or,
// with exact costs, ends the generation).
#include "kernels.hpp"
#include "select_dev.hpp"

namespace hubga {

// Candidate slots for the column-parallel re-evaluation, in island order, up
// to `tot`, each with its island, its candidate number and its child;
// handled[r] candidates of island r get a slot and the rest form the extra
// list (re-evaluated one workgroup each).  One workgroup.
__device__ inline void compact_candidates(const int32_t *__restrict__ cand, const int32_t *__restrict__ cand_cnt,
                                          int R, int m, int tot, int32_t *__restrict__ slot_r,
                                          int32_t *__restrict__ slot_c, int32_t *__restrict__ slot_s,
                                          int32_t *__restrict__ handled, int32_t *__restrict__ total,
                                          int32_t *__restrict__ extra_r, int32_t *__restrict__ extra_c,
                                          int32_t *__restrict__ nextra)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int chunk = (R + nt - 1) / nt;
    const int r0 = min(R, tid * chunk), r1 = min(R, r0 + chunk);
    int sum = 0;
    for (int r = r0; r < r1; ++r) sum += cand_cnt[r];
    int acc;
    int off = block_exclusive_scan(sum, &acc), ex = 0;
    if (tid == 0) *total = min(acc, tot);
    for (int r = r0; r < r1; ++r) {
        const int cnt = cand_cnt[r];
        const int h = max(0, min(cnt, tot - off));
        for (int c = 0; c < h; ++c) {
            slot_r[off + c] = r;
            slot_c[off + c] = c;
            slot_s[off + c] = cand[(size_t)r * m + c];
        }
        handled[r] = h;
        off += cnt;
        ex += cnt - h;
    }
    int eo = block_exclusive_scan(ex, &acc);
    if (tid == 0) *nextra = acc;
    for (int r = r0; r < r1; ++r)
        for (int c = handled[r]; c < cand_cnt[r]; ++c) {
            extra_r[eo] = r;
            extra_c[eo] = c;
            ++eo;
        }
}

// Island r = blk of a grid of nblk = R workgroups (block size: a power of two
// >= m).
__device__ __forceinline__ void select1_body(const SelState &S, const double *__restrict__ cost,
                                             const double *__restrict__ eps, const double *__restrict__ parts,
                                             int32_t *__restrict__ cand, int32_t *__restrict__ cand_cnt, int tot,
                                             int32_t *__restrict__ slot_r, int32_t *__restrict__ slot_c,
                                             int32_t *__restrict__ slot_s,
                                             int32_t *__restrict__ handled, int32_t *__restrict__ total,
                                             int32_t *__restrict__ extra_r, int32_t *__restrict__ extra_c,
                                             int32_t *__restrict__ nextra, int *__restrict__ sync, int blk, int nblk,
                                             bool reserve = false)
{
    __shared__ int wave_cnt[16];
    __shared__ int sh_best, sh_res[3];
    const int m = S.m, p = S.p;
    const int r = blk, tid = threadIdx.x, nt = blockDim.x;
    const int s = r * m + tid;
    const bool live = tid < m;
    __shared__ int sh_anc[kMaxP];
    if (!S.exact && tid < p) sh_anc[tid] = S.anc[(size_t)r * p + tid];
    const double fa = S.anc_cost[r];
    double f = live ? cost[s] : 0.0;
    double lb = f, ub = f;
    bool same_as_anc = false;
    if (!S.exact) __syncthreads();   // sh_anc
    if (!S.exact && live) {
        double e = 2.0 * eps[s] + 8.881784197001252e-16;   // + 2^-50 for the interval arithmetic itself
        lb = f * (1.0 - e);
        ub = f * (1.0 + e);
        // a child identical to the ancestor has the ancestor's exact cost;
        // its hub list is compared 16 ids at a time, all loads in flight
        int diff = 0;
        for (int k0 = 0; k0 < p; k0 += 16) {
            int h[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) h[u] = k0 + u < p ? S.children[(size_t)s * p + k0 + u] : 0;
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (k0 + u < p) diff |= h[u] ^ sh_anc[k0 + u];
        }
        same_as_anc = diff == 0;
        if (same_as_anc) lb = ub = fa;
    }
    // (min ub, index) over the island; exact mode: (min f, lowest j)
    double U;
    const int jbest = block_argmin_entries(ub, live ? tid : -1, &U);
    if (S.exact) {
        if (tid == 0) {
            const int j = jbest;
            sh_best = (!S.elitist || U < fa) ? j : -1;
            cand_cnt[r] = 0;
        }
        __syncthreads();
        const int j = sh_best;
        if (j >= 0) {
            const int sb = r * m + j;
            for (int k = tid; k < p; k += nt) S.anc[(size_t)r * p + k] = S.children[(size_t)sb * p + k];
            if (tid == 0) {
                S.anc_cost[r] = cost[sb];
                for (int c = 0; c < 3; ++c) S.anc_parts[3 * (size_t)r + c] = parts[3 * (size_t)sb + c];
            }
        }
    } else {
        const bool is_cand = live && lb <= U && (!S.elitist || lb < fa) && !(S.elitist && same_as_anc);
        // compact candidates in ascending child order: wave ballots + per-wave offsets
        const unsigned long long mask = __ballot(is_cand);
        const int lane = tid & 63, wave = tid >> 6;
        const int below = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wave_cnt[wave] = __popcll(mask);
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wave; ++w) off += wave_cnt[w];
        if (is_cand) cand[(size_t)r * m + off + below] = s;
        if (tid == 0) {
            int tt = 0;
            for (int w = 0; w < (nt + 63) / 64; ++w) tt += wave_cnt[w];
            cand_cnt[r] = tt;
            if (reserve) {
                // the island's slots [o, o + tt) from the shared counter (zeroed
                // at the start of the generation); past tot they are extras
                const int o = tt > 0 ? atomicAdd(total, tt) : 0;
                const int h = max(0, min(tt, tot - o));
                handled[r] = h;
                sh_res[0] = o;
                sh_res[1] = h;
                sh_res[2] = tt > h ? atomicAdd(nextra, tt - h) : 0;
            }
        }
        if (reserve) {
            // slots in any island order: each candidate's exact cost is its
            // own, so which slot or extra computes it changes no result
            __syncthreads();
            if (is_cand) {
                const int c = off + below, o = sh_res[0], h = sh_res[1];
                if (c < h) {
                    slot_r[o + c] = r;
                    slot_c[o + c] = c;
                    slot_s[o + c] = s;
                } else {
                    extra_r[sh_res[2] + c - h] = r;
                    extra_c[sh_res[2] + c - h] = c;
                }
            }
            return;
        }
    }
    if (!last_block(sync, nblk)) return;
    if (S.exact)
        global_step(S);
    else
        compact_candidates(cand, cand_cnt, S.R, m, tot, slot_r, slot_c, slot_s, handled, total, extra_r, extra_c,
                           nextra);
}

__global__ __launch_bounds__(1024) void k_select1(SelState S, const double *__restrict__ cost,
                                                  const double *__restrict__ eps, const double *__restrict__ parts,
                                                  int32_t *__restrict__ cand, int32_t *__restrict__ cand_cnt, int tot,
                                                  int32_t *__restrict__ slot_r, int32_t *__restrict__ slot_c,
                                                  int32_t *__restrict__ slot_s,
                                                  int32_t *__restrict__ handled, int32_t *__restrict__ total,
                                                  int32_t *__restrict__ extra_r, int32_t *__restrict__ extra_c,
                                                  int32_t *__restrict__ nextra, int *__restrict__ sync, int reserve)
{
    select1_body(S, cost, eps, parts, cand, cand_cnt, tot, slot_r, slot_c, slot_s, handled, total, extra_r, extra_c,
                 nextra, sync, blockIdx.x, gridDim.x, reserve != 0);
}

__global__ __launch_bounds__(1024) void k_select1_group(const GroupHdr *__restrict__ hdr,
                                                        const TickJob *__restrict__ jobs)
{
    if ((int)blockIdx.x >= hdr->blocks[kTickSel1]) return;
    const TickJob &J = jobs[tick_job(jobs, hdr->njobs, kTickSel1, blockIdx.x)];
    const DevPtrs &P = J.P;
    const SelState S = make_sel_state(P, J.d);
    select1_body(S, P.cost, P.eps, P.parts, P.cand, P.cand_cnt, J.d.tot, P.slot_r, P.slot_c, P.slot_s, P.handled,
                 P.total, P.extra_r, P.extra_c, P.nextra, P.sync, blockIdx.x - J.start[kTickSel1],
                 J.blocks[kTickSel1]);
}

// Every island ancestor <- the single solution in best / best_cost (the
// evaluated P0 of Sec. 4.1); generation, counters, grid and slot counters
// reset.
__global__ void k_init_state(int R, int p, int tot, int32_t *__restrict__ anc, double *__restrict__ anc_cost,
                             double *__restrict__ anc_parts, const int32_t *__restrict__ best,
                             const double *__restrict__ best_cost, int64_t *__restrict__ gen,
                             int64_t *__restrict__ stats, int *__restrict__ sync, int32_t *__restrict__ slot_done)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < tot) slot_done[t] = 0;
    if (t < R * p) anc[t] = best[t % p];
    if (t < R) {
        anc_cost[t] = best_cost[0];
        for (int q = 0; q < 3; ++q) anc_parts[3 * (size_t)t + q] = best_cost[1 + q];
    }
    if (t == 0) {
        *gen = 0;
        for (int q = 0; q < 4; ++q) stats[q] = 0;
        sync[0] = sync[1] = 0;
    }
}

hipError_t launch_init_state(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    int span = d.R * d.p > d.R ? d.R * d.p : d.R;
    span = span > d.tot ? span : d.tot;
    k_init_state<<<(span + 255) / 256, 256, 0, st>>>(d.R, d.p, d.tot, P.anc, P.anc_cost, P.anc_parts, P.best,
                                                     P.best_cost, P.gen, P.stats, P.sync, P.slot_done);
    return hipGetLastError();
}


int select_threads(int m)
{
    int bt = 64;   // power of two for the tree reduction
    while (bt < m) bt *= 2;
    return bt;
}

// Selection and the end of the generation: k_select1 (with the global step
// for exact costs), else k_select1 -> k_recheck (exact re-evaluation of the
// candidates, island decisions, global step).  reserve: the candidates take
// their slots from the counters P.total and P.nextra, which the generation's
// allocation kernel zeroed, instead of from the last workgroup's compaction.
hipError_t launch_select(const DevPtrs &P, const Dims &d, int exact, hipStream_t st, int reserve)
{
    const int bt = select_threads(d.m);
    const SelState S = make_sel_state(P, d);
    k_select1<<<d.R, bt, 0, st>>>(S, P.cost, P.eps, P.parts, P.cand, P.cand_cnt, d.tot, P.slot_r, P.slot_c,
                                  P.slot_s, P.handled, P.total, P.extra_r, P.extra_c, P.nextra, P.sync,
                                  exact ? 0 : reserve);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || exact) return e;
    return launch_recheck(P, d, st);
}

hipError_t launch_select1_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, int blocks, int threads,
                                hipStream_t st)
{
    if (njobs <= 0 || blocks <= 0) return hipSuccess;
    k_select1_group<<<blocks, threads, 0, st>>>(hdr, jobs);
    return hipGetLastError();
}

}  // namespace hubga
