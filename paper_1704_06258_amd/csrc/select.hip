// Selection (Sec. 5): each island's best child (argmin, ties to the lowest
// child index) replaces the island ancestor -- only when strictly better in
// elitist mode -- and every n1 generations the best ancestor (ties to the
// lowest island) replaces all ancestors.  Ancestor costs are always exact.
//
// With approximate costs f~ (FP32 or split-bf16) every child carries a
// rigorous bound |f~ - f| <= eps f, hence f in [lb, ub] = f~(1 -+ eps').
// Stage 1 keeps as candidates the children whose interval could hold the
// island minimum (lb <= min ub) and could beat the ancestor (lb < f_anc);
// their exact costs are recomputed (k_recheck) and stage 2 decides on exact
// values, so the decision is the one exact arithmetic would take.
#include "kernels.hpp"

namespace hubga {

__device__ inline bool better(double v, int i, double bv, int bi)
{
    return bi < 0 || v < bv || (v == bv && i < bi);
}

__global__ __launch_bounds__(1024) void k_select1(const double *__restrict__ cost, const double *__restrict__ eps,
                                                  const double *__restrict__ parts, const int32_t *__restrict__ children,
                                                  int m, int p, int exact, int elitist, int32_t *__restrict__ anc,
                                                  double *__restrict__ anc_cost, double *__restrict__ anc_parts,
                                                  int32_t *__restrict__ cand, int32_t *__restrict__ cand_cnt)
{
    __shared__ double sv[1024];
    __shared__ int si[1024];
    __shared__ int wave_cnt[16];
    __shared__ int sh_best;
    const int r = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int s = r * m + tid;
    const bool live = tid < m;
    const double fa = anc_cost[r];
    double f = live ? cost[s] : 0.0;
    double lb = f, ub = f;
    bool same_as_anc = false;
    if (!exact && live) {
        double e = 2.0 * eps[s] + 8.881784197001252e-16;   // + 2^-50 for the interval arithmetic itself
        lb = f * (1.0 - e);
        ub = f * (1.0 + e);
        // a child identical to the ancestor has the ancestor's exact cost
        same_as_anc = true;
        for (int k = 0; k < p; ++k)
            if (children[(size_t)s * p + k] != anc[(size_t)r * p + k]) {
                same_as_anc = false;
                break;
            }
        if (same_as_anc) lb = ub = fa;
    }
    // (min ub, index) over the island; exact mode: (min f, lowest j)
    sv[tid] = ub;
    si[tid] = live ? tid : -1;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
        if (tid < w && si[tid + w] >= 0 && better(sv[tid + w], si[tid + w], sv[tid], si[tid])) {
            sv[tid] = sv[tid + w];
            si[tid] = si[tid + w];
        }
        __syncthreads();
    }
    const double U = sv[0];
    if (exact) {
        if (tid == 0) {
            const int j = si[0];
            sh_best = (!elitist || sv[0] < fa) ? j : -1;
            cand_cnt[r] = 0;
        }
        __syncthreads();
        const int j = sh_best;
        if (j >= 0) {
            const int sb = r * m + j;
            for (int k = tid; k < p; k += nt) anc[(size_t)r * p + k] = children[(size_t)sb * p + k];
            if (tid == 0) {
                anc_cost[r] = cost[sb];
                for (int c = 0; c < 3; ++c) anc_parts[3 * (size_t)r + c] = parts[3 * (size_t)sb + c];
            }
        }
        return;
    }
    const bool is_cand = live && lb <= U && (!elitist || lb < fa) && !(elitist && same_as_anc);
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
        int tot = 0;
        for (int w = 0; w < (nt + 63) / 64; ++w) tot += wave_cnt[w];
        cand_cnt[r] = tot;
    }
}

__global__ __launch_bounds__(64) void k_select2(const int32_t *__restrict__ cand, const int32_t *__restrict__ cand_cnt,
                                                const double *__restrict__ cand_cost,
                                                const double *__restrict__ cand_parts,
                                                const int32_t *__restrict__ children, int m, int p, int elitist,
                                                int32_t *__restrict__ anc, double *__restrict__ anc_cost,
                                                double *__restrict__ anc_parts)
{
    __shared__ double sv[64];
    __shared__ int si[64];
    const int r = blockIdx.x, tid = threadIdx.x;
    const int cnt = cand_cnt[r];
    if (cnt == 0) return;
    double bv = 0.0;
    int bi = -1;
    for (int c = tid; c < cnt; c += 64) {
        double v = cand_cost[(size_t)r * m + c];
        if (better(v, c, bv, bi)) {
            bv = v;
            bi = c;
        }
    }
    sv[tid] = bv;
    si[tid] = bi;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (tid < w && si[tid + w] >= 0 && better(sv[tid + w], si[tid + w], sv[tid], si[tid])) {
            sv[tid] = sv[tid + w];
            si[tid] = si[tid + w];
        }
        __syncthreads();
    }
    const int c = si[0];
    const double v = sv[0];
    if (elitist && !(v < anc_cost[r])) return;
    const int sb = cand[(size_t)r * m + c];
    for (int k = tid; k < p; k += 64) anc[(size_t)r * p + k] = children[(size_t)sb * p + k];
    if (tid == 0) {
        anc_cost[r] = v;
        for (int q = 0; q < 3; ++q) anc_parts[3 * (size_t)r + q] = cand_parts[3 * ((size_t)r * m + c) + q];
    }
}

// End of a generation: counters, the outer-loop global step every n1
// generations, best so far, g <- g + 1.  One workgroup.
__global__ __launch_bounds__(256) void k_global(int R, int p, int S, int n1, int exact,
                                                const int32_t *__restrict__ cand_cnt, int32_t *__restrict__ anc,
                                                double *__restrict__ anc_cost, double *__restrict__ anc_parts,
                                                int32_t *__restrict__ best, double *__restrict__ best_cost,
                                                int64_t *__restrict__ gen, int64_t *__restrict__ stats)
{
    __shared__ double sv[256];
    __shared__ int si[256];
    __shared__ long long sc[256], sr[256];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t g = *gen;
    long long cc = 0, cr = 0;
    if (!exact)
        for (int r = tid; r < R; r += nt) {
            int c = cand_cnt[r];
            cc += c;
            cr += c > 0;
        }
    sc[tid] = cc;
    sr[tid] = cr;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
        if (tid < w) {
            sc[tid] += sc[tid + w];
            sr[tid] += sr[tid + w];
        }
        __syncthreads();
    }
    // argmin over island ancestors (ties to the lowest island)
    auto argmin_anc = [&]() {
        double bv = 0.0;
        int bi = -1;
        for (int r = tid; r < R; r += nt)
            if (better(anc_cost[r], r, bv, bi)) {
                bv = anc_cost[r];
                bi = r;
            }
        __syncthreads();
        sv[tid] = bv;
        si[tid] = bi;
        __syncthreads();
        for (int w = nt / 2; w > 0; w >>= 1) {
            if (tid < w && si[tid + w] >= 0 && better(sv[tid + w], si[tid + w], sv[tid], si[tid])) {
                sv[tid] = sv[tid + w];
                si[tid] = si[tid + w];
            }
            __syncthreads();
        }
        return si[0];
    };
    if ((g + 1) % n1 == 0) {
        const int rs = argmin_anc();
        for (int e = tid; e < R * p; e += nt) {
            int r = e / p, k = e % p;
            if (r != rs) anc[e] = anc[(size_t)rs * p + k];
        }
        for (int r = tid; r < R; r += nt)
            if (r != rs) {
                anc_cost[r] = anc_cost[rs];
                for (int q = 0; q < 3; ++q) anc_parts[3 * (size_t)r + q] = anc_parts[3 * (size_t)rs + q];
            }
        __syncthreads();
    }
    const int rb = argmin_anc();
    const bool improve = anc_cost[rb] < best_cost[0];
    __syncthreads();
    if (improve) {
        for (int k = tid; k < p; k += nt) best[k] = anc[(size_t)rb * p + k];
        if (tid == 0) {
            best_cost[0] = anc_cost[rb];
            for (int q = 0; q < 3; ++q) best_cost[1 + q] = anc_parts[3 * (size_t)rb + q];
        }
    }
    if (tid == 0) {
        *gen = g + 1;
        stats[0] = g + 1;
        stats[1] += sc[0];
        stats[2] += sr[0];
        stats[3] += S;
    }
}

// Every island ancestor <- the single solution in best / best_cost (the
// evaluated P0 of Sec. 4.1); generation and counters reset.
__global__ void k_init_state(int R, int p, int32_t *__restrict__ anc, double *__restrict__ anc_cost,
                             double *__restrict__ anc_parts, const int32_t *__restrict__ best,
                             const double *__restrict__ best_cost, int64_t *__restrict__ gen,
                             int64_t *__restrict__ stats)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < R * p) anc[t] = best[t % p];
    if (t < R) {
        anc_cost[t] = best_cost[0];
        for (int q = 0; q < 3; ++q) anc_parts[3 * (size_t)t + q] = best_cost[1 + q];
    }
    if (t == 0) {
        *gen = 0;
        for (int q = 0; q < 4; ++q) stats[q] = 0;
    }
}

hipError_t launch_init_state(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    int tot = d.R * d.p > d.R ? d.R * d.p : d.R;
    k_init_state<<<(tot + 255) / 256, 256, 0, st>>>(d.R, d.p, P.anc, P.anc_cost, P.anc_parts, P.best, P.best_cost,
                                                    P.gen, P.stats);
    return hipGetLastError();
}

hipError_t launch_select(const DevPtrs &P, const Dims &d, int exact, hipStream_t st)
{
    int bt = 64;   // power of two for the tree reduction
    while (bt < d.m) bt *= 2;
    k_select1<<<d.R, bt, 0, st>>>(P.cost, P.eps, P.parts, P.hubs, d.m, d.p, exact, d.elitist, P.anc, P.anc_cost,
                                  P.anc_parts, P.cand, P.cand_cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || exact) return e;
    e = launch_recheck(P, d, st);
    if (e != hipSuccess) return e;
    k_select2<<<d.R, 64, 0, st>>>(P.cand, P.cand_cnt, P.cand_cost, P.cand_parts, P.hubs, d.m, d.p, d.elitist, P.anc,
                                  P.anc_cost, P.anc_parts);
    return hipGetLastError();
}

hipError_t launch_global(const DevPtrs &P, const Dims &d, int exact, hipStream_t st)
{
    k_global<<<1, 256, 0, st>>>(d.R, d.p, d.S, d.n1, exact, P.cand_cnt, P.anc, P.anc_cost, P.anc_parts, P.best,
                                P.best_cost, P.gen, P.stats);
    return hipGetLastError();
}

}  // namespace hubga
