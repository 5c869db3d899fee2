// Selection steps shared by the selection and exact re-evaluation kernels
// (Sec. 5): island argmin with ancestor update, the outer-loop global step,
// and the grid-level bookkeeping done by the last workgroup of a launch.
#pragma once
#include "common.hpp"

namespace hubga {

__device__ inline bool better(double v, int i, double bv, int bi)
{
    return bi < 0 || v < bv || (v == bv && i < bi);
}

// True in the last workgroup of the grid to get here.  Every workgroup
// publishes its global writes (device-scope fence) before counting itself in;
// the last one fences again before reading them and resets the counter for
// the next launch.
// Device-scope release and acquire fences.  A release writes the XCD's L2
// back; only an acquire invalidates it (a full fence would do both, and the
// invalidation drops what every other workgroup on that XCD has cached).
__device__ __forceinline__ void release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ inline bool last_block(int *counter, int nblocks)
{
    __shared__ int is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        release_agent();
        const int prev = atomicAdd(counter, 1);
        is_last = prev == nblocks - 1;
        if (is_last) atomicExch(counter, 0);
    }
    __syncthreads();
    if (is_last) acquire_agent();
    return is_last != 0;
}

// Block-wide (value, index) argmin of one entry per thread (index < 0: no
// entry); returns the index (-1 if no thread has one).  Ties go to the lower
// index; any workgroup size up to 1024.  (value, index) pairs are totally
// ordered, so the order of the lane and wave merges does not change the
// result.
__device__ inline int block_argmin_entries(double bv, int bi, double *out_value)
{
    __shared__ double wv[16];
    __shared__ int wi[16];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (oi >= 0 && better(ov, oi, bv, bi)) {
            bv = ov;
            bi = oi;
        }
    }
    __syncthreads();   // wv / wi free from a previous call
    if ((tid & 63) == 0) {
        wv[tid >> 6] = bv;
        wi[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < (nt + 63) / 64; ++w)
            if (wi[w] >= 0 && better(wv[w], wi[w], bv, bi)) {
                bv = wv[w];
                bi = wi[w];
            }
        wv[0] = bv;
        wi[0] = bi;
    }
    __syncthreads();
    const int r = wi[0];
    if (out_value) *out_value = wv[0];
    __syncthreads();
    return r;
}

// Block-wide (value, index) argmin over v[0..count) read through f(i);
// returns the index (-1 if count == 0).
template <typename F>
__device__ inline int block_argmin(int count, F f, double *out_value)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    double bv = 0.0;
    int bi = -1;
    for (int i = tid; i < count; i += nt) {
        const double v = f(i);
        if (better(v, i, bv, bi)) {
            bv = v;
            bi = i;
        }
    }
    return block_argmin_entries(bv, bi, out_value);
}

// Exclusive prefix sum of one value per thread in thread order; *sum gets
// the workgroup's total.  Any workgroup size up to 1024.
__device__ inline int block_exclusive_scan(int v, int *sum)
{
    __shared__ int ws[16];
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
    int x = v;   // inclusive scan within the wave
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    __syncthreads();   // ws free from a previous call
    if (lane == 63 || tid == nt - 1) ws[wave] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < (nt + 63) / 64; ++w) {
        const int t = ws[w];
        base += w < wave ? t : 0;
        tot += t;
    }
    *sum = tot;
    return base + x - v;
}

struct SelState {
    int R, m, p, S, n1, elitist, exact;
    const int32_t *children;
    int32_t *anc;
    double *anc_cost, *anc_parts;
    int32_t *best;
    double *best_cost;   // cost, then 3 parts
    int64_t *gen, *stats;
    const int32_t *cand, *cand_cnt;
    const double *cand_cost, *cand_parts;
};

__host__ __device__ inline SelState make_sel_state(const DevPtrs &P, const Dims &d)
{
    SelState S;
    S.R = d.R;
    S.m = d.m;
    S.p = d.p;
    S.S = d.S;
    S.n1 = d.n1;
    S.elitist = d.elitist;
    S.exact = d.prec == kFP64;
    S.children = P.hubs;
    S.anc = P.anc;
    S.anc_cost = P.anc_cost;
    S.anc_parts = P.anc_parts;
    S.best = P.best;
    S.best_cost = P.best_cost;
    S.gen = P.gen;
    S.stats = P.stats;
    S.cand = P.cand;
    S.cand_cnt = P.cand_cnt;
    S.cand_cost = P.cand_cost;
    S.cand_parts = P.cand_parts;
    return S;
}

// End of a generation (one workgroup): counters, the global step every n1
// generations (best ancestor, ties to the lowest island, replaces all), best
// so far, g <- g + 1.
__device__ inline void global_step(const SelState &S)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t g = *S.gen;
    __shared__ long long sc, sr;
    if (tid == 0) {
        long long cc = 0, cr = 0;
        if (!S.exact)
            for (int r = 0; r < S.R; ++r) {
                const int c = S.cand_cnt[r];
                cc += c;
                cr += c > 0;
            }
        sc = cc;
        sr = cr;
    }
    __syncthreads();
    if ((g + 1) % S.n1 == 0) {
        const int rs = block_argmin(S.R, [&](int r) { return S.anc_cost[r]; }, nullptr);
        for (int e = tid; e < S.R * S.p; e += nt) {
            const int r = e / S.p, k = e % S.p;
            if (r != rs) S.anc[e] = S.anc[(size_t)rs * S.p + k];
        }
        for (int r = tid; r < S.R; r += nt)
            if (r != rs) {
                S.anc_cost[r] = S.anc_cost[rs];
                for (int q = 0; q < 3; ++q) S.anc_parts[3 * (size_t)r + q] = S.anc_parts[3 * (size_t)rs + q];
            }
        __syncthreads();
    }
    double bv;
    const int rb = block_argmin(S.R, [&](int r) { return S.anc_cost[r]; }, &bv);
    const bool improve = bv < S.best_cost[0];
    __syncthreads();
    if (improve) {
        for (int k = tid; k < S.p; k += nt) S.best[k] = S.anc[(size_t)rb * S.p + k];
        if (tid == 0) {
            S.best_cost[0] = bv;
            for (int q = 0; q < 3; ++q) S.best_cost[1 + q] = S.anc_parts[3 * (size_t)rb + q];
        }
    }
    if (tid == 0) {
        *S.gen = g + 1;
        S.stats[0] = g + 1;
        S.stats[1] += sc;
        S.stats[2] += sr;
        S.stats[3] += S.S;
    }
    __syncthreads();
}

// Every island decided on the exact costs of its candidates (ties to the
// lower candidate, i.e. the lower child index; elitist mode keeps the ancestor
// unless strictly beaten), then the end of the generation -- counters, the
// global step every n1 generations (the best island, ties to the lowest,
// replaces all), best so far, g <- g + 1 -- in one pass over the islands.
// The best island and the source of its hub list and parts come out of the
// pass itself, so nothing written in it is read back.  One workgroup of any
// size up to 1024; choice: R ints of scratch.
__device__ inline void decide_generation(const SelState &S, int32_t *__restrict__ choice)
{
    __shared__ double wv[16], wp[16][3];
    __shared__ int wi[16], wsb[16], wcc[16], wcr[16];
    __shared__ double sh_parts[3];
    const int tid = threadIdx.x, nt = blockDim.x, m = S.m, p = S.p;
    const int64_t g = *S.gen;
    const double best0 = S.best_cost[0];
    const bool gstep = (g + 1) % S.n1 == 0;
    int64_t st[3] = {0, 0, 0};   // counters, read ahead of the islands' loads
    if (tid == 0)
        for (int q = 0; q < 3; ++q) st[q] = S.stats[1 + q];
    // the best island so far: its cost, index, child and parts (carried
    // through the reductions, so no load waits on them)
    double bv = 0.0, bp[3] = {0.0, 0.0, 0.0};
    int bi = -1, bsb = -1, cc = 0, cr = 0;
    for (int r = tid; r < S.R; r += nt) {
        const int cnt = S.cand_cnt[r];
        const double fa = S.anc_cost[r];
        double ap[3];
        for (int q = 0; q < 3; ++q) ap[q] = S.anc_parts[3 * (size_t)r + q];
        // the first four candidates' costs, children and parts are read
        // together (valid addresses whatever cnt is), the rest in a loop
        constexpr int Q = 4;
        double x[Q], xp[Q][3];
        int xc[Q];
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            const size_t o = (size_t)r * m + (u < m ? u : m - 1);
            x[u] = S.cand_cost[o];
            xc[u] = S.cand[o];
#pragma unroll
            for (int q = 0; q < 3; ++q) xp[u][q] = S.cand_parts[3 * o + q];
        }
        double v = 0.0, vp[3] = {0.0, 0.0, 0.0};
        int c = -1, sb = -1;
#pragma unroll
        for (int u = 0; u < Q; ++u)
            if (u < cnt && (c < 0 || x[u] < v)) {
                v = x[u];
                c = u;
                sb = xc[u];
#pragma unroll
                for (int q = 0; q < 3; ++q) vp[q] = xp[u][q];
            }
        for (int i = Q; i < cnt; ++i) {
            const double y = S.cand_cost[(size_t)r * m + i];
            if (y < v) {
                v = y;
                c = i;
            }
        }
        if (c >= Q) {
            const size_t o = (size_t)r * m + c;
            sb = S.cand[o];
            for (int q = 0; q < 3; ++q) vp[q] = S.cand_parts[3 * o + q];
        }
        const bool take = c >= 0 && (!S.elitist || v < fa);
        if (!take) sb = -1;
        const double fr = take ? v : fa;
        choice[r] = sb;
        if (take) {   // the island's new hub list, its loads issued together
            S.anc_cost[r] = v;
            for (int q = 0; q < 3; ++q) S.anc_parts[3 * (size_t)r + q] = vp[q];
            for (int k0 = 0; k0 < p; k0 += 8) {
                int h[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) h[u] = k0 + u < p ? S.children[(size_t)sb * p + k0 + u] : 0;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (k0 + u < p) S.anc[(size_t)r * p + k0 + u] = h[u];
            }
        }
        cc += cnt;
        cr += cnt > 0;
        if (better(fr, r, bv, bi)) {
            bv = fr;
            bi = r;
            bsb = sb;
            for (int q = 0; q < 3; ++q) bp[q] = take ? vp[q] : ap[q];
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off), osb = __shfl_xor(bsb, off);
        double op[3];
        for (int q = 0; q < 3; ++q) op[q] = __shfl_xor(bp[q], off);
        if (oi >= 0 && better(ov, oi, bv, bi)) {
            bv = ov;
            bi = oi;
            bsb = osb;
            for (int q = 0; q < 3; ++q) bp[q] = op[q];
        }
        cc += __shfl_xor(cc, off);
        cr += __shfl_xor(cr, off);
    }
    if ((tid & 63) == 0) {
        wv[tid >> 6] = bv;
        wi[tid >> 6] = bi;
        wsb[tid >> 6] = bsb;
        for (int q = 0; q < 3; ++q) wp[tid >> 6][q] = bp[q];
        wcc[tid >> 6] = cc;
        wcr[tid >> 6] = cr;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < (nt + 63) / 64; ++w) {
            if (wi[w] >= 0 && better(wv[w], wi[w], bv, bi)) {
                bv = wv[w];
                bi = wi[w];
                bsb = wsb[w];
                for (int q = 0; q < 3; ++q) bp[q] = wp[w][q];
            }
            cc += wcc[w];
            cr += wcr[w];
        }
        wv[0] = bv;
        wi[0] = bi;
        wsb[0] = bsb;
        for (int q = 0; q < 3; ++q) sh_parts[q] = bp[q];
    }
    __syncthreads();
    const int rs = wi[0], sbs = wsb[0];
    const double vs = wv[0];
    auto hub_of_rs = [&](int k) { return sbs >= 0 ? S.children[(size_t)sbs * p + k] : S.anc[(size_t)rs * p + k]; };
    // hub lists: each island took its choice above; the global step gives
    // every other island rs's (island rs's own list is read from the child
    // it took, or is its unchanged ancestor)
    if (gstep)
        for (int e = tid; e < S.R * p; e += nt) {
            const int r = e / p, k = e - r * p;
            if (r != rs) S.anc[e] = hub_of_rs(k);
        }
    if (gstep)
        for (int r = tid; r < S.R; r += nt)
            if (r != rs) {
                S.anc_cost[r] = vs;
                for (int q = 0; q < 3; ++q) S.anc_parts[3 * (size_t)r + q] = sh_parts[q];
            }
    if (vs < best0) {
        for (int k = tid; k < p; k += nt) S.best[k] = hub_of_rs(k);
        if (tid == 0) {
            S.best_cost[0] = vs;
            for (int q = 0; q < 3; ++q) S.best_cost[1 + q] = sh_parts[q];
        }
    }
    if (tid == 0) {
        *S.gen = g + 1;
        S.stats[0] = g + 1;
        S.stats[1] = st[0] + cc;
        S.stats[2] = st[1] + cr;
        S.stats[3] = st[2] + S.S;
    }
    __syncthreads();
}

}  // namespace hubga
