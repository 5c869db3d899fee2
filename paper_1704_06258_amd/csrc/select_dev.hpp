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
__device__ inline bool last_block(int *counter, int nblocks)
{
    __shared__ int is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const int prev = atomicAdd(counter, 1);
        is_last = prev == nblocks - 1;
        if (is_last) atomicExch(counter, 0);
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

// LDS of the block-wide reductions (one instance per kernel).
struct ArgminScratch {
    double v[1024];
    int i[1024];
};
__device__ inline ArgminScratch &argmin_scratch()
{
    __shared__ ArgminScratch s;
    return s;
}

// Block-wide (value, index) argmin over v[0..count) read through f(i);
// returns the index (-1 if count == 0).  Ties go to the lower index.
template <typename F>
__device__ inline int block_argmin(int count, F f, double *out_value)
{
    ArgminScratch &sc = argmin_scratch();
    double *sv = sc.v;
    int *si = sc.i;
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
    const int r = si[0];
    if (out_value) *out_value = sv[0];
    __syncthreads();
    return r;
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

// Island r: the exactly re-evaluated candidates decide (ties to the lower
// candidate, i.e. the lower child index); elitist mode keeps the ancestor
// unless strictly beaten.
__device__ inline void select_island_exact(const SelState &S, int r)
{
    const int cnt = S.cand_cnt[r];
    if (cnt == 0) return;
    double v;
    const int c = block_argmin(cnt, [&](int i) { return S.cand_cost[(size_t)r * S.m + i]; }, &v);
    if (S.elitist && !(v < S.anc_cost[r])) return;
    const int sb = S.cand[(size_t)r * S.m + c];
    for (int k = threadIdx.x; k < S.p; k += blockDim.x) S.anc[(size_t)r * S.p + k] = S.children[(size_t)sb * S.p + k];
    if (threadIdx.x == 0) {
        S.anc_cost[r] = v;
        for (int q = 0; q < 3; ++q) S.anc_parts[3 * (size_t)r + q] = S.cand_parts[3 * ((size_t)r * S.m + c) + q];
    }
    __syncthreads();
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

}  // namespace hubga
