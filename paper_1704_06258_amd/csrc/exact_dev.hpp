// Whole-solution exact evaluation by one workgroup (objective (1) of Sec. 3
// in binary64): lane j accumulates t_j = sum_i W_ij * C[a_i][a_j] over
// ascending i, then T, Cc and Dd are summed in ascending order by one lane.
// No FMA contraction anywhere, so the result is the sequential definition bit
// for bit.  Works for any workgroup size.
#pragma once
#include "common.hpp"

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

// RU: rows whose W loads are in flight together (registers: 8*RU per lane).
// Ctr (may be null): the transfer term's distances (multi-hop routing); C
// itself when null.
template <typename CT, typename WT, int RU = 8>
__device__ void eval_exact_body(const int32_t *__restrict__ hg, const uint16_t *__restrict__ krow, int n, int p,
                                const CT *__restrict__ C, const double *__restrict__ Ctr, const WT *__restrict__ W,
                                const double *__restrict__ O, const double *__restrict__ D, double chi, double alpha,
                                double delta, double scale, double *cost_out, double *parts_out, char *smem)
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
    for (int e = tid; e < p * p; e += nt)
        Ch[e] = Ctr ? Ctr[(size_t)h[e / p] * n + h[e % p]] : (double)C[(size_t)h[e / p] * n + h[e % p]];
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
        // rows in groups of RU: 4*RU loads in flight per lane, then the adds in
        // ascending row order (absent columns read 0 and are discarded)
        int jc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) jc[q] = js[q] < n ? js[q] : 0;
        int i = 0;
        for (; i + RU <= n; i += RU) {
            double w[RU][4];
            int ki[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const WT *wr = W + (size_t)(i + u) * n;
                ki[u] = kid[i + u];
#pragma unroll
                for (int q = 0; q < 4; ++q) w[u][q] = (double)wr[jc[q]];
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
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

}  // namespace hubga
