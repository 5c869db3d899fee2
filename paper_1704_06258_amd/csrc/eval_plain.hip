// Per-individual fitness evaluation, one workgroup per individual (the
// "plain" kernels; Eval of Sec. 4.3 and Sec. 5, objective (1) of Sec. 3).
//
// k_eval_exact: binary64 in the canonical order, bit-identical to a
//   sequential evaluation: lane j accumulates t_j = sum_i W_ij*C[a_i][a_j]
//   over ascending i (coalesced W rows), then T, Cc and Dd are summed in
//   ascending order by one lane from LDS; no FMA contraction anywhere.
// k_eval_fp32: FP32 per-column sums with FMA, FP64 tree reduction of the
//   columns; Cc and Dd come from the allocation kernel.  Returns a rigorous
//   relative error bound with every cost.
#include "kernels.hpp"
#include "exact_dev.hpp"

#include <algorithm>

namespace hubga {

template <typename CT, typename WT>
__global__ __launch_bounds__(256) void k_eval_exact(const int32_t *__restrict__ hubs,
                                                    const uint16_t *__restrict__ kidx, int count, int n, int n_pad,
                                                    int p, const CT *__restrict__ C, const double *__restrict__ Ctr,
                                                    const WT *__restrict__ W,
                                                    const double *__restrict__ O, const double *__restrict__ D,
                                                    double chi, double alpha, double delta, double scale,
                                                    double *__restrict__ cost, double *__restrict__ parts,
                                                    double *__restrict__ eps)
{
    extern __shared__ __align__(16) char smem[];
    const int s = blockIdx.x;
    if (s >= count) return;
    eval_exact_body<CT, WT>(hubs + (size_t)s * p, kidx + (size_t)s * n_pad, n, p, C, Ctr, W, O, D, chi, alpha,
                            delta, scale, cost + s, parts + 3 * (size_t)s, smem);
    if (threadIdx.x == 0 && eps) eps[s] = 0.0;
}

// ------------------------------------------------------------- FP32 --

template <typename CT>
__global__ __launch_bounds__(256) void k_eval_fp32(const int32_t *__restrict__ hubs, const uint16_t *__restrict__ kidx,
                                                   int count, int n, int n_pad, int p, const CT *__restrict__ Ct,
                                                   const double *__restrict__ Ctr, const float *__restrict__ W,
                                                   double chi, double alpha,
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
    for (int e = tid; e < p * p; e += nt)
        Ch[e] = Ctr ? (float)Ctr[(size_t)h[e / p] * n + h[e % p]] : (float)Ct[(size_t)h[e % p] * n + h[e / p]];
    __syncthreads();
    double tsum = 0.0;
    constexpr int RU = 8;   // rows whose W loads are in flight together, as in the binary64 kernel
    for (int j0 = tid; j0 < n; j0 += 4 * nt) {
        int js[4], kj[4], jc[4];
        float acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            js[q] = j0 + q * nt;
            kj[q] = js[q] < n ? kid[js[q]] : 0;
            jc[q] = js[q] < n ? js[q] : 0;   // absent columns read column 0 and are discarded
            acc[q] = 0.0f;
        }
        int i = 0;
        for (; i + RU <= n; i += RU) {
            float w[RU][4];
            int ki[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const float *wr = W + (size_t)(i + u) * n;
                ki[u] = kid[i + u];
#pragma unroll
                for (int q = 0; q < 4; ++q) w[u][q] = wr[jc[q]];
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const float *chr = Ch + (size_t)ki[u] * p;
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = __builtin_fmaf(w[u][q], chr[kj[q]], acc[q]);
            }
        }
        for (; i < n; ++i) {
            const float *wr = W + (size_t)i * n;
            const float *chr = Ch + (size_t)kid[i] * p;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = __builtin_fmaf(wr[jc[q]], chr[kj[q]], acc[q]);
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
                                                             P.Ctr, (const WT *)P.W, P.O, P.D, d.chi, d.alpha, d.delta,
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
                                                                (const float *)P.Ct, P.Ctr, W, d.chi, d.alpha, d.delta,
                                                                d.scale, eb, P.cost, P.parts, P.eps);
    } else {
        k_eval_fp32<double><<<count, eval_block(d.n), sm, st>>>(hubs, kidx, count, d.n, d.n_pad, d.p,
                                                                 (const double *)P.Ct, P.Ctr, W, d.chi, d.alpha, d.delta,
                                                                 d.scale, eb, P.cost, P.parts, P.eps);
    }
    return hipGetLastError();
}

// Raise the dynamic-LDS cap of every kernel here that may need more than the
// default, once per process (never during graph capture).
hipError_t prepare_plain_kernels(int max_lds)
{
    const void *fns[] = {(const void *)k_eval_exact<double, double>, (const void *)k_eval_exact<double, float>,
                         (const void *)k_eval_exact<float, double>,  (const void *)k_eval_exact<float, float>,
                         (const void *)k_eval_fp32<double>,          (const void *)k_eval_fp32<float>};
    for (const void *f : fns) {
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, f);
        if (e != hipSuccess) return e;
        const int dyn = max_lds - (int)fa.sharedSizeBytes;   // the cap excludes the kernel's static LDS
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hubga
