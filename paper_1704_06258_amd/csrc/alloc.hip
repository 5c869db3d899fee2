// Nearest-hub allocation of a batch of hub sets (Sec. 4.1 and Sec. 5): node i
// goes to the hub h_k with the smallest C[i][h_k], scanning k ascending with a
// strict comparison (ties to the smaller hub id); hubs are allocated to
// themselves.  One workgroup per individual; the hub rows of the transposed
// distance matrix are read coalesced (lane = node).
//
// Outputs per individual s: kidx[s][i] = hub position (kNoHub in the padding
// up to n_pad), the largest cluster size, and (when asked) the collection and
// distribution sums Cc = sum_i O_i c_i, Dd = sum_i D_i c_i with c_i =
// C[i][a_i] in binary64 (fixed tree order), and the FP32 hub-to-hub table
// Ch32[s][k][l] = C[h_k][h_l] used by the batched kernel's epilogue.
#include "kernels.hpp"

namespace hubga {

template <typename CT>
__global__ __launch_bounds__(256) void k_alloc(const int32_t *__restrict__ hubs, int count, int n, int n_pad, int p,
                                               const CT *__restrict__ Ct, const float *__restrict__ Ct32,
                                               const double *__restrict__ O,
                                               const double *__restrict__ D, uint16_t *__restrict__ kidx,
                                               double *__restrict__ parts, int32_t *__restrict__ cmax,
                                               float *__restrict__ Ch32, int want_sums)
{
#pragma clang fp contract(off)
    __shared__ int sh_h[kMaxP];
    __shared__ int sh_cnt[kMaxP];
    __shared__ double red_c[256], red_d[256];
    const int s = blockIdx.x;
    if (s >= count) return;
    const int tid = threadIdx.x;
    const int32_t *h = hubs + (size_t)s * p;
    if (tid < p) {
        sh_h[tid] = h[tid];
        sh_cnt[tid] = 0;
    }
    __syncthreads();
    double pc = 0.0, pd = 0.0;
    uint16_t *krow = kidx + (size_t)s * n_pad;
    for (int i = tid; i < n_pad; i += blockDim.x) {
        if (i >= n) {
            krow[i] = kNoHub;
            continue;
        }
        // Scan in FP32: rounding to FP32 is monotone, so a unique FP32
        // minimum is also the unique minimum of the instance values.  When
        // several hubs share the FP32 minimum, rescan in the instance dtype
        // (strict <, ties to the smaller hub id).
        int best = 0;
        float bd = Ct32[(size_t)sh_h[0] * n + i];
        bool tie = false;
        for (int k = 1; k < p; ++k) {
            float v = Ct32[(size_t)sh_h[k] * n + i];
            if (v < bd) {
                bd = v;
                best = k;
                tie = false;
            } else if (v == bd) {
                tie = true;
            }
        }
        if (tie) {
            best = 0;
            CT be = Ct[(size_t)sh_h[0] * n + i];
            for (int k = 1; k < p; ++k) {
                CT v = Ct[(size_t)sh_h[k] * n + i];
                if (v < be) {
                    be = v;
                    best = k;
                }
            }
        }
        // a hub keeps itself: binary search of i in the sorted list
        int lo = 0, hi = p - 1;
        while (lo <= hi) {
            int mid = (lo + hi) >> 1;
            int hv = sh_h[mid];
            if (hv == i) {
                best = mid;
                break;
            }
            if (hv < i)
                lo = mid + 1;
            else
                hi = mid - 1;
        }
        krow[i] = (uint16_t)best;
        atomicAdd(&sh_cnt[best], 1);
        if (want_sums) {
            double ci = (double)Ct[(size_t)sh_h[best] * n + i];
            pc = pc + O[i] * ci;
            pd = pd + D[i] * ci;
        }
    }
    if (Ch32) {
        float *ch = Ch32 + (size_t)s * p * p;
        for (int e = tid; e < p * p; e += blockDim.x) {
            int k = e / p, l = e % p;
            ch[e] = (float)Ct[(size_t)sh_h[l] * n + sh_h[k]];   // C[h_k][h_l]
        }
    }
    if (want_sums) {
        red_c[tid] = pc;
        red_d[tid] = pd;
    }
    __syncthreads();
    if (want_sums) {
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (tid < w) {
                red_c[tid] = red_c[tid] + red_c[tid + w];
                red_d[tid] = red_d[tid] + red_d[tid + w];
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        int m = 0;
        for (int k = 0; k < p; ++k) m = sh_cnt[k] > m ? sh_cnt[k] : m;
        cmax[s] = m;
        if (want_sums) {
            parts[3 * (size_t)s + 0] = red_c[0];
            parts[3 * (size_t)s + 2] = red_d[0];
        }
    }
}

// Copy caller-provided device hub lists into the workspace, clamping every id
// to [0, n) so that malformed input can never address memory out of bounds.
__global__ void k_copy_clamp(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int total, int n)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < total) {
        int v = src[t];
        dst[t] = v < 0 ? 0 : (v >= n ? n - 1 : v);
    }
}

hipError_t launch_copy_clamp(const int32_t *src, int32_t *dst, int total, int n, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    k_copy_clamp<<<(total + 255) / 256, 256, 0, st>>>(src, dst, total, n);
    return hipGetLastError();
}

hipError_t launch_alloc(const DevPtrs &P, const Dims &d, const int32_t *hubs, int count, uint16_t *kidx,
                        int want_sums, int want_ch, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    float *ch = want_ch ? P.Ch32 : nullptr;
    if (d.c_f32)
        k_alloc<float><<<count, 256, 0, st>>>(hubs, count, d.n, d.n_pad, d.p, (const float *)P.Ct, P.Ct32, P.O, P.D,
                                             kidx, P.parts, P.cmax, ch, want_sums);
    else
        k_alloc<double><<<count, 256, 0, st>>>(hubs, count, d.n, d.n_pad, d.p, (const double *)P.Ct, P.Ct32, P.O,
                                              P.D, kidx, P.parts, P.cmax, ch, want_sums);
    return hipGetLastError();
}

}  // namespace hubga
