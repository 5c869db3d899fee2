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

constexpr int kAllocPer = 1;     // individuals per workgroup
constexpr int kScanChunk = 16;   // hub distances loaded together by one lane

// Workgroup blk (of a grid of alloc_blocks(count)) of one context.
template <typename CT>
__device__ __forceinline__ void alloc_body(const int32_t *__restrict__ hubs, int count, int n, int n_pad, int p,
                                           const CT *__restrict__ Ct, const float *__restrict__ Ct32,
                                           const double *__restrict__ O, const double *__restrict__ D,
                                           uint16_t *__restrict__ kidx, double *__restrict__ parts,
                                           int32_t *__restrict__ cmax, float *__restrict__ Ch32, int want_sums,
                                           int blk)
{
#pragma clang fp contract(off)
    __shared__ int sh_h[kAllocPer][kMaxP];
    __shared__ int sh_cnt[kAllocPer][kMaxP];
    __shared__ double red_c[kAllocPer][256], red_d[kAllocPer][256];
    // XCD-major group order: consecutive groups (children of one island) run
    // on the same XCD (workgroup index % 8; a grouped launch starts every
    // context on a multiple of 8) and share its L2.
    const int groups = (count + kAllocPer - 1) / kAllocPer;
    const int per = (groups + 7) / 8;
    const int grp = (blk & 7) * per + (blk >> 3);
    if (grp >= groups) return;
    const int s0 = grp * kAllocPer;
    const int nind = min(kAllocPer, count - s0);
    const int tid = threadIdx.x;
    for (int e = tid; e < kAllocPer * kMaxP; e += 256) {
        const int c = e / kMaxP, k = e % kMaxP;
        sh_cnt[c][k] = 0;
        if (c < nind && k < p) sh_h[c][k] = hubs[(size_t)(s0 + c) * p + k];
    }
    __syncthreads();
    double pc[kAllocPer], pd[kAllocPer];
#pragma unroll
    for (int c = 0; c < kAllocPer; ++c) pc[c] = pd[c] = 0.0;
    for (int i = tid; i < n_pad; i += 256) {
#pragma unroll
        for (int c = 0; c < kAllocPer; ++c) {
            if (c >= nind) break;
            uint16_t *krow = kidx + (size_t)(s0 + c) * n_pad;
            if (i >= n) {
                krow[i] = kNoHub;
                continue;
            }
            const int *h = sh_h[c];
            // Scan in FP32: rounding to FP32 is monotone, so a unique FP32
            // minimum is also the unique minimum of the instance values.  When
            // several hubs share the FP32 minimum, rescan in the instance
            // dtype (strict <, ties to the smaller hub id).
            // The p loads of a chunk are issued before any comparison (a
            // compare-as-you-load loop waits for every load in turn).
            int best = 0;
            float bd = __builtin_huge_valf();
            bool tie = false;
            for (int k0 = 0; k0 < p; k0 += kScanChunk) {
                float v[kScanChunk];
#pragma unroll
                for (int u = 0; u < kScanChunk; ++u)
                    v[u] = k0 + u < p ? Ct32[(size_t)h[k0 + u] * n + i] : __builtin_huge_valf();
#pragma unroll
                for (int u = 0; u < kScanChunk; ++u) {
                    if (v[u] < bd) {
                        bd = v[u];
                        best = k0 + u;
                        tie = false;
                    } else if (v[u] == bd && k0 + u < p) {
                        tie = true;
                    }
                }
            }
            if (tie) {
                best = 0;
                CT be = Ct[(size_t)h[0] * n + i];
                for (int k = 1; k < p; ++k) {
                    const CT v = Ct[(size_t)h[k] * n + i];
                    if (v < be) {
                        be = v;
                        best = k;
                    }
                }
            }
            // a hub keeps itself: binary search of i in the sorted list
            int lo = 0, hi = p - 1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int hv = h[mid];
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
            atomicAdd(&sh_cnt[c][best], 1);
            if (want_sums) {
                const double ci = (double)Ct[(size_t)h[best] * n + i];
                pc[c] = pc[c] + O[i] * ci;
                pd[c] = pd[c] + D[i] * ci;
            }
        }
    }
    if (Ch32) {
        for (int e = tid; e < nind * p * p; e += 256) {
            const int c = e / (p * p), kl = e % (p * p);
            const int k = kl / p, l = kl % p;
            Ch32[(size_t)(s0 + c) * p * p + kl] = (float)Ct[(size_t)sh_h[c][l] * n + sh_h[c][k]];   // C[h_k][h_l]
        }
    }
    if (want_sums) {
#pragma unroll
        for (int c = 0; c < kAllocPer; ++c) {
            red_c[c][tid] = pc[c];
            red_d[c][tid] = pd[c];
        }
    }
    __syncthreads();
    if (want_sums) {
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) {
#pragma unroll
                for (int c = 0; c < kAllocPer; ++c) {
                    red_c[c][tid] = red_c[c][tid] + red_c[c][tid + w];
                    red_d[c][tid] = red_d[c][tid] + red_d[c][tid + w];
                }
            }
            __syncthreads();
        }
    }
    if (tid < nind) {
        const int c = tid;
        int mx = 0;
        for (int k = 0; k < p; ++k) mx = sh_cnt[c][k] > mx ? sh_cnt[c][k] : mx;
        cmax[s0 + c] = mx;
        if (want_sums) {
            parts[3 * (size_t)(s0 + c) + 0] = red_c[c][0];
            parts[3 * (size_t)(s0 + c) + 2] = red_d[c][0];
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

template <typename CT>
__global__ __launch_bounds__(256) void k_alloc(const int32_t *__restrict__ hubs, int count, int n, int n_pad, int p,
                                               const CT *__restrict__ Ct, const float *__restrict__ Ct32,
                                               const double *__restrict__ O, const double *__restrict__ D,
                                               uint16_t *__restrict__ kidx, double *__restrict__ parts,
                                               int32_t *__restrict__ cmax, float *__restrict__ Ch32, int want_sums)
{
    alloc_body<CT>(hubs, count, n, n_pad, p, Ct, Ct32, O, D, kidx, parts, cmax, Ch32, want_sums, blockIdx.x);
}

// Grouped: the children of every context, with their sums and hub tables
// (the split-bf16 generation).
__global__ __launch_bounds__(256) void k_alloc_group(const TickJob *__restrict__ jobs, int njobs)
{
    const TickJob &J = jobs[tick_job(jobs, njobs, kTickAlloc, blockIdx.x)];
    const int blk = blockIdx.x - J.start[kTickAlloc];
    const DevPtrs &P = J.P;
    const Dims &d = J.d;
    if (d.c_f32)
        alloc_body<float>(P.hubs, d.S, d.n, d.n_pad, d.p, (const float *)P.Ct, P.Ct32, P.O, P.D, P.kidx, P.parts,
                          P.cmax, P.Ch32, 1, blk);
    else
        alloc_body<double>(P.hubs, d.S, d.n, d.n_pad, d.p, (const double *)P.Ct, P.Ct32, P.O, P.D, P.kidx,
                           P.parts, P.cmax, P.Ch32, 1, blk);
}

int alloc_blocks(int count)
{
    const int groups = (count + kAllocPer - 1) / kAllocPer;
    return ((groups + 7) / 8) * 8;
}

hipError_t launch_alloc(const DevPtrs &P, const Dims &d, const int32_t *hubs, int count, uint16_t *kidx,
                        int want_sums, int want_ch, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    float *ch = want_ch ? P.Ch32 : nullptr;
    const unsigned grid = (unsigned)alloc_blocks(count);
    if (d.c_f32)
        k_alloc<float><<<grid, 256, 0, st>>>(hubs, count, d.n, d.n_pad, d.p, (const float *)P.Ct, P.Ct32, P.O, P.D,
                                             kidx, P.parts, P.cmax, ch, want_sums);
    else
        k_alloc<double><<<grid, 256, 0, st>>>(hubs, count, d.n, d.n_pad, d.p, (const double *)P.Ct, P.Ct32, P.O,
                                              P.D, kidx, P.parts, P.cmax, ch, want_sums);
    return hipGetLastError();
}

hipError_t launch_alloc_group(const TickJob *jobs, int njobs, int blocks, hipStream_t st)
{
    if (njobs <= 0 || blocks <= 0) return hipSuccess;
    k_alloc_group<<<blocks, 256, 0, st>>>(jobs, njobs);
    return hipGetLastError();
}

}  // namespace hubga
