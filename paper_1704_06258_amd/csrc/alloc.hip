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

constexpr int kScanChunk = 16;   // hub distances loaded together by one lane

// Workgroup blk (of a grid of alloc_blocks(count)) of one context: individual
// s = the workgroup's place in XCD-major order.  The hub ids are read with
// scalar loads (the same for every lane), so each distance load needs no
// per-lane address arithmetic and no LDS round trip; a node-to-position table
// in LDS answers "is node i a hub" with one read.
template <typename CT>
__device__ __forceinline__ void alloc_body(const int32_t *__restrict__ hubs, int count, int n, int n_pad, int p,
                                           const CT *__restrict__ Ct, const float *__restrict__ Ct32,
                                           const double *__restrict__ O, const double *__restrict__ D,
                                           uint16_t *__restrict__ kidx, double *__restrict__ parts,
                                           int32_t *__restrict__ cmax, float *__restrict__ Ch32, int want_sums,
                                           int blk)
{
#pragma clang fp contract(off)
    __shared__ int sh_h[kMaxP];
    __shared__ __align__(16) int sh_off[kMaxP];   // row offsets h*n in the FP32 copy; padding: row n (+inf)
    __shared__ int sh_cnt[kMaxP];
    __shared__ uint8_t sh_pos[kMaxN];   // position of node i in the hub list, 0xFF for spokes
    __shared__ double red_c[256], red_d[256];
    // XCD-major order: consecutive individuals (children of one island) run
    // on the same XCD (workgroup index % 8; a grouped launch starts every
    // context on a multiple of 8) and share its L2.
    const int per = (count + 7) / 8;
    const int s = (blk & 7) * per + (blk >> 3);
    if (s >= count) return;
    const int tid = threadIdx.x;
    const int32_t *__restrict__ hrow = hubs + (size_t)s * p;
    for (int e = tid; e < n; e += 256) sh_pos[e] = 0xFF;
    if (tid < kMaxP) sh_cnt[tid] = 0;
    __syncthreads();
    if (tid < p) {
        const int h = hrow[tid];
        sh_h[tid] = h;
        sh_pos[h] = (uint8_t)tid;
    }
    if (tid < kMaxP) sh_off[tid] = (tid < p ? hrow[tid] : n) * n;
    __syncthreads();
    const int p16 = (p + kScanChunk - 1) / kScanChunk * kScanChunk;
    double pc = 0.0, pd = 0.0;
    uint16_t *krow = kidx + (size_t)s * n_pad;
    for (int i = tid; i < n_pad; i += 256) {
        if (i >= n) {
            krow[i] = kNoHub;
            continue;
        }
        int best;
        const int self = sh_pos[i];
        if (self != 0xFF) {   // a hub keeps itself
            best = self;
        } else {
            // Scan in FP32: rounding to FP32 is monotone, so a unique FP32
            // minimum is also the unique minimum of the instance values.  When
            // several hubs share the FP32 minimum, rescan in the instance
            // dtype (strict <, ties to the smaller hub id).
            // Branch-free: per chunk its minimum, first position and number of
            // hubs at it; merged over chunks (selects, no per-hub branches).
            best = 0;
            float bd = __builtin_huge_valf();
            int at_min = 0;   // hubs at the FP32 minimum so far
            for (int k0 = 0; k0 < p16; k0 += kScanChunk) {
                float v[kScanChunk];
#pragma unroll
                for (int u = 0; u < kScanChunk; ++u) v[u] = Ct32[sh_off[k0 + u] + i];   // padding reads +inf
                float m = v[0];
#pragma unroll
                for (int u = 1; u < kScanChunk; ++u) m = fminf(m, v[u]);
                int first = kScanChunk - 1, cnt = 0;
#pragma unroll
                for (int u = kScanChunk - 1; u >= 0; --u) {
                    const int eq = v[u] == m ? 1 : 0;
                    first = eq ? u : first;
                    cnt += eq;
                }
                const bool lt = m < bd, same = m == bd;
                at_min = lt ? cnt : (same ? at_min + cnt : at_min);
                best = lt ? k0 + first : best;
                bd = lt ? m : bd;
            }
            const bool tie = at_min > 1;   // (+inf padding ties only when every distance is +inf: rescanned)
            if (tie) {
                best = 0;
                CT be = Ct[(size_t)hrow[0] * n + i];
                for (int k = 1; k < p; ++k) {
                    const CT v = Ct[(size_t)hrow[k] * n + i];
                    if (v < be) {
                        be = v;
                        best = k;
                    }
                }
            }
        }
        krow[i] = (uint16_t)best;
        atomicAdd(&sh_cnt[best], 1);
        if (want_sums) {
            const double ci = (double)Ct[(size_t)sh_h[best] * n + i];
            pc = pc + O[i] * ci;
            pd = pd + D[i] * ci;
        }
    }
    if (Ch32)
        for (int e = tid; e < p * p; e += 256) {
            const int k = e / p, l = e % p;
            Ch32[(size_t)s * p * p + e] = (float)Ct[(size_t)sh_h[l] * n + sh_h[k]];   // C[h_k][h_l]
        }
    if (want_sums) {
        red_c[tid] = pc;
        red_d[tid] = pd;
    }
    __syncthreads();
    if (want_sums) {
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) {
                red_c[tid] = red_c[tid] + red_c[tid + w];
                red_d[tid] = red_d[tid] + red_d[tid + w];
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        int mx = 0;
        for (int k = 0; k < p; ++k) mx = sh_cnt[k] > mx ? sh_cnt[k] : mx;
        cmax[s] = mx;
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

int alloc_blocks(int count) { return ((count + 7) / 8) * 8; }

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
