// Nearest-hub allocation of a batch of hub sets (Sec. 4.1 and Sec. 5): node i
// goes to the hub h_k with the smallest C[i][h_k], scanning k ascending with a
// strict comparison (ties to the smaller hub id); hubs are allocated to
// themselves.  One workgroup per individual; the hub rows of the transposed
// distance matrix are read coalesced (lane = node).
//
// Outputs per individual s: kidx[s][i] = hub position (kNoHub in the padding
// up to n_pad), the largest cluster size, and (when asked, in the approximate
// modes) the collection and distribution sums Cc = sum_i O_i c_i, Dd = sum_i
// D_i c_i in binary64 (a fixed summation order) with c_i = C[i][a_i] rounded
// to FP32 -- the scan's own minimum, no second gather; its rounding, 2^-24
// relative, is the one the error bounds already allow for every FP32
// distance -- and the FP32 hub-to-hub table
// Ch32[s][k][l] = C[h_k][h_l] used by the batched kernel's epilogue (the
// shortest-path distance Ctr[h_k][h_l] instead under multi-hop routing).
#include "kernels.hpp"

namespace hubga {

constexpr int kScanHubs = 4;    // hubs per scan chunk
constexpr int kScanNodes = 4;   // nodes per lane scanned together

// Workgroup blk (of a grid of alloc_blocks(count)) of one context: individual
// s = the workgroup's place in XCD-major order.  A lane takes kScanNodes nodes
// i = g0 + t*256 + tid at once and scans the hubs in chunks of kScanHubs: the
// chunk's distances for all its nodes are loaded together, then merged (loads
// past n re-read valid addresses and are not used).  Few registers, so many
// workgroups share a CU and hide each other's load latency.  A
// node-to-position table in LDS answers "is node i a hub" with one read.
template <typename CT>
__device__ __forceinline__ void alloc_body(const int32_t *__restrict__ hubs, int count, int n, int n_pad, int p,
                                           const CT *__restrict__ Ct, const float *__restrict__ Ct32,
                                           const double *__restrict__ O, const double *__restrict__ D,
                                           uint16_t *__restrict__ kidx, double *__restrict__ parts,
                                           int32_t *__restrict__ cmax, float *__restrict__ Ch32, int want_sums,
                                           const double *__restrict__ Ctr, int blk)
{
#pragma clang fp contract(off)
    constexpr int T = kScanNodes, H = kScanHubs;
    __shared__ int sh_h[kMaxP];
    __shared__ __align__(16) int sh_off[kMaxP];   // row offsets h*n in the FP32 copy; padding: row n (+inf)
    __shared__ int sh_cnt[kMaxP];
    __shared__ uint8_t sh_pos[kMaxN];   // position of node i in the hub list, 0xFF for spokes
    __shared__ double red_c[4], red_d[4];
    // XCD-major order: consecutive individuals (children of one island) run
    // on the same XCD (workgroup index % 8; a grouped launch starts every
    // context on a multiple of 8) and share its L2.
    const int per = (count + 7) / 8;
    const int s = (blk & 7) * per + (blk >> 3);
    if (s >= count) return;
    const int tid = threadIdx.x;
    const int32_t *__restrict__ hrow = hubs + (size_t)s * p;
    const int hk = tid < p ? hrow[tid] : n;   // in flight while LDS is cleared
    for (int e = tid; e < n; e += 256) sh_pos[e] = 0xFF;
    if (tid < kMaxP) sh_cnt[tid] = 0;
    __syncthreads();
    if (tid < p) {
        sh_h[tid] = hk;
        sh_pos[hk] = (uint8_t)tid;
    }
    if (tid < kMaxP) sh_off[tid] = hk * n;
    __syncthreads();
    const int nchunks = (p + H - 1) / H;
    // the hub-to-hub table C[h_k][h_l] in FP32: its first 512 entries are
    // gathered now, in flight during the scan, and stored at the end
    float chv[2];
    if (Ch32) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + q * 256;
            chv[q] = e >= p * p ? 0.0f
                     : Ctr ? (float)Ctr[(size_t)sh_h[e / p] * n + sh_h[e % p]]
                           : (float)Ct[(size_t)sh_h[e % p] * n + sh_h[e / p]];
        }
    }
    double pc = 0.0, pd = 0.0;
    uint16_t *krow = kidx + (size_t)s * n_pad;
    for (int g0 = 0; g0 < n_pad; g0 += 256 * T) {
        int ii[T], ic[T];   // nodes, and the same clamped to a valid row position
#pragma unroll
        for (int t = 0; t < T; ++t) {
            ii[t] = g0 + t * 256 + tid;
            ic[t] = ii[t] < n ? ii[t] : n - 1;
        }
        // FP32 scan: rounding to FP32 is monotone, so a unique FP32 minimum is
        // also the unique minimum of the instance values.  Per node: the
        // running minimum, its first hub position and how many hubs are at it.
        float bd[T];
        int best[T], at_min[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            bd[t] = __builtin_huge_valf();
            best[t] = 0;
            at_min[t] = 0;
        }
        float A[T][H];
        auto load = [&](float(&X)[T][H], int c) {
            const int4 o = *(const int4 *)(sh_off + c * H);
            const int off[H] = {o.x, o.y, o.z, o.w};
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int u = 0; u < H; ++u) X[t][u] = Ct32[off[u] + ic[t]];   // padding hubs read +inf
        };
        auto merge = [&](const float(&X)[T][H], int c) {
#pragma unroll
            for (int t = 0; t < T; ++t) {
                float m = X[t][0];
#pragma unroll
                for (int u = 1; u < H; ++u) m = fminf(m, X[t][u]);
                int first = H - 1, cnt = 0;
#pragma unroll
                for (int u = H - 1; u >= 0; --u) {
                    const int eq = X[t][u] == m ? 1 : 0;
                    first = eq ? u : first;
                    cnt += eq;
                }
                const bool lt = m < bd[t], same = m == bd[t];
                at_min[t] = lt ? cnt : (same ? at_min[t] + cnt : at_min[t]);
                best[t] = lt ? c * H + first : best[t];
                bd[t] = lt ? m : bd[t];
            }
        };
        for (int c = 0; c < nchunks; ++c) {
            load(A, c);
            merge(A, c);
        }
        // hubs keep themselves; FP32 ties are rescanned in the instance dtype
        // (strict <, ties to the smaller hub id; +inf padding ties only when
        // every distance is +inf: rescanned too).  c32: the FP32 distance to
        // the chosen hub (a tie's winner has the tied FP32 value).
        float c32[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int i = ii[t];
            c32[t] = bd[t];
            if (i >= n) continue;
            const int self = sh_pos[i];
            if (self != 0xFF) {
                best[t] = self;
                c32[t] = Ct32[(size_t)i * n + i];
            } else if (at_min[t] > 1) {
                int b = 0;
                CT be = Ct[(size_t)hrow[0] * n + i];
                for (int k = 1; k < p; ++k) {
                    const CT v = Ct[(size_t)hrow[k] * n + i];
                    if (v < be) {
                        be = v;
                        b = k;
                    }
                }
                best[t] = b;
            }
        }
        // outputs, two nodes at a time (few registers): position, cluster
        // count, and the binary64 terms O_i c_i and D_i c_i in node order
#pragma unroll
        for (int t0 = 0; t0 < T; t0 += 2) {
            double cv[2], ov[2], dv[2];
            if (want_sums) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int t = t0 + u;
                    cv[u] = (double)c32[t];
                    ov[u] = O[ic[t]];
                    dv[u] = D[ic[t]];
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = t0 + u, i = ii[t];
                if (i >= n_pad) continue;
                if (i >= n) {
                    krow[i] = kNoHub;
                    continue;
                }
                krow[i] = (uint16_t)best[t];
                atomicAdd(&sh_cnt[best[t]], 1);
                if (want_sums) {
                    pc = pc + ov[u] * cv[u];
                    pd = pd + dv[u] * cv[u];
                }
            }
        }
    }
    if (Ch32) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + q * 256;
            if (e < p * p) Ch32[(size_t)s * p * p + e] = chv[q];
        }
        for (int e = tid + 512; e < p * p; e += 256)
            Ch32[(size_t)s * p * p + e] = Ctr ? (float)Ctr[(size_t)sh_h[e / p] * n + sh_h[e % p]]
                                              : (float)Ct[(size_t)sh_h[e % p] * n + sh_h[e / p]];
    }
    // Cc and Dd: each wave's lanes merged by halving distance, then the four
    // waves in order (a fixed order)
    if (want_sums) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            pc = pc + __shfl_xor(pc, off);
            pd = pd + __shfl_xor(pd, off);
        }
        if ((tid & 63) == 0) {
            red_c[tid >> 6] = pc;
            red_d[tid >> 6] = pd;
        }
    }
    __syncthreads();
    if (tid == 0) {
        int mx = 0;
        for (int k = 0; k < p; ++k) mx = sh_cnt[k] > mx ? sh_cnt[k] : mx;
        cmax[s] = mx;
        if (want_sums) {
            parts[3 * (size_t)s + 0] = ((red_c[0] + red_c[1]) + red_c[2]) + red_c[3];
            parts[3 * (size_t)s + 2] = ((red_d[0] + red_d[1]) + red_d[2]) + red_d[3];
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
__global__ __launch_bounds__(256, 8) void k_alloc(const int32_t *__restrict__ hubs, int count, int n, int n_pad, int p,
                                               const CT *__restrict__ Ct, const float *__restrict__ Ct32,
                                               const double *__restrict__ O, const double *__restrict__ D,
                                               uint16_t *__restrict__ kidx, double *__restrict__ parts,
                                               int32_t *__restrict__ cmax, float *__restrict__ Ch32, int want_sums,
                                               const double *__restrict__ Ctr)
{
    alloc_body<CT>(hubs, count, n, n_pad, p, Ct, Ct32, O, D, kidx, parts, cmax, Ch32, want_sums, Ctr, blockIdx.x);
}

// Grouped: the children of every context, with their sums and hub tables
// (the split-bf16 generation).
__global__ __launch_bounds__(256, 8) void k_alloc_group(const GroupHdr *__restrict__ hdr,
                                                       const TickJob *__restrict__ jobs)
{
    if ((int)blockIdx.x >= hdr->blocks[kTickAlloc]) return;
    const TickJob &J = jobs[tick_job(jobs, hdr->njobs, kTickAlloc, blockIdx.x)];
    const int blk = blockIdx.x - J.start[kTickAlloc];
    const DevPtrs &P = J.P;
    const Dims &d = J.d;
    if (d.c_f32)
        alloc_body<float>(P.hubs, d.S, d.n, d.n_pad, d.p, (const float *)P.Ct, P.Ct32, P.O, P.D, P.kidx, P.parts,
                          P.cmax, P.Ch32, 1, P.Ctr, blk);
    else
        alloc_body<double>(P.hubs, d.S, d.n, d.n_pad, d.p, (const double *)P.Ct, P.Ct32, P.O, P.D, P.kidx,
                           P.parts, P.cmax, P.Ch32, 1, P.Ctr, blk);
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
                                             kidx, P.parts, P.cmax, ch, want_sums, P.Ctr);
    else
        k_alloc<double><<<grid, 256, 0, st>>>(hubs, count, d.n, d.n_pad, d.p, (const double *)P.Ct, P.Ct32, P.O,
                                              P.D, kidx, P.parts, P.cmax, ch, want_sums, P.Ctr);
    return hipGetLastError();
}

hipError_t launch_alloc_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, int blocks, hipStream_t st)
{
    if (njobs <= 0 || blocks <= 0) return hipSuccess;
    k_alloc_group<<<blocks, 256, 0, st>>>(hdr, jobs);
    return hipGetLastError();
}

}  // namespace hubga
