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

// ------------------------------------------------- island allocation --
// The children of a generation are their island ancestor with a few hubs
// removed and a few added.  A workgroup takes kIslandKids children of one
// island and 256 nodes: every lane ranks, once, the ancestor's hubs by their
// FP32 distance to its node (the kTop nearest, ties to the lower position),
// and for each child takes the first of them the child kept, then compares it
// with the child's added hubs.  The result is the rule of the paper: a hub
// allocates itself, every other node its nearest hub, ties to the smaller hub
// id.  A node whose ranking has equal FP32 distances, a child with more than
// kMaxAdd added hubs, a child that removed all kTop, and an FP32 tie with an
// added hub take the plain scan in the instance dtype instead.  Each
// workgroup writes its {Cc, Dd} partials per child and node chunk (summed in a
// fixed order by the cost assembly) and adds its cluster sizes into cnt
// (zeroed by the operators).
constexpr int kIslandKids = 16;
constexpr int kTop = 6;
constexpr int kMaxAdd = 8;

__host__ __device__ inline int island_quarters(int m) { return (m + kIslandKids - 1) / kIslandKids; }
__host__ __device__ inline int island_chunks(int n_pad) { return (n_pad + 255) / 256; }
__host__ __device__ inline int island_units(int R, int m, int n_pad) { return R * island_quarters(m) * island_chunks(n_pad); }

template <typename CT>
__device__ __forceinline__ void alloc_island_body(const int32_t *__restrict__ anc, const int32_t *__restrict__ kids,
                                                  int R, int m, int n, int n_pad, int p, const CT *__restrict__ Ct,
                                                  const float *__restrict__ Ct32, const double *__restrict__ O,
                                                  const double *__restrict__ D, uint16_t *__restrict__ kidx,
                                                  double *__restrict__ part_cd, int32_t *__restrict__ cnt,
                                                  float *__restrict__ Ch32, int blk)
{
#pragma clang fp contract(off)
    __shared__ int sA[kMaxP];
    __shared__ int sK[kIslandKids][kMaxP];
    __shared__ unsigned long long sRem[kIslandKids];
    __shared__ int sAdd[kIslandKids][kMaxAdd];
    __shared__ int sNAdd[kIslandKids];
    __shared__ int sCnt[kIslandKids][kMaxP];
    __shared__ double sP[2][kIslandKids][256];
    __shared__ double sSeg[2][kIslandKids][8];
    const int nq = island_quarters(m), nch = island_chunks(n_pad);
    const int units = R * nq * nch;
    const int per = (units + 7) / 8;
    const int u = (blk & 7) * per + (blk >> 3);   // XCD-major: an island's units share one L2
    if (u >= units) return;
    const int c = u % nch, q = (u / nch) % nq, r = u / (nch * nq);
    const int j0 = q * kIslandKids, nk = min(kIslandKids, m - j0);
    const int tid = threadIdx.x;
    const int s0 = r * m + j0;   // first child of this workgroup
    for (int e = tid; e < p; e += 256) sA[e] = anc[(size_t)r * p + e];
    for (int e = tid; e < kIslandKids * kMaxP; e += 256) {
        const int j = e / kMaxP, k = e % kMaxP;
        sCnt[j][k] = 0;
        if (j < nk && k < p) sK[j][k] = kids[(size_t)(s0 + j) * p + k];
    }
    __syncthreads();
    if (tid < nk) {   // merge the sorted lists: removed ancestor positions, added hubs
        unsigned long long rem = 0;
        int na = 0, a = 0, b = 0;
        while (a < p || b < p) {
            const int x = a < p ? sA[a] : 0x7FFFFFFF, y = b < p ? sK[tid][b] : 0x7FFFFFFF;
            if (x == y) {
                ++a;
                ++b;
            } else if (x < y) {
                rem |= 1ull << a;
                ++a;
            } else {
                if (na < kMaxAdd) sAdd[tid][na] = y;
                ++na;
                ++b;
            }
        }
        sRem[tid] = rem;
        sNAdd[tid] = na <= kMaxAdd ? na : -1;
    }
    __syncthreads();

    const int i = c * 256 + tid;
    if (i < n) {
        // the ancestor's kTop nearest hubs (FP32 distance, then position)
        float tv[kTop];
        int tp[kTop];
#pragma unroll
        for (int t = 0; t < kTop; ++t) {
            tv[t] = __builtin_huge_valf();
            tp[t] = -1;
        }
        bool amb = false;
        for (int k0 = 0; k0 < p; k0 += kScanChunk) {
            float v[kScanChunk];
#pragma unroll
            for (int e = 0; e < kScanChunk; ++e)
                v[e] = k0 + e < p ? Ct32[(size_t)sA[k0 + e] * n + i] : __builtin_huge_valf();
#pragma unroll
            for (int e = 0; e < kScanChunk; ++e) {
                if (k0 + e >= p) break;
                float x = v[e];
                int xp = k0 + e;
#pragma unroll
                for (int t = 0; t < kTop; ++t) {
                    amb |= tp[t] >= 0 && x == tv[t];
                    if (x < tv[t]) {   // strict: an equal value stays behind (lower position first)
                        const float fv = tv[t];
                        const int fp = tp[t];
                        tv[t] = x;
                        tp[t] = xp;
                        x = fv;
                        xp = fp;
                    }
                }
            }
        }
        // node i among the ancestor's hubs
        int selfA = -1;
        {
            int lo = 0, hi = p - 1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1, hv = sA[mid];
                if (hv == i) {
                    selfA = mid;
                    break;
                }
                if (hv < i)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
        }
        double ex[kTop];
#pragma unroll
        for (int t = 0; t < kTop; ++t) ex[t] = tp[t] >= 0 ? (double)Ct[(size_t)sA[tp[t]] * n + i] : 0.0;
        const double Oi = O[i], Di = D[i];
        for (int j = 0; j < nk; ++j) {
            const unsigned long long rem = sRem[j];
            const int na = sNAdd[j];
            int wh = -1;          // winning hub id
            double wex = 0.0;     // its exact distance
            bool plain = amb || na < 0;
            if (!plain) {
                if (selfA >= 0 && !((rem >> selfA) & 1ull)) {
                    wh = i;
                } else {
                    for (int e = 0; e < na; ++e)
                        if (sAdd[j][e] == i) wh = i;
                }
                if (wh == i) {
                    wex = (double)Ct[(size_t)i * n + i];
                } else {
                    int t0 = -1;
#pragma unroll
                    for (int t = kTop - 1; t >= 0; --t)
                        if (tp[t] >= 0 && !((rem >> tp[t]) & 1ull)) t0 = t;
                    if (t0 < 0) {
                        plain = true;
                    } else {
                        float wv = tv[0];
                        wex = ex[0];
#pragma unroll
                        for (int t = 1; t < kTop; ++t)
                            if (t == t0) {
                                wv = tv[t];
                                wex = ex[t];
                            }
                        wh = sA[tp[t0]];
                        for (int e = 0; e < na; ++e) {
                            const int h = sAdd[j][e];
                            const float v = Ct32[(size_t)h * n + i];
                            if (v < wv) {
                                wv = v;
                                wh = h;
                                wex = -1.0;   // loaded below
                            } else if (v == wv) {
                                plain = true;
                            }
                        }
                        if (!plain && wex < 0.0) wex = (double)Ct[(size_t)wh * n + i];
                    }
                }
            }
            int pos;
            if (plain) {   // the rule itself: self, else strict minimum in the instance dtype
                pos = -1;
                int lo = 0, hi = p - 1;
                while (lo <= hi) {
                    const int mid = (lo + hi) >> 1, hv = sK[j][mid];
                    if (hv == i) {
                        pos = mid;
                        break;
                    }
                    if (hv < i)
                        lo = mid + 1;
                    else
                        hi = mid - 1;
                }
                if (pos < 0) {
                    pos = 0;
                    CT be = Ct[(size_t)sK[j][0] * n + i];
                    for (int k = 1; k < p; ++k) {
                        const CT v = Ct[(size_t)sK[j][k] * n + i];
                        if (v < be) {
                            be = v;
                            pos = k;
                        }
                    }
                    wex = (double)be;
                } else {
                    wex = (double)Ct[(size_t)i * n + i];
                }
            } else {   // position of the winning hub in the child's sorted list
                int lo = 0, hi = p - 1;
                pos = 0;
                while (lo <= hi) {
                    const int mid = (lo + hi) >> 1, hv = sK[j][mid];
                    if (hv == wh) {
                        pos = mid;
                        break;
                    }
                    if (hv < wh)
                        lo = mid + 1;
                    else
                        hi = mid - 1;
                }
            }
            kidx[(size_t)(s0 + j) * n_pad + i] = (uint16_t)pos;
            atomicAdd(&sCnt[j][pos], 1);
            sP[0][j][tid] = Oi * wex;
            sP[1][j][tid] = Di * wex;
        }
    } else {
        for (int j = 0; j < nk; ++j) {
            if (i < n_pad) kidx[(size_t)(s0 + j) * n_pad + i] = kNoHub;
            sP[0][j][tid] = 0.0;
            sP[1][j][tid] = 0.0;
        }
    }
    __syncthreads();
    // {Cc, Dd} partials of the chunk in a fixed order: 8 segments of 32 nodes
    {
        const int qq = tid >> 7, j = (tid >> 3) & 15, g = tid & 7;
        double acc = 0.0;
        if (j < nk)
            for (int e = 0; e < 32; ++e) acc = acc + sP[qq][j][g * 32 + e];
        sSeg[qq][j][g] = acc;
    }
    if (c == 0)   // FP32 hub-to-hub distances of the children: C[h_k][h_l]
        for (int e = tid; e < nk * p * p; e += 256) {
            const int j = e / (p * p), kl = e % (p * p);
            Ch32[(size_t)(s0 + j) * p * p + kl] = (float)Ct[(size_t)sK[j][kl % p] * n + sK[j][kl / p]];
        }
    __syncthreads();
    if (tid < 2 * nk) {
        const int qq = tid / nk, j = tid % nk;
        double acc = 0.0;
        for (int g = 0; g < 8; ++g) acc = acc + sSeg[qq][j][g];
        part_cd[((size_t)(s0 + j) * nch + c) * 2 + qq] = acc;
    }
    for (int e = tid; e < nk * p; e += 256) {
        const int j = e / p, k = e % p;
        if (sCnt[j][k]) atomicAdd(&cnt[(size_t)(s0 + j) * p + k], sCnt[j][k]);
    }
}

template <typename CT>
__global__ __launch_bounds__(256) void k_alloc_island(const int32_t *__restrict__ anc,
                                                      const int32_t *__restrict__ kids, int R, int m, int n,
                                                      int n_pad, int p, const CT *__restrict__ Ct,
                                                      const float *__restrict__ Ct32, const double *__restrict__ O,
                                                      const double *__restrict__ D, uint16_t *__restrict__ kidx,
                                                      double *__restrict__ part_cd, int32_t *__restrict__ cnt,
                                                      float *__restrict__ Ch32)
{
    alloc_island_body<CT>(anc, kids, R, m, n, n_pad, p, Ct, Ct32, O, D, kidx, part_cd, cnt, Ch32, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_alloc_island_group(const TickJob *__restrict__ jobs, int njobs)
{
    const TickJob &J = jobs[tick_job(jobs, njobs, kTickAlloc, blockIdx.x)];
    const int blk = blockIdx.x - J.start[kTickAlloc];
    const DevPtrs &P = J.P;
    const Dims &d = J.d;
    if (d.c_f32)
        alloc_island_body<float>(P.anc, P.hubs, d.R, d.m, d.n, d.n_pad, d.p, (const float *)P.Ct, P.Ct32, P.O, P.D,
                                 P.kidx, P.part_cd, P.cnt, P.Ch32, blk);
    else
        alloc_island_body<double>(P.anc, P.hubs, d.R, d.m, d.n, d.n_pad, d.p, (const double *)P.Ct, P.Ct32, P.O,
                                  P.D, P.kidx, P.part_cd, P.cnt, P.Ch32, blk);
}

int alloc_island_blocks(const Dims &d) { return ((island_units(d.R, d.m, d.n_pad) + 7) / 8) * 8; }

hipError_t launch_alloc_island(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    const unsigned grid = (unsigned)alloc_island_blocks(d);
    if (d.c_f32)
        k_alloc_island<float><<<grid, 256, 0, st>>>(P.anc, P.hubs, d.R, d.m, d.n, d.n_pad, d.p, (const float *)P.Ct,
                                                    P.Ct32, P.O, P.D, P.kidx, P.part_cd, P.cnt, P.Ch32);
    else
        k_alloc_island<double><<<grid, 256, 0, st>>>(P.anc, P.hubs, d.R, d.m, d.n, d.n_pad, d.p,
                                                     (const double *)P.Ct, P.Ct32, P.O, P.D, P.kidx, P.part_cd,
                                                     P.cnt, P.Ch32);
    return hipGetLastError();
}

hipError_t launch_alloc_island_group(const TickJob *jobs, int njobs, int blocks, hipStream_t st)
{
    if (njobs <= 0 || blocks <= 0) return hipSuccess;
    k_alloc_island_group<<<blocks, 256, 0, st>>>(jobs, njobs);
    return hipGetLastError();
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
