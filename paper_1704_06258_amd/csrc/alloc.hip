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
#include "ga_ops_dev.hpp"

namespace hubga {

constexpr int kScanHubs = 4;    // hubs per scan chunk
constexpr int kScanNodes = 4;   // nodes per lane scanned together

// LDS of one workgroup; the kernels declare it once, so a kernel that
// instantiates several forms of the body still holds one copy.
struct AllocLds {
    int h[kMaxP];
    __align__(16) int off[kMaxP];   // row offsets h*n in the FP32 copy; padding: row n (+inf)
    int cnt[kMaxP];
    __align__(4) uint8_t pos[kMaxN];   // position of node i in the hub list, 0xFF for spokes
    double red_c[4], red_d[4];
    int lists[3][128];   // the child built here (ops): its parents, then the child
};

// Workgroup blk (of a grid of alloc_blocks(count)) of one context: individual
// s = the workgroup's place in XCD-major order.  A lane takes kScanNodes nodes
// at once and scans the hubs in chunks of kScanHubs: the chunk's distances for
// all its nodes are loaded together, then merged (loads past n re-read valid
// addresses and are not used).  With V = 4 (n a multiple of 4) the lane's
// nodes are consecutive, i = g0 + 4*tid + t, and each hub row is read with one
// 16-byte load; with V = 1 they are i = g0 + t*256 + tid, one 4-byte load each.
// Few registers, so many workgroups share a CU and hide each other's load
// latency.  A node-to-position table in LDS answers "is node i a hub" with one
// read.  With ops.anc set (one generation of a context), wave 0 first builds
// child s from its island's ancestor (the operators, ga_child_wave) while the
// other waves clear that table.
template <typename CT, int V>
__device__ __forceinline__ void alloc_body(AllocLds &L, const AllocOps &ops, const int32_t *hubs, int count, int n,
                                           int n_pad, int p,
                                           const CT *__restrict__ Ct, const float *__restrict__ Ct32,
                                           const double *__restrict__ O, const double *__restrict__ D,
                                           uint16_t *__restrict__ kidx, double *__restrict__ parts,
                                           int32_t *__restrict__ cmax, float *__restrict__ Ch32, int want_sums,
                                           const double *__restrict__ Ctr, int blk)
{
#pragma clang fp contract(off)
    constexpr int T = kScanNodes, H = kScanHubs;
    static_assert(V == 1 || V == T, "a lane's nodes are strided or consecutive");
    int *__restrict__ sh_h = L.h;
    int *__restrict__ sh_off = L.off;
    int *__restrict__ sh_cnt = L.cnt;
    uint8_t *__restrict__ sh_pos = L.pos;
    double *__restrict__ red_c = L.red_c;
    double *__restrict__ red_d = L.red_d;
    // XCD-major order: consecutive individuals (children of one island) run
    // on the same XCD (workgroup index % 8; a grouped launch starts every
    // context on a multiple of 8) and share its L2.
    const int per = (count + 7) / 8;
    const int s = (blk & 7) * per + (blk >> 3);
    if (s >= count) return;
    const int tid = threadIdx.x;
    const bool build = ops.anc != nullptr;
    if (build && s == 0 && tid == 0 && ops.slot_counters[0]) {
        *ops.slot_counters[0] = 0;   // candidate slots of this generation's selection
        *ops.slot_counters[1] = 0;
    }
    // the hub list: loaded (in flight while LDS is cleared), or first built
    // here by wave 0 (the generation's operators for child s)
    int hk = !build && tid < p ? hubs[(size_t)s * p + tid] : n;
    if (build && tid < 64)
        ga_child_wave(ops.anc, ops.children, (uint64_t)*ops.gen, n, p, ops.m, ops.seed, s, &L.lists[0][0]);
    for (int e = tid; e < (n + 3) / 4; e += 256) ((uint32_t *)sh_pos)[e] = 0xFFFFFFFFu;
    if (tid < kMaxP) sh_cnt[tid] = 0;
    __syncthreads();
    if (build && tid < p) hk = L.lists[2][tid];
    if (tid < p) {
        sh_h[tid] = hk;
        sh_pos[hk] = (uint8_t)tid;
    }
    if (tid < kMaxP) sh_off[tid] = hk * n;
    __syncthreads();
    const int nchunks = (p + H - 1) / H;
    // the hub-to-hub table C[h_k][h_l] in FP32 (the FP32 copy holds C rounded
    // to FP32): its first 512 entries are gathered now, in flight during the
    // scan, and stored at the end
    float chv[2];
    if (Ch32) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + q * 256;
            chv[q] = e >= p * p ? 0.0f
                     : Ctr ? (float)Ctr[(size_t)sh_h[e / p] * n + sh_h[e % p]]
                           : Ct32[(size_t)sh_h[e % p] * n + sh_h[e / p]];
        }
    }
    double pc = 0.0, pd = 0.0;
    uint16_t *krow = kidx + (size_t)s * n_pad;
    for (int g0 = 0; g0 < n_pad; g0 += 256 * T) {
        int ii[T], ic[T];   // nodes, and the same clamped to a valid row position
#pragma unroll
        for (int t = 0; t < T; ++t) {
            if constexpr (V == 1) {
                ii[t] = g0 + t * 256 + tid;
                ic[t] = ii[t] < n ? ii[t] : n - 1;
            } else {
                const int i0 = g0 + T * tid;
                ii[t] = i0 + t;
                ic[t] = (i0 < n ? i0 : n - T) + t;
            }
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
            if constexpr (V == 1) {
#pragma unroll
                for (int t = 0; t < T; ++t)
#pragma unroll
                    for (int u = 0; u < H; ++u) X[t][u] = Ct32[off[u] + ic[t]];   // padding hubs read +inf
            } else {
#pragma unroll
                for (int u = 0; u < H; ++u) {
                    const float4 r = *(const float4 *)(Ct32 + off[u] + ic[0]);
                    X[0][u] = r.x;
                    X[1][u] = r.y;
                    X[2][u] = r.z;
                    X[3][u] = r.w;
                }
            }
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
                CT be = Ct[(size_t)sh_h[0] * n + i];
                for (int k = 1; k < p; ++k) {
                    const CT v = Ct[(size_t)sh_h[k] * n + i];
                    if (v < be) {
                        be = v;
                        b = k;
                    }
                }
                best[t] = b;
            }
        }
        // outputs: position, cluster count, and the binary64 terms O_i c_i and
        // D_i c_i in the lane's node order
        if constexpr (V == 1) {
            // two nodes at a time (few registers)
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
        } else {
            // n and n_pad are multiples of 4: a lane's four nodes are all
            // real or all padding
            const int i0 = ii[0];
            if (i0 < n) {
                if (want_sums) {
                    const double2 o01 = *(const double2 *)(O + i0), o23 = *(const double2 *)(O + i0 + 2);
                    const double2 d01 = *(const double2 *)(D + i0), d23 = *(const double2 *)(D + i0 + 2);
                    const double ov[T] = {o01.x, o01.y, o23.x, o23.y}, dv[T] = {d01.x, d01.y, d23.x, d23.y};
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        pc = pc + ov[t] * (double)c32[t];
                        pd = pd + dv[t] * (double)c32[t];
                    }
                }
                uint2 w;
                w.x = (uint32_t)best[0] | ((uint32_t)best[1] << 16);
                w.y = (uint32_t)best[2] | ((uint32_t)best[3] << 16);
                *(uint2 *)(krow + i0) = w;
#pragma unroll
                for (int t = 0; t < T; ++t) atomicAdd(&sh_cnt[best[t]], 1);
            } else if (i0 < n_pad) {
                *(uint2 *)(krow + i0) = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);   // kNoHub
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
                                              : Ct32[(size_t)sh_h[e % p] * n + sh_h[e / p]];
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
    // the largest cluster: wave 0 takes the p counts (p <= 64), one per lane
    if (tid < 64) {
        int mx = tid < p ? sh_cnt[tid] : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const int o = __shfl_xor(mx, off);
            mx = o > mx ? o : mx;
        }
        if (tid == 0) {
            cmax[s] = mx;
            if (want_sums) {
                parts[3 * (size_t)s + 0] = ((red_c[0] + red_c[1]) + red_c[2]) + red_c[3];
                parts[3 * (size_t)s + 2] = ((red_d[0] + red_d[1]) + red_d[2]) + red_d[3];
            }
        }
    }
}

// The consecutive-node form needs whole groups of four nodes, 16-byte rows in
// the FP32 copy and 16-byte (O, D) and 8-byte (positions) aligned vectors.
__host__ __device__ inline bool alloc_vec4(int n, const float *Ct32, const double *O, const double *D,
                                           const uint16_t *kidx)
{
    return n % 4 == 0 && (((uintptr_t)Ct32 | (uintptr_t)O | (uintptr_t)D) & 15) == 0 && ((uintptr_t)kidx & 7) == 0;
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

template <typename CT, int V>
__global__ __launch_bounds__(256, 8) void k_alloc(AllocOps ops, const int32_t *hubs, int count, int n, int n_pad, int p,
                                               const CT *__restrict__ Ct, const float *__restrict__ Ct32,
                                               const double *__restrict__ O, const double *__restrict__ D,
                                               uint16_t *__restrict__ kidx, double *__restrict__ parts,
                                               int32_t *__restrict__ cmax, float *__restrict__ Ch32, int want_sums,
                                               const double *__restrict__ Ctr)
{
    __shared__ AllocLds L;
    alloc_body<CT, V>(L, ops, hubs, count, n, n_pad, p, Ct, Ct32, O, D, kidx, parts, cmax, Ch32, want_sums, Ctr, blockIdx.x);
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
    const bool v4 = alloc_vec4(d.n, P.Ct32, P.O, P.D, P.kidx);
    __shared__ AllocLds L;
    if (d.c_f32) {
        if (v4)
            alloc_body<float, 4>(L, AllocOps{}, P.hubs, d.S, d.n, d.n_pad, d.p, (const float *)P.Ct, P.Ct32, P.O, P.D, P.kidx,
                                 P.parts, P.cmax, P.Ch32, 1, P.Ctr, blk);
        else
            alloc_body<float, 1>(L, AllocOps{}, P.hubs, d.S, d.n, d.n_pad, d.p, (const float *)P.Ct, P.Ct32, P.O, P.D, P.kidx,
                                 P.parts, P.cmax, P.Ch32, 1, P.Ctr, blk);
    } else {
        if (v4)
            alloc_body<double, 4>(L, AllocOps{}, P.hubs, d.S, d.n, d.n_pad, d.p, (const double *)P.Ct, P.Ct32, P.O, P.D, P.kidx,
                                  P.parts, P.cmax, P.Ch32, 1, P.Ctr, blk);
        else
            alloc_body<double, 1>(L, AllocOps{}, P.hubs, d.S, d.n, d.n_pad, d.p, (const double *)P.Ct, P.Ct32, P.O, P.D, P.kidx,
                                  P.parts, P.cmax, P.Ch32, 1, P.Ctr, blk);
    }
}

int alloc_blocks(int count) { return ((count + 7) / 8) * 8; }

hipError_t launch_alloc(const DevPtrs &P, const Dims &d, const int32_t *hubs, int count, uint16_t *kidx,
                        int want_sums, int want_ch, hipStream_t st, const AllocOps &ops)
{
    if (count <= 0) return hipSuccess;
    float *ch = want_ch ? P.Ch32 : nullptr;
    const unsigned grid = (unsigned)alloc_blocks(count);
    const bool v4 = alloc_vec4(d.n, P.Ct32, P.O, P.D, kidx);
#define HUBGA_ALLOC(CT, V)                                                                                      \
    k_alloc<CT, V><<<grid, 256, 0, st>>>(ops, hubs, count, d.n, d.n_pad, d.p, (const CT *)P.Ct, P.Ct32, P.O, P.D, kidx, \
                                         P.parts, P.cmax, ch, want_sums, P.Ctr)
    if (d.c_f32) {
        if (v4) HUBGA_ALLOC(float, 4);
        else HUBGA_ALLOC(float, 1);
    } else {
        if (v4) HUBGA_ALLOC(double, 4);
        else HUBGA_ALLOC(double, 1);
    }
#undef HUBGA_ALLOC
    return hipGetLastError();
}

hipError_t launch_alloc_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, int blocks, hipStream_t st)
{
    if (njobs <= 0 || blocks <= 0) return hipSuccess;
    k_alloc_group<<<blocks, 256, 0, st>>>(hdr, jobs);
    return hipGetLastError();
}

}  // namespace hubga
