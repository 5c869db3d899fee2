// Exact re-evaluation of the selection candidates, the island decisions and
// the end of the generation, in one launch (Sec. 5; objective (1) of Sec. 3).
//
// Units of work: every candidate with a slot, evaluated column-parallel, and
// every extra candidate, evaluated whole by one workgroup.  A slot's items are
// its 32-column chunks and one item for its sums Cc = sum_i O_i C[i][a_i] and
// Dd = sum_i D_i C[i][a_i].  Inside a column item, lanes 0..31 of wave 0 own
// the columns -- lane l adds t_j, j = j0 + l, over ascending rows i -- while
// four producer waves form the binary64 products W_ij * C[a_i][a_j] of the
// next 64-row tile into a double-buffered LDS ring.  Each producer holds its W
// rows three tiles ahead in registers (bounds-checked buffer loads), and the
// tile hand-over is a bare workgroup barrier, so those loads stay in flight
// across it.  The last item of a slot to finish (device-scope fence, then a
// counter) sums T = sum_j t_j in ascending order and writes the exact cost.
// The last unit to finish decides every island on exact costs and ends the
// generation.
//
// Every addition is one of the sequential definition, in its order, with no
// FMA contraction (rows past n add a zero, which leaves a sum that started at
// +0.0 unchanged: such a sum is never -0.0), so every cost equals the
// sequential binary64 evaluation bit for bit.
#include "kernels.hpp"
#include "exact_dev.hpp"
#include "wave_sync.hpp"

namespace hubga {

constexpr int kRcCols = 32;        // columns of an item, one owner lane each
constexpr int kRcRows = 64;        // rows of a product tile
constexpr int kRcProducers = 4;    // producer waves
constexpr int kRcPairs = kRcRows / 2 / kRcProducers;   // row pairs of a tile per producer lane
constexpr int kRcThreads = 64 * (1 + kRcProducers);
constexpr size_t kRcRing = (size_t)2 * kRcRows * kRcCols * 8;   // two tiles of binary64 products
constexpr int kRcChain = 1024;     // values per LDS-staged chunk of a candidate sum
static_assert(kRcPairs == 8, "a producer lane forms 8 row pairs of a tile (two 16-byte reads of positions)");
// Word 3 of a gfx9 buffer resource for untyped 32-bit-element access; loads
// past num_records return zero and touch no memory.
constexpr int kBufWord3 = 0x00020000;
static_assert((size_t)3 * kRcChain * 8 <= kRcRing, "the three sums are staged in the ring");

__host__ __device__ inline int rc_chunks(int n) { return (n + kRcCols - 1) / kRcCols; }
// Items of a slot: its column chunks, then one for its sums Cc and Dd.
__host__ __device__ inline int rc_slot_items(int n) { return rc_chunks(n) + 1; }
__host__ __device__ inline int rc_tiles(int n) { return (n + kRcRows - 1) / kRcRows; }

// LDS of a column item: the ring, chT ((p + 1) x 32 binary64 distances), the
// hub positions of tiles*64 rows.
__host__ __device__ inline size_t rc_item_lds(int n, int p)
{
    return kRcRing + (size_t)(p + 1) * kRcCols * 8 + (size_t)rc_tiles(n) * kRcRows * 2;
}

size_t recheck_lds(int n, int p)
{
    const size_t a = rc_item_lds(n, p), b = exact_smem_bytes(n, p);
    return a > b ? a : b;
}

// What one re-evaluation reads and where it writes.
struct RcView {
    const int32_t *children;   // hub lists, p per child
    const uint16_t *kidx;      // hub positions, n_pad per child
    int m;                     // candidates per island: output o = r*m + c
    double *cost_out;          // scaled exact cost at o
    double *parts_out;         // {Cc, T, Dd} at 3o
    int decide;                // the last unit decides the islands and ends the generation
};

__host__ __device__ inline RcView rc_generation_view(const DevPtrs &P, const Dims &d)
{
    RcView v;
    v.children = P.hubs;
    v.kidx = P.kidx;
    v.m = d.m;
    v.cost_out = P.cand_cost;
    v.parts_out = P.cand_parts;
    v.decide = 1;
    return v;
}

// acc + buf[0] + buf[1] + ... + buf[cnt-1], left to right (one lane; buf
// 16-byte aligned, cnt <= kRcChain values of capacity).  Two register sets of
// 16 values take turns: one is added while the other's reads are in flight;
// the reads ahead stay inside the buffer (clamped), so no set is loaded on
// one path only.
__device__ inline double chain_sum(double acc, const double *buf, int cnt)
{
#pragma clang fp contract(off)
    const double2 *b2 = (const double2 *)buf;
    double2 A[8], B[8];
    auto load = [&](double2(&X)[8], int at) {
        at = at < kRcChain - 16 ? at : kRcChain - 16;
#pragma unroll
        for (int u = 0; u < 8; ++u) X[u] = b2[at / 2 + u];
        asm volatile("" ::: "memory");   // the reads are issued here, ahead of the adds that follow
    };
    auto add = [&](const double2(&X)[8]) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            acc = acc + X[u].x;
            acc = acc + X[u].y;
        }
    };
    load(A, 0);
    int i = 0;
    for (; i + 32 <= cnt; i += 32) {
        load(B, i + 16);
        add(A);
        load(A, i + 32);
        add(B);
    }
    if (i + 16 <= cnt) {   // A holds buf[i .. i+15]
        add(A);
        i += 16;
    }
    for (; i < cnt; ++i) acc = acc + buf[i];
    return acc;
}

// Loads of one W element (byte offset; zero past the end of W).
template <typename WT>
__device__ __forceinline__ WT rc_wload1(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ double rc_wload1<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float rc_wload1<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// LDS of an item: the ring, chT ((p + 1) x 32 binary64 distances), the hub
// positions of tiles*64 rows (rows past n: position p).
struct RcLds {
    double *ring;
    double *chT;
    uint16_t *kid;
};
__device__ __forceinline__ RcLds rc_lds(char *smem, int p)
{
    RcLds L;
    L.ring = (double *)smem;
    L.chT = (double *)(smem + kRcRing);
    L.kid = (uint16_t *)(L.chT + (size_t)(p + 1) * kRcCols);
    return L;
}

// The candidate of a slot into LDS: hub list (sh_h) and hub positions.
__device__ __forceinline__ void rc_stage_candidate(const Dims &d, const RcView &V, int s, const RcLds &L, int *sh_h)
{
    const int n = d.n, p = d.p, nt = rc_tiles(n), tid = threadIdx.x;
    if (tid < p) sh_h[tid] = V.children[(size_t)s * p + tid];
    const uint16_t *krow = V.kidx + (size_t)s * d.n_pad;
    for (int e = tid * 8; e < nt * kRcRows; e += kRcThreads * 8)   // n_pad >= nt*64; rows are 256-byte aligned
        *(uint4 *)(L.kid + e) = *(const uint4 *)(krow + e);
    __syncthreads();
    for (int i = n + tid; i < nt * kRcRows; i += kRcThreads) L.kid[i] = (uint16_t)p;
}

// The slot's item is done: device-scope fence, then the slot counter.  True
// in the workgroup that finished the slot's last item.
__device__ __forceinline__ bool rc_item_done(const DevPtrs &P, int slot, int items)
{
    __shared__ int sh_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        sh_last = atomicAdd(&P.slot_done[slot], 1) == items - 1;
        if (sh_last) atomicExch(&P.slot_done[slot], 0);
    }
    __syncthreads();
    if (sh_last) __threadfence();
    return sh_last != 0;
}

// Column item (slot, chunk): t_j for the chunk's columns into tbuf.
template <typename CT, typename WT>
__device__ __forceinline__ void rc_column_item(const DevPtrs &P, const Dims &d, const RcView &V, int slot, int chunk,
                                               char *smem, int *sh_h)
{
#pragma clang fp contract(off)
    const int n = d.n, p = d.p, nt = rc_tiles(n);
    const int tid = threadIdx.x, lane = tid & 63, col = lane & 31, half = lane >> 5;
    const int pw = __builtin_amdgcn_readfirstlane(tid >> 6) - 1;   // producer number (wave-uniform); -1: the owner
    const RcLds L = rc_lds(smem, p);   // ring: [2 tiles][32 row pairs][32 columns][2 rows]
    const int j0 = chunk * kRcCols, j = j0 + col, jc = j < n ? j : n - 1;
    __syncthreads();   // LDS of the previous item free

    // A producer lane forms column j0 + col of rows 2v + half of its row pairs
    // v = 8 pw .. 8 pw + 7 of every tile.  W rows of the first three tiles are
    // loaded first (they do not depend on the candidate).  Rows past n read
    // zero, and their hub position p has a zero chT row.
    const __amdgpu_buffer_rsrc_t wr =
        __builtin_amdgcn_make_buffer_rsrc((void *)P.W, (short)0, (int)((size_t)n * n * sizeof(WT)), kBufWord3);
    const uint32_t rstep = 2u * (uint32_t)n * (uint32_t)sizeof(WT);
    WT w0[kRcPairs], w1[kRcPairs], w2[kRcPairs];
    auto wload = [&](int k, WT(&w)[kRcPairs]) {   // this lane's rows of tile k
        uint32_t off = ((uint32_t)(k * kRcRows + pw * 2 * kRcPairs + half) * (uint32_t)n + (uint32_t)jc) *
                       (uint32_t)sizeof(WT);
#pragma unroll
        for (int u = 0; u < kRcPairs; ++u) {
            w[u] = rc_wload1<WT>(wr, off);
            off += rstep;
        }
    };
    if (pw >= 0) {
        wload(0, w0);
        wload(1, w1);
        wload(2, w2);
    }
    rc_stage_candidate(d, V, P.slot_s[slot], L, sh_h);
    for (int e = tid; e < (p + 1) * kRcCols; e += kRcThreads) {   // chT[k][c] = C[h_k][a_j], j = j0 + c; row p zero
        const int k = e / kRcCols, jj = j0 + e % kRcCols < n ? j0 + e % kRcCols : n - 1;
        const size_t at = (size_t)sh_h[k < p ? k : 0] * n + sh_h[L.kid[jj]];
        L.chT[e] = k < p ? (P.Ctr ? P.Ctr[at] : (double)((const CT *)P.C)[at]) : 0.0;
    }
    lds_wait();
    wg_barrier();

    // producers: tile k's products W_ij * C[a_i][a_j]
    auto produce = [&](int k, const WT(&w)[kRcPairs]) {
        const int i0 = k * kRcRows + pw * 2 * kRcPairs;   // positions of rows i0 .. i0+15, a pair per word
        const uint4 k0 = *(const uint4 *)(L.kid + i0), k1 = *(const uint4 *)(L.kid + i0 + 8);
        const uint32_t kw[kRcPairs] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
        double c[kRcPairs];
#pragma unroll
        for (int u = 0; u < kRcPairs; ++u) c[u] = L.chT[((kw[u] >> (16 * half)) & 0xFFFFu) * kRcCols + col];
        double *dst = L.ring + (((size_t)(k & 1) * (kRcRows / 2) + pw * kRcPairs) * kRcCols + col) * 2 + half;
#pragma unroll
        for (int u = 0; u < kRcPairs; ++u) dst[u * kRcCols * 2] = (double)w[u] * c[u];
    };
    // owner (lanes 0..31): acc + tile k's 64 products of column j, ascending rows
    double acc = 0.0;
    auto consume = [&](int k) {
        const double2 *src = (const double2 *)L.ring + (size_t)(k & 1) * (kRcRows / 2) * kRcCols + col;
        double2 cur[8], nxt[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) cur[u] = src[u * kRcCols];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            if (g < 3) {
#pragma unroll
                for (int u = 0; u < 8; ++u) nxt[u] = src[((g + 1) * 8 + u) * kRcCols];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                acc = acc + cur[u].x;
                acc = acc + cur[u].y;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) cur[u] = nxt[u];
        }
    };
    // Step k: the owner adds tile k while the producers form tile k+1 (from
    // register set (k+1) % 3, then refilled with tile k+4).  Owner and
    // producers run loops of their own with the same barriers, one after
    // tile 0 and one per step; the producers' loop runs whole groups of three
    // steps, so the owner's runs as many, idle past the last tile.
    const int steps = 3 * ((nt + 2) / 3);
    if (pw < 0) {
        lds_wait();
        wg_barrier();
        for (int k = 0; k < steps; ++k) {
            if (k < nt && half == 0) consume(k);
            lds_wait();
            wg_barrier();
        }
        if (half == 0 && j < n) P.tbuf[(size_t)slot * n + j] = acc;
    } else {
        produce(0, w0);
        wload(3, w0);
        lds_wait();
        wg_barrier();
        auto step = [&](int k, WT(&w)[kRcPairs]) {
            if (k + 1 < nt) produce(k + 1, w);
            wload(k + 4, w);
            lds_wait();
            wg_barrier();
        };
        for (int k = 0; k < steps; k += 3) {
            step(k, w1);
            step(k + 1, w2);
            step(k + 2, w0);
        }
    }
}

// Ascending sums of up to three n-vectors, lane 0 of wave v adding vector v
// (bit v of MASK): T = sum_j t_j (tbuf), Cc terms O_i * C[i][a_i], Dd terms
// D_i * C[i][a_i].  Chunks are staged in the LDS ring by every lane, all loads
// of a round issued before its LDS writes.  Results in sums[v].
template <typename CT, int MASK>
__device__ __forceinline__ void rc_sums(const DevPtrs &P, const Dims &d, int slot, const RcLds &L, const int *sh_h,
                                        double *sums)
{
#pragma clang fp contract(off)
    const int n = d.n, tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    double *bt = L.ring, *bc = bt + kRcChain, *bd = bc + kRcChain;
    const double *t = P.tbuf + (size_t)slot * n;
    const CT *C = (const CT *)P.C;
    double acc = 0.0;
    for (int i0 = 0; i0 < n; i0 += kRcChain) {
        const int cnt = n - i0 < kRcChain ? n - i0 : kRcChain;
        for (int q0 = 0; q0 < cnt; q0 += 4 * kRcThreads) {
            double tv[4], cv[4], ov[4], dv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * kRcThreads + tid, i = i0 + (q < cnt ? q : cnt - 1);
                if (MASK & 1) tv[u] = t[i];
                if (MASK & 6) cv[u] = (double)C[(size_t)i * n + sh_h[L.kid[i]]];
                if (MASK & 2) ov[u] = P.O[i];
                if (MASK & 4) dv[u] = P.D[i];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * kRcThreads + tid;
                if (q < cnt) {
                    if (MASK & 1) bt[q] = tv[u];
                    if (MASK & 2) bc[q] = ov[u] * cv[u];
                    if (MASK & 4) bd[q] = dv[u] * cv[u];
                }
            }
        }
        __syncthreads();
        if (lane == 0 && wave < 3 && ((MASK >> wave) & 1))
            acc = chain_sum(acc, wave == 0 ? bt : (wave == 1 ? bc : bd), cnt);
        __syncthreads();
    }
    if (lane == 0 && wave < 3 && ((MASK >> wave) & 1)) sums[wave] = acc;
    __syncthreads();
}

// Sums item of a slot: Cc and Dd into the candidate's parts.
template <typename CT>
__device__ __forceinline__ void rc_ccdd_item(const DevPtrs &P, const Dims &d, const RcView &V, int slot, char *smem,
                                             int *sh_h)
{
    __shared__ double sums[3];
    const RcLds L = rc_lds(smem, d.p);
    __syncthreads();   // LDS of the previous item free
    rc_stage_candidate(d, V, P.slot_s[slot], L, sh_h);
    __syncthreads();
    rc_sums<CT, 6>(P, d, slot, L, sh_h, sums);
    if (threadIdx.x == 0) {
        const size_t o = (size_t)P.slot_r[slot] * V.m + P.slot_c[slot];
        V.parts_out[3 * o + 0] = sums[1];
        V.parts_out[3 * o + 2] = sums[2];
    }
}

// The slot's last item: T, then the cost from Cc and Dd of the sums item.
template <typename CT>
__device__ __forceinline__ void rc_finish_slot(const DevPtrs &P, const Dims &d, const RcView &V, int slot, char *smem,
                                               const int *sh_h)
{
#pragma clang fp contract(off)
    __shared__ double sums[3];
    const RcLds L = rc_lds(smem, d.p);
    size_t o = 0;
    double Cc = 0.0, Dd = 0.0;
    if (threadIdx.x == 0) {   // read while T is summed
        o = (size_t)P.slot_r[slot] * V.m + P.slot_c[slot];
        Cc = V.parts_out[3 * o + 0];
        Dd = V.parts_out[3 * o + 2];
    }
    rc_sums<CT, 1>(P, d, slot, L, sh_h, sums);
    if (threadIdx.x == 0) {
        const double T = sums[0];
        V.cost_out[o] = (((d.chi * Cc) + (d.alpha * T)) + (d.delta * Dd)) * d.scale;
        V.parts_out[3 * o + 1] = T;
    }
}

// Item c of a slot (c < chunks: a column chunk; c == chunks: the sums);
// the slot's last item finishes it.  True when the slot was finished here.
template <typename CT, typename WT>
__device__ __forceinline__ bool rc_slot_item(const DevPtrs &P, const Dims &d, const RcView &V, int slot, int c,
                                             char *smem, int *sh_h)
{
    if (c < rc_chunks(d.n))
        rc_column_item<CT, WT>(P, d, V, slot, c, smem, sh_h);
    else
        rc_ccdd_item<CT>(P, d, V, slot, smem, sh_h);
    if (!rc_item_done(P, slot, rc_slot_items(d.n))) return false;
    rc_finish_slot<CT>(P, d, V, slot, smem, sh_h);
    return true;
}

// A unit (slot or extra candidate) is done: the last one decides.
__device__ inline void rc_unit_done(const DevPtrs &P, const Dims &d, const RcView &V, int units)
{
    if (last_block(P.sync + 1, units) && V.decide) decide_generation(make_sel_state(P, d), P.choice);
}

// Extra candidate e, evaluated whole.
template <typename CT, typename WT>
__device__ __forceinline__ void rc_extra(const DevPtrs &P, const Dims &d, const RcView &V, int e, char *smem)
{
    const int r = P.extra_r[e], c = P.extra_c[e];
    const int s = P.cand[(size_t)r * V.m + c];
    const size_t o = (size_t)r * V.m + c;
    __syncthreads();   // LDS of the previous item free
    eval_exact_body<CT, WT, 2>(V.children + (size_t)s * d.p, V.kidx + (size_t)s * d.n_pad, d.n, d.p, (const CT *)P.C,
                            P.Ctr, (const WT *)P.W, P.O, P.D, d.chi, d.alpha, d.delta, d.scale, V.cost_out + o,
                            V.parts_out + 3 * o, smem);
}

// Workgroup blk of nblk (a multiple of 8) on one context.  With eight or more
// items per slot, item c of every slot runs on XCD c % 8, so the slots share
// that column strip of W in one L2.
template <typename CT, typename WT>
__device__ __forceinline__ void rc_body(const DevPtrs &P, const Dims &d, const RcView &V, char *smem, int blk, int nblk)
{
    __shared__ int sh_h[kMaxP];
    const int total = *P.total, nextra = *P.nextra, units = total + nextra;
    const int nch = rc_slot_items(d.n);
    if (units == 0) {
        if (blk == 0 && V.decide) decide_generation(make_sel_state(P, d), P.choice);
        return;
    }
    auto column = [&](int slot, int c) {
        if (rc_slot_item<CT, WT>(P, d, V, slot, c, smem, sh_h)) rc_unit_done(P, d, V, units);
    };
    if (nch >= 8) {
        const int x = blk & 7, q = blk >> 3, nq = nblk >> 3;
        const int a = (nch - x + 7) / 8;   // chunks x, x + 8, ...
        for (int li = q; li < a * total; li += nq) column(li % total, x + 8 * (li / total));
    } else {
        for (int g = blk; g < nch * total; g += nblk) column(g / nch, g % nch);
    }
    for (int e = blk; e < nextra; e += nblk) {
        rc_extra<CT, WT>(P, d, V, e, smem);
        rc_unit_done(P, d, V, units);
    }
}

template <typename CT, typename WT>
__global__ __launch_bounds__(kRcThreads, 3) void k_recheck(DevPtrs P, Dims d, RcView V)
{
    extern __shared__ __align__(16) char smem[];
    rc_body<CT, WT>(P, d, V, smem, blockIdx.x, gridDim.x);
}

// Grouped re-evaluation (split-bf16 generations of several contexts): the
// items of all contexts, concatenated in context order, form one pool shared
// by every workgroup of the launch.  A context without candidates has one
// item, its decision.

// Exclusive prefix of one count per context (njobs <= kMaxPoolJobs = 4 x 64):
// pre[j] = items of the contexts before j; returns all items.  Wave 0 scans,
// four contexts per lane.
template <typename F>
__device__ inline int pool_prefix(int njobs, F count, int *pre)
{
    static_assert(kMaxPoolJobs == 4 * 64, "four contexts per lane of one wave");
    const int tid = threadIdx.x;
    if (tid < 64) {
        int v[4], sum = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * tid + u;
            v[u] = j < njobs ? count(j) : 0;
            sum += v[u];
        }
        int incl = sum;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off);
            if (tid >= off) incl += t;
        }
        int e = incl - sum;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pre[4 * tid + u] = e;
            e += v[u];
        }
        if (tid == 63) pre[kMaxPoolJobs] = incl;
    }
    __syncthreads();
    return pre[njobs];
}

__device__ inline int pool_job(const int *pre, int njobs, int g)   // last j with pre[j] <= g
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ inline int rc_items(const TickJob &J)
{
    const int u = *J.P.total * rc_slot_items(J.d.n) + *J.P.nextra;
    return u > 0 ? u : 1;
}

template <typename CT, typename WT>
__device__ __forceinline__ void rc_group_item(const TickJob &J, int item, char *smem, int *sh_h)
{
    const DevPtrs &P = J.P;
    const Dims &d = J.d;
    const RcView V = rc_generation_view(P, d);
    const int total = *P.total, units = total + *P.nextra, nch = rc_slot_items(d.n);
    if (units == 0) {
        decide_generation(make_sel_state(P, d), P.choice);
    } else if (item < total * nch) {
        if (rc_slot_item<CT, WT>(P, d, V, item % total, item / total, smem, sh_h)) rc_unit_done(P, d, V, units);
    } else {
        rc_extra<CT, WT>(P, d, V, item - total * nch, smem);
        rc_unit_done(P, d, V, units);
    }
}

__global__ __launch_bounds__(kRcThreads) void k_recheck_group(const GroupHdr *__restrict__ hdr,
                                                              const TickJob *__restrict__ jobs)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int pre[kMaxPoolJobs + 1];
    __shared__ int sh_h[kMaxP];
    const int njobs = hdr->njobs;
    const int items = pool_prefix(njobs, [&](int j) { return rc_items(jobs[j]); }, pre);
    for (int g = blockIdx.x; g < items; g += gridDim.x) {
        const int j = pool_job(pre, njobs, g);
        const TickJob &J = jobs[j];
        const int item = g - pre[j];
        if (J.d.c_f32) {
            if (J.d.w_f32) rc_group_item<float, float>(J, item, smem, sh_h);
            else rc_group_item<float, double>(J, item, smem, sh_h);
        } else {
            if (J.d.w_f32) rc_group_item<double, float>(J, item, smem, sh_h);
            else rc_group_item<double, double>(J, item, smem, sh_h);
        }
    }
}

// The exact cost of the single solution in best (P0 of Sec. 4.1) through the
// same column-parallel path, as one slot: the result is the sequential
// definition, bit for bit, in best_cost (cost, then Cc, T, Dd).  The slot
// arrays are unused before the first generation.
__global__ void k_p0_index(DevPtrs P)
{
    if (threadIdx.x == 0) {
        P.cand[0] = P.slot_r[0] = P.slot_c[0] = P.slot_s[0] = 0;
        *P.total = 1;
        *P.nextra = 0;
        P.slot_done[0] = 0;
        P.sync[1] = 0;
    }
}

template <typename CT, typename WT>
static hipError_t rc_launch(const DevPtrs &P, const Dims &d, const RcView &V, hipStream_t st)
{
    k_recheck<CT, WT><<<kRecheckBlocks, kRcThreads, recheck_lds(d.n, d.p), st>>>(P, d, V);
    return hipGetLastError();
}

static hipError_t rc_dispatch(const DevPtrs &P, const Dims &d, const RcView &V, hipStream_t st)
{
    if (d.c_f32 && d.w_f32) return rc_launch<float, float>(P, d, V, st);
    if (d.c_f32) return rc_launch<float, double>(P, d, V, st);
    if (d.w_f32) return rc_launch<double, float>(P, d, V, st);
    return rc_launch<double, double>(P, d, V, st);
}

hipError_t launch_recheck(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    return rc_dispatch(P, d, rc_generation_view(P, d), st);
}

hipError_t launch_p0_exact(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    k_p0_index<<<1, 64, 0, st>>>(P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    RcView V;
    V.children = P.best;
    V.kidx = P.kidx_one;
    V.m = 1;
    V.cost_out = P.best_cost;
    V.parts_out = P.best_cost + 1;
    V.decide = 0;
    return rc_dispatch(P, d, V, st);
}

hipError_t launch_recheck_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, size_t lds, hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    if (njobs > kMaxPoolJobs) return hipErrorInvalidValue;
    k_recheck_group<<<kRecheckBlocks, kRcThreads, lds, st>>>(hdr, jobs);
    return hipGetLastError();
}

static size_t g_group_lds_cap = 0;   // dynamic LDS limit of k_recheck_group

size_t recheck_group_lds_cap() { return g_group_lds_cap; }

// Raise the dynamic-LDS caps, once per process (never during graph capture).
hipError_t prepare_recheck_kernels(int max_lds)
{
    const void *fns[] = {(const void *)k_recheck<double, double>, (const void *)k_recheck<double, float>,
                         (const void *)k_recheck<float, double>, (const void *)k_recheck<float, float>,
                         (const void *)k_recheck_group};
    for (const void *f : fns) {
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, f);
        if (e != hipSuccess) return e;
        const int dyn = max_lds - (int)fa.sharedSizeBytes;   // the cap excludes the kernel's static LDS
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        if (e != hipSuccess) return e;
        if (f == (const void *)k_recheck_group) g_group_lds_cap = (size_t)dyn;
    }
    return hipSuccess;
}

}  // namespace hubga
