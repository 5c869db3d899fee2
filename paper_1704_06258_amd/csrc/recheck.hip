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
// Bursts of candidates (every island has one or more in the first
// generations) go to a second kernel, k_recheck_wide, launched after this
// one; each returns at once unless the number of slots in use is in its
// range (the wide one from kRcWideMin slots).  A column item there is 64
// columns of four slots: wave w owns slot 4g + w, each lane one column, and
// adds its own products, its candidate's p x p distances in LDS.  The four
// waves read the same W values, which the whole workgroup moves into a
// double-buffered LDS ring 16 rows at a time, the next kRwDepth such stages
// in flight in registers (a quarter of each stage per thread).  W is then
// read once per four slots, not once per slot, and column chunk c goes to
// XCD c mod 8, so the four-slot groups on an XCD share its chunks in L2.
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

constexpr int kRcWideThreads = 256;   // the wide kernel's workgroup: four waves
constexpr int kRwSlots = 4;            // slots of a wide column item, one per wave
constexpr int kRwCols = 64;            // its columns, one per lane
constexpr int kRwRows = 32;            // W rows of a ring stage
constexpr int kRwDepth = 4;            // stages in flight in registers
constexpr int kRwSum = 1024;           // tbuf values a wave stages at a time to sum a slot's T
constexpr int kRcWideMin = 24;         // slots in use from which the wide kernel takes a launch
constexpr int kRcWideBlocks = 512;     // its persistent workgroups (two to a CU fit)
// Wide item LDS: the W ring (two stages of binary64 or FP32 values), the
// stages' hub positions ([2][slot][row]), then the four slots' p x p tables.
constexpr size_t kRwRing = (size_t)2 * kRwRows * kRwCols * 8;
constexpr size_t kRwPos = (size_t)2 * kRwSlots * kRwRows * 2;

constexpr int kRwMaxP = 56;            // largest p whose four tables fit a wide item's LDS

// The wide kernel serves a launch with at least kRcWideMin slots in use when
// its LDS holds p; the narrow one serves every other.
__host__ __device__ inline bool rc_wide(int total, int p) { return total >= kRcWideMin && p <= kRwMaxP; }
__host__ __device__ inline int rc_chunks(int n) { return (n + kRcCols - 1) / kRcCols; }
__host__ __device__ inline int rc_wide_chunks(int n) { return (n + kRwCols - 1) / kRwCols; }
// Items of a slot: its column chunks, then one for its sums Cc and Dd (both
// kernels; a wide column item counts once for each of its slots).
__host__ __device__ inline int rc_slot_items(int n, bool wide) { return (wide ? rc_wide_chunks(n) : rc_chunks(n)) + 1; }
__host__ __device__ inline int rc_tiles(int n) { return (n + kRcRows - 1) / kRcRows; }
__host__ __device__ inline size_t rc_wide_item_lds(int p)
{
    const size_t item = kRwRing + kRwPos + (size_t)kRwSlots * p * p * 8, sum = (size_t)kRwSlots * kRwSum * 8;
    return item > sum ? item : sum;
}

// LDS of a column item: the ring, chT ((p + 1) x 32 binary64 distances), the
// hub positions of tiles*64 rows.
__host__ __device__ inline size_t rc_item_lds(int n, int p)
{
    return kRcRing + (size_t)(p + 1) * kRcCols * 8 + (size_t)rc_tiles(n) * kRcRows * 2;
}

// Dynamic LDS of the narrow kernel (its items or a whole-candidate
// evaluation) and of the wide one (its column items, its sums items or a
// whole-candidate evaluation).
size_t recheck_lds(int n, int p)
{
    const size_t a = rc_item_lds(n, p), b = exact_smem_bytes(n, p);
    return a > b ? a : b;
}
size_t recheck_wide_lds(int n, int p)
{
    if (p > kRwMaxP) return 0;   // never the wide kernel's: it returns at once
    const size_t a = rc_wide_item_lds(p), b = exact_smem_bytes(n, p);
    const size_t c = (size_t)3 * kRcChain * 8 + (size_t)rc_tiles(n) * kRcRows * 2;
    const size_t ab = a > b ? a : b;
    return ab > c ? ab : c;
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
// 16-byte aligned, cnt <= CAP values of capacity).  SETS (2 or 3) register
// sets of 16 values take turns: while one is added, the reads of the others
// are in flight (three sets hide a longer LDS latency, for 32 more
// registers).  The reads ahead stay inside the buffer (clamped), so no set is
// loaded on one path only; a clamped set is never added.
template <int CAP = kRcChain, int SETS = 2>
__device__ inline double chain_sum(double acc, const double *buf, int cnt)
{
#pragma clang fp contract(off)
    static_assert(SETS == 2 || SETS == 3, "two or three register sets");
    const double2 *b2 = (const double2 *)buf;
    double2 A[8], B[8], C[8];
    auto load = [&](double2(&X)[8], int at) {
        at = at < CAP - 16 ? at : CAP - 16;
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
    if constexpr (SETS == 3) {
        load(B, 16);
        for (; i + 48 <= cnt; i += 48) {
            load(C, i + 32);
            add(A);
            load(A, i + 48);
            add(B);
            load(B, i + 64);
            add(C);
        }
        if (i + 16 <= cnt) {   // A and B hold buf[i .. i+31]
            add(A);
            i += 16;
            if (i + 16 <= cnt) {
                add(B);
                i += 16;
            }
        }
    } else {
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
// The wide kernel's sums items use only the three staged chunks of the ring
// and no chT: its layout is the ring's first 3 x kRcChain values, then kid.
template <bool WIDE = false>
__device__ __forceinline__ RcLds rc_lds(char *smem, int p)
{
    RcLds L;
    L.ring = (double *)smem;
    L.chT = (double *)(smem + (WIDE ? (size_t)3 * kRcChain * 8 : kRcRing));
    L.kid = WIDE ? (uint16_t *)L.chT : (uint16_t *)(L.chT + (size_t)(p + 1) * kRcCols);
    return L;
}

// The candidate of a slot into LDS: hub list (sh_h) and hub positions.
__device__ __forceinline__ void rc_stage_candidate(const Dims &d, const RcView &V, int s, const RcLds &L, int *sh_h)
{
    const int n = d.n, p = d.p, nt = rc_tiles(n), tid = threadIdx.x;
    if (tid < p) sh_h[tid] = V.children[(size_t)s * p + tid];
    const uint16_t *krow = V.kidx + (size_t)s * d.n_pad;
    const int nth = blockDim.x;
    for (int e = tid * 8; e < nt * kRcRows; e += nth * 8)   // n_pad >= nt*64; rows are 256-byte aligned
        *(uint4 *)(L.kid + e) = *(const uint4 *)(krow + e);
    __syncthreads();
    for (int i = n + tid; i < nt * kRcRows; i += nth) L.kid[i] = (uint16_t)p;
}

// An item is done for slots s0 .. s0 + k - 1: one device-scope release,
// then each slot's counter.  Bit w of the result is set where this workgroup
// finished slot s0 + w's last item (it then holds an acquire).
__device__ __forceinline__ unsigned rc_items_done(const DevPtrs &P, int s0, int k, int items)
{
    __shared__ unsigned sh_mask;
    __syncthreads();
    if (threadIdx.x == 0) {
        release_agent();
        unsigned m = 0;
        for (int w = 0; w < k; ++w)
            if (atomicAdd(&P.slot_done[s0 + w], 1) == items - 1) {
                atomicExch(&P.slot_done[s0 + w], 0);
                m |= 1u << w;
            }
        sh_mask = m;
    }
    __syncthreads();
    const unsigned m = sh_mask;
    if (m) acquire_agent();
    return m;
}
__device__ __forceinline__ bool rc_item_done(const DevPtrs &P, int slot, int items)
{
    return rc_items_done(P, slot, 1, items) != 0;
}

// The wide kernel's completion counters: slot s counts in 16-bit field s % 4
// of the 64-bit word s / 4 over slot_done (zero between launches, as the
// narrow kernel's per-slot counters), so an item of four slots is one
// atomic.  The slots s0 + w (s0 a multiple of 4) whose bit w is set in
// fields had an item done; bit w of the result is set where this workgroup
// did the slot's last one (it then holds an acquire).
__device__ __forceinline__ unsigned rc_group_done(const DevPtrs &P, int s0, unsigned fields, int items)
{
    __shared__ unsigned sh_mask;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long add = 0;
        for (int w = 0; w < kRwSlots; ++w)
            if ((fields >> w) & 1u) add += 1ull << (16 * w);
        unsigned long long *word = (unsigned long long *)P.slot_done + s0 / kRwSlots;
        release_agent();
        const unsigned long long old = atomicAdd(word, add);
        unsigned m = 0;
        unsigned long long clear = 0;
        for (int w = 0; w < kRwSlots; ++w)
            if (((fields >> w) & 1u) && (int)((old >> (16 * w)) & 0xffffu) == items - 1) {
                m |= 1u << w;
                clear |= 0xffffull << (16 * w);
            }
        if (m) atomicAnd(word, ~clear);
        sh_mask = m;
    }
    __syncthreads();
    const unsigned m = sh_mask;
    if (m) acquire_agent();
    return m;
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

// Wide column item (group g, chunk c): t_j for columns 64c .. 64c + 63 of
// slots 4g .. 4g + 3 (those below total) into tbuf.  Workgroup of
// kRcWideThreads; wave w adds slot 4g + w.  VEC: W rows are 16-byte aligned
// (n * sizeof(WT) a multiple of 16, n >= 64), so a stage moves in 16-byte
// pieces.
template <typename CT, typename WT, bool VEC>
__device__ __forceinline__ void rc_column_item_wide(const DevPtrs &P, const Dims &d, const RcView &V, int total,
                                                    int g, int chunk, char *smem)
{
#pragma clang fp contract(off)
    constexpr int EPC = 16 / (int)sizeof(WT);          // elements of a 16-byte piece
    constexpr int CPR = kRwCols / EPC;                 // pieces of a stage row
    constexpr int NPC = kRwRows * CPR / kRcWideThreads;   // pieces per thread and stage (VEC)
    constexpr int NQ = kRwRows / 4;                    // elements per thread and stage (else)
    constexpr int SD = kRwRows * (int)sizeof(WT) / 16;   // staged 32-bit words per thread and stage
    constexpr int WPS = kRwRows / 2;                   // 32-bit words of hub positions per slot and stage
    static_assert(NPC * 4 == SD && NQ * (int)sizeof(WT) == SD * 4, "stage split");
    static_assert(kRwRows % 8 == 0 && kRwSlots * WPS <= kRcWideThreads, "position words");
    __shared__ int sh_h4[kRwSlots][kMaxP];
    const int n = d.n, p = d.p, pp = p * p, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    WT *ring = (WT *)smem;                                      // [2][kRwRows][kRwCols]
    uint16_t *pos = (uint16_t *)(smem + kRwRing);               // [2][kRwSlots][kRwRows]
    double *Ch = (double *)(smem + kRwRing + kRwPos);           // [kRwSlots][p][p]
    const int slot0 = g * kRwSlots, c0 = chunk * kRwCols;
    const int j = c0 + lane, jc = j < n ? j : n - 1;
    const int nst = (n + kRwRows - 1) / kRwRows;
    const WT *W = (const WT *)P.W;
    // This thread's share of a stage, as 32-bit words: VEC, pieces
    // e = tid + 256 v (row e / CPR, columns EPC (e % CPR) ..); else the
    // elements of rows 4q + wave at column jc.  Also one word of hub
    // positions, rows 2(t % WPS) and 2(t % WPS) + 1 of slot (t / WPS) % 4
    // (threads below 4 WPS store theirs).  W comes through bounds-checked buffer loads at a
    // fixed per-thread byte offset plus the stage's: rows past n read zero.
    // Rows past n are masked again when stored (weight zero, position 0).
    // Loads take no branch -- the positions of stages past the last reread
    // it -- so the only waits on them are the stores'.
    const int ps = slot0 + ((tid / WPS) & 3) < total ? slot0 + ((tid / WPS) & 3) : total - 1;
    const uint32_t *prow = (const uint32_t *)(V.kidx + (size_t)P.slot_s[ps] * d.n_pad) + tid % WPS;
    const __amdgpu_buffer_rsrc_t wrs =
        __builtin_amdgcn_make_buffer_rsrc((void *)W, (short)0, (int)((size_t)n * n * sizeof(WT)), kBufWord3);
    const uint32_t stage_bytes = (uint32_t)kRwRows * (uint32_t)n * (uint32_t)sizeof(WT);
    constexpr int NV = VEC ? NPC : NQ;
    uint32_t voff[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if constexpr (VEC) {
            const int e = tid + kRcWideThreads * v;
            const int col = c0 + (e % CPR) * EPC < n - EPC ? c0 + (e % CPR) * EPC : n - EPC;
            voff[v] = ((uint32_t)(e / CPR) * (uint32_t)n + (uint32_t)col) * (uint32_t)sizeof(WT);
        } else {
            voff[v] = ((uint32_t)(4 * v + wave) * (uint32_t)n + (uint32_t)jc) * (uint32_t)sizeof(WT);
        }
    }
    auto load = [&](int st, uint32_t(&w)[SD], uint32_t &pv) {
        const uint32_t sb = (uint32_t)st * stage_bytes;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if constexpr (VEC) {
                const auto x = __builtin_amdgcn_raw_buffer_load_b128(wrs, voff[v] + sb, 0, 0);
                w[4 * v] = x[0];
                w[4 * v + 1] = x[1];
                w[4 * v + 2] = x[2];
                w[4 * v + 3] = x[3];
            } else if constexpr (sizeof(WT) == 8) {
                const auto x = __builtin_amdgcn_raw_buffer_load_b64(wrs, voff[v] + sb, 0, 0);
                w[2 * v] = x[0];
                w[2 * v + 1] = x[1];
            } else {
                w[v] = __builtin_amdgcn_raw_buffer_load_b32(wrs, voff[v] + sb, 0, 0);
            }
        }
        pv = prow[(st < nst ? st : nst - 1) * WPS];   // n_pad >= nst * kRwRows: in bounds
    };
    auto store = [&](int st, const uint32_t(&w)[SD], uint32_t pv) {
        const int buf = st & 1;
        if constexpr (VEC) {
#pragma unroll
            for (int v = 0; v < NPC; ++v) {
                const int e = tid + kRcWideThreads * v, r = e / CPR, i = st * kRwRows + r;
                const uint4 x = i < n ? make_uint4(w[4 * v], w[4 * v + 1], w[4 * v + 2], w[4 * v + 3])
                                      : make_uint4(0u, 0u, 0u, 0u);
                *(uint4 *)(ring + (buf * kRwRows + r) * kRwCols + (e % CPR) * EPC) = x;
            }
        } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int i = st * kRwRows + 4 * q + wave;
                WT x;
                if constexpr (sizeof(WT) == 8)
                    x = __builtin_bit_cast(double, (uint64_t)w[2 * q] | ((uint64_t)w[2 * q + 1] << 32));
                else
                    x = __builtin_bit_cast(float, w[q]);
                ring[(buf * kRwRows + 4 * q + wave) * kRwCols + lane] = i < n ? x : (WT)0;
            }
        }
        if (tid < kRwSlots * WPS) {   // stored as table offsets k(i) p (below 2^16: p <= 64)
            const int i = st * kRwRows + 2 * (tid % WPS);
            ((uint32_t *)pos)[(buf * kRwSlots + tid / WPS) * WPS + tid % WPS] =
                (i < n ? (pv & 0xffffu) * (uint32_t)p : 0u) | (i + 1 < n ? (pv >> 16) * (uint32_t)p << 16 : 0u);
        }
    };
    __syncthreads();   // LDS of the previous item free
    uint32_t wr[kRwDepth][SD];
    uint32_t pr[kRwDepth];
#pragma unroll
    for (int u = 0; u < kRwDepth; ++u) load(u, wr[u], pr[u]);   // independent of the candidates
    // the four slots' hub lists and distance tables
    for (int e = tid; e < kRwSlots * p; e += kRcWideThreads) {
        const int w = e / p, sl = slot0 + w < total ? slot0 + w : total - 1;
        sh_h4[w][e % p] = V.children[(size_t)P.slot_s[sl] * p + e % p];
    }
    const int my = slot0 + wave;   // this wave's slot
    const bool active = my < total;
    const int kj = V.kidx[(size_t)P.slot_s[active ? my : total - 1] * d.n_pad + jc];
    __syncthreads();
    for (int e = tid; e < kRwSlots * pp; e += kRcWideThreads) {
        const int w = e / pp, r = e % pp;
        const size_t at = (size_t)sh_h4[w][r / p] * n + sh_h4[w][r % p];
        Ch[e] = P.Ctr ? P.Ctr[at] : (double)((const CT *)P.C)[at];
    }
    store(0, wr[0], pr[0]);
    load(kRwDepth, wr[0], pr[0]);
    __syncthreads();
    const double *chl = Ch + (size_t)wave * pp + kj;   // chl[k p] = C[h_k][h_{k(j)}] of this wave's slot
    double acc = 0.0;
    // stages past the last (up to a multiple of kRwDepth) are all rows past n
    for (int t0 = 0; t0 < nst; t0 += kRwDepth) {
#pragma unroll
        for (int u = 0; u < kRwDepth; ++u) {
            const int t = t0 + u, nx = (u + 1) % kRwDepth;
            store(t + 1, wr[nx], pr[nx]);   // that buffer was read before the last barrier
            load(t + 1 + kRwDepth, wr[nx], pr[nx]);
            if (active) {
                // the stage's table offsets first (one address for all lanes),
                // then the reads of each 8 rows issued before the previous 8
                // rows are added
                const WT *rw = ring + (t & 1) * kRwRows * kRwCols + lane;
                const uint16_t *pw = pos + ((t & 1) * kRwSlots + wave) * kRwRows;
                uint32_t kw[kRwRows / 2];
#pragma unroll
                for (int q = 0; q < kRwRows / 8; ++q) {
                    const uint4 x = *(const uint4 *)(pw + 8 * q);
                    kw[4 * q] = x.x;
                    kw[4 * q + 1] = x.y;
                    kw[4 * q + 2] = x.z;
                    kw[4 * q + 3] = x.w;
                }
                double wv[2][8], cv[2][8];
                auto issue = [&](int b, int r0) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) wv[b][q] = (double)rw[(r0 + q) * kRwCols];
#pragma unroll
                    for (int q = 0; q < 8; ++q) cv[b][q] = chl[(kw[(r0 + q) >> 1] >> (16 * ((r0 + q) & 1))) & 0xffffu];
                };
                issue(0, 0);
#pragma unroll
                for (int r0 = 0; r0 < kRwRows; r0 += 8) {
                    const int b = (r0 >> 3) & 1;
                    if (r0 + 8 < kRwRows) issue(b ^ 1, r0 + 8);
#pragma unroll
                    for (int q = 0; q < 8; ++q) acc = acc + wv[b][q] * cv[b][q];
                }
            }
            __syncthreads();
        }
    }
    if (active && j < n) P.tbuf[(size_t)my * n + j] = acc;
}

// T = sum_j t_j in ascending order for the slots s0 + w whose bit w is set in
// mask -- wave w adds slot s0 + w, all in parallel -- then each slot's cost
// from Cc and Dd of its sums item.
__device__ __forceinline__ void rc_finish_group(const DevPtrs &P, const Dims &d, const RcView &V, int s0,
                                                unsigned mask, char *smem)
{
#pragma clang fp contract(off)
    const int n = d.n, lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool mine = (mask >> wave) & 1u;
    double *buf = (double *)smem + (size_t)wave * kRwSum;
    const double *t = P.tbuf + (size_t)(s0 + wave) * n;
    double acc = 0.0;
    __syncthreads();   // LDS of the item free
    for (int i0 = 0; i0 < n; i0 += kRwSum) {
        const int cnt = n - i0 < kRwSum ? n - i0 : kRwSum;
        if (mine) {
            double v[kRwSum / 64];
#pragma unroll
            for (int u = 0; u < kRwSum / 64; ++u) {
                const int q = u * 64 + lane;
                v[u] = t[i0 + (q < cnt ? q : cnt - 1)];
            }
#pragma unroll
            for (int u = 0; u < kRwSum / 64; ++u)
                if (u * 64 + lane < cnt) buf[u * 64 + lane] = v[u];
        }
        __syncthreads();
        if (mine && lane == 0) acc = chain_sum<kRwSum, 3>(acc, buf, cnt);
        __syncthreads();
    }
    if (mine && lane == 0) {
        const int slot = s0 + wave;
        const size_t o = (size_t)P.slot_r[slot] * V.m + P.slot_c[slot];
        const double Cc = V.parts_out[3 * o + 0], Dd = V.parts_out[3 * o + 2];
        V.cost_out[o] = (((d.chi * Cc) + (d.alpha * acc)) + (d.delta * Dd)) * d.scale;
        V.parts_out[3 * o + 1] = acc;
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
    const int nth = blockDim.x;
    double *bt = L.ring, *bc = bt + kRcChain, *bd = bc + kRcChain;
    const double *t = P.tbuf + (size_t)slot * n;
    const CT *C = (const CT *)P.C;
    double acc = 0.0;
    for (int i0 = 0; i0 < n; i0 += kRcChain) {
        const int cnt = n - i0 < kRcChain ? n - i0 : kRcChain;
        for (int q0 = 0; q0 < cnt; q0 += 4 * nth) {
            double tv[4], cv[4], ov[4], dv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * nth + tid, i = i0 + (q < cnt ? q : cnt - 1);
                if (MASK & 1) tv[u] = t[i];
                if (MASK & 6) cv[u] = (double)C[(size_t)i * n + sh_h[L.kid[i]]];
                if (MASK & 2) ov[u] = P.O[i];
                if (MASK & 4) dv[u] = P.D[i];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * nth + tid;
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
template <typename CT, bool WIDE>
__device__ __forceinline__ void rc_ccdd_item(const DevPtrs &P, const Dims &d, const RcView &V, int slot, char *smem,
                                             int *sh_h)
{
    __shared__ double sums[3];
    const RcLds L = rc_lds<WIDE>(smem, d.p);
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
template <typename CT, bool WIDE>
__device__ __forceinline__ void rc_finish_slot(const DevPtrs &P, const Dims &d, const RcView &V, int slot, char *smem,
                                               const int *sh_h)
{
#pragma clang fp contract(off)
    __shared__ double sums[3];
    const RcLds L = rc_lds<WIDE>(smem, d.p);
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

// One item of the slot is done; the slot's last one finishes it.  True when
// the slot was finished here.
template <typename CT, bool WIDE>
__device__ __forceinline__ bool rc_slot_done(const DevPtrs &P, const Dims &d, const RcView &V, int slot, char *smem,
                                             const int *sh_h)
{
    if (!rc_item_done(P, slot, rc_slot_items(d.n, WIDE))) return false;
    rc_finish_slot<CT, WIDE>(P, d, V, slot, smem, sh_h);
    return true;
}

// Item c of a slot in the narrow kernel (c < chunks: a column chunk;
// c == chunks: the sums); the slot's last item finishes it.  True when the
// slot was finished here.
template <typename CT, typename WT>
__device__ __forceinline__ bool rc_slot_item(const DevPtrs &P, const Dims &d, const RcView &V, int slot, int c,
                                             char *smem, int *sh_h)
{
    if (c < rc_chunks(d.n))
        rc_column_item<CT, WT>(P, d, V, slot, c, smem, sh_h);
    else
        rc_ccdd_item<CT, false>(P, d, V, slot, smem, sh_h);
    return rc_slot_done<CT, false>(P, d, V, slot, smem, sh_h);
}

// A unit (slot or extra candidate) is done: the last one decides.
__device__ inline void rc_unit_done(const DevPtrs &P, const Dims &d, const RcView &V, int units)
{
    if (last_block(P.sync + 1, units) && V.decide) decide_generation(make_sel_state(P, d), P.choice);
}

// k units done at once: the last one decides.
__device__ inline void rc_units_done(const DevPtrs &P, const Dims &d, const RcView &V, int units, int k)
{
    __shared__ int is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        release_agent();
        is_last = atomicAdd(P.sync + 1, k) + k == units;
        if (is_last) atomicExch(P.sync + 1, 0);
    }
    __syncthreads();
    if (is_last) {
        acquire_agent();
        if (V.decide) decide_generation(make_sel_state(P, d), P.choice);
    }
}

// Wide column item (g, c), then the completion of its slots.
template <typename CT, typename WT>
__device__ __forceinline__ void rc_wide_column(const DevPtrs &P, const Dims &d, const RcView &V, int total, int units,
                                               int g, int c, char *smem)
{
    if ((d.n * (int)sizeof(WT)) % 16 == 0 && d.n >= kRwCols)
        rc_column_item_wide<CT, WT, true>(P, d, V, total, g, c, smem);
    else
        rc_column_item_wide<CT, WT, false>(P, d, V, total, g, c, smem);
    const int s0 = g * kRwSlots, k = total - s0 < kRwSlots ? total - s0 : kRwSlots;
    const unsigned m = rc_group_done(P, s0, (1u << k) - 1u, rc_slot_items(d.n, true));
    if (m) {
        rc_finish_group(P, d, V, s0, m, smem);
        rc_units_done(P, d, V, units, __builtin_popcount(m));
    }
}

// Sums item of slot e in the wide kernel, then the slot's completion.
template <typename CT>
__device__ __forceinline__ void rc_wide_sums(const DevPtrs &P, const Dims &d, const RcView &V, int units, int e,
                                             char *smem, int *sh_h)
{
    rc_ccdd_item<CT, true>(P, d, V, e, smem, sh_h);
    const int s0 = e & ~(kRwSlots - 1);
    const unsigned m = rc_group_done(P, s0, 1u << (e - s0), rc_slot_items(d.n, true));
    if (m) {
        rc_finish_group(P, d, V, s0, m, smem);
        rc_units_done(P, d, V, units, 1);
    }
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
// that column strip of W in one L2; the wide kernel maps its column chunks
// the same way and takes the sums items from the last workgroup down.
// WIDE: the wide kernel's body, which serves only launches with
// rc_wide(total, p); the other serves the rest.
template <typename CT, typename WT, bool WIDE>
__device__ __forceinline__ void rc_body(const DevPtrs &P, const Dims &d, const RcView &V, char *smem, int blk, int nblk)
{
    __shared__ int sh_h[kMaxP];
    const int total = min(*P.total, d.tot), nextra = *P.nextra, units = total + nextra;
    if (rc_wide(total, d.p) != WIDE) return;
    if (units == 0) {
        if (blk == 0 && V.decide) decide_generation(make_sel_state(P, d), P.choice);
        return;
    }
    if constexpr (WIDE) {
        const int nct = rc_wide_chunks(d.n), ng = (total + kRwSlots - 1) / kRwSlots;
        const int x = blk & 7, q = blk >> 3, nq = nblk >> 3;
        const int a = (nct - x + 7) / 8;   // chunks x, x + 8, ...
        for (int li = q; li < a * ng; li += nq)
            rc_wide_column<CT, WT>(P, d, V, total, units, li % ng, x + 8 * (li / ng), smem);
        for (int e = nblk - 1 - blk; e < total; e += nblk) rc_wide_sums<CT>(P, d, V, units, e, smem, sh_h);
        for (int e = blk; e < nextra; e += nblk) {
            rc_extra<CT, WT>(P, d, V, e, smem);
            rc_unit_done(P, d, V, units);
        }
        return;
    }
    const int nch = rc_slot_items(d.n, false);
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
    rc_body<CT, WT, false>(P, d, V, smem, blockIdx.x, gridDim.x);
}

template <typename CT, typename WT>
__global__ __launch_bounds__(kRcWideThreads, 2) void k_recheck_wide(DevPtrs P, Dims d, RcView V)
{
    extern __shared__ __align__(16) char smem[];
    rc_body<CT, WT, true>(P, d, V, smem, blockIdx.x, gridDim.x);
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

// Items of context J in the WIDE kernel's pool: none unless the context's
// slot count is in that kernel's range.
// Column items of a context in the wide kernel (groups of four slots by
// column chunks); its sums items follow them.
__device__ inline int rc_wide_columns(int n, int total)
{
    return rc_wide_chunks(n) * ((total + kRwSlots - 1) / kRwSlots);
}

template <bool WIDE>
__device__ inline int rc_items(const TickJob &J)
{
    const int total = min(*J.P.total, J.d.tot);
    if (rc_wide(total, J.d.p) != WIDE) return 0;
    const int u = (WIDE ? rc_wide_columns(J.d.n, total) + total : total * rc_slot_items(J.d.n, false)) + *J.P.nextra;
    return u > 0 ? u : 1;
}

template <typename CT, typename WT, bool WIDE>
__device__ __forceinline__ void rc_group_item(const TickJob &J, int item, char *smem, int *sh_h)
{
    const DevPtrs &P = J.P;
    const Dims &d = J.d;
    const RcView V = rc_generation_view(P, d);
    const int total = min(*P.total, d.tot), units = total + *P.nextra;
    const int slot_items = WIDE ? rc_wide_columns(d.n, total) + total : total * rc_slot_items(d.n, false);
    if (units == 0) {
        decide_generation(make_sel_state(P, d), P.choice);
    } else if (item < slot_items) {
        if constexpr (WIDE) {
            const int ncol = rc_wide_columns(d.n, total), ng = (total + kRwSlots - 1) / kRwSlots;
            if (item < ncol) {
                rc_wide_column<CT, WT>(P, d, V, total, units, item % ng, item / ng, smem);
            } else {
                rc_wide_sums<CT>(P, d, V, units, item - ncol, smem, sh_h);
            }
        } else if (rc_slot_item<CT, WT>(P, d, V, item % total, item / total, smem, sh_h)) {
            rc_unit_done(P, d, V, units);
        }
    } else {
        rc_extra<CT, WT>(P, d, V, item - slot_items, smem);
        rc_unit_done(P, d, V, units);
    }
}

template <bool WIDE>
__device__ __forceinline__ void rc_group_body(const GroupHdr *__restrict__ hdr, const TickJob *__restrict__ jobs,
                                              char *smem)
{
    __shared__ int pre[kMaxPoolJobs + 1];
    __shared__ int sh_h[kMaxP];
    const int njobs = hdr->njobs;
    const int items = pool_prefix(njobs, [&](int j) { return rc_items<WIDE>(jobs[j]); }, pre);
    for (int g = blockIdx.x; g < items; g += gridDim.x) {
        const int j = pool_job(pre, njobs, g);
        const TickJob &J = jobs[j];
        const int item = g - pre[j];
        if (J.d.c_f32) {
            if (J.d.w_f32) rc_group_item<float, float, WIDE>(J, item, smem, sh_h);
            else rc_group_item<float, double, WIDE>(J, item, smem, sh_h);
        } else {
            if (J.d.w_f32) rc_group_item<double, float, WIDE>(J, item, smem, sh_h);
            else rc_group_item<double, double, WIDE>(J, item, smem, sh_h);
        }
    }
}

__global__ __launch_bounds__(kRcThreads) void k_recheck_group(const GroupHdr *__restrict__ hdr,
                                                              const TickJob *__restrict__ jobs)
{
    extern __shared__ __align__(16) char smem[];
    rc_group_body<false>(hdr, jobs, smem);
}

__global__ __launch_bounds__(kRcWideThreads, 2) void k_recheck_group_wide(const GroupHdr *__restrict__ hdr,
                                                                       const TickJob *__restrict__ jobs)
{
    extern __shared__ __align__(16) char smem[];
    rc_group_body<true>(hdr, jobs, smem);
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

// The two kernels back to back; the slot count, known only on the device,
// lets one of them work.  wide = false launches the narrow kernel alone (a
// single slot).
template <typename CT, typename WT>
static hipError_t rc_launch(const DevPtrs &P, const Dims &d, const RcView &V, bool wide, hipStream_t st)
{
    k_recheck<CT, WT><<<kRecheckBlocks, kRcThreads, recheck_lds(d.n, d.p), st>>>(P, d, V);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !wide) return e;
    k_recheck_wide<CT, WT><<<kRcWideBlocks, kRcWideThreads, recheck_wide_lds(d.n, d.p), st>>>(P, d, V);
    return hipGetLastError();
}

static hipError_t rc_dispatch(const DevPtrs &P, const Dims &d, const RcView &V, bool wide, hipStream_t st)
{
    if (d.c_f32 && d.w_f32) return rc_launch<float, float>(P, d, V, wide, st);
    if (d.c_f32) return rc_launch<float, double>(P, d, V, wide, st);
    if (d.w_f32) return rc_launch<double, float>(P, d, V, wide, st);
    return rc_launch<double, double>(P, d, V, wide, st);
}

hipError_t launch_recheck(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    return rc_dispatch(P, d, rc_generation_view(P, d), true, st);
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
    return rc_dispatch(P, d, V, false, st);
}

hipError_t launch_recheck_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, size_t lds, size_t lds_wide,
                                hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    if (njobs > kMaxPoolJobs) return hipErrorInvalidValue;
    k_recheck_group<<<kRecheckBlocks, kRcThreads, lds, st>>>(hdr, jobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_recheck_group_wide<<<kRcWideBlocks, kRcWideThreads, lds_wide, st>>>(hdr, jobs);
    return hipGetLastError();
}

static size_t g_group_lds_cap = 0;   // dynamic LDS limit of both grouped kernels

size_t recheck_group_lds_cap() { return g_group_lds_cap; }

// Raise the dynamic-LDS caps, once per process (never during graph capture).
hipError_t prepare_recheck_kernels(int max_lds)
{
    const void *fns[] = {(const void *)k_recheck<double, double>, (const void *)k_recheck<double, float>,
                         (const void *)k_recheck<float, double>, (const void *)k_recheck<float, float>,
                         (const void *)k_recheck_wide<double, double>, (const void *)k_recheck_wide<double, float>,
                         (const void *)k_recheck_wide<float, double>, (const void *)k_recheck_wide<float, float>,
                         (const void *)k_recheck_group, (const void *)k_recheck_group_wide};
    size_t cap = ~(size_t)0;
    for (const void *f : fns) {
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, f);
        if (e != hipSuccess) return e;
        const int dyn = max_lds - (int)fa.sharedSizeBytes;   // the cap excludes the kernel's static LDS
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
        if (e != hipSuccess) return e;
        if ((f == (const void *)k_recheck_group || f == (const void *)k_recheck_group_wide) && (size_t)dyn < cap)
            cap = (size_t)dyn;
    }
    g_group_lds_cap = cap;
    return hipSuccess;
}

}  // namespace hubga
