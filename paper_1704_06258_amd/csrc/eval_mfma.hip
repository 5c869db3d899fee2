// Batched fitness evaluation of a whole population on bf16 matrix cores.
//
// The transfer term of objective (1) (Sec. 3) for individual s is
//     T_s = sum_i sum_l G_s[i][l] * C[h_{k(i)}][h_l],   G_s = W A_s,
// where A_s is the one-hot n x p allocation matrix (A_s[j][l] = 1 iff node j
// is allocated to hub l).  Stacking the population, G = W [A_1 ... A_S] is a
// dense GEMM with M = K = n and N = S*p.  W is split into bf16 hi and lo parts
// (|W - hi - lo| <= 2^-16 W); A is exact in bf16.  Both passes accumulate in
// the same FP32 registers (v_mfma_f32_32x32x16_bf16), and the epilogue folds
// each output column (s, l) against the hub-to-hub distances in binary64,
// writing one partial per (row tile, column).  G is never stored.
//
// Workgroup: 4 waves side by side along N; every wave covers all rows of the
// tile (ROWB blocks of 32) and COLB blocks of 32 columns.  The hi/lo tiles of
// W are staged through LDS (double buffered, K tile 32) and shared by the four
// waves; one-hot B fragments are built in registers from the 16-bit hub
// positions.  Tiles are assigned so that each XCD walks a contiguous range of
// row tiles (row-tile major), keeping its row panel of W in its own L2.
#include "kernels.hpp"
#include "wave_sync.hpp"

#include <type_traits>

namespace hubga {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));


__device__ __forceinline__ uint32_t onehot2(uint32_t kk, uint32_t lq)
{
    uint32_t lo = ((kk & 0xFFFFu) == lq) ? 0x3F80u : 0u;
    uint32_t hi = ((kk >> 16) == lq) ? 0x3F800000u : 0u;
    return lo | hi;
}

// The same for the pipelined kernels, in three packed 16-bit operations: with
// d = positions xor (l, l), min(d, 1) is 0 where a position equals l, and
// m * 0xC080 + 0x3F80 (mod 2^16) is then bf16 1.0 for m = 0 and 0 for m = 1.
// lq2 holds l in both halves.  The three constants come from registers the
// compiler cannot see into (it would turn the arithmetic back into compares
// and selects, twice the instructions).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
struct OneHotK {
    u16x2 one, mul, add;
};
__device__ __forceinline__ u16x2 opaque_u16x2(int v)
{
    uint32_t r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "i"(v));
    return __builtin_bit_cast(u16x2, r);
}
__device__ __forceinline__ OneHotK onehot_consts()
{
    return OneHotK{opaque_u16x2(0x00010001), opaque_u16x2((int)0xC080C080u), opaque_u16x2(0x3F803F80)};
}
__device__ __forceinline__ uint32_t onehot2_packed(uint32_t kk, uint32_t lq2, const OneHotK &c)
{
    const u16x2 d = __builtin_bit_cast(u16x2, kk ^ lq2);
    const u16x2 m = __builtin_elementwise_min(d, c.one);
    return __builtin_bit_cast(uint32_t, m * c.mul + c.add);
}

// NP: parts of the split of W (2: hi, lo; 3: hi, lo, mid), all accumulated
// into the same FP32 registers.
template <int ROWB, int COLB, int KT, int OCC, int NP = 2>
__global__ __launch_bounds__(256, OCC) void k_eval_mfma(const uint16_t *__restrict__ Whi,
                                                      const uint16_t *__restrict__ Wlo,
                                                      const uint16_t *__restrict__ Wmd,
                                                      const uint16_t *__restrict__ kidx,
                                                      const float *__restrict__ Ch32, int n, int n_pad, int p,
                                                      int NS, int n_mt, int n_nt, double *__restrict__ partial)
{
    constexpr int MT = 32 * ROWB;            // rows per tile
    constexpr int NT = 4 * 32 * COLB;        // columns per tile
    constexpr int LDS_ROW = KT + 8;          // bf16 per LDS row (16-byte pad against bank conflicts)
    constexpr int A_ELEMS = MT * LDS_ROW;    // one matrix, one stage
    constexpr int KSTEPS = KT / 16;
    __shared__ __align__(16) uint16_t sA[2][NP][A_ELEMS];   // [stage][hi/lo(/mid)]
    const uint16_t *const Wpart[3] = {Whi, Wlo, Wmd};

    // XCD-aware tile order: XCD x (= blockIdx % 8) gets the contiguous tile
    // range [x*per, (x+1)*per), row-tile major.
    const int tiles = n_mt * n_nt;
    const int per = (tiles + 7) / 8;
    const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tile >= tiles) return;
    const int mt = tile / n_nt, nt = tile % n_nt;
    const int M0 = mt * MT, N0 = nt * NT;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, l32 = lane & 31;

    // columns of this lane and the kidx row each one reads
    int col[COLB];
    uint32_t lq[COLB];
    const uint16_t *krow[COLB];
#pragma unroll
    for (int b = 0; b < COLB; ++b) {
        col[b] = N0 + wave * 32 * COLB + b * 32 + l32;
        int ind = 0;
        if (col[b] < NS) {
            ind = col[b] / p;
            lq[b] = (uint32_t)(col[b] % p);
        } else {
            lq[b] = 0xFFFFu;   // matches no hub position: zero column
        }
        krow[b] = kidx + (size_t)ind * n_pad + half * 8;
    }

    f32x16 acc[ROWB][COLB];
#pragma unroll
    for (int a = 0; a < ROWB; ++a)
#pragma unroll
        for (int b = 0; b < COLB; ++b) acc[a][b] = (f32x16)(0.0f);

    // global -> LDS staging: each matrix tile is MT rows x KT k = MT*KT/8 chunks of 16 B
    constexpr int CHUNKS = MT * (KT / 8);
    constexpr int PER_THREAD = CHUNKS / 256;   // per matrix
    static_assert(CHUNKS % 256 == 0, "tile must split evenly over 256 threads");
    u32x4 stage[NP][PER_THREAD];
    u32x4 knext[KSTEPS][COLB], kcur[KSTEPS][COLB];

    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            int c = tid + q * 256;
            int row = c / (KT / 8), kq = (c % (KT / 8)) * 8;
            size_t off = (size_t)(M0 + row) * n_pad + k0 + kq;
#pragma unroll
            for (int part = 0; part < NP; ++part) stage[part][q] = *(const u32x4 *)(Wpart[part] + off);
        }
#pragma unroll
        for (int kk = 0; kk < KSTEPS; ++kk)
#pragma unroll
            for (int b = 0; b < COLB; ++b) knext[kk][b] = *(const u32x4 *)(krow[b] + k0 + kk * 16);
    };
    auto lstore = [&](int st) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            int c = tid + q * 256;
            int row = c / (KT / 8), kq = (c % (KT / 8)) * 8;
#pragma unroll
            for (int part = 0; part < NP; ++part) *(u32x4 *)(&sA[st][part][row * LDS_ROW + kq]) = stage[part][q];
        }
#pragma unroll
        for (int kk = 0; kk < KSTEPS; ++kk)
#pragma unroll
            for (int b = 0; b < COLB; ++b) kcur[kk][b] = knext[kk][b];
    };

    const int ktiles = n_pad / KT;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < ktiles) gload((kt + 1) * KT);
#pragma unroll
        for (int kk = 0; kk < KSTEPS; ++kk) {
            bf16x8 bfrag[COLB];
#pragma unroll
            for (int b = 0; b < COLB; ++b) {
                const u32x4 kv = kcur[kk][b];
                const uint32_t l2 = lq[b];
                u32x4 bb;
                bb.x = onehot2(kv.x, l2);
                bb.y = onehot2(kv.y, l2);
                bb.z = onehot2(kv.z, l2);
                bb.w = onehot2(kv.w, l2);
                bfrag[b] = __builtin_bit_cast(bf16x8, bb);
            }
            // hi pass over every accumulator, then lo (then mid): consecutive
            // MFMAs never feed each other
#pragma unroll
            for (int part = 0; part < NP; ++part) {
#pragma unroll
                for (int a = 0; a < ROWB; ++a) {
                    const int lrow = (a * 32 + l32) * LDS_ROW + kk * 16 + half * 8;
                    bf16x8 af = __builtin_bit_cast(bf16x8, *(const u32x4 *)(&sA[cur][part][lrow]));
#pragma unroll
                    for (int b = 0; b < COLB; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bfrag[b], acc[a][b], 0, 0, 0);
                }
            }
        }
        if (kt + 1 < ktiles) lstore(cur ^ 1);
        __syncthreads();
    }

    // epilogue: sum_i G[i][(s,l)] * C[h_k(i)][h_l] over this tile's rows, binary64.
    // Accumulator v of a 32x32 block holds row 8*(v/4) + 4*half + (v%4), column l32.
#pragma unroll
    for (int b = 0; b < COLB; ++b) {
        double sum = 0.0;
        if (col[b] < NS) {
            const int s = col[b] / p;
            const uint16_t *kr = kidx + (size_t)s * n_pad;
            const float *ch = Ch32 + (size_t)s * p * p + lq[b];
#pragma unroll
            for (int a = 0; a < ROWB; ++a) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int i = M0 + a * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
                    if (i < n) {
                        const int k = kr[i];
                        sum = __builtin_fma((double)acc[a][b][v], (double)ch[k * p], sum);
                    }
                }
            }
        }
        sum += __shfl_xor(sum, 32);
        if (half == 0 && col[b] < NS) partial[(size_t)mt * NS + col[b]] = sum;
    }
}

// ---------------------------------------------------------------------------
// Pipelined variant.  W hi/lo are read from a fragment-ordered ("swizzled")
// copy in which every (64-row group, 16-k step, k half) is one contiguous 1 KB
// run of 64 16-byte chunks -- exactly the lane order of one wave's operand
// fragment.  Each K tile (32) of W and of every wave's hub positions is moved
// global -> LDS by global_load_lds_dwordx4 (no register staging) into a ring
// of NST stages, NST-1 tiles ahead of the matrix cores.  Waits are explicit
// vmcnt counts (in-order completion of the wave's own loads) followed by a
// bare workgroup barrier; the ring is read with ds_read_b128 issued as inline
// assembly and an explicit lgkmcnt wait, so the compiler never drains the
// whole pipeline before an LDS read.
typedef __attribute__((address_space(3))) void lds_void;

template <int OFF>
__device__ __forceinline__ u32x4 ds_read16(uint32_t addr)
{
    u32x4 v;
    asm volatile("ds_read_b128 %0, %1 offset:%2" : "=v"(v) : "v"(addr), "i"(OFF));
    return v;
}
__device__ __forceinline__ void pin(u32x4 &v) { asm volatile("" : "+v"(v)); }
// An FP32 read from LDS byte address addr.
__device__ __forceinline__ float lds_f32(uint32_t addr)
{
    return *(const __attribute__((address_space(3))) float *)(uintptr_t)addr;
}

// One context's operands for the batched kernel (also one entry of a grouped
// launch over several contexts).
// n_rt row tiles by n_nt column tiles are the work units; n_mt is the number
// of partials per column (one per row tile: n_mt == n_rt).
struct MfmaJob {
    const u32x4 *Whsw, *Wlsw;   // W in fragment order, the folded W when fold is set
    const uint16_t *kidx;
    const float *Ch32;
    double *partial;
    int n, n_pad, p, count, NS, n_mt, n_nt, tile_start, n_rt, fold;
};

// Ring size in 16-byte chunks; MODE 2 stages K tiles of 64 (the rest 32).
template <int ROWB, int COLB, int NST, int KINS, int MODE = 0>
constexpr int pipe_ring_chunks()
{
    constexpr int KH = MODE == 2 ? 2 : 1;   // 32-deep halves of the K tile
    return NST * (2 * (2 * KH) * 2 * 32 * ROWB + 4 * KINS * KH * 64);
}

// Individuals [s_lo, s_lo + nind) whose columns column tile nt touches.
template <int NT>
__device__ __forceinline__ int2 tile_individuals(const MfmaJob &J, int nt)
{
    const int N0 = nt * NT;
    const int s_lo = min(N0, J.NS - 1) / J.p, s_hi = min(N0 + NT - 1, J.NS - 1) / J.p;
    return make_int2(s_lo, s_hi - s_lo + 1);
}

// LDS bytes of a tile's staged epilogue operands: the hub positions of its MT
// rows for each of its individuals ([ind][row], 16-bit), then their FP32
// hub-distance tables ([ind][k][l]).
template <int MT, int NT>
__device__ __forceinline__ int epi_stage_bytes(const MfmaJob &J, int nt)
{
    const int nind = tile_individuals<NT>(J, nt).y;
    return nind * MT * 2 + nind * J.p * J.p * 4;
}

// Moves those operands global -> LDS at dst with the waves' direct loads
// (no register round trip; completion is each wave's vmcnt).  The hub
// positions go in 16-byte pieces of MT/8 per individual; the tables in
// 16-byte pieces when p*p is a multiple of 4 (every piece then starts
// aligned and ends inside the last individual's table), else in 4-byte ones.
template <int MT, int NT>
__device__ __forceinline__ void epi_stage_issue(const MfmaJob &J, int mt, int nt, u32x4 *dst)
{
    const int2 ind = tile_individuals<NT>(J, nt);
    const int s_lo = ind.x, nind = ind.y, pp = J.p * J.p;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int CPI = MT / 8;   // 16-byte pieces of hub positions per individual
    const int nk = nind * CPI;
    for (int b = wave * 64; b < nk; b += 256) {
        const int c = b + lane;
        if (c < nk)
            __builtin_amdgcn_global_load_lds(
                (const void *)(J.kidx + (size_t)(s_lo + c / CPI) * J.n_pad + mt * MT + (c % CPI) * 8),
                (lds_void *)(dst + b), 16, 0, 0);
    }
    const float *src = J.Ch32 + (size_t)s_lo * pp;
    if (pp % 4 == 0) {
        const int nc = nind * pp / 4;
        for (int b = wave * 64; b < nc; b += 256) {
            const int c = b + lane;
            if (c < nc)
                __builtin_amdgcn_global_load_lds((const void *)(src + 4 * c), (lds_void *)(dst + nk + b), 16, 0, 0);
        }
    } else {
        uint32_t *dl = (uint32_t *)(dst + nk);
        const int nc = nind * pp;
        for (int b = wave * 64; b < nc; b += 256) {
            const int c = b + lane;
            if (c < nc) __builtin_amdgcn_global_load_lds((const void *)(src + c), (lds_void *)(dl + b), 4, 0, 0);
        }
    }
}

// Epilogue of a pipelined tile: sum_i G[i][(s,l)] * C[h_k(i)][h_l] over the
// tile's rows in binary64, one partial per column in slot `slot`.  Both
// factors are FP32, so their product is exact in binary64 and a fused
// multiply-add rounds exactly as the product-then-sum does.  The
// operands are staged in LDS so the gathers hit LDS: at pre when the K loop
// already issued them there, else into the ring (ring_chunks 16-byte chunks,
// free once every wave has left the K loop) if they fit, else the gathers go
// to global memory.
template <int ROWB, int COLB>
__device__ __forceinline__ void pipe_epilogue(const MfmaJob &J, f32x16 (&acc)[ROWB][COLB], const int (&col)[COLB],
                                              const uint32_t (&lq)[COLB], int mt, int nt, u32x4 *ring,
                                              int ring_chunks, int slot, u32x4 *pre)
{
    constexpr int MT = 32 * ROWB, NT = 128 * COLB;
    const uint16_t *__restrict__ kidx = J.kidx;
    const float *__restrict__ Ch32 = J.Ch32;
    double *__restrict__ partial = J.partial;
    const int n = J.n, n_pad = J.n_pad, p = J.p, NS = J.NS;
    const int M0 = mt * MT;
    const int tid = threadIdx.x, half = (tid & 63) >> 5;
    // Accumulator v of a 32x32 block holds row 8*(v/4) + 4*half + (v%4).
    wg_barrier();   // every wave has left the K loop
    const int2 ti = tile_individuals<NT>(J, nt);
    const int s_lo = ti.x, nind = ti.y;
    u32x4 *sd = pre;
    if (!sd && epi_stage_bytes<MT, NT>(J, nt) <= (int)sizeof(u32x4) * ring_chunks) {
        epi_stage_issue<MT, NT>(J, mt, nt, ring);
        sd = ring;
    }
    const bool staged = sd != nullptr;
    // Indices into the staged arrays are offsets from their start (never a
    // pointer moved before it): LDS pointer arithmetic is 32-bit, and a
    // negative intermediate would leave the LDS aperture of a flat address.
    uint16_t *lk = (uint16_t *)sd;                       // [ind][row - M0]
    float *lch = (float *)(sd + nind * (MT / 8));        // [ind][k][l]
    const uint32_t lch_addr = staged ? (uint32_t)(uintptr_t)(lds_void *)lch : 0u, p4 = 4u * (uint32_t)p;
    if (staged) {
        vm_wait<0>();
        wg_barrier();   // every wave's copies have landed
        if (M0 + MT > n) {
            // rows past n (kNoHub in kidx) get position 0: their products are
            // exactly zero (W is zero-padded), which keeps the sum below free
            // of branches
            for (int e = tid; e < nind * MT; e += 256)
                if (M0 + e % MT >= n) lk[e] = 0;
            __syncthreads();
        }
    }
#pragma unroll
    for (int b = 0; b < COLB; ++b) {
        double part[4] = {0.0, 0.0, 0.0, 0.0};
        if (col[b] < NS) {
            const int s = col[b] / p;
            if (staged) {
                // rows a*32 + 8j + 4*half + t (t = 0..3) are 4 consecutive
                // positions; the factor C[h_k][h_l] is at LDS byte address
                // k*4p + cb, one full-rate 24-bit multiply-add (k*4p < 2^24)
                const int kb = (s - s_lo) * MT + 4 * half;
                const uint32_t cb = lch_addr + 4u * (uint32_t)((s - s_lo) * p * p + (int)lq[b]);
#pragma unroll
                for (int a = 0; a < ROWB; ++a) {
                    // the row block's 16 factors are all read before its products
                    float f[16];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint2 k4 = *(const uint2 *)(lk + kb + a * 32 + 8 * j);
                        f[4 * j + 0] = lds_f32(__umul24(k4.x & 0xFFFFu, p4) + cb);
                        f[4 * j + 1] = lds_f32(__umul24(k4.x >> 16, p4) + cb);
                        f[4 * j + 2] = lds_f32(__umul24(k4.y & 0xFFFFu, p4) + cb);
                        f[4 * j + 3] = lds_f32(__umul24(k4.y >> 16, p4) + cb);
                    }
#pragma unroll
                    for (int v = 0; v < 16; ++v)
                        part[v & 3] = __builtin_fma((double)acc[a][b][v], (double)f[v], part[v & 3]);
                }
            } else {
                const uint16_t *kr = kidx + (size_t)s * n_pad;
                const float *ch = Ch32 + (size_t)s * p * p + lq[b];
#pragma unroll
                for (int a = 0; a < ROWB; ++a) {
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int i = M0 + a * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
                        if (i < n) part[v & 3] = __builtin_fma((double)acc[a][b][v], (double)ch[kr[i] * p], part[v & 3]);
                    }
                }
            }
        }
        double sum = (part[0] + part[1]) + (part[2] + part[3]);
        sum += __shfl_xor(sum, 32);
        if (half == 0 && col[b] < NS) partial[(size_t)slot * NS + col[b]] = sum;
    }
}

// EARLY: the LDS reads of every k-step of a tile are issued up front, so the
// reads of step k+1 land while step k's products run.
template <int ROWB, int COLB, int NST, int KINS, int EARLY>
__device__ __forceinline__ void mfma_pipe_tile(const MfmaJob &J, int tile, u32x4 *ring)
{
    constexpr int MT = 32 * ROWB, NT = 128 * COLB, KTILE = 32, KSTEPS = KTILE / 16;
    constexpr int A_CHUNKS = 2 * KSTEPS * 2 * MT;   // [hi/lo][kk][half][row] 16-byte chunks per stage
    constexpr int K_CHUNKS = 4 * KINS * 64;         // [wave][ins][lane]
    constexpr int STAGE = A_CHUNKS + K_CHUNKS;
    constexpr int A_INS = A_CHUNKS / 64 / 4;        // 1 KB transfers per wave per tile for W
    constexpr int LPT = A_INS + KINS;               // vector-memory instructions per wave per tile
    static_assert(MT % 64 == 0 && (A_CHUNKS / 64) % 4 == 0, "tile shape");
    const u32x4 *__restrict__ Whsw = J.Whsw;
    const u32x4 *__restrict__ Wlsw = J.Wlsw;
    const uint16_t *__restrict__ kidx = J.kidx;
    const int n_pad = J.n_pad, p = J.p, count = J.count, NS = J.NS, n_nt = J.n_nt;
    const int mt = tile / n_nt, nt = tile % n_nt;
    const int N0 = nt * NT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int KS = n_pad / 16;

    // this wave's columns and the individuals they belong to
    const int c_first = min(N0 + wave * 32 * COLB, NS - 1);
    const int s_first = c_first / p;
    int col[COLB], li[COLB];
    uint32_t lq[COLB];
#pragma unroll
    for (int b = 0; b < COLB; ++b) {
        col[b] = N0 + wave * 32 * COLB + b * 32 + l32;
        if (col[b] < NS) {
            li[b] = col[b] / p - s_first;
            lq[b] = (uint32_t)(col[b] % p);
        } else {
            li[b] = 0;
            lq[b] = 0xFFFFu;
        }
    }
    uint32_t lq2[COLB];
#pragma unroll
    for (int b = 0; b < COLB; ++b) lq2[b] = lq[b] | (lq[b] << 16);
    const OneHotK ohk = onehot_consts();

    const uint32_t ring_addr = (uint32_t)(uintptr_t)(lds_void *)ring;
    auto issue = [&](int kt) {
        const int st = kt % NST;
        u32x4 *stage = ring + st * STAGE;
#pragma unroll
        for (int q = 0; q < A_INS; ++q) {
            const int ins = wave + 4 * q;                    // ((mat*KSTEPS + kk)*2 + h)*(MT/64) + gl
            const int gl = ins % (MT / 64), t = ins / (MT / 64);
            const int h = t & 1, kk = (t >> 1) % KSTEPS, mat = (t >> 1) / KSTEPS;
            const size_t gchunk = (((size_t)(mt * (MT / 64) + gl) * KS + kt * KSTEPS + kk) * 2 + h) * 64;
            const u32x4 *src = (mat ? Wlsw : Whsw) + gchunk + lane;
            __builtin_amdgcn_global_load_lds((const void *)src, (lds_void *)(stage + ins * 64), 16, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < KINS; ++q) {
            const int si = min(s_first + q * 16 + (lane >> 2), count - 1);
            const uint16_t *src = kidx + (size_t)si * n_pad + kt * KTILE + (lane & 3) * 8;
            __builtin_amdgcn_global_load_lds((const void *)src,
                                             (lds_void *)(stage + A_CHUNKS + (wave * KINS + q) * 64), 16, 0, 0);
        }
    };

    f32x16 acc[ROWB][COLB];
#pragma unroll
    for (int a = 0; a < ROWB; ++a)
#pragma unroll
        for (int b = 0; b < COLB; ++b) acc[a][b] = (f32x16)(0.0f);

    const int ktiles = n_pad / KTILE;
#pragma unroll
    for (int t = 0; t < NST - 1; ++t)
        if (t < ktiles) issue(t);
    // per-lane LDS byte addresses (stage 0); per-stage offset added below
    const uint32_t a_lane = ring_addr + (uint32_t)((half * MT + l32) * 16);
    uint32_t k_lane[COLB];
#pragma unroll
    for (int b = 0; b < COLB; ++b)
        k_lane[b] = ring_addr + (uint32_t)((A_CHUNKS + wave * KINS * 64 + li[b] * 4 + half) * 16);

    for (int kt = 0; kt < ktiles; ++kt) {
        // this wave's loads of tile kt are done once at most (younger tiles)*LPT remain
        const int younger = min(NST - 2, ktiles - 1 - kt);
        static_for<NST - 1>([&](auto Y) {
            if (younger == Y.value) vm_wait<Y.value * LPT>();
        });
        wg_barrier();
        if (kt + NST - 1 < ktiles) issue(kt + NST - 1);
        const uint32_t soff = (uint32_t)((kt % NST) * STAGE * 16);
        constexpr int RPK = 2 * ROWB + COLB;   // LDS reads per k-step
        u32x4 af[KSTEPS][2][ROWB], kv[KSTEPS][COLB];
        auto reads = [&](auto KK) {
            constexpr int kk = KK.value;
            static_for<2>([&](auto M) {
                static_for<ROWB>([&](auto A) {
                    af[kk][M.value][A.value] =
                        ds_read16<((M.value * KSTEPS + kk) * 2 * MT + A.value * 32) * 16>(a_lane + soff);
                });
            });
            static_for<COLB>([&](auto B) { kv[kk][B.value] = ds_read16<kk * 32>(k_lane[B.value] + soff); });
        };
        if constexpr (EARLY) static_for<KSTEPS>(reads);
        static_for<KSTEPS>([&](auto KK) {
            constexpr int kk = KK.value;
            if constexpr (EARLY) {
                lds_wait_n<(KSTEPS - 1 - kk) * RPK>();
            } else {
                reads(KK);
                lds_wait();
            }
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int a = 0; a < ROWB; ++a) pin(af[kk][m][a]);
#pragma unroll
            for (int b = 0; b < COLB; ++b) pin(kv[kk][b]);
            bf16x8 bfrag[COLB];
#pragma unroll
            for (int b = 0; b < COLB; ++b) {
                u32x4 bb;
                bb.x = onehot2_packed(kv[kk][b].x, lq2[b], ohk);
                bb.y = onehot2_packed(kv[kk][b].y, lq2[b], ohk);
                bb.z = onehot2_packed(kv[kk][b].z, lq2[b], ohk);
                bb.w = onehot2_packed(kv[kk][b].w, lq2[b], ohk);
                bfrag[b] = __builtin_bit_cast(bf16x8, bb);
            }
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int a = 0; a < ROWB; ++a) {
                    const bf16x8 afr = __builtin_bit_cast(bf16x8, af[kk][m][a]);
#pragma unroll
                    for (int b = 0; b < COLB; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr, bfrag[b], acc[a][b], 0, 0, 0);
                }
            // keep this step's products ahead of the next step's wait
            if constexpr (EARLY) __builtin_amdgcn_sched_barrier(0);
        });
    }

    pipe_epilogue<ROWB, COLB>(J, acc, col, lq, mt, nt, ring, NST * STAGE, mt, nullptr);
}

// K tiles of 64 (four 16-deep k-steps between barriers) with a rolling
// register pipeline: the LDS reads of step k+1 are in flight while step k's
// products run, the one-hot fragment of the second column block is built
// between the products of the first, and the barrier that hands over the
// next K tile is taken before the last step's products, whose operands are
// already in registers.
// K tiles kb..ke-1 (ke > kb) of row tile mt and column tile nt, summed into
// partial slot `slot` of each column.
template <int ROWB, int COLB, int NST, int KINS>
__device__ __forceinline__ void mfma_pipe_piece64(const MfmaJob &J, int mt, int nt, int kb, int ke, int slot,
                                                  u32x4 *ring)
{
    constexpr int MT = 32 * ROWB, NT = 128 * COLB, KTILE = 64, KSTEPS = KTILE / 16, KH = 2;
    constexpr int A_CHUNKS = 2 * KSTEPS * 2 * MT;   // [hi/lo][kk][half][row] 16-byte chunks per stage
    constexpr int K_CHUNKS = 4 * KINS * KH * 64;    // [wave][ins][k half][lane]
    constexpr int STAGE = A_CHUNKS + K_CHUNKS;
    constexpr int A_INS = A_CHUNKS / 64 / 4;        // 1 KB transfers per wave per tile for W
    constexpr int LPT = A_INS + KINS * KH;          // vector-memory instructions per wave per tile
    constexpr int RPK = 2 * ROWB + COLB;            // LDS reads per k-step
    static_assert(MT % 64 == 0 && (A_CHUNKS / 64) % 4 == 0 && RPK <= 15, "tile shape");
    static_assert(NST * STAGE == pipe_ring_chunks<ROWB, COLB, NST, KINS, 2>(), "ring size");
    const u32x4 *__restrict__ Whsw = J.Whsw;
    const u32x4 *__restrict__ Wlsw = J.Wlsw;
    const uint16_t *__restrict__ kidx = J.kidx;
    const int n_pad = J.n_pad, p = J.p, count = J.count, NS = J.NS;
    const int N0 = nt * NT;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: addresses stay scalar
    const int half = lane >> 5, l32 = lane & 31;
    const int KS = n_pad / 16;

    const int c_first = min(N0 + wave * 32 * COLB, NS - 1);
    const int s_first = c_first / p;
    int col[COLB], li[COLB];
    uint32_t lq[COLB];
#pragma unroll
    for (int b = 0; b < COLB; ++b) {
        col[b] = N0 + wave * 32 * COLB + b * 32 + l32;
        if (col[b] < NS) {
            li[b] = col[b] / p - s_first;
            lq[b] = (uint32_t)(col[b] % p);
        } else {
            li[b] = 0;
            lq[b] = 0xFFFFu;
        }
    }
    uint32_t lq2[COLB];
#pragma unroll
    for (int b = 0; b < COLB; ++b) lq2[b] = lq[b] | (lq[b] << 16);
    const OneHotK ohk = onehot_consts();

    const uint32_t ring_addr = (uint32_t)(uintptr_t)(lds_void *)ring;
    auto issue = [&](int kt) {   // K tile kb + kt
        u32x4 *stage = ring + (kt % NST) * STAGE;
        const int ka = kb + kt;
#pragma unroll
        for (int q = 0; q < A_INS; ++q) {
            const int ins = wave + 4 * q;                    // ((mat*KSTEPS + kk)*2 + h)*(MT/64) + gl
            const int gl = ins % (MT / 64), t = ins / (MT / 64);
            const int h = t & 1, kk = (t >> 1) % KSTEPS, mat = (t >> 1) / KSTEPS;
            const size_t gchunk = (((size_t)(mt * (MT / 64) + gl) * KS + ka * KSTEPS + kk) * 2 + h) * 64;
            const u32x4 *src = (mat ? Wlsw : Whsw) + gchunk + lane;
            __builtin_amdgcn_global_load_lds((const void *)src, (lds_void *)(stage + ins * 64), 16, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < KINS; ++q) {
            const int si = min(s_first + q * 16 + (lane >> 2), count - 1);
#pragma unroll
            for (int kh = 0; kh < KH; ++kh) {
                const uint16_t *src = kidx + (size_t)si * n_pad + ka * KTILE + kh * 32 + (lane & 3) * 8;
                __builtin_amdgcn_global_load_lds((const void *)src,
                                                 (lds_void *)(stage + A_CHUNKS + ((wave * KINS + q) * KH + kh) * 64),
                                                 16, 0, 0);
            }
        }
    };
    auto wait_tile = [&](int kt) {   // this wave's transfers of tile kt have landed
        const int younger = min(NST - 2, ke - kb - 1 - kt);
        static_for<NST - 1>([&](auto Y) {
            if (younger == Y.value) vm_wait<Y.value * LPT>();
        });
    };

    f32x16 acc[ROWB][COLB];
#pragma unroll
    for (int a = 0; a < ROWB; ++a)
#pragma unroll
        for (int b = 0; b < COLB; ++b) acc[a][b] = (f32x16)(0.0f);

    const uint32_t a_lane = ring_addr + (uint32_t)((half * MT + l32) * 16);
    uint32_t k_lane[COLB];
#pragma unroll
    for (int b = 0; b < COLB; ++b)
        k_lane[b] = ring_addr +
                    (uint32_t)((A_CHUNKS + (wave * KINS + li[b] / 16) * KH * 64 + (li[b] % 16) * 4 + half) * 16);

    u32x4 af[2][2][ROWB], kv[2][COLB];   // [register set][hi/lo][row block]
    auto reads = [&](auto R, auto KK, uint32_t soff) {
        constexpr int r = decltype(R)::value, kk = decltype(KK)::value;
        static_for<2>([&](auto M) {
            static_for<ROWB>([&](auto A) {
                af[r][M.value][A.value] =
                    ds_read16<((M.value * KSTEPS + kk) * 2 * MT + A.value * 32) * 16>(a_lane + soff);
            });
        });
        static_for<COLB>([&](auto B) {
            kv[r][B.value] = ds_read16<((kk / 2) * 64 + (kk % 2) * 2) * 16>(k_lane[B.value] + soff);
        });
    };

    const int ktiles = ke - kb;
#pragma unroll
    for (int t = 0; t < NST - 1; ++t)
        if (t < ktiles) issue(t);
    wait_tile(0);
    wg_barrier();
    if (NST - 1 < ktiles) issue(NST - 1);
    // The epilogue's operands go to the stage after the last K tile's, free
    // from the hand-over before the last tile on (from the start if there are
    // fewer K tiles than stages), and land while the last tile's products run.
    const bool early = epi_stage_bytes<MT, NT>(J, nt) <= (int)sizeof(u32x4) * STAGE;
    u32x4 *const pre = ring + (ktiles % NST) * STAGE;
    if (early && ktiles < NST) epi_stage_issue<MT, NT>(J, mt, nt, pre);
    reads(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{}, 0u);

    for (int kt = 0; kt < ktiles; ++kt) {
        const uint32_t soff = (uint32_t)((kt % NST) * STAGE * 16);
        static_for<KSTEPS>([&](auto KK) {
            constexpr int kk = KK.value, r = kk & 1;
            if constexpr (kk + 1 < KSTEPS) {
                reads(std::integral_constant<int, r ^ 1>{}, std::integral_constant<int, kk + 1>{}, soff);
                lds_wait_n<RPK>();
            } else {
                lds_wait_n<0>();   // every read of tile kt has landed
                if (kt + 1 < ktiles) {
                    wait_tile(kt + 1);
                    wg_barrier();   // tile kt+1 visible to all waves; tile kt's stage is free
                    if (kt + NST < ktiles)
                        issue(kt + NST);
                    else if (early && kt + NST == ktiles)
                        epi_stage_issue<MT, NT>(J, mt, nt, pre);
                    reads(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{},
                          (uint32_t)(((kt + 1) % NST) * STAGE * 16));
                }
            }
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int a = 0; a < ROWB; ++a) pin(af[r][m][a]);
#pragma unroll
            for (int b = 0; b < COLB; ++b) pin(kv[r][b]);
            bf16x8 bfrag[COLB];
#pragma unroll
            for (int b = 0; b < COLB; ++b) {
                u32x4 bb;
                bb.x = onehot2_packed(kv[r][b].x, lq2[b], ohk);
                bb.y = onehot2_packed(kv[r][b].y, lq2[b], ohk);
                bb.z = onehot2_packed(kv[r][b].z, lq2[b], ohk);
                bb.w = onehot2_packed(kv[r][b].w, lq2[b], ohk);
                bfrag[b] = __builtin_bit_cast(bf16x8, bb);
            }
            // column block by column block, so that the next block's one-hot
            // fragment is built while this block's products run
#pragma unroll
            for (int b = 0; b < COLB; ++b)
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int a = 0; a < ROWB; ++a)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, af[r][m][a]), bfrag[b], acc[a][b], 0, 0, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);   // one-hot of block 0
            static_for<COLB - 1>([&](auto) {
                static_for<2 * ROWB>([&](auto) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
                });
            });
            __builtin_amdgcn_sched_group_barrier(0x008, 2 * ROWB, 0);
            __builtin_amdgcn_sched_barrier(0);
        });
    }

    pipe_epilogue<ROWB, COLB>(J, acc, col, lq, mt, nt, ring, NST * STAGE, slot, early ? pre : nullptr);
}

// Work unit `tile` (row-tile major over the column tiles) of the K-64
// product: row tile mt over K tiles 0..KT-1, or, on the folded W (C
// symmetric; zero below the diagonal), over K tiles KPR*mt..KT-1 only (KPR K
// tiles per row tile).  Folded units shrink with mt, so the row-tile-major
// order hands them out longest first.
template <int ROWB, int COLB, int NST, int KINS>
__device__ __forceinline__ void mfma_pipe_unit64(const MfmaJob &J, int tile, u32x4 *ring)
{
    constexpr int KPR = 32 * ROWB / 64;
    const int mt = tile / J.n_nt, nt = tile % J.n_nt;
    mfma_pipe_piece64<ROWB, COLB, NST, KINS>(J, mt, nt, J.fold ? KPR * mt : 0, J.n_pad / 64, mt, ring);
}

// Workgroup -> tile.  XCD-major (blockIdx % 8 picks the XCD, which walks a
// contiguous range of tiles, so its L2 keeps its own W row panels) for equal
// tiles; round robin (consecutive tiles on consecutive XCDs, every XCD
// stepping through the row tiles together) for the folded product, whose
// tiles shrink along the list.
__device__ __forceinline__ int pipe_tile_of_block(int tiles, bool round_robin)
{
    if (round_robin) return blockIdx.x;
    const int per = (tiles + 7) / 8;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

template <int ROWB, int COLB, int NST, int KINS, int OCC, int EARLY>
__global__ __launch_bounds__(256, OCC) void k_eval_mfma_pipe(MfmaJob J)
{
    __shared__ __align__(16) u32x4 ring[pipe_ring_chunks<ROWB, COLB, NST, KINS, EARLY>()];
    const int tiles = J.n_rt * J.n_nt;
    const int tile = pipe_tile_of_block(tiles, J.fold);
    if (tile >= tiles) return;
    if constexpr (EARLY == 2)
        mfma_pipe_unit64<ROWB, COLB, NST, KINS>(J, tile, ring);
    else
        mfma_pipe_tile<ROWB, COLB, NST, KINS, EARLY>(J, tile, ring);
}

// One launch over the tiles of several contexts: the concatenated tile list
// (each context row-tile major) is split into 8 contiguous ranges, one per
// XCD (blockIdx % 8), so every XCD walks whole row panels; round robin when
// a context is folded.  The grid may exceed the composition's tiles (a
// captured graph's capacity): the extra workgroups return.
template <int ROWB, int COLB, int NST, int KINS, int OCC, int EARLY>
__global__ __launch_bounds__(256, OCC) void k_eval_mfma_pipe_group(const GroupHdr *__restrict__ hdr,
                                                                   const MfmaJob *__restrict__ jobs)
{
    __shared__ __align__(16) u32x4 ring[pipe_ring_chunks<ROWB, COLB, NST, KINS, EARLY>()];
    const int total_tiles = hdr->total_tiles, round_robin = hdr->round_robin, njobs = hdr->njobs;
    if (!round_robin && (int)(blockIdx.x >> 3) >= (total_tiles + 7) / 8) return;
    const int t = pipe_tile_of_block(total_tiles, round_robin);
    if (t >= total_tiles) return;
    int lo = 0, hi = njobs - 1;   // last job with tile_start <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_start <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    const MfmaJob J = jobs[lo];
    if constexpr (EARLY == 2)
        mfma_pipe_unit64<ROWB, COLB, NST, KINS>(J, t - J.tile_start, ring);
    else
        mfma_pipe_tile<ROWB, COLB, NST, KINS, EARLY>(J, t - J.tile_start, ring);
}

// T_s = sum of the individual's p*n_mt partials (partial[t][column], row tile
// t, the individual's p columns contiguous in each), one wave per individual
// with a fixed reduction order; cost assembly
// f = ((chi*Cc) + (alpha*T)) + (delta*Dd) and its relative error bound.
// resid: the split's residual bound; terms: non-zero addends per output and
// cluster member (2 or 3 parts).
__device__ __forceinline__ void finalize_body(const double *__restrict__ partial, const int32_t *__restrict__ cmax,
                                              int count, int p, int n_mt, int n, int c_f32, double chi, double alpha,
                                              double delta, double scale, double resid, double terms,
                                              double *__restrict__ cost, double *__restrict__ parts,
                                              double *__restrict__ eps, int blk)
{
    const int s = blk * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= count) return;
    const int len = p * n_mt;
    const size_t NS = (size_t)count * p;
    const double *ps = partial + (size_t)s * p;
    double v = 0.0;
    constexpr int MAXIT = 8;
    if (len <= 64 * MAXIT) {
        // every load of the lane issued before its sum (the same sum)
        double x[MAXIT];
#pragma unroll
        for (int it = 0; it < MAXIT; ++it) {
            const int e = lane + 64 * it;
            x[it] = e < len ? ps[(size_t)(e / p) * NS + e % p] : 0.0;
        }
#pragma unroll
        for (int it = 0; it < MAXIT; ++it)
            if (lane + 64 * it < len) v += x[it];
    } else {
        for (int e = lane; e < len; e += 64) v += ps[(size_t)(e / p) * NS + e % p];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) {
        const double T = v;
        const double Cc = parts[3 * (size_t)s], Dd = parts[3 * (size_t)s + 2];
        parts[3 * (size_t)s + 1] = T;
        cost[s] = (((chi * Cc) + (alpha * T)) + (delta * Dd)) * scale;
        // split residual + FP32 accumulation of at most terms*cmax non-zero
        // addends per output (any faithful rounding, relative to the mass of
        // the parts) + FP32 hub distances + binary64 sums
        eps[s] = resid + gamma_k(terms * cmax[s], kU32Faithful) * kHiLoMass + (c_f32 ? 0.0 : kU32) +
                 gamma_k((double)n + (double)len + 8.0, kU64) + gamma_k(n + 2.0, kU64) + gamma_k(8.0, kU64) + 1e-9;
    }
}

__global__ __launch_bounds__(256) void k_finalize_split(const double *__restrict__ partial,
                                                        const int32_t *__restrict__ cmax, int count, int p, int n_mt,
                                                        int n, int c_f32, double chi, double alpha, double delta,
                                                        double scale, double resid, double terms,
                                                        double *__restrict__ cost, double *__restrict__ parts,
                                                        double *__restrict__ eps)
{
    finalize_body(partial, cmax, count, p, n_mt, n, c_f32, chi, alpha, delta, scale, resid, terms, cost, parts, eps,
                  blockIdx.x);
}

__global__ __launch_bounds__(256) void k_finalize_group(const GroupHdr *__restrict__ hdr,
                                                        const TickJob *__restrict__ jobs)
{
    if ((int)blockIdx.x >= hdr->blocks[kTickFinal]) return;
    const TickJob &J = jobs[tick_job(jobs, hdr->njobs, kTickFinal, blockIdx.x)];
    const DevPtrs &P = J.P;
    const Dims &d = J.d;
    finalize_body(P.partial, P.cmax, d.S, d.p, J.n_mt, d.n, d.c_f32, d.chi, d.alpha, d.delta, d.scale, kSplitResidual,
                  2.0, P.cost, P.parts, P.eps, blockIdx.x - J.start[kTickFinal]);
}

template <int ROWB, int COLB, int KT, int OCC, int NP = 2>
static hipError_t mfma_launch(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st)
{
    const int MT = 32 * ROWB, NT = 128 * COLB;
    const int NS = count * d.p;
    const int n_mt = d.n_pad / MT;
    const int n_nt = (NS + NT - 1) / NT;
    const int tiles = n_mt * n_nt;
    const int per = (tiles + 7) / 8;
    k_eval_mfma<ROWB, COLB, KT, OCC, NP><<<per * 8, 256, 0, st>>>(P.Whi, P.Wlo, P.Wmd, kidx, P.Ch32, d.n, d.n_pad,
                                                                 d.p, NS, n_mt, n_nt, P.partial);
    return hipGetLastError();
}

// Tile configurations the three-part split runs in (register-staged, and
// their three LDS stages within the static limit).
bool mfma_split3_config(int cfg) { return cfg == 0 || cfg == 2 || cfg == 3 || cfg == 5; }

template <int ROWB, int COLB, int NST, int KINS, int OCC, int EARLY>
static hipError_t pipe_launch(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st)
{
    const int MT = 32 * ROWB, NT = 128 * COLB;
    const int NS = count * d.p;
    const int n_mt = d.n_pad / MT;
    const int n_nt = (NS + NT - 1) / NT;
    const int tiles = n_mt * n_nt;
    const int per = (tiles + 7) / 8;
    const int fold = EARLY == 2 && d.sym;
    MfmaJob J{(const u32x4 *)(fold ? P.Wfhsw : P.Whsw), (const u32x4 *)(fold ? P.Wflsw : P.Wlsw), kidx, P.Ch32,
              P.partial, d.n, d.n_pad, d.p, count, NS, n_mt, n_nt, 0, n_mt, fold};
    k_eval_mfma_pipe<ROWB, COLB, NST, KINS, OCC, EARLY><<<per * 8, 256, 0, st>>>(J);
    return hipGetLastError();
}

// Individuals one wave's columns can touch, in 16-individual transfers.
static int kidx_transfers(int colb, int p) { return (((32 * colb + p - 2) / p + 2) + 15) / 16; }

template <int ROWB, int COLB, int NST, int OCC, int EARLY = 0>
static hipError_t pipe_dispatch(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st)
{
    const int kins = kidx_transfers(COLB, d.p);
    if (kins <= 1) return pipe_launch<ROWB, COLB, NST, 1, OCC, EARLY>(P, d, kidx, count, st);
    if (kins <= 2) return pipe_launch<ROWB, COLB, NST, 2, OCC, EARLY>(P, d, kidx, count, st);
    return mfma_launch<4, 2, 32, 2>(P, d, kidx, count, st);   // few hubs: per-lane fragment loads
}

// Tile configurations of the batched kernel: {rows/32 per wave, columns/32
// per wave, K tile, minimum workgroups per CU, pipeline stages (0: register
// staging, double-buffered LDS)}.
struct MfmaCfg { int rowb, colb, kt, occ, nst; };
static const MfmaCfg kMfmaCfgs[] = {{4, 2, 32, 2, 0}, {4, 2, 64, 1, 0}, {4, 4, 32, 1, 0}, {2, 4, 32, 2, 0},
                                    {4, 4, 64, 1, 0}, {2, 2, 64, 2, 0}, {4, 2, 32, 1, 4}, {4, 2, 32, 2, 3},
                                    {4, 4, 32, 1, 4}, {4, 4, 32, 1, 3}, {2, 4, 32, 2, 4},
                                    // the same shapes with early LDS reads
                                    {4, 2, 32, 2, 3}, {4, 2, 32, 1, 4}, {2, 4, 32, 2, 4},
                                    // four stages at two workgroups per CU (fits for one hub-position transfer)
                                    {4, 2, 32, 2, 4}, {4, 2, 32, 2, 4},
                                    // K tiles of 64 with the rolling register pipeline
                                    {4, 2, 64, 2, 2}, {4, 2, 64, 1, 3},
                                    // ... and 128 x 512 workgroup tiles, one workgroup per CU
                                    {4, 4, 64, 1, 3}, {4, 4, 64, 1, 2},
                                    // ... and 64 x 512 workgroup tiles, two workgroups per CU
                                    {2, 4, 64, 2, 3}, {2, 4, 64, 2, 2}};
constexpr int kNumMfmaCfgs = sizeof(kMfmaCfgs) / sizeof(kMfmaCfgs[0]);

int mfma_num_configs() { return kNumMfmaCfgs; }
int mfma_rows_per_tile(int cfg) { return 32 * kMfmaCfgs[cfg].rowb; }
int mfma_pipelined(int cfg) { return kMfmaCfgs[cfg].nst > 0; }
int mfma_cols_per_tile(int cfg) { return 128 * kMfmaCfgs[cfg].colb; }
int mfma_k_tile(int cfg) { return kMfmaCfgs[cfg].kt; }

hipError_t launch_mfma(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (d.prec == kSplit3BF16) {
        switch (d.mfma_cfg) {
        case 0: return mfma_launch<4, 2, 32, 2, 3>(P, d, kidx, count, st);
        case 2: return mfma_launch<4, 4, 32, 1, 3>(P, d, kidx, count, st);
        case 3: return mfma_launch<2, 4, 32, 2, 3>(P, d, kidx, count, st);
        case 5: return mfma_launch<2, 2, 64, 2, 3>(P, d, kidx, count, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (d.mfma_cfg) {
    case 0: return mfma_launch<4, 2, 32, 2>(P, d, kidx, count, st);
    case 1: return mfma_launch<4, 2, 64, 1>(P, d, kidx, count, st);
    case 2: return mfma_launch<4, 4, 32, 1>(P, d, kidx, count, st);
    case 3: return mfma_launch<2, 4, 32, 2>(P, d, kidx, count, st);
    case 4: return mfma_launch<4, 4, 64, 1>(P, d, kidx, count, st);
    case 5: return mfma_launch<2, 2, 64, 2>(P, d, kidx, count, st);
    case 6: return pipe_dispatch<4, 2, 4, 1>(P, d, kidx, count, st);
    case 7: return pipe_dispatch<4, 2, 3, 2>(P, d, kidx, count, st);
    case 8: return pipe_dispatch<4, 4, 4, 1>(P, d, kidx, count, st);
    case 9: return pipe_dispatch<4, 4, 3, 1>(P, d, kidx, count, st);
    case 10: return pipe_dispatch<2, 4, 4, 2>(P, d, kidx, count, st);
    case 11: return pipe_dispatch<4, 2, 3, 2, 1>(P, d, kidx, count, st);
    case 12: return pipe_dispatch<4, 2, 4, 1, 1>(P, d, kidx, count, st);
    case 13: return pipe_dispatch<2, 4, 4, 2, 1>(P, d, kidx, count, st);
    case 14: return pipe_dispatch<4, 2, 4, 2>(P, d, kidx, count, st);
    case 15: return pipe_dispatch<4, 2, 4, 2, 1>(P, d, kidx, count, st);
    case 16: return pipe_dispatch<4, 2, 2, 2, 2>(P, d, kidx, count, st);
    case 17: return pipe_dispatch<4, 2, 3, 1, 2>(P, d, kidx, count, st);
    case 18: return pipe_dispatch<4, 4, 3, 1, 2>(P, d, kidx, count, st);
    case 19: return pipe_dispatch<4, 4, 2, 1, 2>(P, d, kidx, count, st);
    case 20: return pipe_dispatch<2, 4, 3, 2, 2>(P, d, kidx, count, st);
    default: return pipe_dispatch<2, 4, 2, 2, 2>(P, d, kidx, count, st);
    }
}

// Whether configuration cfg evaluates a context on the folded W: the K-64
// pipelined kernels do when C is symmetric.
bool mfma_folds(const Dims &d, int cfg)
{
    const MfmaCfg &c = kMfmaCfgs[cfg];
    return d.sym && c.nst > 0 && c.kt == 64 && kidx_transfers(c.colb, d.p) <= 2;
}

// The layout of the W split that configuration cfg reads for this context:
// the register-staged kernels (and the few-hub fallback of the pipelined
// ones) read it row-major, the pipelined ones in fragment order, of the
// folded W when they fold.
int mfma_w_layout(const Dims &d, int cfg)
{
    const MfmaCfg &c = kMfmaCfgs[cfg];
    if (c.nst == 0 || kidx_transfers(c.colb, d.p) > 2) return kWRowMajor;
    return mfma_folds(d, cfg) ? kWFragFolded : kWFrag;
}

// Row tiles the partials of configuration cfg use for p hubs.
int mfma_partial_tiles(const Dims &d, int cfg)
{
    int rows = mfma_rows_per_tile(cfg);
    if (mfma_pipelined(cfg) && kidx_transfers(kMfmaCfgs[cfg].colb, d.p) > 2) rows = 128;
    return d.n_pad / rows;
}

hipError_t launch_finalize(const DevPtrs &P, const Dims &d, int count, int cfg, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int n_mt = mfma_partial_tiles(d, cfg);
    const bool three = d.prec == kSplit3BF16;
    k_finalize_split<<<(count + 3) / 4, 256, 0, st>>>(P.partial, P.cmax, count, d.p, n_mt, d.n, d.c_f32, d.chi,
                                                      d.alpha, d.delta, d.scale, three ? kSplit3Residual : kSplitResidual,
                                                      three ? 3.0 : 2.0, P.cost, P.parts, P.eps);
    return hipGetLastError();
}

int finalize_blocks(int count) { return (count + 3) / 4; }

hipError_t launch_finalize_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, int blocks, hipStream_t st)
{
    if (njobs <= 0 || blocks <= 0) return hipSuccess;
    k_finalize_group<<<blocks, 256, 0, st>>>(hdr, jobs);
    return hipGetLastError();
}

hipError_t launch_eval_split(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st,
                             hipEvent_t ev0, hipEvent_t ev1)
{
    if (count <= 0) return hipSuccess;
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    if ((e = launch_mfma(P, d, kidx, count, st)) != hipSuccess) return e;
    if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
    return launch_finalize(P, d, count, d.mfma_cfg, st);
}

// Grouped launch over several contexts' populations (one tile configuration,
// pipelined, at least 3 hubs per context).
bool mfma_groupable(const Dims &d, int cfg)
{
    return mfma_pipelined(cfg) && kidx_transfers(kMfmaCfgs[cfg].colb, d.p) <= 2;
}

size_t mfma_job_bytes() { return sizeof(MfmaJob); }

// Fill jobs (host array, one per context) and return the total tile count.
int mfma_fill_jobs(const DevPtrs *const *P, const Dims *const *d, int njobs, int cfg, void *jobs_host)
{
    MfmaJob *J = (MfmaJob *)jobs_host;
    const int MT = mfma_rows_per_tile(cfg), NT = mfma_cols_per_tile(cfg);
    int start = 0;
    for (int j = 0; j < njobs; ++j) {
        const int NS = d[j]->S * d[j]->p;
        const int n_rt = d[j]->n_pad / MT, n_nt = (NS + NT - 1) / NT;
        const int fold = mfma_folds(*d[j], cfg);
        J[j] = MfmaJob{(const u32x4 *)(fold ? P[j]->Wfhsw : P[j]->Whsw), (const u32x4 *)(fold ? P[j]->Wflsw : P[j]->Wlsw),
                       P[j]->kidx, P[j]->Ch32, P[j]->partial, d[j]->n, d[j]->n_pad, d[j]->p, d[j]->S, NS,
                       n_rt, n_nt, start, n_rt, fold};
        start += n_rt * n_nt;
    }
    return start;
}

template <int ROWB, int COLB, int NST, int KINS, int OCC, int EARLY>
static hipError_t group_launch(const GroupHdr *hdr, const void *d_jobs, int grid, hipStream_t st)
{
    k_eval_mfma_pipe_group<ROWB, COLB, NST, KINS, OCC, EARLY><<<grid, 256, 0, st>>>(hdr, (const MfmaJob *)d_jobs);
    return hipGetLastError();
}

template <int ROWB, int COLB, int NST, int OCC, int EARLY = 0>
static hipError_t group_dispatch(int kins, const GroupHdr *hdr, const void *d_jobs, int grid, hipStream_t st)
{
    if (kins <= 1) return group_launch<ROWB, COLB, NST, 1, OCC, EARLY>(hdr, d_jobs, grid, st);
    return group_launch<ROWB, COLB, NST, 2, OCC, EARLY>(hdr, d_jobs, grid, st);
}

int mfma_group_kins(int cfg, int min_p) { return kidx_transfers(kMfmaCfgs[cfg].colb, min_p); }

// grid: workgroups, a multiple of 8 and at least the composition's tiles
// rounded up to one; kins: hub-position transfers the kernel stages (enough
// for the smallest hub count of the composition).
hipError_t launch_mfma_group(const GroupHdr *hdr, const void *d_jobs, int grid, int cfg, int kins, hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    if (kins > 2 || grid % 8) return hipErrorInvalidValue;
    switch (cfg) {
    case 6: return group_dispatch<4, 2, 4, 1>(kins, hdr, d_jobs, grid, st);
    case 7: return group_dispatch<4, 2, 3, 2>(kins, hdr, d_jobs, grid, st);
    case 8: return group_dispatch<4, 4, 4, 1>(kins, hdr, d_jobs, grid, st);
    case 9: return group_dispatch<4, 4, 3, 1>(kins, hdr, d_jobs, grid, st);
    case 10: return group_dispatch<2, 4, 4, 2>(kins, hdr, d_jobs, grid, st);
    case 11: return group_dispatch<4, 2, 3, 2, 1>(kins, hdr, d_jobs, grid, st);
    case 12: return group_dispatch<4, 2, 4, 1, 1>(kins, hdr, d_jobs, grid, st);
    case 13: return group_dispatch<2, 4, 4, 2, 1>(kins, hdr, d_jobs, grid, st);
    case 14: return group_dispatch<4, 2, 4, 2>(kins, hdr, d_jobs, grid, st);
    case 15: return group_dispatch<4, 2, 4, 2, 1>(kins, hdr, d_jobs, grid, st);
    case 16: return group_dispatch<4, 2, 2, 2, 2>(kins, hdr, d_jobs, grid, st);
    case 17: return group_dispatch<4, 2, 3, 1, 2>(kins, hdr, d_jobs, grid, st);
    case 18: return group_dispatch<4, 4, 3, 1, 2>(kins, hdr, d_jobs, grid, st);
    case 19: return group_dispatch<4, 4, 2, 1, 2>(kins, hdr, d_jobs, grid, st);
    case 20: return group_dispatch<2, 4, 3, 2, 2>(kins, hdr, d_jobs, grid, st);
    case 21: return group_dispatch<2, 4, 2, 2, 2>(kins, hdr, d_jobs, grid, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hubga
