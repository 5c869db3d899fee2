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

namespace hubga {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int KT = 32;            // K tile staged per iteration
constexpr int LDS_ROW = KT + 8;   // bf16 elements per LDS row (16-byte pad against bank conflicts)

__device__ __forceinline__ uint32_t onehot2(uint32_t kk, uint32_t lq)
{
    uint32_t lo = ((kk & 0xFFFFu) == lq) ? 0x3F80u : 0u;
    uint32_t hi = ((kk >> 16) == lq) ? 0x3F800000u : 0u;
    return lo | hi;
}

template <int ROWB, int COLB>
__global__ __launch_bounds__(256) void k_eval_mfma(const uint16_t *__restrict__ Whi, const uint16_t *__restrict__ Wlo,
                                                   const uint16_t *__restrict__ kidx, const float *__restrict__ Ch32,
                                                   int n, int n_pad, int p, int NS, int n_mt, int n_nt,
                                                   double *__restrict__ partial)
{
    constexpr int MT = 32 * ROWB;            // rows per tile
    constexpr int NT = 4 * 32 * COLB;        // columns per tile
    constexpr int A_ELEMS = MT * LDS_ROW;    // one matrix, one stage
    __shared__ __align__(16) uint16_t sA[2][2][A_ELEMS];   // [stage][hi/lo]

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
    int col[COLB], ind[COLB];
    uint32_t lq[COLB];
#pragma unroll
    for (int b = 0; b < COLB; ++b) {
        col[b] = N0 + wave * 32 * COLB + b * 32 + l32;
        if (col[b] < NS) {
            ind[b] = col[b] / p;
            lq[b] = (uint32_t)(col[b] % p);
        } else {
            ind[b] = 0;
            lq[b] = 0xFFFFu;   // matches no hub position: zero column
        }
    }

    f32x16 acc[ROWB][COLB];
#pragma unroll
    for (int a = 0; a < ROWB; ++a)
#pragma unroll
        for (int b = 0; b < COLB; ++b) acc[a][b] = (f32x16)(0.0f);

    // global -> LDS staging: each matrix tile is MT rows x KT k = MT*4 chunks of 16 B
    constexpr int CHUNKS = MT * (KT / 8);
    constexpr int PER_THREAD = CHUNKS / 256;   // per matrix
    static_assert(CHUNKS % 256 == 0, "tile must split evenly over 256 threads");
    u32x4 stage_hi[PER_THREAD], stage_lo[PER_THREAD];

    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            int c = tid + q * 256;
            int row = c >> 2, kq = (c & 3) * 8;
            size_t off = (size_t)(M0 + row) * n_pad + k0 + kq;
            stage_hi[q] = *(const u32x4 *)(Whi + off);
            stage_lo[q] = *(const u32x4 *)(Wlo + off);
        }
    };
    auto lstore = [&](int st) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            int c = tid + q * 256;
            int row = c >> 2, kq = (c & 3) * 8;
            *(u32x4 *)(&sA[st][0][row * LDS_ROW + kq]) = stage_hi[q];
            *(u32x4 *)(&sA[st][1][row * LDS_ROW + kq]) = stage_lo[q];
        }
    };

    const int ktiles = n_pad / KT;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < ktiles) gload((kt + 1) * KT);
#pragma unroll
        for (int kk = 0; kk < KT / 16; ++kk) {
            const int kbase = kt * KT + kk * 16 + half * 8;
            bf16x8 bfrag[COLB];
#pragma unroll
            for (int b = 0; b < COLB; ++b) {
                u32x4 kv = *(const u32x4 *)(kidx + (size_t)ind[b] * n_pad + kbase);
                uint32_t l2 = lq[b];
                u32x4 bb;
                bb.x = onehot2(kv.x, l2);
                bb.y = onehot2(kv.y, l2);
                bb.z = onehot2(kv.z, l2);
                bb.w = onehot2(kv.w, l2);
                bfrag[b] = __builtin_bit_cast(bf16x8, bb);
            }
#pragma unroll
            for (int a = 0; a < ROWB; ++a) {
                const int lrow = (a * 32 + l32) * LDS_ROW + kk * 16 + half * 8;
                bf16x8 ahi = __builtin_bit_cast(bf16x8, *(const u32x4 *)(&sA[cur][0][lrow]));
                bf16x8 alo = __builtin_bit_cast(bf16x8, *(const u32x4 *)(&sA[cur][1][lrow]));
#pragma unroll
                for (int b = 0; b < COLB; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bfrag[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bfrag[b], acc[a][b], 0, 0, 0);
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
            const int s = ind[b];
            const uint16_t *krow = kidx + (size_t)s * n_pad;
            const float *ch = Ch32 + (size_t)s * p * p + lq[b];
#pragma unroll
            for (int a = 0; a < ROWB; ++a) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int i = M0 + a * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
                    if (i < n) {
                        const int k = krow[i];
                        sum += (double)acc[a][b][v] * (double)ch[k * p];
                    }
                }
            }
        }
        sum += __shfl_xor(sum, 32);
        if (half == 0 && col[b] < NS) partial[(size_t)mt * NS + col[b]] = sum;
    }
}

// T_s = sum over l, then over row tiles, of the partials; cost assembly
// f = ((chi*Cc) + (alpha*T)) + (delta*Dd) and its relative error bound.
__global__ void k_finalize_split(const double *__restrict__ partial, const int32_t *__restrict__ cmax, int count,
                                 int p, int n_mt, int n, int c_f32, double chi, double alpha, double delta,
                                 double scale, double *__restrict__ cost, double *__restrict__ parts,
                                 double *__restrict__ eps)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const int NS = count * p;
    double T = 0.0;
    for (int l = 0; l < p; ++l)
        for (int mt = 0; mt < n_mt; ++mt) T += partial[(size_t)mt * NS + (size_t)s * p + l];
    const double Cc = parts[3 * (size_t)s], Dd = parts[3 * (size_t)s + 2];
    parts[3 * (size_t)s + 1] = T;
    cost[s] = (((chi * Cc) + (alpha * T)) + (delta * Dd)) * scale;
    // split residual + FP32 accumulation of at most 2*cmax non-zero addends per
    // output (any faithful rounding) + FP32 hub distances + binary64 sums
    double e = kSplitResidual + gamma_k(2.0 * cmax[s], kU32Faithful) + (c_f32 ? 0.0 : kU32) +
               gamma_k((double)n + (double)p * n_mt + 4.0, kU64) + gamma_k(n + 2.0, kU64) + gamma_k(8.0, kU64) + 1e-9;
    eps[s] = e;
}

template <int ROWB, int COLB>
static hipError_t mfma_launch(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st)
{
    const int MT = 32 * ROWB, NT = 128 * COLB;
    const int NS = count * d.p;
    const int n_mt = d.n_pad / MT;
    const int n_nt = (NS + NT - 1) / NT;
    const int tiles = n_mt * n_nt;
    const int per = (tiles + 7) / 8;
    k_eval_mfma<ROWB, COLB><<<per * 8, 256, 0, st>>>(P.Whi, P.Wlo, kidx, P.Ch32, d.n, d.n_pad, d.p, NS, n_mt, n_nt,
                                                     P.partial);
    return hipGetLastError();
}

int mfma_row_tiles(const Dims &d) { return d.n_pad / kMfmaRowsPerTile; }

hipError_t launch_eval_split(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st,
                             hipEvent_t ev0, hipEvent_t ev1)
{
    if (count <= 0) return hipSuccess;
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    e = mfma_launch<4, 2>(P, d, kidx, count, st);
    if (e != hipSuccess) return e;
    if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
    const int n_mt = d.n_pad / kMfmaRowsPerTile;
    k_finalize_split<<<(count + 255) / 256, 256, 0, st>>>(P.partial, P.cmax, count, d.p, n_mt, d.n, d.c_f32, d.chi,
                                                          d.alpha, d.delta, d.scale, P.cost, P.parts, P.eps);
    return hipGetLastError();
}

}  // namespace hubga
