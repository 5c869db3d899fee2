// Internal declarations shared by the HIP translation units of libhubga.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hubga {

constexpr int kMaxP = 64;          // hub lists live in LDS; p*p doubles fit easily
constexpr int kMaxN = 8192;        // canonical kernel keeps n partial sums t_j in LDS
constexpr int kMaxIsland = 1024;   // one island per workgroup in selection
constexpr uint16_t kNoHub = 0xFFFF;
constexpr int kMfmaMinRows = 64;        // smallest row tile of the batched kernel (sizes its partials)
constexpr int kPad = 128;               // n is padded to a multiple of this for the bf16 copies

enum Precision { kFP64 = 0, kFP32 = 1, kSplitBF16 = 2, kSplit3BF16 = 3 };
// Modes whose fitness is the bf16 matrix-core product (two or three parts of W).
__host__ __device__ inline bool split_mode(int prec) { return prec == kSplitBF16 || prec == kSplit3BF16; }
// Layouts of the bf16 hi/lo split of W (one pair of buffers per context).
enum WLayout { kWRowMajor = 0, kWFrag = 1, kWFragFolded = 2 };

// Running state of an exhaustive search (enumerate.hip).
struct EnumState {
    double best_cost;       // exact scaled cost of the best set so far (+inf before any)
    double best_parts[3];   // its {Cc, T, Dd}
    int64_t best_rank;      // its lexicographic rank (-1 before any)
    int64_t rechecks;       // sets re-evaluated exactly
    int cand_count;         // sets listed for exact re-evaluation in the current chunk
    int pad;
};

// Device pointers of one context, carved out of the workspace.
struct DevPtrs {
    void *C;            // n*n, instance dtype
    void *Ct;           // n*n transposed (== C when C is symmetric): hub rows for allocation
    float *Ct32;        // Ct rounded to FP32 (== Ct for an FP32 instance)
    void *W;            // n*n, instance dtype
    double *Ctr;        // n*n all-pairs shortest-path distances of C (multi-hop routing), else null:
                        //   the transfer term's C[h_k][h_l] is read from here when set
    float *W32;         // n*n FP32 copy (FP32 mode with a binary64 instance), else null
    // The bf16 hi/lo split of W: n_pad*n_pad bf16 bits each (split mode), else
    // null.  One pair of buffers holds the layout the current tile
    // configuration reads (WLayout), rewritten when the configuration needs
    // another; the names below alias it by layout:
    uint16_t *Whi;      //   row-major
    uint16_t *Wlo;
    uint16_t *Wmd;      //   the middle part of the three-part split (row-major), else null
    uint16_t *Whsw;     //   fragment order: 16-byte chunk (row r, k 8c..8c+7) at
    uint16_t *Wlsw;     //   ((r/64 * n_pad/16 + k/16)*2 + (k/8)%2)*64 + r%64
    uint16_t *Wfhsw;    //   fragment order of the folded W (C symmetric): W_rk + W_kr above
    uint16_t *Wflsw;    //   the diagonal, W_rr on it, zero below
    double *O, *D, *dsum;
    int32_t *hubs;      // S*p current batch / children (sorted)
    uint16_t *kidx;     // S*n_pad hub positions (kNoHub in the padding)
    double *cost;       // S scaled cost (approximate in FP32/split modes)
    double *parts;      // S*3 {Cc, T, Dd}
    double *eps;        // S relative error bounds
    int32_t *cmax;      // S largest cluster size
    float *Ch32;        // S*p*p hub-to-hub distances (split mode)
    double *partial;    // S*p*(n_pad/64) epilogue partials (split mode), [row tile][column]
    // GA state
    int32_t *anc;       // R*p
    double *anc_cost;   // R
    double *anc_parts;  // R*3
    int32_t *best;      // p
    double *best_cost;  // 1 (+3 parts following)
    int64_t *gen;       // generation counter g
    int64_t *stats;     // 4 counters
    int32_t *cand;      // R*m candidate child indices
    int32_t *cand_cnt;  // R
    double *cand_cost;  // R*m exact costs of candidates
    double *cand_parts; // R*m*3
    uint16_t *kidx_one; // n_pad hub positions of a single solution (best so far)
    uint8_t *scratch;   // n bytes (middle-node selection)
    double *tbuf;       // tot*n column sums t_j of candidates under exact re-evaluation
    int32_t *slot_r, *slot_c;   // tot candidate slots (island, candidate)
    int32_t *slot_s;    // tot: the child of each slot
    int32_t *slot_done; // tot: finished column items of each slot, zero between launches
    int32_t *handled;   // R: candidates of each island that got a slot
    int32_t *choice;    // R: the child each island takes in the exact decision, or -1
    int32_t *total;     // 1: slots in use
    int32_t *extra_r, *extra_c;   // S: candidates beyond the slots
    int32_t *nextra;    // 1
    int *sync;          // 2 grid counters (last workgroup of the selection, last unit of the
                        // re-evaluation), zero between launches
    // exhaustive search
    EnumState *enum_state;
    int32_t *enum_best; // p: hub set of the best so far
    uint64_t *binom;    // (n+1)*(p+1): C(m, j) at [m*(p+1) + j], saturated at 2^63
};

struct Dims {
    int n, p, S, m, R, n_pad, n_mtiles, n1, elitist, prec;
    int kern;           // ga_kernel: 0 plain (one workgroup per individual), 1 batched
    int tot;            // candidate slots of the column-parallel exact re-evaluation
    int mfma_cfg;       // tile configuration of the batched kernel
    int c_f32, w_f32;   // instance dtypes (1 = FP32)
    int sym;            // C == C^T: the batched K-64 configurations use the folded W
    int multihop;       // transfer term through the shortest-path distances Ctr
    double chi, alpha, delta, scale;
    uint64_t seed;
};

// ----------------------------------------------------- grouped launches --
// One generation of several contexts with one launch per step: the grid is
// the concatenation of the contexts' own grids, start[phase] being the first
// workgroup of context j, so every workgroup serves exactly one context.
enum TickPhase { kTickOps = 0, kTickAlloc, kTickFinal, kTickSel1, kTickPhases };
constexpr int kMaxPoolJobs = 256;      // grouped contexts per batch
constexpr int kRecheckBlocks = 512;    // persistent workgroups of the exact re-evaluation (one context or all)

struct TickJob {
    DevPtrs P;
    Dims d;
    int n_mt;                  // row tiles of the epilogue partials
    int start[kTickPhases];
    int blocks[kTickPhases];
};

// The composition of a grouped generation, in device memory ahead of the job
// tables: the grouped kernels read their job count and sizes from here, so a
// graph captured with grids of some capacity serves every composition that
// fits it (workgroups past a phase's total return at once).
struct GroupHdr {
    int njobs;
    int total_tiles;           // matrix-core work units
    int round_robin;           // some context is folded: units go round robin over the XCDs
    int pad;
    int blocks[kTickPhases];   // workgroups of each phase
};

// The context owning workgroup b of a grouped launch (last job with start <= b).
__device__ inline int tick_job(const TickJob *__restrict__ jobs, int njobs, int phase, int b)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].start[phase] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ----------------------------------------------------------------- RNG --
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies with the halves crossed and xored with the round key,
// the key bumped by two Weyl constants between rounds.
struct U64x4 { uint64_t x[4]; };

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    U64x4 o; o.x[0] = c0; o.x[1] = c1; o.x[2] = c2; o.x[3] = c3;
    return o;
}

// Draw for (generation, index, operator, repeat) under the GA key.
__device__ __forceinline__ U64x4 ga_draw(uint64_t seed, uint64_t g, uint64_t idx, uint64_t op, uint64_t t)
{
    return philox4x64_10(g, idx, op, t, seed, 0x4741ull);
}

// floor(w * m / 2^64): uniform index in [0, m).
__device__ __forceinline__ int uindex(uint64_t w, int m) { return (int)__umul64hi(w, (uint64_t)m); }

// Unit roundoffs used in the error bounds.
constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53
constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24
constexpr double kU32Faithful = 1.1920928955078125e-07;  // 2^-23 (any faithful FP32 rounding)
constexpr double kSplitResidual = 1.52587890625e-05;     // 2^-16: |W - hi - lo| <= 2^-16 W
constexpr double kSplit3Residual = 5.9604644775390625e-08;  // 2^-24: |W - hi - mid - lo| <= 2^-24 W
// The FP32 accumulators add hi and lo parts, whose magnitudes sum to at most
// (1 + 2^-8) W + (1 + 2^-8) 2^-8 W <= (1 + 2^-6) W (bf16 unit roundoff 2^-8),
// so the accumulation bound is taken relative to that mass, not to W.
constexpr double kHiLoMass = 1.015625;                   // 1 + 2^-6

__host__ __device__ inline double gamma_k(double k, double u) { return k * u / (1.0 - k * u); }

}  // namespace hubga
