// Batched FP32 evaluation on the vector units (GA_PREC_FP32 with
// GA_KERN_BATCHED): the comparator of the matrix-core path that does only the
// useful work.  The transfer term of objective (1) (Sec. 3) for individual s,
//     T_s = sum_j t_j,   t_j = sum_i W_ij * C[h_{k(i)}][h_{k(j)}],
// costs n^2 multiply-adds per individual whatever p is, against the 4 n^2 p
// matrix-core flops of the one-hot product; what it pays instead is a gather
// from the individual's p x p distance table per term.
//
// Workgroup: a strip of 64 columns j (one per lane) by a group of G
// individuals, whose FP32 distance tables sit in LDS.  The four waves take a
// quarter of the rows each; every W element a lane loads serves all G
// individuals.  Per term: the row's table offset k(i)*p (staged in LDS,
// read wave-uniform four rows at a time), one LDS gather Ch_s[k(i)][k(j)]
// and one FMA.  The waves' FP32 column sums are
// added in binary64, then the strip's 64 columns (fixed order), into one
// partial per (strip, individual); k_finalize_vec adds an individual's
// partials in strip order and assembles the cost.  The error bound is the
// FP32 plain kernel's (a column's FP32 chain here is a quarter as long).
#include "kernels.hpp"

namespace hubga {

constexpr int kVecCols = 64;

// Individuals per workgroup for p hubs: their tables fill at most 48 KB.
int vec_group(int p)
{
    const int per = p * p * 4;
    return per * 8 <= 49152 ? 8 : per * 4 <= 49152 ? 4 : per * 2 <= 49152 ? 2 : 1;
}

constexpr int kVecChunk = 256;   // rows whose table offsets are staged at a time (64 per wave)

template <int G>
__global__ __launch_bounds__(256, 2) void k_eval_vec(const float *__restrict__ W, const uint16_t *__restrict__ kidx,
                                                     const float *__restrict__ Ch32, int count, int n, int n_pad,
                                                     int p, int n_ct, double *__restrict__ partial)
{
#pragma clang fp contract(off)
    extern __shared__ __align__(16) float sCh[];      // [G][p*p]
    __shared__ __align__(16) uint32_t offs[G][kVecChunk];   // g*p*p + k_g(i)*p of the chunk's rows
    __shared__ double red[4][G][kVecCols];
    // strips in XCD-major order: XCD x (blockIdx % 8) walks a contiguous range
    // of strips, so the groups reading one strip of W share an L2
    const int ngroups = (count + G - 1) / G;
    const int units = n_ct * ngroups;
    const int per = (units + 7) / 8;
    const int u = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (u >= units) return;
    const int ct = u / ngroups, grp = u % ngroups;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int pp = p * p;
    const int s0 = grp * G;
    for (int e = tid; e < G * pp; e += 256) {
        const int g = e / pp, s = s0 + g < count ? s0 + g : count - 1;
        sCh[e] = Ch32[(size_t)s * pp + e % pp];
    }
    const int j = ct * kVecCols + lane;
    const int jc = j < n ? j : n - 1;   // absent columns compute column n-1 and are discarded
    int kj[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int s = s0 + g < count ? s0 + g : count - 1;
        kj[g] = kidx[(size_t)s * n_pad + jc];
    }
    float acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = 0.0f;
    const float *wcol = W + jc;
    // Chunks of 256 rows: the table offsets of the group's hub positions are
    // staged in LDS (coalesced loads by every lane), then each wave takes 64
    // rows, eight at a time with the next eight rows' W loads in flight.
    for (int c0 = 0; c0 < n; c0 += kVecChunk) {
        __syncthreads();   // the previous chunk's offsets are consumed
        for (int e = tid; e < G * kVecChunk; e += 256) {
            const int g = e / kVecChunk, r = c0 + e % kVecChunk;
            const int s = s0 + g < count ? s0 + g : count - 1;
            offs[g][e % kVecChunk] = r < n ? (uint32_t)(g * pp + (int)kidx[(size_t)s * n_pad + r] * p) : 0u;
        }
        __syncthreads();
        const int rb = c0 + wave * 64;
        const int nr = n - rb < 64 ? n - rb : 64;   // rows of this wave in the chunk (may be <= 0)
        if (nr <= 0) continue;
        // rows past the wave's last one load a valid row and weigh it 0: with
        // finite non-negative terms, adding 0 leaves every sum unchanged
        float wc[8], wn[8];
        auto wload = [&](float(&w)[8], int t0) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float v = wcol[(size_t)(rb + (t0 + t < nr ? t0 + t : nr - 1)) * n];
                w[t] = t0 + t < nr ? v : 0.0f;
            }
        };
        // all gathers of eight rows first (independent LDS reads in flight
        // together), then the multiply-adds
        auto apply = [&](const float(&w)[8], int t0) {
            float cv[G][8];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const uint4 o0 = *(const uint4 *)&offs[g][wave * 64 + t0];
                const uint4 o1 = *(const uint4 *)&offs[g][wave * 64 + t0 + 4];
                const uint32_t ov[8] = {o0.x, o0.y, o0.z, o0.w, o1.x, o1.y, o1.z, o1.w};
#pragma unroll
                for (int t = 0; t < 8; ++t) cv[g][t] = sCh[kj[g] + ov[t]];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t)
#pragma unroll
                for (int g = 0; g < G; ++g) acc[g] = __builtin_fmaf(w[t], cv[g][t], acc[g]);
        };
        wload(wc, 0);
        for (int t0 = 0; t0 < nr; t0 += 8) {
            if (t0 + 8 < nr) wload(wn, t0 + 8);
            apply(wc, t0);
#pragma unroll
            for (int t = 0; t < 8; ++t) wc[t] = wn[t];
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) red[wave][g][lane] = (double)acc[g];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double t = j < n ? ((red[0][g][lane] + red[1][g][lane]) + red[2][g][lane]) + red[3][g][lane] : 0.0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) t = t + __shfl_xor(t, off);
            if (lane == 0 && s0 + g < count) partial[(size_t)ct * count + s0 + g] = t;
        }
    }
}

// T_s = sum of individual s's strip partials in strip order; cost assembly
// f = ((chi*Cc) + (alpha*T)) + (delta*Dd) with Cc, Dd from the allocation.
__global__ __launch_bounds__(256) void k_finalize_vec(const double *__restrict__ partial, int count, int n_ct,
                                                      double chi, double alpha, double delta, double scale,
                                                      double eps_bound, double *__restrict__ cost,
                                                      double *__restrict__ parts, double *__restrict__ eps)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    double T = 0.0;
    for (int c = 0; c < n_ct; ++c) T = T + partial[(size_t)c * count + s];
    const double Cc = parts[3 * (size_t)s], Dd = parts[3 * (size_t)s + 2];
    parts[3 * (size_t)s + 1] = T;
    cost[s] = (((chi * Cc) + (alpha * T)) + (delta * Dd)) * scale;
    eps[s] = eps_bound;
}

template <int G>
static hipError_t vec_launch(const DevPtrs &P, const Dims &d, const float *W, const uint16_t *kidx, int count,
                             hipStream_t st)
{
    const int n_ct = (d.n + kVecCols - 1) / kVecCols;
    const int units = n_ct * ((count + G - 1) / G);
    const size_t lds = (size_t)G * d.p * d.p * 4;
    k_eval_vec<G><<<((units + 7) / 8) * 8, 256, lds, st>>>(W, kidx, P.Ch32, count, d.n, d.n_pad, d.p, n_ct,
                                                           P.partial);
    return hipGetLastError();
}

hipError_t launch_eval_vec(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st,
                           hipEvent_t ev0, hipEvent_t ev1)
{
    if (count <= 0) return hipSuccess;
    const float *W = d.w_f32 ? (const float *)P.W : P.W32;
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    switch (vec_group(d.p)) {
    case 8: e = vec_launch<8>(P, d, W, kidx, count, st); break;
    case 4: e = vec_launch<4>(P, d, W, kidx, count, st); break;
    case 2: e = vec_launch<2>(P, d, W, kidx, count, st); break;
    default: e = vec_launch<1>(P, d, W, kidx, count, st); break;
    }
    if (e != hipSuccess) return e;
    if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
    const int n_ct = (d.n + kVecCols - 1) / kVecCols;
    k_finalize_vec<<<(count + 255) / 256, 256, 0, st>>>(P.partial, count, n_ct, d.chi, d.alpha, d.delta, d.scale,
                                                        fp32_eps_bound(d.n), P.cost, P.parts, P.eps);
    return hipGetLastError();
}

size_t vec_partial_bytes(const Dims &d) { return (size_t)((d.n + kVecCols - 1) / kVecCols) * d.S * 8; }

}  // namespace hubga
