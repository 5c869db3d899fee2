// Instance preparation, once per context (copy of C and W to GPU global
// memory, Sec. 5 host steps; middle nodes of Sec. 4.1):
//   O_i = sum_j W_ij, D_j = sum_i W_ij, d_i = sum_j C_ij in binary64, ascending;
//   transposed C for coalesced hub-row reads;
//   FP32 copy of W; bf16 hi/lo split of W padded with zeros to n_pad.
#include "kernels.hpp"

namespace hubga {

// Sums of the rows (ROWS) or columns of M in binary64, each in ascending
// index order, one output per lane of a 64-line workgroup: tiles of 64 x 64
// are loaded coalesced by all 256 lanes (the next tile's loads are in flight
// while the current one is summed) and each line's owner adds its 64 values
// in order.
template <typename T, bool ROWS>
__global__ __launch_bounds__(256) void k_line_sums(const T *__restrict__ M, int n, double *__restrict__ out)
{
#pragma clang fp contract(off)
    __shared__ double tile[64][65];
    const int tid = threadIdx.x, base = blockIdx.x * 64;
    const int nt = (n + 63) / 64;
    T reg[16];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = tid + 256 * q, l = e / 64, k = e % 64;   // line l, index k within the tile
            const int line = base + l, idx = k0 + k;
            reg[q] = (line < n && idx < n) ? (ROWS ? M[(size_t)line * n + idx] : M[(size_t)idx * n + line]) : (T)0;
        }
    };
    double acc = 0.0;
    load(0);
    for (int t = 0; t < nt; ++t) {
        const int k0 = t * 64;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = tid + 256 * q;
            tile[e / 64][e % 64] = (double)reg[q];
        }
        __syncthreads();
        if (t + 1 < nt) load(k0 + 64);
        if (tid < 64) {
            const int cnt = min(64, n - k0);
            for (int k = 0; k < cnt; ++k) acc = acc + tile[tid][k];
        }
        __syncthreads();
    }
    if (tid < 64 && base + tid < n) out[base + tid] = acc;
}

template <typename T>
__global__ void k_transpose(const T *__restrict__ src, T *__restrict__ dst, int n)
{
    __shared__ T tile[32][33];
    int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
    for (int r = ty; r < 32; r += 8) {
        int i = by + r, j = bx + tx;
        if (i < n && j < n) tile[r][tx] = src[(size_t)i * n + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int i = bx + r, j = by + tx;
        if (i < n && j < n) dst[(size_t)i * n + j] = tile[tx][r];
    }
}

// Round-to-nearest-even of a binary64 value to bfloat16 (8 significant bits,
// exponent range of binary32), in one rounding step: scale by the bf16
// quantum of x's binade, round to an integer with ties to even, scale back.
__device__ inline uint16_t bf16_rne_bits(double x)
{
    if (x == 0.0) return 0;
    double ax = fabs(x);
    int e = ilogb(ax);                 // ax in [2^e, 2^(e+1))
    int qe = (e < -126 ? -126 : e) - 7;
    double r = rint(ldexp(ax, -qe));   // exact scaling, RNE to integer
    float v = (float)ldexp(r, qe);     // exactly representable in bf16, hence in binary32
    uint32_t b = __float_as_uint(v) >> 16;
    return (uint16_t)(b | (x < 0.0 ? 0x8000u : 0u));
}

__device__ inline double bf16_to_double(uint16_t b) { return (double)__uint_as_float(((uint32_t)b) << 16); }

// mid non-null: the three-part split hi, mid, lo, each the bf16 rounding of
// what the parts before it leave (the remainders are exact in binary64).
template <typename T>
__global__ void k_split_bf16(const T *__restrict__ W, int n, int n_pad, uint16_t *__restrict__ hi,
                             uint16_t *__restrict__ lo, uint16_t *__restrict__ mid)
{
#pragma clang fp contract(off)
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)n_pad * n_pad;
    if (idx >= total) return;
    int i = (int)(idx / n_pad), j = (int)(idx % n_pad);
    uint16_t h = 0, m = 0, l = 0;
    if (i < n && j < n) {
        double x = (double)W[(size_t)i * n + j];
        h = bf16_rne_bits(x);
        double rem = x - bf16_to_double(h);   // exact (Sterbenz)
        if (mid) {
            m = bf16_rne_bits(rem);
            rem = rem - bf16_to_double(m);    // exact
        }
        l = bf16_rne_bits(rem);
    }
    hi[idx] = h;
    lo[idx] = l;
    if (mid) mid[idx] = m;
}

// The same split written in fragment order: one thread per 16-byte chunk of
// 8 consecutive k of one row; chunk ((g*KS + ks)*2 + h)*64 + rl holds row
// g*64 + rl, k = ks*16 + h*8 .. +7 (KS = n_pad/16).  FOLD splits the folded
// matrix instead: W_rk + W_kr (one binary64 rounding) for k > r, W_rr for
// k = r, zero for k < r.  With C symmetric, sum_{r,k} W_rk C[a(r)][a(k)] is
// the same sum over the folded matrix, whose non-zeros lie on and above the
// diagonal.
template <typename T, bool FOLD = false>
__global__ void k_split_bf16_swz(const T *__restrict__ W, int n, int n_pad, uint16_t *__restrict__ hi,
                                 uint16_t *__restrict__ lo)
{
#pragma clang fp contract(off)
    size_t chunk = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)n_pad * n_pad / 8;
    if (chunk >= total) return;
    const int KS = n_pad / 16;
    const int rl = (int)(chunk % 64);
    size_t t = chunk / 64;
    const int h = (int)(t % 2);
    t /= 2;
    const int ks = (int)(t % KS), g = (int)(t / KS);
    const int r = g * 64 + rl, k0 = ks * 16 + h * 8;
    uint16_t vh[8], vl[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        uint16_t a = 0, b = 0;
        if (r < n && k < n && (!FOLD || k >= r)) {
            double x = (double)W[(size_t)r * n + k];
            if (FOLD && k > r) x = x + (double)W[(size_t)k * n + r];
            a = bf16_rne_bits(x);
            b = bf16_rne_bits(x - bf16_to_double(a));
        }
        vh[e] = a;
        vl[e] = b;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        hi[chunk * 8 + e] = vh[e];
        lo[chunk * 8 + e] = vl[e];
    }
}

__global__ void k_to_f32(const double *__restrict__ src, float *__restrict__ dst, size_t count)
{
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < count) dst[idx] = (float)src[idx];
}

// The p nodes with the smallest d_i (ties to the smaller index), sorted.
// One workgroup; p rounds of a (value, index) argmin over the untaken nodes.
__global__ void k_middle_select(const double *__restrict__ d, int n, int p, int32_t *__restrict__ hubs,
                                uint8_t *__restrict__ taken)
{
    __shared__ double sv[1024];
    __shared__ int si[1024];
    int tid = threadIdx.x;
    for (int i = tid; i < n; i += blockDim.x) taken[i] = 0;
    __syncthreads();
    for (int k = 0; k < p; ++k) {
        double bv = 0.0;
        int bi = -1;
        for (int i = tid; i < n; i += blockDim.x) {
            if (taken[i]) continue;
            double v = d[i];
            if (bi < 0 || v < bv) { bv = v; bi = i; }   // ascending i: ties keep the smaller i
        }
        sv[tid] = bv;
        si[tid] = bi;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (tid < s) {
                int oi = si[tid + s];
                double ov = sv[tid + s];
                int mi = si[tid];
                if (oi >= 0 && (mi < 0 || ov < sv[tid] || (ov == sv[tid] && oi < mi))) {
                    sv[tid] = ov;
                    si[tid] = oi;
                }
            }
            __syncthreads();
        }
        if (tid == 0) taken[si[0]] = 1;
        __syncthreads();
    }
    if (tid == 0) {
        int c = 0;
        for (int i = 0; i < n && c < p; ++i)
            if (taken[i]) hubs[c++] = i;
    }
}

// Row n of the FP32 hub-distance copy: +inf, read for the padding hubs of the
// allocation scan.
__global__ void k_inf_row(float *__restrict__ row, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) row[t] = __builtin_huge_valf();
}

// Multi-hop routing (eq. (4) of Sec. 3 lets inter-hub flow use every arc):
// the transfer term reads the all-pairs shortest-path distances of C,
// Floyd-Warshall in binary64.  One launch per intermediate node k updates
// every entry: out[i][j] takes out[i][k] + out[k][j] when strictly smaller.
// Row k and column k cannot change during step k (out[k][k] >= 0 and adding a
// non-negative number never decreases a binary64 sum), so the entries read in
// step k are those of the sequential algorithm and the result is its result
// bit for bit.
template <typename T>
__global__ void k_to_f64(const T *__restrict__ src, double *__restrict__ dst, size_t count)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < count) dst[idx] = (double)src[idx];
}

__global__ void k_fw_step(double *__restrict__ D, int n, int k)
{
#pragma clang fp contract(off)
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= n) return;
    const double via = D[(size_t)i * n + k] + D[(size_t)k * n + j];
    if (via < D[(size_t)i * n + j]) D[(size_t)i * n + j] = via;
}

hipError_t launch_shortest_paths(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    if (!P.Ctr) return hipSuccess;
    const int n = d.n, tb = 256;
    const size_t cnt = (size_t)n * n;
    const unsigned g = (unsigned)((cnt + tb - 1) / tb);
    if (d.c_f32)
        k_to_f64<float><<<g, tb, 0, st>>>((const float *)P.C, P.Ctr, cnt);
    else
        k_to_f64<double><<<g, tb, 0, st>>>((const double *)P.C, P.Ctr, cnt);
    const dim3 grid((n + tb - 1) / tb, n);
    for (int k = 0; k < n; ++k) k_fw_step<<<grid, tb, 0, st>>>(P.Ctr, n, k);
    return hipGetLastError();
}

// ------------------------------------------------------------ launchers --

hipError_t launch_prep(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    const int n = d.n;
    const int tb = 256;
    const int nb = (n + tb - 1) / tb;
    const int nl = (n + 63) / 64;   // 64 lines per workgroup
    if (d.w_f32) {
        k_line_sums<float, true><<<nl, 256, 0, st>>>((const float *)P.W, n, P.O);
        k_line_sums<float, false><<<nl, 256, 0, st>>>((const float *)P.W, n, P.D);
    } else {
        k_line_sums<double, true><<<nl, 256, 0, st>>>((const double *)P.W, n, P.O);
        k_line_sums<double, false><<<nl, 256, 0, st>>>((const double *)P.W, n, P.D);
    }
    if (d.c_f32)
        k_line_sums<float, true><<<nl, 256, 0, st>>>((const float *)P.C, n, P.dsum);
    else
        k_line_sums<double, true><<<nl, 256, 0, st>>>((const double *)P.C, n, P.dsum);
    if (P.Ct != P.C) {
        dim3 g((n + 31) / 32, (n + 31) / 32);
        if (d.c_f32)
            k_transpose<float><<<g, 256, 0, st>>>((const float *)P.C, (float *)P.Ct, n);
        else
            k_transpose<double><<<g, 256, 0, st>>>((const double *)P.C, (double *)P.Ct, n);
    }
    if (P.W32) {
        size_t cnt = (size_t)n * n;
        k_to_f32<<<(unsigned)((cnt + tb - 1) / tb), tb, 0, st>>>((const double *)P.W, P.W32, cnt);
    }
    if (!d.c_f32) {
        size_t cnt = (size_t)n * n;
        k_to_f32<<<(unsigned)((cnt + tb - 1) / tb), tb, 0, st>>>((const double *)P.Ct, P.Ct32, cnt);
    }
    k_inf_row<<<nb, tb, 0, st>>>(P.Ct32 + (size_t)n * n, n);
    return hipGetLastError();
}

// The bf16 hi/lo split of W into the context's one pair of split buffers, in
// the layout the selected tile configuration reads: row-major, fragment
// order, or fragment order of the folded W.
hipError_t launch_w_layout(const DevPtrs &P, const Dims &d, int layout, hipStream_t st)
{
    if (!P.Whi) return hipSuccess;
    const int n = d.n, tb = 256;
    const size_t cnt = (size_t)d.n_pad * d.n_pad;
    if (layout == kWRowMajor) {
        const unsigned g = (unsigned)((cnt + tb - 1) / tb);
        if (d.w_f32)
            k_split_bf16<float><<<g, tb, 0, st>>>((const float *)P.W, n, d.n_pad, P.Whi, P.Wlo, P.Wmd);
        else
            k_split_bf16<double><<<g, tb, 0, st>>>((const double *)P.W, n, d.n_pad, P.Whi, P.Wlo, P.Wmd);
        return hipGetLastError();
    }
    const unsigned gs = (unsigned)((cnt / 8 + tb - 1) / tb);
    const bool fold = layout == kWFragFolded;
    if (d.w_f32 && fold)
        k_split_bf16_swz<float, true><<<gs, tb, 0, st>>>((const float *)P.W, n, d.n_pad, P.Whi, P.Wlo);
    else if (d.w_f32)
        k_split_bf16_swz<float><<<gs, tb, 0, st>>>((const float *)P.W, n, d.n_pad, P.Whi, P.Wlo);
    else if (fold)
        k_split_bf16_swz<double, true><<<gs, tb, 0, st>>>((const double *)P.W, n, d.n_pad, P.Whi, P.Wlo);
    else
        k_split_bf16_swz<double><<<gs, tb, 0, st>>>((const double *)P.W, n, d.n_pad, P.Whi, P.Wlo);
    return hipGetLastError();
}

hipError_t launch_middle_nodes(const DevPtrs &P, const Dims &d, int32_t *hubs_out, uint8_t *scratch, hipStream_t st)
{
    k_middle_select<<<1, 1024, 0, st>>>(P.dsum, d.n, d.p, hubs_out, scratch);
    return hipGetLastError();
}

}  // namespace hubga
