// Genetic operators of one generation (Sec. 4.1, 4.2 and 5), integer only.
// Child s of island r = s / m is built from the island ancestor:
//   1. both parents of the pair q = s / 2 are the ancestor with one hub
//      swapped for one spoke (operator 0, index = parent slot 2q or 2q+1);
//   2. single-point crossover of the pair at cut c in [1, n-1] (operator 1,
//      index q): the even child takes the first parent's hubs below c and the
//      second parent's hubs from c on, the odd child the opposite;
//   3. mutation: one hub<->spoke swap when 0 < count < n (operator 2);
//   4. correction to exactly p hubs, one draw per removal or addition
//      (operator 3, repeat t = 0, 1, ...).
// A swap removes the hub at position floor(w0*count/2^64) and adds the
// spoke of rank floor(w1*(n-count)/2^64) among the spokes, ranked before the
// removal.  Draws are Philox4x64-10 words addressed by (g, index, operator,
// t), so an operator that does nothing never shifts later draws.
//
// One lane per child; hub lists are kept sorted in LDS, strided by the block
// size so that lanes touch distinct banks.
#include "kernels.hpp"

namespace hubga {

namespace {

struct List {
    uint16_t *a;   // element k at a[k * stride]
    int stride;
    __device__ int get(int k) const { return a[k * stride]; }
    __device__ void set(int k, int v) { a[k * stride] = (uint16_t)v; }
};

__device__ int nth_spoke(const List &x, int cnt, int r)
{
    int v = r;
    for (int k = 0; k < cnt; ++k) {
        if (x.get(k) <= v)
            ++v;
        else
            break;
    }
    return v;
}

__device__ void remove_at(List &x, int &cnt, int pos)
{
    for (int k = pos; k + 1 < cnt; ++k) x.set(k, x.get(k + 1));
    --cnt;
}

__device__ void insert_sorted(List &x, int &cnt, int v)
{
    int k = cnt;
    while (k > 0 && x.get(k - 1) > v) {
        x.set(k, x.get(k - 1));
        --k;
    }
    x.set(k, v);
    ++cnt;
}

__device__ void swap_move(int n, List &x, int &cnt, uint64_t w_pos, uint64_t w_rank)
{
    int pos = uindex(w_pos, cnt);
    int v = nth_spoke(x, cnt, uindex(w_rank, n - cnt));
    remove_at(x, cnt, pos);
    insert_sorted(x, cnt, v);
}

}  // namespace

__global__ __launch_bounds__(64) void k_ga_ops(const int32_t *__restrict__ anc, int32_t *__restrict__ children,
                                               const int64_t *__restrict__ gen, int n, int p, int S, int m,
                                               uint64_t seed)
{
    extern __shared__ uint16_t lds[];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const int B = blockDim.x, tid = threadIdx.x;
    const uint64_t g = (uint64_t)*gen;
    List pa{lds + tid, B}, pb{lds + (size_t)p * B + tid, B}, cx{lds + (size_t)2 * p * B + tid, B};
    const int r = s / m, q = s / 2;
    const int32_t *a = anc + (size_t)r * p;
    for (int k = 0; k < p; ++k) {
        pa.set(k, a[k]);
        pb.set(k, a[k]);
    }
    int ca = p, cb = p;
    if (p < n) {
        U64x4 w = ga_draw(seed, g, (uint64_t)(2 * q), 0, 0);
        swap_move(n, pa, ca, w.x[0], w.x[1]);
        w = ga_draw(seed, g, (uint64_t)(2 * q + 1), 0, 0);
        swap_move(n, pb, cb, w.x[0], w.x[1]);
    }
    U64x4 w = ga_draw(seed, g, (uint64_t)q, 1, 0);
    const int cut = 1 + uindex(w.x[0], n - 1);
    const List &first = (s & 1) ? pb : pa;
    const List &second = (s & 1) ? pa : pb;
    const int cf = (s & 1) ? cb : ca, cs = (s & 1) ? ca : cb;
    int cnt = 0;
    for (int k = 0; k < cf; ++k) {
        int v = first.get(k);
        if (v < cut) cx.set(cnt++, v);
    }
    for (int k = 0; k < cs; ++k) {
        int v = second.get(k);
        if (v >= cut) cx.set(cnt++, v);
    }
    w = ga_draw(seed, g, (uint64_t)s, 2, 0);
    if (cnt > 0 && cnt < n) swap_move(n, cx, cnt, w.x[0], w.x[1]);
    uint64_t t = 0;
    while (cnt > p) {
        w = ga_draw(seed, g, (uint64_t)s, 3, t++);
        remove_at(cx, cnt, uindex(w.x[0], cnt));
    }
    while (cnt < p) {
        w = ga_draw(seed, g, (uint64_t)s, 3, t++);
        insert_sorted(cx, cnt, nth_spoke(cx, cnt, uindex(w.x[0], n - cnt)));
    }
    int32_t *out = children + (size_t)s * p;
    for (int k = 0; k < p; ++k) out[k] = cx.get(k);
}

hipError_t launch_ga_ops(const DevPtrs &P, const Dims &d, hipStream_t st)
{
    const int B = 64;
    size_t sm = (size_t)(4 * d.p + 2) * B * sizeof(uint16_t);
    k_ga_ops<<<(d.S + B - 1) / B, B, sm, st>>>(P.anc, P.hubs, P.gen, d.n, d.p, d.S, d.m, d.seed);
    return hipGetLastError();
}

}  // namespace hubga
