// Genetic operators of one generation (Sec. 4.1, 4.2 and 5), integer only,
// one wave per child: shared by the operators kernel and the allocation
// kernel that builds its own child first.
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
// One wave per child.  A sorted hub list lives in LDS with element k owned by
// lane k (and lane k-64 for k >= 64).  With x sorted and distinct, x[k] - k
// is the number of spokes below x[k] and is non-decreasing in k, so the spoke
// of rank r is r + #{k : x[k] - k <= r}: one ballot.  Removing position pos
// and inserting v moves element k to k - [k > pos] + [x[k] > v].
#pragma once
#include "common.hpp"

namespace hubga {

// Sorted list of up to 128 node ids; slots k and k+64 belong to lane k.
struct WList {
    int *a;
    __device__ int lo(int lane) const { return a[lane]; }
    __device__ int hi(int lane) const { return a[lane + 64]; }
};

__device__ __forceinline__ int popc(unsigned long long m) { return __popcll(m); }

// Spoke of rank r for the list x[0..cnt).
__device__ __forceinline__ int wave_nth_spoke(const WList &x, int cnt, int r, int lane)
{
    const int e0 = lane < cnt ? x.lo(lane) - lane : 0x7FFFFFFF;
    const int e1 = lane + 64 < cnt ? x.hi(lane) - (lane + 64) : 0x7FFFFFFF;
    return r + popc(__ballot(e0 <= r)) + popc(__ballot(e1 <= r));
}

// Remove position pos (or none when pos < 0) and insert v (or none when v < 0).
__device__ __forceinline__ void wave_edit(WList &x, int &cnt, int pos, int v, int lane)
{
    const bool in0 = lane < cnt, in1 = lane + 64 < cnt;
    const int x0 = in0 ? x.lo(lane) : 0, x1 = in1 ? x.hi(lane) : 0;
    const bool keep0 = in0 && lane != pos, keep1 = in1 && lane + 64 != pos;
    int ins = 0;
    if (v >= 0) ins = popc(__ballot(keep0 && x0 < v)) + popc(__ballot(keep1 && x1 < v));
    const int d0 = lane - (pos >= 0 && lane > pos ? 1 : 0) + (v >= 0 && x0 > v ? 1 : 0);
    const int d1 = lane + 64 - (pos >= 0 && lane + 64 > pos ? 1 : 0) + (v >= 0 && x1 > v ? 1 : 0);
    __builtin_amdgcn_wave_barrier();
    if (keep0) x.a[d0] = x0;
    if (keep1) x.a[d1] = x1;
    if (v >= 0 && lane == 0) x.a[ins] = v;
    __builtin_amdgcn_wave_barrier();
    cnt += (v >= 0 ? 1 : 0) - (pos >= 0 ? 1 : 0);
}

// Hub<->spoke swap with the spoke ranked before the removal.
__device__ __forceinline__ void wave_swap(int n, WList &x, int &cnt, uint64_t w_pos, uint64_t w_rank, int lane)
{
    const int pos = uindex(w_pos, cnt);
    const int v = wave_nth_spoke(x, cnt, uindex(w_rank, n - cnt), lane);
    wave_edit(x, cnt, pos, v, lane);
}


// Child s (island s / m) built by one whole wave from the island ancestors
// anc and generation g's draws, in lists (3 x 128 ints of LDS: the two
// parents, then the child), and written to children[s*p ..); on return
// lists[256 + k] holds the child's k-th hub for k < p.
__device__ __forceinline__ void ga_child_wave(const int32_t *__restrict__ anc, int32_t *children, uint64_t g, int n,
                                              int p, int m, uint64_t seed, int s, int *lists)
{
    const int lane = threadIdx.x & 63;
    WList pa{lists}, pb{lists + 128}, cx{lists + 256};
    const int r = s / m, q = s / 2;
    const int32_t *a = anc + (size_t)r * p;
    if (lane < p) {
        pa.a[lane] = a[lane];
        pb.a[lane] = a[lane];
    }
    __builtin_amdgcn_wave_barrier();
    // The child's first eight draws, one per lane (they are addressed by their
    // counters, so drawing one that is not used changes nothing):
    // 0, 1: perturbation of parent slots 2q, 2q+1; 2: crossover; 3: mutation;
    // 4..7: corrections t = 0..3.
    U64x4 mine;
    {
        const int k = lane & 7;
        const uint64_t idx = k == 0 ? (uint64_t)(2 * q) : k == 1 ? (uint64_t)(2 * q + 1) : k == 2 ? (uint64_t)q
                                                                                                  : (uint64_t)s;
        const uint64_t op = k < 2 ? 0 : (k == 2 ? 1 : (k == 3 ? 2 : 3));
        mine = ga_draw(seed, g, idx, op, k >= 4 ? (uint64_t)(k - 4) : 0);
    }
    auto word = [&](int k, int w) -> uint64_t {   // word w of draw k, from lane k
        const uint64_t v = mine.x[w];
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, k);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), k);
        return ((uint64_t)hi << 32) | lo;
    };
    int ca = p, cb = p;
    if (p < n) {
        wave_swap(n, pa, ca, word(0, 0), word(0, 1), lane);
        wave_swap(n, pb, cb, word(1, 0), word(1, 1), lane);
    }
    // crossover: first parent's hubs below the cut, second parent's from it on
    const int cut = 1 + uindex(word(2, 0), n - 1);
    const WList &first = (s & 1) ? pb : pa;
    const WList &second = (s & 1) ? pa : pb;
    const int f = lane < p ? first.lo(lane) : 0x7FFFFFFF;
    const int sc = lane < p ? second.lo(lane) : -1;
    const int nf = popc(__ballot(lane < p && f < cut));
    const int ns_below = popc(__ballot(lane < p && sc < cut));
    __builtin_amdgcn_wave_barrier();
    if (lane < p && f < cut) cx.a[lane] = f;
    if (lane < p && sc >= cut) cx.a[nf + lane - ns_below] = sc;
    __builtin_amdgcn_wave_barrier();
    int cnt = nf + (p - ns_below);
    // mutation
    if (cnt > 0 && cnt < n) wave_swap(n, cx, cnt, word(3, 0), word(3, 1), lane);
    // correction
    int t = 0;
    auto corr = [&]() -> uint64_t {   // word 0 of correction draw t, then t + 1
        const uint64_t w0 = t < 4 ? word(4 + t, 0) : ga_draw(seed, g, (uint64_t)s, 3, (uint64_t)t).x[0];
        ++t;
        return w0;
    };
    while (cnt > p) wave_edit(cx, cnt, uindex(corr(), cnt), -1, lane);
    while (cnt < p) wave_edit(cx, cnt, -1, wave_nth_spoke(cx, cnt, uindex(corr(), n - cnt), lane), lane);
    if (lane < p) children[(size_t)s * p + lane] = cx.a[lane];
}

}  // namespace hubga
