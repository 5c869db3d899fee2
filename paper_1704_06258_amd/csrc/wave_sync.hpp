// Wave-level synchronisation helpers for gfx950 kernels that keep global
// loads in flight across workgroup barriers: __syncthreads() waits for every
// outstanding memory operation of the wave, these wait only for what is named.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace hubga {

template <int N, typename F, int I = 0>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, F, I + 1>(static_cast<F &&>(f));
    }
}

__device__ __forceinline__ void lds_wait() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
// Wait until at most N LDS reads of this wave are outstanding (they complete in
// order when nothing else counted by lgkmcnt is in flight).
template <int N>
__device__ __forceinline__ void lds_wait_n()
{
    static_assert(N >= 0 && N <= 15, "lgkmcnt range");
    asm volatile("s_waitcnt lgkmcnt(%0)" ::"n"(N) : "memory");
}
// s_waitcnt vmcnt(N), other counters untouched (gfx9 encoding).
template <int N>
__device__ __forceinline__ void vm_wait()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

__device__ __forceinline__ void wg_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

}  // namespace hubga
