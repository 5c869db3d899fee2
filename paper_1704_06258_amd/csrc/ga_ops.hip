// Genetic operators of one generation (Sec. 4.1, 4.2 and 5) for grouped
// launches over several contexts; the operators themselves are in
// ga_ops_dev.hpp, and a single context's generation builds its children in
// the allocation kernel.
#include "kernels.hpp"
#include "ga_ops_dev.hpp"

namespace hubga {

// Workgroup blk of a context: children 4*blk .. 4*blk+3, one per wave.
__device__ __forceinline__ void ga_ops_body(const int32_t *__restrict__ anc, int32_t *__restrict__ children,
                                            const int64_t *__restrict__ gen, int n, int p, int S, int m,
                                            uint64_t seed, int blk)
{
    __shared__ int lists[4][3][128];   // per wave: parent a, parent b, child
    const int wave = threadIdx.x >> 6;
    const int s = blk * 4 + wave;
    if (s >= S) return;
    ga_child_wave(anc, children, (uint64_t)*gen, n, p, m, seed, s, &lists[wave][0][0]);
}

__global__ __launch_bounds__(256) void k_ga_ops_group(const GroupHdr *__restrict__ hdr, const TickJob *__restrict__ jobs)
{
    if ((int)blockIdx.x >= hdr->blocks[kTickOps]) return;
    const TickJob &J = jobs[tick_job(jobs, hdr->njobs, kTickOps, blockIdx.x)];
    ga_ops_body(J.P.anc, J.P.hubs, J.P.gen, J.d.n, J.d.p, J.d.S, J.d.m, J.d.seed, blockIdx.x - J.start[kTickOps]);
}

int ga_ops_blocks(const Dims &d) { return (d.S + 3) / 4; }

hipError_t launch_ga_ops_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, int blocks, hipStream_t st)
{
    if (njobs <= 0 || blocks <= 0) return hipSuccess;
    k_ga_ops_group<<<blocks, 256, 0, st>>>(hdr, jobs);
    return hipGetLastError();
}

}  // namespace hubga
