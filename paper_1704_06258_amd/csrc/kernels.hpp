// Launchers of the device kernels of libhubga (internal).
#pragma once
#include "common.hpp"
#include "select_dev.hpp"

namespace hubga {

// instance preparation (prep.hip)
hipError_t launch_prep(const DevPtrs &P, const Dims &d, hipStream_t st);
hipError_t launch_w_layout(const DevPtrs &P, const Dims &d, int layout, hipStream_t st);
hipError_t launch_shortest_paths(const DevPtrs &P, const Dims &d, hipStream_t st);
hipError_t launch_middle_nodes(const DevPtrs &P, const Dims &d, int32_t *hubs_out, uint8_t *scratch, hipStream_t st);

// nearest-hub allocation (alloc.hip); with ops.anc set, each workgroup first
// builds its child (the generation's operators) into ops.children and
// allocates that
struct AllocOps {
    const int32_t *anc = nullptr;
    int32_t *children = nullptr;
    const int64_t *gen = nullptr;
    uint64_t seed = 0;
    int m = 0;
    int32_t *slot_counters[2] = {nullptr, nullptr};   // zeroed by the workgroup of individual 0
};
hipError_t launch_alloc(const DevPtrs &P, const Dims &d, const int32_t *hubs, int count, uint16_t *kidx,
                        int want_sums, int want_ch, hipStream_t st, const AllocOps &ops = AllocOps{});
hipError_t launch_copy_clamp(const int32_t *src, int32_t *dst, int total, int n, hipStream_t st);
int alloc_blocks(int count);
hipError_t launch_alloc_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, int blocks, hipStream_t st);

// per-individual evaluation (eval_plain.hip)
hipError_t launch_eval_exact(const DevPtrs &P, const Dims &d, const int32_t *hubs, const uint16_t *kidx, int count,
                             double *cost, double *parts, double *eps, hipStream_t st);
hipError_t launch_eval_fp32(const DevPtrs &P, const Dims &d, const int32_t *hubs, const uint16_t *kidx, int count,
                            hipStream_t st);
double fp32_eps_bound(int n);

// batched FP32 evaluation on the vector units (eval_vec.hip)
hipError_t launch_eval_vec(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st,
                           hipEvent_t ev0, hipEvent_t ev1);
size_t vec_partial_bytes(const Dims &d);
int vec_group(int p);
hipError_t prepare_plain_kernels(int max_lds);

// exact re-evaluation of candidates, island decisions, P0 (recheck.hip)
hipError_t launch_recheck(const DevPtrs &P, const Dims &d, hipStream_t st);
hipError_t launch_p0_exact(const DevPtrs &P, const Dims &d, hipStream_t st);
size_t recheck_lds(int n, int p);
size_t recheck_wide_lds(int n, int p);
size_t recheck_group_lds_cap();
hipError_t launch_recheck_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, size_t lds, size_t lds_wide,
                                hipStream_t st);
hipError_t prepare_recheck_kernels(int max_lds);

// batched matrix-core evaluation (eval_mfma.hip)
hipError_t launch_eval_split(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st,
                             hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_mfma(const DevPtrs &P, const Dims &d, const uint16_t *kidx, int count, hipStream_t st);
hipError_t launch_finalize(const DevPtrs &P, const Dims &d, int count, int cfg, hipStream_t st);
int mfma_partial_tiles(const Dims &d, int cfg);
bool mfma_folds(const Dims &d, int cfg);
int mfma_w_layout(const Dims &d, int cfg);
bool mfma_split3_config(int cfg);
int finalize_blocks(int count);
hipError_t launch_finalize_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, int blocks, hipStream_t st);
bool mfma_groupable(const Dims &d, int cfg);
size_t mfma_job_bytes();
int mfma_fill_jobs(const DevPtrs *const *P, const Dims *const *d, int njobs, int cfg, void *jobs_host);
hipError_t launch_mfma_group(const GroupHdr *hdr, const void *d_jobs, int grid, int cfg, int kins, hipStream_t st);
int mfma_group_kins(int cfg, int min_p);
int mfma_pipelined(int cfg);
int mfma_num_configs();
int mfma_rows_per_tile(int cfg);
int mfma_cols_per_tile(int cfg);
int mfma_k_tile(int cfg);

// exhaustive search over hub sets (enumerate.hip)
hipError_t launch_enum_init(const DevPtrs &P, hipStream_t st);
hipError_t launch_enum_unrank(const DevPtrs &P, const Dims &d, int64_t first, int count, hipStream_t st);
hipError_t launch_enum_select(const DevPtrs &P, const Dims &d, int64_t first, int count, hipStream_t st);
hipError_t prepare_enum_kernels(int max_lds);

// GA (ga_ops.hip, select.hip)
int ga_ops_blocks(const Dims &d);
hipError_t launch_ga_ops_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, int blocks, hipStream_t st);
int select_threads(int m);
hipError_t launch_select1_group(const GroupHdr *hdr, const TickJob *jobs, int njobs, int blocks, int threads,
                                hipStream_t st);
hipError_t launch_select(const DevPtrs &P, const Dims &d, int exact, hipStream_t st, int reserve = 0);
hipError_t launch_init_state(const DevPtrs &P, const Dims &d, hipStream_t st);

}  // namespace hubga
