// Launchers of flat per-MB kernels outside the search: reference padding,
// and the batch's fused forms of classification and MC.
#pragma once
#include <hip/hip_runtime.h>

#include "me_internal.h"

namespace me {

// MPEG-4 padding of each job's reference VOP (cur / cur_a -> out_u8);
// `cls_all` holds total_mbs class bytes (job i's at its mb_base), `max_mbs`
// is the largest job's MB count.
hipError_t launch_pad(const JobDesc *jobs, int n, int max_mbs, uint8_t *cls_all, hipStream_t s);

// Classification as launch_classify that also sets z0[0, n0) and z1[0, n1)
// to zero (32-bit words; scratch that later kernels of the stream expect
// cleared).
hipError_t launch_classify_zeroing(const JobDesc *jobs, int n, int total_mbs, uint32_t *z0, size_t n0, uint32_t *z1,
                                   size_t n1, hipStream_t s, const KernelTimer *t, int per_cu);

// MC sums without a prediction frame, added atomically to acc[2 j] (SSE)
// and acc[2 j + 1] (pixel count) of job j: acc must be zero before.
hipError_t launch_mc_sums_acc(const JobDesc *jobs, int n, int total_mbs, unsigned long long *acc, uint32_t *status,
                              hipStream_t s, const KernelTimer *t, int per_cu);

}  // namespace me
