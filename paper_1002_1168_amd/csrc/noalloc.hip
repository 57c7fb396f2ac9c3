// Allocation-free motion compensation + masked SSE: the same kernels as
// me_motion_compensate_sse, with every buffer beyond the caller's inputs and
// outputs (the job table, the per-MB partial sums, the status slot) in one
// fixed array in device memory, so that the call allocates nothing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.h"
#include "me_internal.h"

using namespace me;
using namespace me::host;

namespace {

constexpr int kMaxJobs = 1024;
constexpr int kMaxMbs = 1 << 19;
constexpr size_t kDescBytes = sizeof(JobDesc) * kMaxJobs;  // 160 KiB
constexpr size_t kPartBytes = (size_t)kMaxMbs * 8;         // two u32 per MB: 4 MiB
constexpr size_t kStatusBytes = 256;
constexpr size_t kScratchBytes = kDescBytes + kPartBytes + kStatusBytes;
constexpr int kMaxDevices = 64;
constexpr int kChunk = 16;  // descriptors per upload launch, passed as kernel arguments (2.5 KiB)

}  // namespace

// One copy per GPU, resident until the process ends.  Host code reaches it
// only through the address hipGetSymbolAddress returns on each device.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

struct DescChunk {
    JobDesc d[kChunk];
};

// Copy `count` descriptors from the kernel arguments into the job table.
__global__ __launch_bounds__(64) void put_descs(DescChunk c, int count, JobDesc *dst) {
    const uint32_t *src = (const uint32_t *)&c;
    uint32_t *out = (uint32_t *)dst;
    const int words = count * (int)(sizeof(JobDesc) / 4);
    for (int i = threadIdx.x; i < words; i += 64) out[i] = src[i];
}

std::mutex g_mu;
uint8_t *g_scratch[kMaxDevices] = {};

// The scratch address on device `dev` (current), looked up once per device.
int scratch_on(int dev, uint8_t **out) {
    if (dev < 0 || dev >= kMaxDevices) return ME_ENODEV;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ME_EHIP;
        g_scratch[dev] = (uint8_t *)p;
    }
    *out = g_scratch[dev];
    return ME_OK;
}

}  // namespace

extern "C" int me_motion_compensate_sse_noalloc(const me_job *jobs, int n, uint8_t *const *pred, uint64_t *sums,
                                                void *stream) {
    if (n < 0 || (n > 0 && (!jobs || !sums))) return ME_EINVAL;
    if (((uintptr_t)sums & 7u) != 0) return ME_EALIGN;
    if (n > kMaxJobs) return ME_EINVAL;
    long long total = 0;
    for (int i = 0; i < n; ++i) {
        JobDesc d;
        int rc = mc_desc(jobs[i], pred ? pred[i] : nullptr, &d);
        if (rc) return rc;
        total += (long long)d.wm * d.hm;
    }
    if (total > kMaxMbs) return ME_EINVAL;
    if (n == 0) return ME_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ME_ENODEV;
    int rc = check_device(dev);
    if (rc) return rc;
    uint8_t *base = nullptr;
    rc = scratch_on(dev, &base);
    if (rc) return rc;
    JobDesc *table = (JobDesc *)base;
    uint32_t *part = (uint32_t *)(base + kDescBytes);
    uint32_t *status = (uint32_t *)(base + kDescBytes + kPartBytes);
    hipStream_t s = (hipStream_t)stream;
    // the job table, kChunk descriptors per launch (kernel arguments are
    // copied at launch, so nothing on the host outlives the call)
    long long mb = 0;
    for (int c0 = 0; c0 < n; c0 += kChunk) {
        DescChunk c;
        const int count = n - c0 < kChunk ? n - c0 : kChunk;
        for (int i = 0; i < count; ++i) {
            mc_desc(jobs[c0 + i], pred ? pred[c0 + i] : nullptr, &c.d[i]);
            c.d[i].mb_base = (int32_t)mb;
            mb += (long long)c.d[i].wm * c.d[i].hm;
        }
        hipLaunchKernelGGL(put_descs, dim3(1), dim3(64), 0, s, c, count, table + c0);
        if (hipGetLastError() != hipSuccess) return ME_EHIP;
    }
    // the status slot starts clear on every call; every MB's partials are
    // written by the prediction kernel before the per-job sums read them
    rc = hip_err(launch_fill_u32(status, kStatusBytes / 4, 0u, s));
    if (rc) return rc;
    bool sums_only = true;
    for (int i = 0; pred && i < n; ++i) sums_only = sums_only && pred[i] == nullptr;
    return hip_err(launch_mc(table, n, (int)total, part, (unsigned long long *)sums, status, s, nullptr, 8, false,
                             sums_only));
}
