// C ABI of the learned motion-vector proposal network: creation from given
// initial weights, inference (seeds for the pel-recursive start), the
// gradient on labelled MBs, a momentum-SGD step (separately or fused),
// weight read-back, and checkpoints (versioned, checksummed files).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "host.h"
#include "me_internal.h"

using namespace me;
using namespace me::host;

struct me_net {
    int device = 0;
    float *P = nullptr, *V = nullptr;  // fp32 master weights and momentum
    uint16_t *wb = nullptr;            // bf16 copies
    uint8_t *buf = nullptr;            // per-call scratch
    size_t cap = 0;
    void *host[2] = {nullptr, nullptr};  // pinned job-table staging
    size_t host_cap[2] = {0, 0};
    hipEvent_t ev[2] = {nullptr, nullptr};
    int slot = 0;
    double *host_loss = nullptr;
    int cus = 256;
    int scale = 2;  // window scale f: reference window [-(12f-8), 12f+8) box-averaged f x f
    std::mutex mu;
};

namespace {

void release(me_net *m) {
    if (!m) return;
    hipDeviceSynchronize();
    if (m->P) hipFree(m->P);
    if (m->V) hipFree(m->V);
    if (m->wb) hipFree(m->wb);
    if (m->buf) hipFree(m->buf);
    for (int s = 0; s < 2; ++s) {
        if (m->host[s]) hipHostFree(m->host[s]);
        if (m->ev[s]) hipEventDestroy(m->ev[s]);
    }
    if (m->host_loss) hipHostFree(m->host_loss);
    delete m;
}

// Validated job table (flat MB order) for the network calls; `aux` per job
// is the label field (training) or the prediction output (inference).
int net_table(const me_job *jobs, int n, const void *const *aux, bool need_aux, std::vector<JobDesc> &desc,
              long long &total) {
    if (n <= 0 || !jobs) return ME_EINVAL;
    desc.resize(n);
    total = 0;
    for (int i = 0; i < n; ++i) {
        const me_job &j = jobs[i];
        int rc = check_frame(j.cur, false);
        if (rc) return rc;
        rc = check_frame(j.ref, false);
        if (rc) return rc;
        if (j.cur.width != j.ref.width || j.cur.height != j.ref.height || j.cur.stride != j.ref.stride)
            return ME_EINVAL;
        const void *x = aux ? aux[i] : nullptr;
        if (need_aux && !x) return ME_EINVAL;
        if ((x && !al4(x)) || (j.seed && !al4(j.seed))) return ME_EALIGN;
        JobDesc d;
        std::memset(&d, 0, sizeof(d));
        d.cur = j.cur.luma;
        d.ref = j.ref.luma;
        d.cls = j.mb_class;
        d.seed = (const int16_t *)j.seed;
        if (need_aux)
            d.tf = (const int16_t *)x;
        else
            d.out_u32 = (uint32_t *)const_cast<void *>(x);
        d.width = j.cur.width;
        d.height = j.cur.height;
        d.stride = j.cur.stride;
        d.wm = d.width / 16;
        d.hm = d.height / 16;
        d.mb_base = (int32_t)total;
        d.dep_line_base = -1;
        total += (long long)d.wm * d.hm;
        desc[i] = d;
    }
    if (total > (1ll << 30) || n > 65535) return ME_EINVAL;
    for (const auto &d : desc)
        if (d.wm * d.hm > 65536) return ME_EINVAL;  // list entries keep 16 bits of MB index
    return ME_OK;
}

int ensure(me_net &m, size_t bytes, hipStream_t s) {
    if (bytes <= m.cap) return ME_OK;
    if (m.buf) {
        if (hipStreamSynchronize(s) != hipSuccess) return ME_EHIP;
        hipFree(m.buf);
        m.buf = nullptr;
        m.cap = 0;
    }
    const size_t cap = std::max(bytes + bytes / 4, (size_t)1 << 20);
    if (hipMalloc(&m.buf, cap) != hipSuccess) return ME_ENOMEM;
    m.cap = cap;
    return ME_OK;
}

int upload_table(me_net &m, const std::vector<JobDesc> &desc, hipStream_t s) {
    const size_t bytes = desc.size() * sizeof(JobDesc);
    const int k = m.slot;
    m.slot ^= 1;
    if (hipEventSynchronize(m.ev[k]) != hipSuccess) return ME_EHIP;
    if (m.host_cap[k] < bytes) {
        if (m.host[k]) hipHostFree(m.host[k]);
        m.host[k] = nullptr;
        m.host_cap[k] = 0;
        if (hipHostMalloc(&m.host[k], std::max(bytes, (size_t)4096), hipHostMallocDefault) != hipSuccess)
            return ME_ENOMEM;
        m.host_cap[k] = std::max(bytes, (size_t)4096);
    }
    std::memcpy(m.host[k], desc.data(), bytes);
    if (hipMemcpyAsync(m.buf, m.host[k], bytes, hipMemcpyHostToDevice, s) != hipSuccess) return ME_EHIP;
    if (hipEventRecord(m.ev[k], s) != hipSuccess) return ME_EHIP;
    return ME_OK;
}

int check_lds(int dev, bool train) {
    int lim = 0;
    if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return ME_EHIP;
    return net_lds_bytes(train) <= (size_t)lim ? ME_OK : ME_ENOMEM;
}

}  // namespace

namespace me {
namespace host {

// Seeds of every opaque MB of `jobs` (their `seed` buffers) from `net`
// (used by me_texture_recursive before the search).
int net_seed_jobs(me_net *net, const me_job *jobs, int n, void *stream) {
    for (int i = 0; i < n; ++i)
        if (!jobs[i].seed) return ME_EINVAL;
    return me_net_forward(net, jobs, n, nullptr, stream);
}

size_t net_table_scratch(int total_mbs) { return net_list_scratch(total_mbs); }

// Seeds for an already uploaded job table (used inside captured graphs: no
// allocation, no host synchronisation; `t` = events captured around the
// forward kernel, or none).
hipError_t net_forward_table(me_net *net, const JobDesc *table, int n, int total_mbs, uint8_t *scratch,
                             hipStream_t s, const KernelTimer *t) {
    const uint32_t *list = nullptr, *count = nullptr;
    hipError_t e = launch_net_list(table, n, total_mbs, scratch, &list, &count, s);
    if (e != hipSuccess) return e;
    const int groups = (int)std::min<long long>(total_mbs, (long long)net->cus * 3);
    return launch_net(false, table, n, list, count, net->P, net->wb, nullptr, groups, net->scale, s, t);
}

}  // namespace host
}  // namespace me

extern "C" {

namespace {

// Device net from host weights and (nullable) momentum.
int create_net(const float *init, const float *mom, int32_t scale, me_net **out) {
    if (!out) return ME_EINVAL;
    *out = nullptr;
    if (!init || (scale != 2 && scale != 4)) return ME_EINVAL;
    for (int i = 0; i < kNetParams; ++i)
        if (!std::isfinite(init[i]) || (mom && !std::isfinite(mom[i]))) return ME_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || check_device(dev) != ME_OK) return ME_ENODEV;
    int rc = check_lds(dev, false);
    if (rc) return rc;
    me_net *m = new me_net();
    m->device = dev;
    m->scale = scale;
    hipDeviceGetAttribute(&m->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (m->cus <= 0) m->cus = 256;
    if (hipMalloc(&m->P, kNetParams * 4) != hipSuccess || hipMalloc(&m->V, kNetParams * 4) != hipSuccess ||
        hipMalloc(&m->wb, kNetBf16 * 2) != hipSuccess ||
        hipHostMalloc((void **)&m->host_loss, sizeof(double), hipHostMallocDefault) != hipSuccess) {
        release(m);
        return ME_ENOMEM;
    }
    for (int s = 0; s < 2; ++s)
        if (hipEventCreateWithFlags(&m->ev[s], hipEventDisableTiming) != hipSuccess) {
            release(m);
            return ME_EHIP;
        }
    std::vector<float> zero(kNetParams, 0.f);
    if (hipMemcpy(m->P, init, kNetParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->V, mom ? mom : zero.data(), kNetParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
        launch_net_refresh(m->P, m->wb, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        release(m);
        return ME_EHIP;
    }
    *out = m;
    return ME_OK;
}

// Checkpoint layout (little-endian): 8-byte magic, u32 version, u32 number
// of parameters, u32 window scale, u32 reserved (0), the fp32 weights, the
// fp32 momentum, then the 64-bit FNV-1a hash of every byte before it.
constexpr char kMagic[8] = {'M', 'E', '-', 'N', 'E', 'T', '\0', '\0'};
constexpr uint32_t kVersion = 1;
constexpr size_t kHeader = 24;
constexpr size_t kFileBytes = kHeader + 8 * (size_t)kNetParams + 8;

// 64-bit FNV-1a: the published offset basis and prime.
uint64_t fnv1a64(const uint8_t *p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

}  // namespace

int me_net_create(const float *init, int32_t scale, me_net **out) { return create_net(init, nullptr, scale, out); }

int me_net_save(me_net *net, const char *path) {
    if (!net || !path) return ME_EINVAL;
    std::vector<uint8_t> buf(kFileBytes, 0);
    std::memcpy(buf.data(), kMagic, 8);
    const uint32_t hdr[4] = {kVersion, (uint32_t)kNetParams, (uint32_t)net->scale, 0u};
    std::memcpy(buf.data() + 8, hdr, 16);
    int rc = me_net_weights(net, (float *)(buf.data() + kHeader), (float *)(buf.data() + kHeader + 4 * kNetParams));
    if (rc) return rc;
    const uint64_t h = fnv1a64(buf.data(), kFileBytes - 8);
    std::memcpy(buf.data() + kFileBytes - 8, &h, 8);
    FILE *f = std::fopen(path, "wb");
    if (!f) return ME_EIO;
    const bool ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
    const bool closed = std::fclose(f) == 0;
    return ok && closed ? ME_OK : ME_EIO;
}

int me_net_load(const char *path, me_net **out) {
    if (!out) return ME_EINVAL;
    *out = nullptr;
    if (!path) return ME_EINVAL;
    FILE *f = std::fopen(path, "rb");
    if (!f) return ME_EIO;
    std::vector<uint8_t> buf(kFileBytes + 1);
    const size_t got = std::fread(buf.data(), 1, buf.size(), f);
    std::fclose(f);
    if (got != kFileBytes) return ME_EFORMAT;  // truncated or trailing bytes
    uint32_t hdr[4];
    std::memcpy(hdr, buf.data() + 8, 16);
    uint64_t h = 0;
    std::memcpy(&h, buf.data() + kFileBytes - 8, 8);
    if (std::memcmp(buf.data(), kMagic, 8) != 0 || hdr[0] != kVersion || hdr[1] != (uint32_t)kNetParams ||
        hdr[3] != 0u || h != fnv1a64(buf.data(), kFileBytes - 8))
        return ME_EFORMAT;
    std::vector<float> w(2 * (size_t)kNetParams);
    std::memcpy(w.data(), buf.data() + kHeader, 8 * (size_t)kNetParams);
    const int rc = create_net(w.data(), w.data() + kNetParams, (int32_t)hdr[2], out);
    return rc == ME_EINVAL ? ME_EFORMAT : rc;
}

void me_net_destroy(me_net *net) { release(net); }

int me_net_weights(me_net *net, float *weights, float *momentum) {
    if (!net || !weights) return ME_EINVAL;
    std::lock_guard<std::mutex> lk(net->mu);
    if (hipDeviceSynchronize() != hipSuccess) return ME_EHIP;
    if (hipMemcpy(weights, net->P, kNetParams * 4, hipMemcpyDeviceToHost) != hipSuccess) return ME_EHIP;
    if (momentum && hipMemcpy(momentum, net->V, kNetParams * 4, hipMemcpyDeviceToHost) != hipSuccess) return ME_EHIP;
    return ME_OK;
}

int me_net_forward(me_net *net, const me_job *jobs, int n, float *const *pred, void *stream) {
    if (!net) return ME_EINVAL;
    std::vector<JobDesc> desc;
    long long total = 0;
    int rc = net_table(jobs, n, (const void *const *)pred, false, desc, total);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(net->mu);
    hipStream_t s = (hipStream_t)stream;
    const size_t o_list = align_up(desc.size() * sizeof(JobDesc), 256);
    rc = ensure(*net, o_list + net_list_scratch((int)total), s);
    if (rc) return rc;
    rc = upload_table(*net, desc, s);
    if (rc) return rc;
    const uint32_t *list = nullptr, *count = nullptr;
    const JobDesc *tab = (const JobDesc *)net->buf;
    if (launch_net_list(tab, n, (int)total, net->buf + o_list, &list, &count, s) != hipSuccess) return ME_EHIP;
    const int groups = (int)std::min<long long>(total, (long long)net->cus * 3);
    KernelTimer kt;
    const bool timed = kernel_timer(stream, ME_KT_NET, &kt);
    return hip_err(launch_net(false, tab, n, list, count, net->P, net->wb, nullptr, groups, net->scale, s,
                              timed ? &kt : nullptr));
}

namespace {

// Forward + backward on the served MBs of `jobs` into per-workgroup
// partials, then their fixed-order sum into `grad` / `loss` (device), and,
// with `apply`, momentum SGD.  The loss is read back when `loss_host` is set.
int net_step(me_net *net, const me_job *jobs, int n, const me_mv *const *labels, float lr, float momentum,
             bool apply, float *grad, double *loss_host, void *stream) {
    if (!net || !labels) return ME_EINVAL;
    if (!std::isfinite(lr) || lr < 0.f || !std::isfinite(momentum) || momentum < 0.f || momentum >= 1.f)
        return ME_EINVAL;
    if (grad && !al4(grad)) return ME_EALIGN;
    std::vector<JobDesc> desc;
    long long total = 0;
    int rc = net_table(jobs, n, (const void *const *)labels, true, desc, total);
    if (rc) return rc;
    rc = check_lds(net->device, true);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(net->mu);
    hipStream_t s = (hipStream_t)stream;
    const int groups = (int)std::min<long long>(total, (long long)net->cus);
    const size_t o_list = align_up(desc.size() * sizeof(JobDesc), 256);
    const size_t o_part = o_list + align_up(net_list_scratch((int)total), 256);
    const size_t o_loss = o_part + align_up((size_t)groups * (kNetParams + 1) * 4, 256);
    rc = ensure(*net, o_loss + 256, s);
    if (rc) return rc;
    rc = upload_table(*net, desc, s);
    if (rc) return rc;
    const uint32_t *list = nullptr, *count = nullptr;
    const JobDesc *tab = (const JobDesc *)net->buf;
    if (launch_net_list(tab, n, (int)total, net->buf + o_list, &list, &count, s) != hipSuccess) return ME_EHIP;
    float *part = (float *)(net->buf + o_part);
    double *dloss = (double *)(net->buf + o_loss);
    KernelTimer kt;
    const bool timed = kernel_timer(stream, ME_KT_NET_TRAIN, &kt);
    if (launch_net(true, tab, n, list, count, net->P, net->wb, part, groups, net->scale, s, timed ? &kt : nullptr) !=
        hipSuccess)
        return ME_EHIP;
    if (launch_net_sgd(net->P, net->V, net->wb, part, groups, lr, momentum, grad, dloss, s, apply) != hipSuccess)
        return ME_EHIP;
    if (loss_host) {
        if (hipMemcpyAsync(net->host_loss, dloss, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
            return ME_EHIP;
        if (hipStreamSynchronize(s) != hipSuccess) return ME_EHIP;
        *loss_host = *net->host_loss;
    }
    return ME_OK;
}

}  // namespace

int me_net_train_step(me_net *net, const me_job *jobs, int n, const me_mv *const *labels, float lr, float momentum,
                      float *grad, double *loss, void *stream) {
    return net_step(net, jobs, n, labels, lr, momentum, true, grad, loss, stream);
}

int me_net_backward(me_net *net, const me_job *jobs, int n, const me_mv *const *labels, float *grad, double *loss,
                    void *stream) {
    if (!grad) return ME_EINVAL;
    return net_step(net, jobs, n, labels, 0.f, 0.f, false, grad, loss, stream);
}

int me_net_sgd_step(me_net *net, const float *grad, float lr, float momentum, void *stream) {
    if (!net || !grad) return ME_EINVAL;
    if (!std::isfinite(lr) || lr < 0.f || !std::isfinite(momentum) || momentum < 0.f || momentum >= 1.f)
        return ME_EINVAL;
    if (!al4(grad)) return ME_EALIGN;
    std::lock_guard<std::mutex> lk(net->mu);
    return hip_err(launch_net_apply(net->P, net->V, net->wb, grad, lr, momentum, (hipStream_t)stream));
}

int me_net_scale(const me_net *net) { return net ? net->scale : ME_EINVAL; }

}  // extern "C"
