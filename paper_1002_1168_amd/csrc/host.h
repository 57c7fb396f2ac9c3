// Host-side helpers shared by the C-ABI entry points: argument validation,
// job descriptors, and the chain / ticket tables of the pipelined search.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "me.h"
#include "me_internal.h"

namespace me {
namespace host {

constexpr int kMaxDim = 4096;  // ticket packing: 8 bits per MB coordinate
constexpr int kMaxChains = 65536;
constexpr int kSpinLimit = 1 << 22;
// With learned seeds a dropped seed adds the plain recursion's candidates to
// its own (at most 2 k_max), and iteration counts are stored in a byte.
constexpr int kMaxSeededKmax = 127;

// The last search call's prepared launch (reused when the next call passes
// byte-identical jobs and parameters).
struct PaMemo {
    std::vector<uint8_t> key;  // jobs + params + mode
    std::vector<uint8_t> blob;
    size_t o_jobs = 0, o_ch = 0, o_tk = 0, o_bands = 0;
    int n = 0, total_mbs = 0, nlines = 0, mask_words = 0, nchains = 0;
    int nbands = 0;          // bands of kRowWaves rows (job sets without chains)
    bool unchained = false;  // no job's T field is written in the same call
    std::vector<int> order;  // chain-ordered descriptor i describes job order[i]
    std::vector<int> prod;   // per job: the earlier job whose mv_int is its T field, or -1
    bool valid = false;
};

int hip_err(hipError_t e);
// ME_OK when `dev` is a gfx950 device (cached after the first query).
int check_device(int dev);
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
// Flags whose boundary-MB texture reads only the one-wave line worker has.
inline bool one_wave_lines(uint32_t flags) { return (flags & (ME_FLAG_T_TEXTURE | ME_FLAG_MASKED_PRS)) != 0; }
inline bool al4(const void *p) { return ((uintptr_t)p & 3u) == 0; }

// Append `count` objects to `b` at a 64-byte boundary; returns their offset.
template <class T>
inline size_t put(std::vector<uint8_t> &b, const T *p, size_t count) {
    size_t off = align_up(b.size(), 64);
    b.resize(off + sizeof(T) * count);
    if (count) std::memcpy(b.data() + off, p, sizeof(T) * count);
    return off;
}

int check_frame(const me_frame &f, bool need_alpha);
int check_params(const me_params *p);
int check_job(const me_job &j, bool need_alpha);
KParams kparams(const me_params *p, bool shape_only);
JobDesc job_desc(const me_job &j);
// Checked descriptor of one motion-compensation job (prediction out `pred`,
// nullable); mb_base is left 0.
int mc_desc(const me_job &j, uint8_t *pred, JobDesc *out);
// Chains, chain-ordered descriptors and the ticket order of a job set.
int build_pa(const me_job *jobs, int n, PaMemo &m);
// Event pair for the main kernel of a call of timing kind `kind` (ME_KT_*)
// on `stream`; false when timing is off.
bool kernel_timer(void *stream, int kind, KernelTimer *out);
// Whether calls of timing kind `kind` (ME_KT_*) record kernel events now.
bool timing_enabled(int kind);
// Network seeds for a job table already on the device (graph-capturable);
// `scratch` holds net_table_scratch(total_mbs) bytes.
size_t net_table_scratch(int total_mbs);
hipError_t net_forward_table(me_net *net, const JobDesc *table, int n, int total_mbs, uint8_t *scratch,
                             hipStream_t s, const KernelTimer *t = nullptr);
// Proposal-network seeds into every job's seed buffer (all must be set).
int net_seed_jobs(me_net *net, const me_job *jobs, int n, void *stream);

}  // namespace host
}  // namespace me
