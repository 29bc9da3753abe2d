// Host-side state of one simulation and the runtime helpers shared by the
// single-lattice API and the batched pool.
#pragma once

#include "ce_internal.hpp"

namespace ce {
namespace host {

constexpr size_t kAlign = 256;
constexpr long long kStagingElems = 1LL << 24;  // 128 MiB of FP64 per staging chunk (a 256^3 field in one)

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t field_bytes;   // one array of one field
    size_t off_fields;    // 4 * nf arrays
    size_t off_scalars, off_partials, off_ticket, off_ring, off_maxabs, off_staging;
    size_t total;
    long long staging_elems;
    int nblocks;
};


// Record a failure for ce_last_error() and return `st`.
ce_status fail(ce_status st, const char *fmt, ...);

#define CE_HIP(call)                                                                                    \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return ::ce::host::fail(CE_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)
long long sites_of(const ce_params *p);
Layout layout_of(const ce_params *p);
ce_status validate(const ce_params *p);
ce_status device_cus(int *cus);

}  // namespace host
}  // namespace ce

struct ce_sim {
    ce_params p;
    ce::host::Layout lay;
    ce::Lattice lat;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    char *base = nullptr;
    bool own_mem = false;
    double *staging = nullptr;
    unsigned int *maxabs = nullptr;
    int cur = 0;            // buffer holding the current state
    long long step = 0;
    unsigned loaded = 0;    // bit per field
    bool started = false;
    int step_block = 32;
    double m_host[CE_MAX_FIELDS] = {0, 0, 0};  // homogeneous references at load time
    ce_launch launch{CE_KERNEL_DIRECT, 0, 0, 0, 0, 0};
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // step block starting from buffer 0 / 1
    int graph_k = 0;
};

namespace ce {
namespace host {

// Validate a launch configuration for the simulation and apply it.
ce_status apply_launch(ce_sim *s, const ce_launch &cfg);
// Every field is present (loaded or generated): check leapfrog stability with
// the recorded field maxima and queue the start-up half step.
ce_status start_run(ce_sim *s);
void drop_graphs(ce_sim *s);

}  // namespace host
}  // namespace ce
