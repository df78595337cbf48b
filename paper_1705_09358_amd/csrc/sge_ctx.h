// Context state and the common launch path shared by the single-instance,
// batch and serve entry points.
#pragma once

#include <chrono>
#include <map>
#include <memory>
#include <mutex>

#include "sge_internal.h"

namespace sge {

// A growable device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t reserve(size_t bytes);
    void release();
};

// A growable pinned host buffer.
struct HostBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t reserve(size_t bytes);
    void release();
};

// One search to run: which graphs, how, and where rows go.
struct InstanceSpec {
    const Target *t = nullptr;
    const Pattern *p = nullptr;
    int mode = SGE_RI;
    bool labelled = true;
    uint32_t *rows = nullptr;   // device pointer or null
    uint64_t cap_rows = 0;
};

struct InstanceOut {
    sge_status status = SGE_OK;
    bool timed_out = false;
    uint64_t matches = 0, states = 0, candidates = 0, steals = 0;
};

struct Server;
struct ServerDeleter {
    void operator()(Server *s) const;
};

}  // namespace sge

struct sge_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int labelled = 1;
    int mode = SGE_RI;
    uint64_t cap = 0;
    uint64_t time_limit_ms = 120000;   // every search launch ends by this time
    uint32_t root_lo = 0, root_hi = 0xFFFFFFFFu;
    int lanes = 0, dense = -1, donate = 1;
    uint32_t root_chunk = 0;
    int batch_policy = 0;
    int num_cus = 0;
    size_t lds_per_cu = 0;
    std::map<uint32_t, std::unique_ptr<sge::Target>> targets;
    std::map<uint32_t, std::unique_ptr<sge::Pattern>> patterns;
    uint32_t next_handle = 1;
    sge::DevWork work;
    sge::DevBuf d_blob, d_rows;
    sge::HostBuf h_blob, h_ctr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::unique_ptr<sge::Server, sge::ServerDeleter> server;
    std::mutex serve_mu;
};

namespace sge {

sge_status fail(sge_ctx *c, sge_status code, const std::string &msg);
sge_status hip_fail(sge_ctx *c, hipError_t e, const char *what);

// Plan, upload and search `specs` in one persistent launch.  With `graph`
// the uploads, the launch and the read-back are captured in a HIP graph and
// replayed.  Fills `out` and the prep / search times (ms).
sge_status run_instances(sge_ctx *c, const std::vector<InstanceSpec> &specs, std::vector<InstanceOut> &out,
                         double &ms_prep, double &ms_search, bool graph, int policy);

// Device memory for a target's resident data.
sge_status upload_target(sge_ctx *c, Target &t);
void free_target(Target &t);

}  // namespace sge
