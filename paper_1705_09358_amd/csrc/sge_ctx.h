// Context state and the common launch path shared by the single-instance,
// batch and serve entry points.
#pragma once

#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>

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
    uint64_t matches = 0, states = 0, candidates = 0, steals = 0, steps = 0, bytes = 0;
};

// Buffers of one launch stream.
struct LaunchBufs {
    DevWork work;
    DevBuf d_blob;    // uploaded: search descriptors and plan requests (+ chunk prefix, device-written)
    DevBuf d_arena;   // device-written: plans, domains, per-position bitsets, candidate lists
    HostBuf h_blob, h_ctr;
    void release();
};

// A batch launch shape chosen by the autotuner.
struct BatchTune {
    int policy = 2, lanes = 0, donate = 1, per_cu = 0;
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
    int per_cu = 0;   // resident search blocks per compute unit (0 = as many as fit)
    uint32_t root_chunk = 0;
    int batch_policy = 0;
    int plan_where = -1;   // -1 automatic, 0 host, 1 device
    int count_bytes = 1;   // search launches count each instance's algorithmic bytes
    int check_uniform = 0; // search launches verify that a unit's lanes agree on its state
    // batch autotuner's choice by job list (hash); cleared when tuning changes
    std::map<uint64_t, sge::BatchTune> batch_tune;
    // by job list (the same hash): the steps each job took in its last launch
    std::map<uint64_t, std::vector<uint64_t>> batch_steps;
    int num_cus = 0;
    size_t lds_per_cu = 0;
    // resident graphs by handle (hashed: a 4096-job batch looks up 8192 handles per call)
    std::unordered_map<uint32_t, std::unique_ptr<sge::Target>> targets;
    std::unordered_map<uint32_t, std::unique_ptr<sge::Pattern>> patterns;
    uint32_t next_handle = 1;
    sge::LaunchBufs bufs;
    sge::DevBuf d_rows;
    double last_ms[3] = {0, 0, 0};   // last launch: kernel, until the last task finished, until done was set
    double last_busy_ms = 0;         // last launch: unit-milliseconds spent holding tasks
    uint32_t last_units = 0;         // last launch: units that entered the search loop
    int last_lanes = 0;              // last launch: lanes per search unit
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // around the search kernel of count, enumerate and batch launches
    bool graph_extras = true;          // captures take the event nodes around the search kernel
    std::string graph_extras_error;    // why a capture refused them (then graph_extras is false)
    const char *enqueue_step = "";     // the step enqueue_pack was at (for error messages)
    double last_event_ms = 0;                  // last launch: the search kernel between ev0 and ev1
    // the last batch launch's executable graph and the key of everything it
    // captured (sizes, launch shape, buffer addresses, settings)
    hipGraphExec_t gexec = nullptr;
    uint64_t gexec_key = 0;
    bool gexec_timed = false;   // it holds the kernel's event nodes
    hipEvent_t gev0 = nullptr, gev1 = nullptr;   // those event nodes' events (new ones for every capture)
    std::unique_ptr<sge::Server, sge::ServerDeleter> server;
    std::mutex serve_mu;
};

namespace sge {

sge_status fail(sge_ctx *c, sge_status code, const std::string &msg);
sge_status hip_fail(sge_ctx *c, hipError_t e, const char *what);

// Upload the job descriptors of `specs`, plan every instance on the device
// and search them all in one persistent launch.  With `graph` the upload, the
// kernels and the read-back are captured in a HIP graph and replayed.  Fills
// `out` and the host-preparation / search times (ms).
sge_status run_instances(sge_ctx *c, const std::vector<InstanceSpec> &specs, std::vector<InstanceOut> &out,
                         double &ms_prep, double &ms_search, bool graph, int policy);

// The pieces of run_instances, also used by the server.
// Whether these instances are searched by the dense-bitset kernel.
bool choose_dense(const sge_ctx *c, const std::vector<InstanceSpec> &specs);
bool choose_dense(const sge_ctx *c, const InstanceSpec *specs, size_t m);
// Candidate-list entries one instance may need (parentless positions).
uint64_t list_entries(const InstanceSpec &s);
// Device bytes one instance holds during a launch (descriptors, plan, domains,
// per-position bitsets, candidate lists).
uint64_t instance_device_bytes(const InstanceSpec &s);

// The layout of one launch: descriptors and plan requests in the uploaded
// blob, the device-written plan data in the arena.
struct Pack {
    LaunchCfg cfg;
    uint32_t m = 0;
    int policy = 2;
    bool device_plan = true;           // planned by the plan kernel (else uploaded host plans)
    uint64_t units = 1;                // approximate search units (root chunk sizing)
    double ms_work = 0, ms_done = 0;   // filled by read_pack
    double busy_ms = 0;                // unit-milliseconds holding tasks (read_pack)
    uint32_t units_run = 0;            // units that entered the search loop (read_pack)
    bool bad_task = false;             // filled by read_pack: the work queue delivered an invalid task
    bool bad_unit = false;             // filled by read_pack: a unit's lanes disagreed on its state
    size_t blob = 0, upload = 0, arena = 0, ctr_bytes = 0;
    size_t off_req = 0, off_pref = 0;  // in the blob
    std::vector<size_t> dom_at;        // in the arena: instance j's domains by pattern node
};

// The launch shape of a set of instances: sizes, kernel variant, unit
// width, donation, used-set mode (fills pk.cfg, pk.m, pk.policy, pk.units).
void launch_config(const sge_ctx *c, const InstanceSpec *const *specs, size_t m, bool dense, int policy, Pack &pk);
// Lay out the descriptors and plan requests of `specs` (every one with k > 0)
// in the pinned blob, with device addresses in bufs.d_blob / bufs.d_arena.
sge_status pack_instances(sge_ctx *c, const std::vector<const InstanceSpec *> &specs, bool dense, int policy,
                          LaunchBufs &bufs, Pack &pk);
// The same launch with plans built on the host (plans[j] / bits[j] belong to
// specs[j]; none of them empty): plans, lists and bitsets are uploaded.
sge_status pack_host_planned(sge_ctx *c, const std::vector<const InstanceSpec *> &specs,
                             const std::vector<const Plan *> &plans,
                             const std::vector<const std::vector<uint64_t> *> &bits, bool dense, int policy,
                             LaunchBufs &bufs, Pack &pk);
// Whether a launch of `ninst` instances is planned on the device: batches
// are (the plan kernel runs one workgroup per instance side by side); single
// searches and small launches are planned on the host, where the short serial
// work of one plan finishes sooner.
constexpr size_t PLAN_DEVICE_MIN_INSTANCES = 64;
bool plan_on_device(const sge_ctx *c, const std::vector<const InstanceSpec *> &specs);
// A search with a directed graph, or edge labels that are compared.
bool general_instance(const InstanceSpec &s);
// Indices 0..n-1 by decreasing key, ties in increasing index (a stable order).
void order_by_desc(const uint64_t *key, uint32_t n, uint32_t *perm);
// Upload, plan, reset, search and read back on `s` (asynchronous).  With
// events, e0 and e1 are recorded right before and after the search kernel
// (not while the stream is being captured: a batch graph gets event nodes
// added after its capture).
hipError_t enqueue_pack(sge_ctx *c, const Pack &pk, LaunchBufs &bufs, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
// Upload and plan only (the plan of instance 0 is then read back by the caller).
hipError_t enqueue_plan_only(const Pack &pk, LaunchBufs &bufs, uint32_t root_chunk, hipStream_t s);
// After the stream has drained: per-instance results and the kernel time.
void read_pack(const sge_ctx *c, Pack &pk, const LaunchBufs &bufs, const std::vector<const InstanceSpec *> &specs,
               std::vector<InstanceOut *> &out, double &ms_search);

// The allocation-free count's static scratch array: record its address on
// `device` (the current device), once per device.
hipError_t noalloc_init(int device);

// Device memory for a target's / pattern's resident data.
sge_status upload_target(sge_ctx *c, Target &t);
void free_target(Target &t);
sge_status upload_pattern(sge_ctx *c, Pattern &p);
void free_pattern(Pattern &p);

}  // namespace sge
