// C ABI entry points: contexts, resident targets, patterns, settings, and the
// common path that plans, uploads and searches a set of instances in one
// persistent launch.
#include <algorithm>
#include <cstring>
#include <thread>

#include "sge_ctx.h"

using namespace sge;
using clk = std::chrono::steady_clock;

namespace sge {

hipError_t DevBuf::reserve(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    release();
    size_t want = std::max(bytes, cap * 2);
    want = (want + 4095) & ~size_t(4095);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) { p = nullptr; return e; }
    cap = want;
    return hipSuccess;
}
void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
}
hipError_t HostBuf::reserve(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    release();
    size_t want = std::max(bytes, cap * 2);
    want = (want + 4095) & ~size_t(4095);
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) { p = nullptr; return e; }
    cap = want;
    return hipSuccess;
}
void HostBuf::release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
}

sge_status fail(sge_ctx *c, sge_status code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}
sge_status hip_fail(sge_ctx *c, hipError_t e, const char *what) {
    return fail(c, SGE_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Dense adjacency rows are kept for targets up to this many nodes; larger
// targets test back-edges by binary search in the CSR row.
static constexpr uint32_t ADJ_BITSET_MAX_N = 65536;

sge_status upload_target(sge_ctx *c, Target &t) {
    const HostGraph &g = t.g;
    std::vector<NodeRec> rec(g.n);
    for (uint32_t v = 0; v < g.n; v++) rec[v] = NodeRec{g.rp[v], g.outdeg(v), t.dlab[v], g.indeg(v)};
    size_t mcol = std::max<size_t>(g.col.size(), 1);
    hipError_t e;
    if ((e = hipMalloc(&t.d_col, mcol * 4)) != hipSuccess) return hip_fail(c, e, "hipMalloc(col)");
    if ((e = hipMalloc(&t.d_node, std::max<size_t>(g.n, 1) * sizeof(NodeRec))) != hipSuccess)
        return hip_fail(c, e, "hipMalloc(node)");
    t.dev_bytes = mcol * 4 + std::max<size_t>(g.n, 1) * sizeof(NodeRec);
    if (g.col.size() && (e = hipMemcpy(t.d_col, g.col.data(), g.col.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "upload col");
    if (g.n && (e = hipMemcpy(t.d_node, rec.data(), g.n * sizeof(NodeRec), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "upload node records");
    auto up = [&](uint32_t *&dst, const std::vector<uint32_t> &src, const char *what) -> sge_status {
        const size_t bytes = std::max<size_t>(src.size(), 1) * 4;
        hipError_t e2 = hipMalloc(&dst, bytes);
        if (e2 != hipSuccess) return hip_fail(c, e2, what);
        if (!src.empty() && (e2 = hipMemcpy(dst, src.data(), src.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(c, e2, what);
        t.dev_bytes += bytes;
        return SGE_OK;
    };
    sge_status st;
    if (g.directed) {
        if ((st = up(t.d_irp, g.irp, "upload in-edge rows")) != SGE_OK) return st;
        if ((st = up(t.d_icol, g.icol, "upload in-edges")) != SGE_OK) return st;
    }
    if (g.has_elab()) {
        if ((st = up(t.d_elab, g.elab, "upload edge labels")) != SGE_OK) return st;
        if (g.directed && (st = up(t.d_ielab, g.ielab, "upload in-edge labels")) != SGE_OK) return st;
    }
    // wide CSR (undirected targets): a candidate's id, row start, degree and
    // label in one 16-byte load, so the search step needs no second
    // dependent load for the node record
    if (!g.directed && !g.col.empty()) {
        std::vector<WideEntry> w(g.col.size());
        for (size_t e = 0; e < g.col.size(); e++) {
            const uint32_t x = g.col[e];
            w[e] = WideEntry{x, g.rp[x], g.outdeg(x), t.dlab[x]};
        }
        hipError_t e2 = hipMalloc(&t.d_wcol, w.size() * sizeof(WideEntry));
        if (e2 != hipSuccess) return hip_fail(c, e2, "hipMalloc(wide CSR)");
        if ((e2 = hipMemcpy(t.d_wcol, w.data(), w.size() * sizeof(WideEntry), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(c, e2, "upload wide CSR");
        t.dev_bytes += w.size() * sizeof(WideEntry);
    }
    // adjacency rows (undirected targets: the dense search and direct edge tests)
    if (g.n && g.n <= ADJ_BITSET_MAX_N && !g.directed) {
        std::vector<uint64_t> adj((size_t)g.n * t.W, 0);
        for (uint32_t v = 0; v < g.n; v++)
            for (uint32_t i = g.rp[v]; i < g.rp[v + 1]; i++) {
                uint32_t w = g.col[i];
                adj[(size_t)v * t.W + (w >> 6)] |= 1ull << (w & 63);
            }
        if ((e = hipMalloc(&t.d_adj, adj.size() * 8)) != hipSuccess) return hip_fail(c, e, "hipMalloc(adj)");
        if ((e = hipMemcpy(t.d_adj, adj.data(), adj.size() * 8, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(c, e, "upload adjacency bitsets");
        t.dev_bytes += adj.size() * 8;
    }
    // neighbour-degree table (the plan kernel's first arc-consistency round)
    if (!g.directed && !g.has_elab() && !t.nbr_deg.empty()) {
        if ((e = hipMalloc(&t.d_nbr_deg, t.nbr_deg.size())) != hipSuccess) return hip_fail(c, e, "hipMalloc(table)");
        if ((e = hipMemcpy(t.d_nbr_deg, t.nbr_deg.data(), t.nbr_deg.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(c, e, "upload neighbour-degree table");
        t.dev_bytes += t.nbr_deg.size();
    }
    const size_t nk = std::max<size_t>(t.label_keys.size(), 1);
    if ((e = hipMalloc(&t.d_label_keys, nk * 4)) != hipSuccess) return hip_fail(c, e, "hipMalloc(label keys)");
    if (!t.label_keys.empty() &&
        (e = hipMemcpy(t.d_label_keys, t.label_keys.data(), t.label_keys.size() * 4, hipMemcpyHostToDevice)) !=
            hipSuccess)
        return hip_fail(c, e, "upload label keys");
    t.dev_bytes += nk * 4;
    return SGE_OK;
}

void free_target(Target &t) {
    if (t.d_col) (void)hipFree(t.d_col);
    if (t.d_node) (void)hipFree(t.d_node);
    if (t.d_adj) (void)hipFree(t.d_adj);
    if (t.d_label_keys) (void)hipFree(t.d_label_keys);
    for (uint32_t *q : {t.d_irp, t.d_icol, t.d_elab, t.d_ielab})
        if (q) (void)hipFree(q);
    if (t.d_wcol) (void)hipFree(t.d_wcol);
    if (t.d_nbr_deg) (void)hipFree(t.d_nbr_deg);
    t.d_nbr_deg = nullptr;
    t.d_irp = t.d_icol = t.d_elab = t.d_ielab = nullptr;
    t.d_wcol = nullptr;
    t.d_col = nullptr;
    t.d_node = nullptr;
    t.d_adj = nullptr;
    t.d_label_keys = nullptr;
}

sge_status upload_pattern(sge_ctx *c, Pattern &p) {
    const HostGraph &g = p.g;
    DevPattern dp{};
    dp.k = g.n;
    // connected components: each begins one parentless position of the order
    std::vector<uint32_t> comp(g.n, 0xFFFFFFFFu), stack;
    for (uint32_t s = 0; s < g.n; s++) {
        if (comp[s] != 0xFFFFFFFFu) continue;
        comp[s] = dp.ncomp;
        stack.assign(1, s);
        while (!stack.empty()) {
            const uint32_t u = stack.back();
            stack.pop_back();
            // arcs in either direction join a component
            for (int dir = 0; dir < 2; dir++) {
                const std::vector<uint32_t> &rp = dir ? g.in_rp() : g.rp, &cl = dir ? g.in_col() : g.col;
                for (uint32_t e = rp[u]; e < rp[u + 1]; e++)
                    if (comp[cl[e]] == 0xFFFFFFFFu) {
                        comp[cl[e]] = dp.ncomp;
                        stack.push_back(cl[e]);
                    }
            }
        }
        dp.ncomp++;
    }
    for (uint32_t u = 0; u < g.n; u++) {
        for (uint32_t e = g.rp[u]; e < g.rp[u + 1]; e++) dp.nb[u] |= 1ull << g.col[e];
        dp.deg[u] = g.rp[u + 1] - g.rp[u];
        dp.label[u] = g.lab[u];
    }
    // the RI order depends on the pattern alone: the plan kernel copies it
    // (it is the one that kernel computes for an undirected pattern)
    constraint_first_order(dp.nb, dp.deg, nullptr, g.n, false, false, dp.ri_order);
    p.ncomp = dp.ncomp;
    hipError_t e;
    if ((e = hipMalloc(&p.d_pat, sizeof(DevPattern))) != hipSuccess) return hip_fail(c, e, "hipMalloc(pattern)");
    if ((e = hipMemcpy(p.d_pat, &dp, sizeof(DevPattern), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "upload pattern");
    return SGE_OK;
}

void free_pattern(Pattern &p) {
    if (p.d_pat) (void)hipFree(p.d_pat);
    p.d_pat = nullptr;
}

}  // namespace sge

// ------------------------------------------------------------------ C ABI
extern "C" {

sge_status sge_create(int device, void *hip_stream, sge_ctx **out) {
    if (!out) return SGE_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return SGE_E_DEVICE;
    if (device < 0 || device >= ndev) return SGE_E_INVAL;
    if ((e = hipSetDevice(device)) != hipSuccess) return SGE_E_DEVICE;
    auto *c = new sge_ctx();
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
        delete c;
        return SGE_E_DEVICE;
    }
    (void)hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device);
    int lds = 0;
    (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device);
    c->lds_per_cu = lds > 0 ? (size_t)lds : 65536;
    if (c->num_cus <= 0) c->num_cus = 1;
    (void)hipEventCreate(&c->ev0);
    (void)hipEventCreate(&c->ev1);
    // the allocation-free count's scratch array: its address on this device
    // (a failure leaves that entry point reporting the error)
    (void)noalloc_init(device);
    *out = c;
    return SGE_OK;
}

void sge_serve_shutdown_internal(sge_ctx *c);
bool sge_serve_holds(sge_ctx *c, const Target *t, const Pattern *p);

void sge_destroy(sge_ctx *c) {
    if (!c) return;
    sge_serve_shutdown_internal(c);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &kv : c->targets) free_target(*kv.second);
    for (auto &kv : c->patterns) free_pattern(*kv.second);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->gev0) (void)hipEventDestroy(c->gev0);
    if (c->gev1) (void)hipEventDestroy(c->gev1);
    c->bufs.release();
    c->d_rows.release();
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}

const char *sge_last_error(const sge_ctx *c) { return c ? c->err.c_str() : "no context"; }

sge_status sge_last_launch_timing(const sge_ctx *c, double *ms) {
    if (!c || !ms) return SGE_E_INVAL;
    for (int i = 0; i < 3; i++) ms[i] = c->last_ms[i];
    return SGE_OK;
}

sge_status sge_last_kernel_ms(const sge_ctx *c, double *ms) {
    if (!c || !ms) return SGE_E_INVAL;
    *ms = c->last_event_ms;
    return SGE_OK;
}

sge_status sge_set_checks(sge_ctx *c, int on) {
    if (!c) return SGE_E_INVAL;
    c->check_uniform = on ? 1 : 0;
    return SGE_OK;
}

sge_status sge_set_count_bytes(sge_ctx *c, int on) {
    if (!c) return SGE_E_INVAL;
    c->count_bytes = on ? 1 : 0;
    return SGE_OK;
}

sge_status sge_last_launch_occupancy(const sge_ctx *c, double *busy_unit_ms, uint32_t *units) {
    if (!c || !busy_unit_ms || !units) return SGE_E_INVAL;
    *busy_unit_ms = c->last_busy_ms;
    *units = c->last_units;
    return SGE_OK;
}

sge_status sge_load_target(sge_ctx *c, uint32_t n, const uint32_t *row_ptr, const uint32_t *col,
                           const uint32_t *labels, uint32_t *handle) {
    return sge_load_target_ex(c, n, row_ptr, col, labels, nullptr, 0, handle);
}

sge_status sge_load_target_ex(sge_ctx *c, uint32_t n, const uint32_t *row_ptr, const uint32_t *col,
                              const uint32_t *labels, const uint32_t *edge_labels, int directed, uint32_t *handle) {
    if (!c || !handle) return SGE_E_INVAL;
    auto t = std::make_unique<Target>();
    std::string why = normalise_graph(n, row_ptr, col, labels, edge_labels, directed != 0, t->g);
    if (!why.empty()) return fail(c, SGE_E_INVAL, "target: " + why);
    index_target(*t);
    (void)hipSetDevice(c->device);
    sge_status st = upload_target(c, *t);
    if (st != SGE_OK) {
        free_target(*t);
        return st;
    }
    uint32_t h = c->next_handle++;
    c->targets[h] = std::move(t);
    *handle = h;
    return SGE_OK;
}

sge_status sge_unload_target(sge_ctx *c, uint32_t handle) {
    if (!c) return SGE_E_INVAL;
    auto it = c->targets.find(handle);
    if (it == c->targets.end()) return fail(c, SGE_E_HANDLE, "unknown target handle");
    if (sge_serve_holds(c, it->second.get(), nullptr))
        return fail(c, SGE_E_BUSY, "the target is in use by server queries in flight");
    (void)hipStreamSynchronize(c->stream);
    free_target(*it->second);
    c->targets.erase(it);
    return SGE_OK;
}

sge_status sge_load_pattern(sge_ctx *c, uint32_t k, const uint32_t *row_ptr, const uint32_t *col,
                            const uint32_t *labels, uint32_t *handle) {
    return sge_load_pattern_ex(c, k, row_ptr, col, labels, nullptr, 0, handle);
}

sge_status sge_load_pattern_ex(sge_ctx *c, uint32_t k, const uint32_t *row_ptr, const uint32_t *col,
                               const uint32_t *labels, const uint32_t *edge_labels, int directed,
                               uint32_t *handle) {
    if (!c || !handle) return SGE_E_INVAL;
    if (k > KMAX) return fail(c, SGE_E_INVAL, "pattern has more than 64 nodes");
    auto p = std::make_unique<Pattern>();
    std::string why = normalise_graph(k, row_ptr, col, labels, edge_labels, directed != 0, p->g);
    if (!why.empty()) return fail(c, SGE_E_INVAL, "pattern: " + why);
    (void)hipSetDevice(c->device);
    sge_status st = upload_pattern(c, *p);
    if (st != SGE_OK) {
        free_pattern(*p);
        return st;
    }
    uint32_t h = c->next_handle++;
    c->patterns[h] = std::move(p);
    *handle = h;
    return SGE_OK;
}

sge_status sge_unload_pattern(sge_ctx *c, uint32_t handle) {
    if (!c) return SGE_E_INVAL;
    auto it = c->patterns.find(handle);
    if (it == c->patterns.end()) return fail(c, SGE_E_HANDLE, "unknown pattern handle");
    if (sge_serve_holds(c, nullptr, it->second.get()))
        return fail(c, SGE_E_BUSY, "the pattern is in use by server queries in flight");
    (void)hipStreamSynchronize(c->stream);
    free_pattern(*it->second);
    c->patterns.erase(it);
    return SGE_OK;
}

sge_status sge_set_labelled(sge_ctx *c, int labelled) {
    if (!c) return SGE_E_INVAL;
    c->labelled = labelled ? 1 : 0;
    return SGE_OK;
}

sge_status sge_set_mode(sge_ctx *c, int mode) {
    if (!c) return SGE_E_INVAL;
    if (mode < SGE_RI || mode > SGE_RIDS_SI_FC) return fail(c, SGE_E_INVAL, "unknown mode");
    c->mode = mode;
    return SGE_OK;
}

sge_status sge_set_state_cap(sge_ctx *c, uint64_t cap) {
    if (!c) return SGE_E_INVAL;
    c->cap = cap;
    return SGE_OK;
}

sge_status sge_set_time_limit(sge_ctx *c, uint64_t ms) {
    if (!c) return SGE_E_INVAL;
    c->time_limit_ms = ms;
    return SGE_OK;
}

sge_status sge_set_root_range(sge_ctx *c, uint32_t lo, uint32_t hi) {
    if (!c) return SGE_E_INVAL;
    if (lo > hi) return fail(c, SGE_E_INVAL, "root range lo > hi");
    c->root_lo = lo;
    c->root_hi = hi;
    return SGE_OK;
}

sge_status sge_set_plan_location(sge_ctx *c, int where) {
    if (!c) return SGE_E_INVAL;
    if (where < -1 || where > 1) return fail(c, SGE_E_INVAL, "plan location must be -1, 0 or 1");
    c->plan_where = where;
    return SGE_OK;
}

sge_status sge_set_tuning(sge_ctx *c, int lanes, uint32_t root_chunk, int donate, int dense) {
    if (!c) return SGE_E_INVAL;
    if (lanes != 0 && lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64)
        return fail(c, SGE_E_INVAL, "lanes per unit must be 0, 8, 16, 32 or 64");
    if (dense < -1 || dense > 1) return fail(c, SGE_E_INVAL, "dense must be -1, 0 or 1");
    c->lanes = lanes;
    c->root_chunk = root_chunk;
    c->donate = donate < 0 ? 0 : donate;
    c->dense = dense;
    c->batch_tune.clear();
    return SGE_OK;
}

sge_status sge_set_blocks_per_cu(sge_ctx *c, int blocks_per_cu) {
    if (!c) return SGE_E_INVAL;
    if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(c, SGE_E_INVAL, "blocks per CU must be 0..64");
    c->per_cu = blocks_per_cu;
    c->batch_tune.clear();
    return SGE_OK;
}

static sge_status single(sge_ctx *c, uint32_t target, uint32_t pattern, uint32_t *rows, uint64_t cap_rows,
                         sge_result *res) {
    if (!c || !res) return SGE_E_INVAL;
    auto it = c->targets.find(target);
    if (it == c->targets.end()) return fail(c, SGE_E_HANDLE, "unknown target handle");
    auto ip = c->patterns.find(pattern);
    if (ip == c->patterns.end()) return fail(c, SGE_E_HANDLE, "unknown pattern handle");
    (void)hipSetDevice(c->device);
    InstanceSpec s;
    s.t = it->second.get();
    s.p = ip->second.get();
    s.mode = c->mode;
    s.labelled = c->labelled != 0;
    const uint32_t k = s.p->g.n;
    uint32_t *host_rows = nullptr;
    if (rows && cap_rows && k) {
        hipPointerAttribute_t attr;
        bool on_device = hipPointerGetAttributes(&attr, rows) == hipSuccess && attr.type == hipMemoryTypeDevice;
        (void)hipGetLastError();
        if (on_device) {
            s.rows = rows;
        } else {
            hipError_t e = c->d_rows.reserve(cap_rows * k * 4);
            if (e != hipSuccess) return hip_fail(c, e, "device row buffer");
            s.rows = (uint32_t *)c->d_rows.p;
            host_rows = rows;
        }
        s.cap_rows = cap_rows;
    }
    std::vector<InstanceOut> out;
    double mp = 0, ms = 0;
    sge_status st = run_instances(c, {s}, out, mp, ms, false, 2);
    if (st != SGE_OK) return st;
    res->matches = out[0].matches;
    res->states = out[0].states;
    res->candidates = out[0].candidates;
    res->alg_bytes = out[0].bytes;
    res->steals = out[0].steals;
    res->steps = out[0].steps;
    res->ms_prep = mp;
    res->ms_search = ms;
    if (k == 0 && rows) { /* one empty row: nothing to write */ }
    if (host_rows && res->matches) {
        uint64_t nr = std::min<uint64_t>(res->matches, cap_rows);
        hipError_t e = hipMemcpy(host_rows, s.rows, nr * k * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(c, e, "copy rows");
    }
    if (out[0].timed_out) return fail(c, SGE_E_ABORTED, "search stopped at the time limit; counters are partial");
    if (out[0].status == SGE_E_ABORTED) return fail(c, SGE_E_ABORTED, "state cap exceeded");
    if (rows && k && res->matches > cap_rows) return fail(c, SGE_E_OVERFLOW, "more matches than rows");
    return SGE_OK;
}

sge_status sge_count(sge_ctx *c, uint32_t target, uint32_t pattern, sge_result *res) {
    return single(c, target, pattern, nullptr, 0, res);
}

sge_status sge_enumerate(sge_ctx *c, uint32_t target, uint32_t pattern, uint32_t *rows, uint64_t cap_rows,
                         sge_result *res) {
    if (!rows && cap_rows) return fail(c, SGE_E_INVAL, "rows is NULL");
    return single(c, target, pattern, rows, cap_rows, res);
}

sge_status sge_plan_device(sge_ctx *c, uint32_t target, uint32_t pattern, int mode, int labelled, uint32_t *order,
                           int32_t *parent, uint64_t *dom, uint32_t *nroot, int *empty) {
    if (!c || !order || !parent || !nroot || !empty) return SGE_E_INVAL;
    if (mode < SGE_RI || mode > SGE_RIDS_SI_FC) return fail(c, SGE_E_INVAL, "unknown mode");
    auto it = c->targets.find(target);
    if (it == c->targets.end()) return fail(c, SGE_E_HANDLE, "unknown target handle");
    auto ip = c->patterns.find(pattern);
    if (ip == c->patterns.end()) return fail(c, SGE_E_HANDLE, "unknown pattern handle");
    const uint32_t k = ip->second->g.n;
    *empty = 0;
    *nroot = 0;
    if (k == 0) return SGE_OK;
    (void)hipSetDevice(c->device);
    InstanceSpec s;
    s.t = it->second.get();
    s.p = ip->second.get();
    s.mode = mode;
    s.labelled = labelled != 0;
    if (general_instance(s)) return fail(c, SGE_E_INVAL, "the plan kernel covers undirected graphs without edge labels");
    std::vector<const InstanceSpec *> sp{&s};
    Pack pk;
    sge_status st = pack_instances(c, sp, false, 2, c->bufs, pk);
    if (st != SGE_OK) return st;
    hipError_t e = enqueue_plan_only(pk, c->bufs, c->root_chunk, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "device plan");
    DevPlan dp;
    if ((e = hipMemcpy(&dp, c->bufs.d_arena.p, sizeof(DevPlan), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(c, e, "read device plan");
    *empty = dp.empty ? 1 : 0;
    if (dp.empty) return SGE_OK;
    std::memcpy(order, dp.order, k * 4);
    std::memcpy(parent, dp.parent, k * 4);
    *nroot = dp.list_len[0];
    if (dom && mode != SGE_RI) {
        const size_t words = (size_t)k * s.t->W;
        if ((e = hipMemcpy(dom, (char *)c->bufs.d_arena.p + pk.dom_at[0], words * 8, hipMemcpyDeviceToHost)) !=
            hipSuccess)
            return hip_fail(c, e, "read device domains");
    }
    return SGE_OK;
}

sge_status sge_plan_host(uint32_t k, const uint32_t *p_rp, const uint32_t *p_col, const uint32_t *p_lab, uint32_t n,
                         const uint32_t *t_rp, const uint32_t *t_col, const uint32_t *t_lab, int mode, int labelled,
                         uint32_t *order, int32_t *parent, uint64_t *dom, int *empty) {
    return sge_plan_host_ex(k, p_rp, p_col, p_lab, nullptr, 0, n, t_rp, t_col, t_lab, nullptr, 0, mode, labelled, order,
                            parent, dom, empty);
}

sge_status sge_plan_host_ex(uint32_t k, const uint32_t *p_rp, const uint32_t *p_col, const uint32_t *p_lab,
                            const uint32_t *p_elab, int p_dir, uint32_t n, const uint32_t *t_rp, const uint32_t *t_col,
                            const uint32_t *t_lab, const uint32_t *t_elab, int t_dir, int mode, int labelled,
                            uint32_t *order, int32_t *parent, uint64_t *dom, int *empty) {
    if (k > KMAX || !order || !parent || !empty) return SGE_E_INVAL;
    if (mode < SGE_RI || mode > SGE_RIDS_SI_FC) return SGE_E_INVAL;
    Target t;
    if (!normalise_graph(n, t_rp, t_col, t_lab, t_elab, t_dir != 0, t.g).empty()) return SGE_E_INVAL;
    HostGraph p;
    if (!normalise_graph(k, p_rp, p_col, p_lab, p_elab, p_dir != 0, p).empty()) return SGE_E_INVAL;
    index_target(t);
    Plan pl;
    std::vector<uint64_t> bits;
    build_plan(t, p, mode, labelled != 0, 0, 0xFFFFFFFFu, pl, false, bits);
    *empty = pl.empty ? 1 : 0;
    if (dom && mode != SGE_RI) std::memcpy(dom, pl.dom_node.data(), pl.dom_node.size() * 8);
    if (!pl.empty) {
        std::memcpy(order, pl.order, k * 4);
        std::memcpy(parent, pl.parent, k * 4);
    }
    return SGE_OK;
}

}  // extern "C"
