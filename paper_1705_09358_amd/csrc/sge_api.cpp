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
    for (uint32_t v = 0; v < g.n; v++) rec[v] = NodeRec{g.rp[v], g.rp[v + 1] - g.rp[v], t.dlab[v], 0};
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
    if (g.n && g.n <= ADJ_BITSET_MAX_N) {
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
    return SGE_OK;
}

void free_target(Target &t) {
    if (t.d_col) (void)hipFree(t.d_col);
    if (t.d_node) (void)hipFree(t.d_node);
    if (t.d_adj) (void)hipFree(t.d_adj);
    t.d_col = nullptr;
    t.d_node = nullptr;
    t.d_adj = nullptr;
}

static int auto_lanes(const std::vector<const Target *> &ts) {
    double deg = 0;
    uint64_t cnt = 0;
    for (const Target *t : ts) {
        deg += (double)t->g.col.size();
        cnt += t->g.n;
    }
    double avg = cnt ? deg / (double)cnt : 0;
    if (avg <= 12) return 16;
    if (avg <= 24) return 32;
    return 64;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

sge_status run_instances(sge_ctx *c, const std::vector<InstanceSpec> &specs, std::vector<InstanceOut> &out,
                         double &ms_prep, double &ms_search, bool graph, int policy) {
    auto t0 = clk::now();
    const size_t N = specs.size();
    out.assign(N, InstanceOut{});
    std::vector<Plan> plans(N);
    std::vector<std::vector<uint64_t>> bits(N);
    std::vector<char> active(N, 0);

    auto plan_one = [&](size_t i) {
        const InstanceSpec &s = specs[i];
        if (s.p->g.n == 0) {          // the empty pattern has one (empty) match
            out[i].matches = 1;
            return;
        }
        bool want_bits = s.mode != SGE_RI;
        uint32_t lo = c->root_lo, hi = c->root_hi;
        build_plan(*s.t, s.p->g, s.mode, s.labelled, lo, hi, plans[i], want_bits, bits[i]);
        active[i] = !plans[i].empty;
    };
    if (N >= 64) {
        unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (unsigned w = 0; w < nt; w++)
            th.emplace_back([&, w]() {
                for (size_t i = w; i < N; i += nt) plan_one(i);
            });
        for (auto &x : th) x.join();
    } else {
        for (size_t i = 0; i < N; i++) plan_one(i);
    }

    std::vector<size_t> idx;
    for (size_t i = 0; i < N; i++)
        if (active[i]) idx.push_back(i);
    const uint32_t m = (uint32_t)idx.size();
    if (m == 0) {
        ms_prep = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
        ms_search = 0;
        return SGE_OK;
    }

    // launch shape
    LaunchCfg cfg;
    std::vector<const Target *> ts;
    for (size_t i : idx) {
        cfg.kmax = std::max(cfg.kmax, plans[i].k);
        cfg.nmax = std::max(cfg.nmax, plans[i].n);
        ts.push_back(specs[i].t);
    }
    cfg.lanes = c->lanes ? c->lanes : auto_lanes(ts);
    cfg.donate = c->donate;
    // approximate number of search units (for the root chunk size)
    uint64_t units = (uint64_t)c->num_cus * 4 * 8 * (64 / cfg.lanes) / 2;

    // blob layout: plans | descs | chunk prefix | lists | bits
    size_t off_plan = 0;
    size_t off_desc = align_up(off_plan + m * sizeof(DevPlan), 256);
    size_t off_pref = align_up(off_desc + m * sizeof(InstDesc), 256);
    size_t off_list = align_up(off_pref + (m + 1) * sizeof(unsigned), 256);
    std::vector<size_t> list_at(m), bits_at(m);
    size_t cur = off_list;
    for (uint32_t j = 0; j < m; j++) {
        list_at[j] = cur;
        cur = align_up(cur + plans[idx[j]].lists.size() * 4, 16);
    }
    cur = align_up(cur, 256);
    for (uint32_t j = 0; j < m; j++) {
        bits_at[j] = cur;
        cur = align_up(cur + bits[idx[j]].size() * 8, 16);
    }
    const size_t blob = std::max<size_t>(cur, 256);
    hipError_t e;
    if ((e = c->d_blob.reserve(blob)) != hipSuccess) return hip_fail(c, e, "device plan buffer");
    if ((e = c->h_blob.reserve(blob)) != hipSuccess) return hip_fail(c, e, "pinned plan buffer");
    const size_t ctr_bytes = align_up(m * sizeof(InstCounters), 64);
    if ((e = c->h_ctr.reserve(ctr_bytes + sizeof(Sched))) != hipSuccess) return hip_fail(c, e, "pinned counters");
    char *hb = (char *)c->h_blob.p;
    char *db = (char *)c->d_blob.p;

    uint64_t total_roots = 0;
    for (size_t i : idx) total_roots += plans[i].list_len[0];
    unsigned *pref = (unsigned *)(hb + off_pref);
    pref[0] = 0;
    for (uint32_t j = 0; j < m; j++) {
        const Plan &pl = plans[idx[j]];
        const InstanceSpec &s = specs[idx[j]];
        DevPlan &dp = ((DevPlan *)(hb + off_plan))[j];
        std::memset(&dp, 0, sizeof(dp));
        dp.k = pl.k;
        dp.W = pl.W;
        dp.n = pl.n;
        dp.use_dom = pl.mode != SGE_RI;
        dp.labelled = pl.labelled;
        for (uint32_t i = 0; i < pl.k; i++) {
            dp.parent[i] = pl.parent[i];
            dp.back[i] = pl.back[i];
            dp.plabel[i] = pl.plabel[i];
            dp.pdeg[i] = pl.pdeg[i];
            dp.order[i] = pl.order[i];
            dp.list_off[i] = pl.list_off[i];
            dp.list_len[i] = pl.list_len[i];
        }
        std::memcpy(hb + list_at[j], pl.lists.data(), pl.lists.size() * 4);
        std::memcpy(hb + bits_at[j], bits[idx[j]].data(), bits[idx[j]].size() * 8);
        InstDesc &d = ((InstDesc *)(hb + off_desc))[j];
        d.col = s.t->d_col;
        d.node = s.t->d_node;
        d.adj = s.t->d_adj;
        d.plan = (const DevPlan *)(db + off_plan) + j;
        d.bits = bits[idx[j]].empty() ? nullptr : (const uint64_t *)(db + bits_at[j]);
        d.lists = (const uint32_t *)(db + list_at[j]);
        d.rows = s.rows;
        d.cap_rows = s.rows ? s.cap_rows : 0;
        d.nroot = pl.list_len[0];
        uint32_t chunk;
        if (policy == 1) chunk = std::max<uint32_t>(1, d.nroot);
        else if (c->root_chunk) chunk = c->root_chunk;
        else chunk = (uint32_t)std::max<uint64_t>(1, total_roots / (4 * units));
        d.chunk = chunk;
        d.nchunks = d.nroot ? (d.nroot + chunk - 1) / chunk : 0;
        pref[j + 1] = pref[j] + d.nchunks;
    }
    // device work state
    DevWork &w = c->work;
    w.inst = (InstDesc *)(db + off_desc);
    w.chunk_prefix = (unsigned *)(db + off_pref);
    if (!w.sched) {
        if ((e = hipMalloc(&w.sched, sizeof(Sched))) != hipSuccess) return hip_fail(c, e, "hipMalloc(sched)");
        if ((e = hipMalloc(&w.queue, sizeof(QTask) * QUEUE_SLOTS)) != hipSuccess)
            return hip_fail(c, e, "hipMalloc(queue)");
    }
    if (w.ctr_cap < m) {
        if (w.ctr) (void)hipFree(w.ctr);
        w.ctr = nullptr;
        size_t cap = std::max<size_t>(m, 1024);
        if ((e = hipMalloc(&w.ctr, cap * sizeof(InstCounters))) != hipSuccess) return hip_fail(c, e, "hipMalloc(ctr)");
        w.ctr_cap = cap;
    }

    hipStream_t s = c->stream;
    // the search kernel is bracketed by ev0/ev1, so ms_search is kernel-only time
    auto enqueue = [&](bool timed) -> hipError_t {
        hipError_t r;
        if ((r = hipMemcpyAsync(db, hb, blob, hipMemcpyHostToDevice, s)) != hipSuccess) return r;
        if ((r = launch_reset(w, m, s)) != hipSuccess) return r;
        if (timed && (r = hipEventRecord(c->ev0, s)) != hipSuccess) return r;
        if ((r = launch_search(cfg, w, m, pref[m], c->cap, c->time_limit_ms, s, c->num_cus)) != hipSuccess) return r;
        if (timed && (r = hipEventRecord(c->ev1, s)) != hipSuccess) return r;
        if ((r = hipMemcpyAsync(c->h_ctr.p, w.ctr, m * sizeof(InstCounters), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return r;
        return hipMemcpyAsync((char *)c->h_ctr.p + ctr_bytes, w.sched, sizeof(Sched), hipMemcpyDeviceToHost, s);
    };
    auto t1 = clk::now();
    ms_prep = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (graph) {
        // one graph: plan upload, scheduler reset, the persistent search, read-back
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(c, e, "hipStreamBeginCapture");
        hipError_t er = enqueue(false);
        e = hipStreamEndCapture(s, &g);
        if (er != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(c, er != hipSuccess ? er : e, "capture search graph");
        }
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
        // the executable graph owns the launch's kernel arguments: it is destroyed
        // only after the stream has drained
        if ((e = hipEventRecord(c->ev0, s)) == hipSuccess && (e = hipGraphLaunch(ge, s)) == hipSuccess)
            e = hipEventRecord(c->ev1, s);
        hipError_t es = hipStreamSynchronize(s);
        (void)hipGraphExecDestroy(ge);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
        if (es != hipSuccess) return hip_fail(c, es, "search");
    } else {
        if ((e = enqueue(true)) != hipSuccess) return hip_fail(c, e, "search launch");
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "search");
    float ms = 0;
    (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);

    const InstCounters *hc = (const InstCounters *)c->h_ctr.p;
    const Sched *hs = (const Sched *)((char *)c->h_ctr.p + ctr_bytes);
    if (hs->abort) c->err = "search stopped at the time limit; counters are partial";
    // kernel time from the device clock (100 MHz): first block start to last wave exit
    ms_search = hs->t_end > hs->t_start ? (double)(hs->t_end - hs->t_start) / 1e5 : (double)ms;
    for (uint32_t j = 0; j < m; j++) {
        InstanceOut &o = out[idx[j]];
        o.matches = hc[j].matches;
        o.states = hc[j].states;
        o.candidates = hc[j].candidates;
        o.steals = hc[j].steals;
        if (hs->abort) {
            o.status = SGE_E_ABORTED;
            o.timed_out = true;
        } else if (c->cap && o.states > c->cap) {
            o.status = SGE_E_ABORTED;
        }
        else if (specs[idx[j]].rows && o.matches > specs[idx[j]].cap_rows) o.status = SGE_E_OVERFLOW;
    }
    return SGE_OK;
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
    *out = c;
    return SGE_OK;
}

void sge_serve_shutdown_internal(sge_ctx *c);

void sge_destroy(sge_ctx *c) {
    if (!c) return;
    sge_serve_shutdown_internal(c);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &kv : c->targets) free_target(*kv.second);
    c->d_blob.release();
    c->d_rows.release();
    c->h_blob.release();
    c->h_ctr.release();
    if (c->work.sched) (void)hipFree(c->work.sched);
    if (c->work.queue) (void)hipFree(c->work.queue);
    if (c->work.ctr) (void)hipFree(c->work.ctr);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}

const char *sge_last_error(const sge_ctx *c) { return c ? c->err.c_str() : "no context"; }

sge_status sge_load_target(sge_ctx *c, uint32_t n, const uint32_t *row_ptr, const uint32_t *col,
                           const uint32_t *labels, uint32_t *handle) {
    if (!c || !handle) return SGE_E_INVAL;
    auto t = std::make_unique<Target>();
    std::string why = normalise_graph(n, row_ptr, col, labels, t->g);
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
    (void)hipStreamSynchronize(c->stream);
    free_target(*it->second);
    c->targets.erase(it);
    return SGE_OK;
}

sge_status sge_load_pattern(sge_ctx *c, uint32_t k, const uint32_t *row_ptr, const uint32_t *col,
                            const uint32_t *labels, uint32_t *handle) {
    if (!c || !handle) return SGE_E_INVAL;
    if (k > KMAX) return fail(c, SGE_E_INVAL, "pattern has more than 64 nodes");
    auto p = std::make_unique<Pattern>();
    std::string why = normalise_graph(k, row_ptr, col, labels, p->g);
    if (!why.empty()) return fail(c, SGE_E_INVAL, "pattern: " + why);
    uint32_t h = c->next_handle++;
    c->patterns[h] = std::move(p);
    *handle = h;
    return SGE_OK;
}

sge_status sge_unload_pattern(sge_ctx *c, uint32_t handle) {
    if (!c) return SGE_E_INVAL;
    if (!c->patterns.erase(handle)) return fail(c, SGE_E_HANDLE, "unknown pattern handle");
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

sge_status sge_set_tuning(sge_ctx *c, int lanes, uint32_t root_chunk, int donate, int dense) {
    if (!c) return SGE_E_INVAL;
    if (lanes != 0 && lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64)
        return fail(c, SGE_E_INVAL, "lanes per unit must be 0, 8, 16, 32 or 64");
    if (dense < -1 || dense > 1) return fail(c, SGE_E_INVAL, "dense must be -1, 0 or 1");
    c->lanes = lanes;
    c->root_chunk = root_chunk;
    c->donate = donate ? 1 : 0;
    c->dense = dense;
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
    res->steals = out[0].steals;
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

sge_status sge_plan_host(uint32_t k, const uint32_t *p_rp, const uint32_t *p_col, const uint32_t *p_lab, uint32_t n,
                         const uint32_t *t_rp, const uint32_t *t_col, const uint32_t *t_lab, int mode, int labelled,
                         uint32_t *order, int32_t *parent, uint64_t *dom, int *empty) {
    if (k > KMAX || !order || !parent || !empty) return SGE_E_INVAL;
    if (mode < SGE_RI || mode > SGE_RIDS_SI_FC) return SGE_E_INVAL;
    Target t;
    if (!normalise_graph(n, t_rp, t_col, t_lab, t.g).empty()) return SGE_E_INVAL;
    HostGraph p;
    if (!normalise_graph(k, p_rp, p_col, p_lab, p).empty()) return SGE_E_INVAL;
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
