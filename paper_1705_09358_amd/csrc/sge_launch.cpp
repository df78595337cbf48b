// One persistent search launch over a set of instances: the host lays out a
// descriptor and a plan request per instance (pattern and target are
// resident on the device), uploads them, and the device plans every instance,
// sets the root chunking, resets the scheduler and searches; the counters are
// read back.  Used by the single-instance calls, by batches (in a HIP graph)
// and by the server (asynchronously, one stream per launch lane).
#include <algorithm>
#include <cstring>
#include <thread>

#include "sge_ctx.h"

using clk = std::chrono::steady_clock;

namespace sge {

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

void LaunchBufs::release() {
    d_blob.release();
    d_arena.release();
    h_blob.release();
    h_ctr.release();
    if (work.sched) (void)hipFree(work.sched);
    if (work.queue) (void)hipFree(work.queue);
    if (work.ctr) (void)hipFree(work.ctr);
    work = DevWork{};
}

bool general_instance(const InstanceSpec &s) {
    return s.t->g.directed || s.p->g.directed || (s.labelled && (s.t->g.has_elab() || s.p->g.has_elab()));
}

bool choose_dense(const sge_ctx *c, const std::vector<InstanceSpec> &specs) {
    return choose_dense(c, specs.data(), specs.size());
}

bool choose_dense(const sge_ctx *c, const InstanceSpec *specs, size_t m) {
    // dense-bitset search when every target has adjacency rows and is dense
    // enough that a row of W words costs no more than walking a neighbour list;
    // directed or edge-labelled searches take the CSR kernel
    if (c->dense == 0 || m == 0) return false;
    bool all_adj = true;
    double deg = 0, words = 0;
    LaunchCfg probe;   // every search unit holds k rows of W words in LDS: the launch must fit
    probe.dense = 1;
    for (size_t j = 0; j < m; j++) {
        const InstanceSpec &s = specs[j];
        if (general_instance(s)) return false;
        all_adj &= s.t->d_adj != nullptr;
        deg += s.t->g.n ? (double)s.t->g.col.size() / s.t->g.n : 0.0;
        words += s.t->W;
        probe.kmax = std::max(probe.kmax, s.p->g.n);
        probe.nmax = std::max(probe.nmax, s.t->g.n);
        probe.wmax = std::max(probe.wmax, s.t->W);
    }
    if (!all_adj) return false;
    probe.lanes = c->lanes ? c->lanes : 8;
    if (!c->lanes)
        while (probe.lanes < 64 && (uint32_t)probe.lanes < probe.wmax) probe.lanes *= 2;
    if (search_block_threads(probe) == 0) return false;
    return c->dense == 1 || deg >= 2.0 * words;
}

// Candidate-list entries of one instance: a parentless position either
// starts a pattern component (at most n candidates) or, in the RI-DS modes,
// holds a singleton domain placed first (one candidate).
// Indices 0..n-1 by decreasing key, equal keys in increasing index (what a
// stable sort by `key > key` gives): a least-significant-digit radix sort of
// (largest key - key), 11 bits per pass over the bits in use.  For the 4096
// jobs of a batch it takes a fifth of the comparison sort's time.
void order_by_desc(const uint64_t *key, uint32_t n, uint32_t *perm) {
    uint64_t mx = 0;
    for (uint32_t i = 0; i < n; i++) mx = std::max(mx, key[i]);
    std::vector<uint64_t> k(n), k2(n);
    std::vector<uint32_t> p2(n);
    for (uint32_t i = 0; i < n; i++) {
        k[i] = mx - key[i];
        perm[i] = i;
    }
    int bits = 0;
    while (bits < 64 && (mx >> bits)) bits++;
    uint32_t *pa = perm, *pb = p2.data();
    uint64_t *ka = k.data(), *kb = k2.data();
    for (int sh = 0; sh < bits; sh += 11) {
        uint32_t cnt[2049] = {0};
        for (uint32_t i = 0; i < n; i++) cnt[((ka[i] >> sh) & 2047u) + 1]++;
        for (int d = 0; d < 2048; d++) cnt[d + 1] += cnt[d];
        for (uint32_t i = 0; i < n; i++) {
            const uint32_t at = cnt[(ka[i] >> sh) & 2047u]++;
            kb[at] = ka[i];
            pb[at] = pa[i];
        }
        std::swap(ka, kb);
        std::swap(pa, pb);
    }
    if (pa != perm) std::copy(pa, pa + n, perm);
}

uint64_t list_entries(const InstanceSpec &s) {
    return (uint64_t)std::max<uint32_t>(s.p->ncomp, 1) * s.t->g.n + s.p->g.n;
}

bool plan_on_device(const sge_ctx *c, const std::vector<const InstanceSpec *> &specs) {
    for (const InstanceSpec *s : specs)
        if (general_instance(*s)) return false;   // the plan kernel covers undirected graphs without edge labels
    if (c->plan_where >= 0) return c->plan_where == 1;
    return specs.size() >= PLAN_DEVICE_MIN_INSTANCES;
}

uint64_t instance_device_bytes(const InstanceSpec &s) {
    const uint64_t k = s.p->g.n, W = s.t->W;
    return sizeof(DevPlan) + sizeof(InstDesc) + sizeof(PlanIn) + sizeof(InstCounters) + 2 * k * W * 8 +
           list_entries(s) * 4 + (W > PLAN_LDS_WORDS ? W * 8 : 0);
}

static int auto_lanes(const InstanceSpec *const *specs, size_t m) {
    double deg = 0;
    uint64_t cnt = 0;
    for (size_t j = 0; j < m; j++) {
        const InstanceSpec *s = specs[j];
        deg += (double)s->t->g.col.size();
        cnt += s->t->g.n;
    }
    // a step evaluates one candidate per lane: wide units pay off once
    // neighbour lists are longer than a few entries
    double avg = cnt ? deg / (double)cnt : 0;
    if (avg <= 6) return 32;
    return 64;
}

static hipError_t ensure_work(DevWork &w, uint32_t m) {
    hipError_t e;
    if (!w.sched) {
        if ((e = hipMalloc(&w.sched, sizeof(Sched))) != hipSuccess) return e;
        if ((e = hipMalloc(&w.queue, sizeof(QTask) * QUEUE_SLOTS)) != hipSuccess) return e;
    }
    if (w.ctr_cap < m) {
        if (w.ctr) (void)hipFree(w.ctr);
        w.ctr = nullptr;
        size_t cap = std::max<size_t>(m, 1024);
        if ((e = hipMalloc(&w.ctr, cap * sizeof(InstCounters))) != hipSuccess) return e;
        w.ctr_cap = cap;
    }
    return hipSuccess;
}

// Launch shape shared by both packings: sizes, kernel variant, unit width.
void launch_config(const sge_ctx *c, const InstanceSpec *const *specs, size_t m, bool dense, int policy, Pack &pk) {
    pk = Pack{};
    pk.m = (uint32_t)m;
    pk.policy = policy;
    LaunchCfg &cfg = pk.cfg;
    for (size_t j = 0; j < m; j++) {
        const InstanceSpec *sp = specs[j];
        cfg.kmax = std::max(cfg.kmax, sp->p->g.n);
        cfg.nmax = std::max(cfg.nmax, sp->t->g.n);
        cfg.wmax = std::max(cfg.wmax, sp->t->W);
        cfg.general |= general_instance(*sp) ? 1 : 0;
    }
    cfg.dense = dense ? 1 : 0;
    if (c->lanes) {
        cfg.lanes = c->lanes;
    } else if (dense) {
        cfg.lanes = 8;
        while (cfg.lanes < 64 && (uint32_t)cfg.lanes < cfg.wmax) cfg.lanes *= 2;
    } else {
        cfg.lanes = auto_lanes(specs, m);
    }
    cfg.donate = c->donate;
    cfg.per_cu = c->per_cu;
    // a used-node bitset per search unit (n bits of LDS) unless it would
    // shrink the block; larger targets compare candidates with the mapped
    // prefix instead (at most 63 entries), which fits any n
    cfg.used_bitset = 0;
    const int without = search_block_threads(cfg);
    cfg.used_bitset = 1;
    if (!dense && search_block_threads(cfg) < without) cfg.used_bitset = 0;
    cfg.count_bytes = c->count_bytes;
    cfg.check_uniform = c->check_uniform;
    cfg.root_lo = c->root_lo;
    cfg.root_hi = c->root_hi;
    // approximate number of search units (for the root chunk size): up to
    // four blocks of four waves per CU
    pk.units = (uint64_t)c->num_cus * (c->per_cu > 0 ? std::min(c->per_cu, 4) : 4) * 4 * (64 / cfg.lanes);
}

sge_status pack_instances(sge_ctx *c, const std::vector<const InstanceSpec *> &specs, bool dense, int policy,
                          LaunchBufs &bufs, Pack &pk) {
    const uint32_t m = (uint32_t)specs.size();
    launch_config(c, specs.data(), specs.size(), dense, policy, pk);
    pk.device_plan = true;
    // blob (uploaded): descriptors | plan requests | chunk prefix (device-written)
    const size_t off_desc = 0;
    pk.off_req = align_up(off_desc + m * sizeof(InstDesc), 256);
    pk.off_pref = align_up(pk.off_req + m * sizeof(PlanIn), 256);
    pk.upload = pk.off_pref;
    pk.blob = std::max<size_t>(align_up(pk.off_pref + (m + 1) * sizeof(unsigned), 256), 256);
    // arena (device-written): plans | per instance: domains, bitsets, lists, support scratch
    const size_t off_plans = 0;
    size_t cur = align_up(off_plans + m * sizeof(DevPlan), 256);
    pk.dom_at.resize(m);
    std::vector<size_t> pos_at(m), list_at(m), sup_at(m);
    for (uint32_t j = 0; j < m; j++) {
        const InstanceSpec &sp = *specs[j];
        const size_t kw = (size_t)sp.p->g.n * sp.t->W;
        pk.dom_at[j] = cur;
        cur = align_up(cur + kw * 8, 64);
        pos_at[j] = cur;
        if (dense || sp.mode != SGE_RI) cur = align_up(cur + kw * 8, 64);
        list_at[j] = cur;
        cur = align_up(cur + list_entries(sp) * 4, 64);
        sup_at[j] = cur;
        if (sp.t->W > PLAN_LDS_WORDS) cur = align_up(cur + (size_t)sp.t->W * 8, 64);
    }
    pk.arena = std::max<size_t>(cur, 256);
    pk.ctr_bytes = align_up(m * sizeof(InstCounters), 64);
    hipError_t e;
    if ((e = bufs.d_blob.reserve(pk.blob)) != hipSuccess) return hip_fail(c, e, "device descriptor buffer");
    if ((e = bufs.d_arena.reserve(pk.arena)) != hipSuccess) return hip_fail(c, e, "device plan arena");
    if ((e = bufs.h_blob.reserve(pk.blob)) != hipSuccess) return hip_fail(c, e, "pinned descriptor buffer");
    if ((e = bufs.h_ctr.reserve(pk.ctr_bytes + sizeof(Sched))) != hipSuccess) return hip_fail(c, e, "pinned counters");
    if ((e = ensure_work(bufs.work, m)) != hipSuccess) return hip_fail(c, e, "scheduler buffers");
    char *hb = (char *)bufs.h_blob.p;
    char *db = (char *)bufs.d_blob.p;
    char *da = (char *)bufs.d_arena.p;
    InstDesc *hdesc = (InstDesc *)(hb + off_desc);
    PlanIn *hreq = (PlanIn *)(hb + pk.off_req);
    // plan requests in decreasing order of estimated work (pattern size x
    // target size, arc-consistency counted four times), so the workgroups
    // of the largest plans start first and the kernel has no long tail;
    // each request carries its own output addresses, so the order is free
    std::vector<uint32_t> by_cost(m), slot(m);
    std::vector<uint64_t> cost(m);   // computed once: the sort then reads one array
    for (uint32_t j = 0; j < m; j++) {
        const InstanceSpec &sp = *specs[j];
        by_cost[j] = j;
        cost[j] = (uint64_t)sp.p->g.n * sp.t->g.n * (sp.mode != SGE_RI ? 4u : 1u);
    }
    order_by_desc(cost.data(), m, by_cost.data());
    for (uint32_t r = 0; r < m; r++) slot[by_cost[r]] = r;
    for (uint32_t j = 0; j < m; j++) {
        const InstanceSpec &sp = *specs[j];
        const bool with_bits = dense || sp.mode != SGE_RI;
        InstDesc &d = hdesc[j];
        d = InstDesc{};
        d.col = sp.t->d_col;
        d.node = sp.t->d_node;
        d.wcol = sp.t->d_wcol;
        d.adj = sp.t->d_adj;
        d.plan = (const DevPlan *)(da + off_plans) + j;
        d.bits = with_bits ? (const uint64_t *)(da + pos_at[j]) : nullptr;
        d.lists = (const uint32_t *)(da + list_at[j]);
        d.rows = sp.rows;
        d.cap_rows = sp.rows ? sp.cap_rows : 0;
        PlanIn &r = hreq[slot[j]];
        r = PlanIn{};
        r.pat = sp.p->d_pat;
        r.label_keys = sp.t->d_label_keys;
        r.nlabels = (uint32_t)sp.t->label_keys.size();
        r.nbr_deg = sp.t->d_nbr_deg;
        r.nbr_cols = sp.t->nbr_cols;
        r.nbr_stride = sp.t->nbr_stride;
        r.mode = (uint32_t)sp.mode;
        r.labelled = sp.labelled ? 1u : 0u;
        r.n = sp.t->g.n;
        r.W = sp.t->W;
        r.root_lo = c->root_lo;
        r.root_hi = c->root_hi;
        r.desc = (InstDesc *)(db + off_desc) + j;
        r.plan = (DevPlan *)(da + off_plans) + j;
        r.dom = (uint64_t *)(da + pk.dom_at[j]);
        r.pos_bits = with_bits ? (uint64_t *)(da + pos_at[j]) : nullptr;
        r.lists = (uint32_t *)(da + list_at[j]);
        r.list_cap = (uint32_t)std::min<uint64_t>(list_entries(sp), 0xFFFFFFFFull);
        r.support = sp.t->W > PLAN_LDS_WORDS ? (uint64_t *)(da + sup_at[j]) : nullptr;
        // an adjacency row (W words) is cheaper than a neighbour list once the
        // mean degree reaches W
        r.rows = sp.t->d_adj && sp.t->g.n && sp.t->g.col.size() >= (uint64_t)sp.t->g.n * sp.t->W ? 1u : 0u;
        r.deg_mean = sp.t->g.n ? (uint32_t)std::min<uint64_t>((sp.t->g.col.size() + sp.t->g.n - 1) / sp.t->g.n, 0xFFFFFFFFull) : 0u;
    }
    bufs.work.inst = (InstDesc *)(db + off_desc);
    bufs.work.chunk_prefix = (unsigned *)(db + pk.off_pref);
    return SGE_OK;
}

sge_status pack_host_planned(sge_ctx *c, const std::vector<const InstanceSpec *> &specs,
                             const std::vector<const Plan *> &plans,
                             const std::vector<const std::vector<uint64_t> *> &bits, bool dense, int policy,
                             LaunchBufs &bufs, Pack &pk) {
    const uint32_t m = (uint32_t)specs.size();
    launch_config(c, specs.data(), specs.size(), dense, policy, pk);
    pk.device_plan = false;
    // blob (uploaded whole): descriptors | chunk prefix | plans | lists | bits
    const size_t off_desc = 0;
    pk.off_pref = align_up(off_desc + m * sizeof(InstDesc), 256);
    const size_t off_plan = align_up(pk.off_pref + (m + 1) * sizeof(unsigned), 256);
    size_t cur = align_up(off_plan + m * sizeof(DevPlan), 256);
    std::vector<size_t> list_at(m), bits_at(m), lmat_at(m);
    for (uint32_t j = 0; j < m; j++) {
        list_at[j] = cur;
        cur = align_up(cur + plans[j]->lists.size() * 4, 16);
        lmat_at[j] = cur;
        cur = align_up(cur + plans[j]->lmat.size() * 4, 16);
    }
    cur = align_up(cur, 256);
    for (uint32_t j = 0; j < m; j++) {
        bits_at[j] = cur;
        cur = align_up(cur + bits[j]->size() * 8, 16);
    }
    pk.blob = pk.upload = std::max<size_t>(cur, 256);
    pk.ctr_bytes = align_up(m * sizeof(InstCounters), 64);
    hipError_t e;
    if ((e = bufs.d_blob.reserve(pk.blob)) != hipSuccess) return hip_fail(c, e, "device plan buffer");
    if ((e = bufs.h_blob.reserve(pk.blob)) != hipSuccess) return hip_fail(c, e, "pinned plan buffer");
    if ((e = bufs.h_ctr.reserve(pk.ctr_bytes + sizeof(Sched))) != hipSuccess) return hip_fail(c, e, "pinned counters");
    if ((e = ensure_work(bufs.work, m)) != hipSuccess) return hip_fail(c, e, "scheduler buffers");
    char *hb = (char *)bufs.h_blob.p;
    char *db = (char *)bufs.d_blob.p;
    uint64_t total_roots = 0;
    for (uint32_t j = 0; j < m; j++) total_roots += plans[j]->list_len[0];
    unsigned *pref = (unsigned *)(hb + pk.off_pref);
    pref[0] = 0;
    for (uint32_t j = 0; j < m; j++) {
        const Plan &pl = *plans[j];
        const InstanceSpec &sp = *specs[j];
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
            dp.pindeg[i] = pl.pindeg[i];
            dp.bout[i] = pl.bout[i];
            dp.bin[i] = pl.bin[i];
        }
        dp.flags = pl.flags;
        dp.pdir_out = pl.pdir_out;
        dp.pboth = pl.pboth;
        std::memcpy(hb + list_at[j], pl.lists.data(), pl.lists.size() * 4);
        std::memcpy(hb + lmat_at[j], pl.lmat.data(), pl.lmat.size() * 4);
        std::memcpy(hb + bits_at[j], bits[j]->data(), bits[j]->size() * 8);
        InstDesc &d = ((InstDesc *)(hb + off_desc))[j];
        d = InstDesc{};
        d.col = sp.t->d_col;
        d.node = sp.t->d_node;
        d.wcol = sp.t->d_wcol;
        d.adj = sp.t->d_adj;
        d.irp = sp.t->d_irp;
        d.icol = sp.t->d_icol;
        d.elab = sp.t->d_elab;
        d.ielab = sp.t->d_ielab;
        d.lmat = pl.lmat.empty() ? nullptr : (const uint32_t *)(db + lmat_at[j]);
        d.plan = (const DevPlan *)(db + off_plan) + j;
        d.bits = bits[j]->empty() ? nullptr : (const uint64_t *)(db + bits_at[j]);
        d.lists = (const uint32_t *)(db + list_at[j]);
        d.rows = sp.rows;
        d.cap_rows = sp.rows ? sp.cap_rows : 0;
        d.nroot = pl.list_len[0];
        uint32_t chunk;
        if (policy == 1) chunk = std::max<uint32_t>(1, d.nroot);
        else if (c->root_chunk) chunk = c->root_chunk;
        else chunk = (uint32_t)std::max<uint64_t>(1, total_roots / (4 * pk.units));
        d.chunk = chunk;
        d.nchunks = d.nroot ? (d.nroot + chunk - 1) / chunk : 0;
        pref[j + 1] = pref[j] + d.nchunks;
    }
    bufs.work.inst = (InstDesc *)(db + off_desc);
    bufs.work.chunk_prefix = (unsigned *)(db + pk.off_pref);
    return SGE_OK;
}

hipError_t enqueue_plan_only(const Pack &pk, LaunchBufs &bufs, uint32_t root_chunk, hipStream_t s) {
    hipError_t r;
    if ((r = hipMemcpyAsync(bufs.d_blob.p, bufs.h_blob.p, pk.upload, hipMemcpyHostToDevice, s)) != hipSuccess)
        return r;
    return launch_plan((const PlanIn *)((char *)bufs.d_blob.p + pk.off_req), pk.m, pk.cfg.wmax, pk.cfg.kmax,
                       bufs.work.inst, bufs.work.chunk_prefix, pk.policy, root_chunk, pk.units, s);
}

hipError_t enqueue_pack(sge_ctx *c, const Pack &pk, LaunchBufs &bufs, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    hipError_t r;
    c->enqueue_step = pk.device_plan ? "upload and plan kernels" : "upload";
    if (pk.device_plan) r = enqueue_plan_only(pk, bufs, c->root_chunk, s);
    else r = hipMemcpyAsync(bufs.d_blob.p, bufs.h_blob.p, pk.upload, hipMemcpyHostToDevice, s);
    if (r != hipSuccess) return r;
    c->enqueue_step = "reset kernel";
    if ((r = launch_reset(bufs.work, pk.m, s)) != hipSuccess) return r;
    c->enqueue_step = "record the kernel's start event";
    if (e0 && (r = hipEventRecord(e0, s)) != hipSuccess) return r;
    c->enqueue_step = "search kernel";
    if ((r = launch_search(pk.cfg, bufs.work, pk.m, c->cap, c->time_limit_ms, s, c->num_cus)) != hipSuccess)
        return r;
    c->enqueue_step = "record the kernel's end event";
    if (e1 && (r = hipEventRecord(e1, s)) != hipSuccess) return r;
    c->enqueue_step = "read-back";
    if ((r = hipMemcpyAsync(bufs.h_ctr.p, bufs.work.ctr, pk.m * sizeof(InstCounters), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
        return r;
    return hipMemcpyAsync((char *)bufs.h_ctr.p + pk.ctr_bytes, bufs.work.sched, sizeof(Sched), hipMemcpyDeviceToHost,
                          s);
}

void read_pack(const sge_ctx *c, Pack &pk, const LaunchBufs &bufs, const std::vector<const InstanceSpec *> &specs,
               std::vector<InstanceOut *> &out, double &ms_search) {
    const InstCounters *hc = (const InstCounters *)bufs.h_ctr.p;
    const Sched *hs = (const Sched *)((const char *)bufs.h_ctr.p + pk.ctr_bytes);
    // kernel time from the device clock (100 MHz): first block start to last wave exit
    auto since = [&](unsigned long long t) { return t > hs->t_start ? (double)(t - hs->t_start) / 1e5 : 0.0; };
    ms_search = since(hs->t_end);
    pk.ms_work = since(hs->t_work);
    pk.ms_done = since(hs->t_done);
    pk.busy_ms = (double)hs->t_busy / 1e5;
    pk.units_run = hs->units;
    pk.bad_task = hs->bad == 1;
    pk.bad_unit = hs->bad == 2;
    for (uint32_t j = 0; j < pk.m; j++) {
        InstanceOut &o = *out[j];
        o.matches = hc[j].matches;
        o.states = hc[j].states;
        o.candidates = hc[j].candidates;
        o.steals = hc[j].steals;
        o.steps = hc[j].steps;
        o.bytes = hc[j].bytes;
        o.status = SGE_OK;
        if (pk.bad_task || pk.bad_unit) {
            o.status = SGE_E_DEVICE;
        } else if (hs->abort) {
            o.status = SGE_E_ABORTED;
            o.timed_out = true;
        } else if (c->cap && o.states > c->cap) {
            o.status = SGE_E_ABORTED;
        } else if (specs[j]->rows && o.matches > specs[j]->cap_rows) {
            o.status = SGE_E_OVERFLOW;
        }
    }
}

// Event-record nodes around the search kernel's node of a captured graph:
// e0 after everything the kernel waits for, the kernel after e0, e1 after
// the kernel (the nodes after the kernel keep waiting on it directly).
static hipError_t add_kernel_events(hipGraph_t g, const void *fn, hipEvent_t e0, hipEvent_t e1) {
    if (!fn || !e0 || !e1) return hipErrorInvalidValue;
    size_t n = 0;
    hipError_t e = hipGraphGetNodes(g, nullptr, &n);
    if (e != hipSuccess) return e;
    std::vector<hipGraphNode_t> nodes(n);
    if ((e = hipGraphGetNodes(g, nodes.data(), &n)) != hipSuccess) return e;
    hipGraphNode_t kern = nullptr;
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType t;
        if (hipGraphNodeGetType(nd, &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp{};
        if (hipGraphKernelNodeGetParams(nd, &kp) == hipSuccess && kp.func == fn) {
            kern = nd;
            break;
        }
    }
    if (!kern) return hipErrorNotFound;
    size_t nd = 0;
    if ((e = hipGraphNodeGetDependencies(kern, nullptr, &nd)) != hipSuccess) return e;
    std::vector<hipGraphNode_t> deps(nd);
    if (nd && (e = hipGraphNodeGetDependencies(kern, deps.data(), &nd)) != hipSuccess) return e;
    hipGraphNode_t n0 = nullptr, n1 = nullptr;
    if ((e = hipGraphAddEventRecordNode(&n0, g, deps.data(), nd, e0)) != hipSuccess) return e;
    if ((e = hipGraphAddDependencies(g, &n0, &kern, 1)) != hipSuccess) return e;
    return hipGraphAddEventRecordNode(&n1, g, &kern, 1, e1);
}

// Everything a captured batch graph depends on besides the contents of the
// descriptor buffer: the stream, the pack's sizes and launch shape, the
// buffer addresses and the context settings the kernels receive.
static uint64_t graph_key(const sge_ctx *c, const Pack &pk, const LaunchBufs &b, hipStream_t s) {
    uint64_t h = 1469598103934665603ull;   // FNV-1a over 64-bit words
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; i++) {
            h ^= (v >> (8 * i)) & 0xFFu;
            h *= 1099511628211ull;
        }
    };
    const LaunchCfg &g = pk.cfg;
    for (uint64_t v : {(uint64_t)(uintptr_t)s, (uint64_t)pk.device_plan, (uint64_t)pk.m, (uint64_t)pk.upload,
                       (uint64_t)pk.off_req, (uint64_t)pk.ctr_bytes, (uint64_t)pk.policy, (uint64_t)pk.units,
                       (uint64_t)g.lanes, (uint64_t)g.dense, (uint64_t)g.donate, (uint64_t)g.kmax, (uint64_t)g.nmax,
                       (uint64_t)g.wmax, (uint64_t)g.blocks, (uint64_t)g.per_cu, (uint64_t)g.used_bitset,
                       (uint64_t)g.general, (uint64_t)g.count_bytes, (uint64_t)g.check_uniform,
                       (uint64_t)g.root_lo, (uint64_t)g.root_hi,
                       (uint64_t)(uintptr_t)b.d_blob.p, (uint64_t)(uintptr_t)b.h_blob.p,
                       (uint64_t)(uintptr_t)b.h_ctr.p, (uint64_t)(uintptr_t)b.work.sched,
                       (uint64_t)(uintptr_t)b.work.queue, (uint64_t)(uintptr_t)b.work.ctr,
                       (uint64_t)(uintptr_t)b.work.inst, (uint64_t)(uintptr_t)b.work.chunk_prefix,
                       (uint64_t)c->root_chunk, (uint64_t)c->cap, (uint64_t)c->time_limit_ms, (uint64_t)c->num_cus})
        mix(v);
    return h;
}

sge_status run_instances(sge_ctx *c, const std::vector<InstanceSpec> &specs, std::vector<InstanceOut> &out,
                         double &ms_prep, double &ms_search, bool graph, int policy) {
    auto t0 = clk::now();
    const size_t N = specs.size();
    out.assign(N, InstanceOut{});
    std::vector<const InstanceSpec *> sp;
    std::vector<InstanceOut *> op;
    for (size_t i = 0; i < N; i++) {
        if (specs[i].p->g.n == 0) {   // the empty pattern has one (empty) match
            out[i].matches = 1;
            continue;
        }
        sp.push_back(&specs[i]);
        op.push_back(&out[i]);
    }
    ms_search = 0;
    c->last_event_ms = 0;
    if (sp.empty()) {
        ms_prep = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
        return SGE_OK;
    }
    const bool dense = choose_dense(c, specs);
    if (c->dense == 1 && !dense) {
        for (const InstanceSpec *x : sp)
            if (general_instance(*x)) return fail(c, SGE_E_INVAL, "the dense search covers undirected graphs without edge labels");
    }
    if (c->plan_where == 1) {
        for (const InstanceSpec *x : sp)
            if (general_instance(*x))
                return fail(c, SGE_E_INVAL, "the plan kernel covers undirected graphs without edge labels");
    }
    Pack pk;
    sge_status st;
    if (plan_on_device(c, sp)) {
        st = pack_instances(c, sp, dense, policy, c->bufs, pk);
    } else {
        // host plans (threads for larger sets); an empty domain answers its
        // instance at once
        const size_t M = sp.size();
        std::vector<Plan> plans(M);
        std::vector<std::vector<uint64_t>> bits(M);
        auto plan_one = [&](size_t i) {
            build_plan(*sp[i]->t, sp[i]->p->g, sp[i]->mode, sp[i]->labelled, c->root_lo, c->root_hi, plans[i],
                       dense || sp[i]->mode != SGE_RI, bits[i]);
        };
        if (M >= 64) {
            const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
            std::vector<std::thread> th;
            for (unsigned w = 0; w < nt; w++)
                th.emplace_back([&, w]() {
                    for (size_t i = w; i < M; i += nt) plan_one(i);
                });
            for (auto &x : th) x.join();
        } else {
            for (size_t i = 0; i < M; i++) plan_one(i);
        }
        std::vector<const InstanceSpec *> sp2;
        std::vector<InstanceOut *> op2;
        std::vector<const Plan *> pp;
        std::vector<const std::vector<uint64_t> *> bp;
        for (size_t i = 0; i < M; i++)
            if (!plans[i].empty) {
                sp2.push_back(sp[i]);
                op2.push_back(op[i]);
                pp.push_back(&plans[i]);
                bp.push_back(&bits[i]);
            }
        sp.swap(sp2);
        op.swap(op2);
        if (sp.empty()) {
            ms_prep = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
            return SGE_OK;
        }
        st = pack_host_planned(c, sp, pp, bp, dense, policy, c->bufs, pk);
    }
    if (st != SGE_OK) return st;
    hipStream_t s = c->stream;
    ms_prep = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    hipError_t e;
    if (graph) {
        // one graph: plan upload, scheduler reset, the persistent search,
        // read-back.  The executable graph is kept and launched again while
        // everything it captured is unchanged: the launch shape, the sizes, the
        // buffer addresses and the settings passed to the kernels.  Its upload
        // node copies the pinned descriptor buffer as the host has just
        // refilled it, so each launch plans and searches the current jobs.
        const uint64_t key = graph_key(c, pk, c->bufs, s);
        if (!c->gexec || c->gexec_key != key) {
            if (c->gexec) {
                (void)hipGraphExecDestroy(c->gexec);   // the stream is idle: every launch was waited for
                c->gexec = nullptr;
            }
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            // with event-record nodes right before and after the search
            // kernel's node; should the runtime refuse them, the graph is
            // captured again without them (the events then time nothing) and
            // later captures leave them out
            if (c->gev0) (void)hipEventDestroy(c->gev0);
            if (c->gev1) (void)hipEventDestroy(c->gev1);
            c->gev0 = c->gev1 = nullptr;
            if (c->graph_extras &&
                (hipEventCreate(&c->gev0) != hipSuccess || hipEventCreate(&c->gev1) != hipSuccess)) {
                c->graph_extras = false;
                c->graph_extras_error = "hipEventCreate";
            }
            hipError_t er = hipSuccess;
            for (int attempt = c->graph_extras ? 0 : 1; attempt < 2; attempt++) {
                (void)hipGetLastError();
                if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                    return hip_fail(c, e, "hipStreamBeginCapture");
                er = enqueue_pack(c, pk, c->bufs, s, nullptr, nullptr);
                e = hipStreamEndCapture(s, &g);
                if (er == hipSuccess && e == hipSuccess && attempt == 0) {
                    c->enqueue_step = "event nodes around the search kernel";
                    er = add_kernel_events(g, search_kernel_fn(pk.cfg), c->gev0, c->gev1);
                }
                if (er == hipSuccess && e == hipSuccess) break;
                if (g) (void)hipGraphDestroy(g);
                g = nullptr;
                if (attempt == 1) return hip_fail(c, er != hipSuccess ? er : e, "capture search graph");
                c->graph_extras = false;
                c->graph_extras_error = (er != hipSuccess ? std::string("enqueue (") + c->enqueue_step + "): "
                                                          : std::string("end capture: ")) +
                                        hipGetErrorString(er != hipSuccess ? er : e);
                // not an error of this call: kept as the context's message for inspection
                c->err = "batch graph captured without the kernel's event nodes (" + c->graph_extras_error + ")";
            }
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
            c->gexec = ge;
            c->gexec_key = key;
            c->gexec_timed = c->graph_extras;
        }
        e = hipGraphLaunch(c->gexec, s);
        hipError_t es = hipStreamSynchronize(s);
        if (e != hipSuccess || es != hipSuccess) {
            // an executable graph whose launch failed is not reused
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
        if (es != hipSuccess) return hip_fail(c, es, "search");
    } else {
        if ((e = enqueue_pack(c, pk, c->bufs, s, c->ev0, c->ev1)) != hipSuccess)
            return hip_fail(c, e, "search launch");
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "search");
    }
    read_pack(c, pk, c->bufs, sp, op, ms_search);
    float ev_ms = 0;
    // this launch recorded the kernel's events: plain records, or the event
    // nodes of the graph
    hipEvent_t k0 = graph ? (c->gexec_timed ? c->gev0 : nullptr) : c->ev0;
    hipEvent_t k1 = graph ? (c->gexec_timed ? c->gev1 : nullptr) : c->ev1;
    c->last_event_ms = k0 && k1 && hipEventElapsedTime(&ev_ms, k0, k1) == hipSuccess ? (double)ev_ms : 0.0;
    c->last_ms[0] = ms_search;
    c->last_ms[1] = pk.ms_work;
    c->last_ms[2] = pk.ms_done;
    c->last_busy_ms = pk.busy_ms;
    c->last_units = pk.units_run;
    c->last_lanes = pk.cfg.lanes;
    if (pk.bad_task) return fail(c, SGE_E_DEVICE, "the work queue delivered an invalid task; counters are unreliable");
    if (pk.bad_unit)
        return fail(c, SGE_E_DEVICE, "the lanes of a search unit disagreed on its state; counters are unreliable");
    if (op[0]->timed_out) c->err = "search stopped at the time limit; counters are partial";
    return SGE_OK;
}

}  // namespace sge
