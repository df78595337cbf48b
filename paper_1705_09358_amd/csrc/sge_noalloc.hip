// The allocation-free count: sge_count with every device buffer of the launch
// -- the job descriptor and plan request, the device plan, the instance's
// domains, per-position bitsets and candidate lists, the scheduler words,
// the work queue and the counters -- carved out of one static device array,
// and the plan made by the plan kernel (no host planning buffers).  For
// callers that cannot allocate (code under graph capture, tight serving
// loops, harnesses that forbid allocation).  The target and pattern are
// loaded beforehand, as for sge_count.
//
// Every call on a device uses that device's one copy of the array, which
// keeps the last call's contents: the reset kernel clears the scheduler
// words, counters and queue tickets at the head of each launch, the plan
// kernel overwrites the plan area, and the descriptor is uploaded anew.
// Calls that overlap on one device race for the array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "sge_ctx.h"

namespace sge {

constexpr size_t SCRATCH_BYTES = 16ull << 20;   // per device
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char *g_scratch[MAX_DEVICES] = {};   // the array's device address, per device

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Byte offsets in the array of everything one launch holds.
struct Layout {
    size_t desc, req, pref, plan, dom, pos, lists, support, sched, queue, ctr, end;
};

Layout layout(const InstanceSpec &s, bool dense) {
    const size_t kw = (size_t)s.p->g.n * s.t->W;
    Layout L;
    L.desc = 0;
    L.req = align_up(L.desc + sizeof(InstDesc), 256);
    L.pref = align_up(L.req + sizeof(PlanIn), 256);
    L.plan = align_up(L.pref + 2 * sizeof(unsigned), 256);
    L.dom = align_up(L.plan + sizeof(DevPlan), 256);
    L.pos = align_up(L.dom + kw * 8, 256);
    const bool with_bits = dense || s.mode != SGE_RI;
    L.lists = align_up(L.pos + (with_bits ? kw * 8 : 0), 256);
    L.support = align_up(L.lists + list_entries(s) * 4, 256);
    L.sched = align_up(L.support + (s.t->W > PLAN_LDS_WORDS ? (size_t)s.t->W * 8 : 0), 256);
    L.queue = align_up(L.sched + sizeof(Sched), 256);
    L.ctr = align_up(L.queue + sizeof(QTask) * QUEUE_SLOTS, 256);
    L.end = align_up(L.ctr + sizeof(InstCounters), 256);
    return L;
}

}  // namespace

// Called once per device by sge_create, with that device current: the
// array's address on this device (each device holds its own copy).
hipError_t noalloc_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();   // not left for the next launch check to find
        return e;
    }
    g_scratch[device] = (unsigned char *)p;
    return hipSuccess;
}

}  // namespace sge

using namespace sge;

extern "C" sge_status sge_count_noalloc(sge_ctx *c, uint32_t target, uint32_t pattern, sge_result *res) {
    if (!c || !res) return SGE_E_INVAL;
    auto it = c->targets.find(target);
    if (it == c->targets.end()) return fail(c, SGE_E_HANDLE, "unknown target handle");
    auto ip = c->patterns.find(pattern);
    if (ip == c->patterns.end()) return fail(c, SGE_E_HANDLE, "unknown pattern handle");
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (c->device >= 0 && c->device < MAX_DEVICES) base = g_scratch[c->device];
    }
    if (!base) return fail(c, SGE_E_DEVICE, "the allocation-free scratch array has no address on this device");
    (void)hipSetDevice(c->device);
    *res = sge_result{};
    c->last_event_ms = 0;
    InstanceSpec s;
    s.t = it->second.get();
    s.p = ip->second.get();
    s.mode = c->mode;
    s.labelled = c->labelled != 0;
    const uint32_t k = s.p->g.n;
    if (k == 0) {   // the empty pattern has one (empty) match
        res->matches = 1;
        return SGE_OK;
    }
    if (general_instance(s))
        return fail(c, SGE_E_INVAL, "the allocation-free count plans on the device: undirected graphs without "
                                    "compared edge labels only");
    const bool dense = choose_dense(c, &s, 1);
    const Layout L = layout(s, dense);
    if (L.end > SCRATCH_BYTES)
        return fail(c, SGE_E_INVAL, "instance needs " + std::to_string(L.end) +
                                        " bytes of device scratch; the allocation-free count has " +
                                        std::to_string(SCRATCH_BYTES));
    const InstanceSpec *sp = &s;
    Pack pk;
    launch_config(c, &sp, 1, dense, 2, pk);
    if (search_block_threads(pk.cfg) == 0) return fail(c, SGE_E_INVAL, "search units do not fit in LDS");

    // the descriptor and plan request, as the batch packer writes them
    const bool with_bits = dense || s.mode != SGE_RI;
    InstDesc d{};
    d.col = s.t->d_col;
    d.node = s.t->d_node;
    d.wcol = s.t->d_wcol;
    d.adj = s.t->d_adj;
    d.plan = (const DevPlan *)(base + L.plan);
    d.bits = with_bits ? (const uint64_t *)(base + L.pos) : nullptr;
    d.lists = (const uint32_t *)(base + L.lists);
    PlanIn r{};
    r.pat = s.p->d_pat;
    r.label_keys = s.t->d_label_keys;
    r.nlabels = (uint32_t)s.t->label_keys.size();
    r.nbr_deg = s.t->d_nbr_deg;
    r.nbr_cols = s.t->nbr_cols;
    r.nbr_stride = s.t->nbr_stride;
    r.mode = (uint32_t)s.mode;
    r.labelled = s.labelled ? 1u : 0u;
    r.n = s.t->g.n;
    r.W = s.t->W;
    r.root_lo = c->root_lo;
    r.root_hi = c->root_hi;
    r.desc = (InstDesc *)(base + L.desc);
    r.plan = (DevPlan *)(base + L.plan);
    r.dom = (uint64_t *)(base + L.dom);
    r.pos_bits = with_bits ? (uint64_t *)(base + L.pos) : nullptr;
    r.lists = (uint32_t *)(base + L.lists);
    r.list_cap = (uint32_t)std::min<uint64_t>(list_entries(s), 0xFFFFFFFFull);
    r.support = s.t->W > PLAN_LDS_WORDS ? (uint64_t *)(base + L.support) : nullptr;
    r.rows = s.t->d_adj && s.t->g.n && s.t->g.col.size() >= (uint64_t)s.t->g.n * s.t->W ? 1u : 0u;
    r.deg_mean = s.t->g.n ? (uint32_t)std::min<uint64_t>((s.t->g.col.size() + s.t->g.n - 1) / s.t->g.n, 0xFFFFFFFFull) : 0u;

    DevWork w;
    w.sched = (Sched *)(base + L.sched);
    w.queue = (QTask *)(base + L.queue);
    w.ctr = (InstCounters *)(base + L.ctr);
    w.inst = (InstDesc *)(base + L.desc);
    w.chunk_prefix = (unsigned *)(base + L.pref);

    InstCounters hc{};
    Sched hs{};
    hipStream_t st = c->stream;
    hipError_t e = hipMemcpyAsync(base + L.desc, &d, sizeof(d), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(base + L.req, &r, sizeof(r), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_plan((const PlanIn *)(base + L.req), 1, s.t->W, k, w.inst, w.chunk_prefix, 2, c->root_chunk,
                        pk.units, st);
    if (e == hipSuccess) e = launch_reset(w, 1, st);
    if (e == hipSuccess && c->ev0) e = hipEventRecord(c->ev0, st);
    if (e == hipSuccess) e = launch_search(pk.cfg, w, 1, c->cap, c->time_limit_ms, st, c->num_cus);
    if (e == hipSuccess && c->ev1) e = hipEventRecord(c->ev1, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&hc, w.ctr, sizeof(hc), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&hs, w.sched, sizeof(hs), hipMemcpyDeviceToHost, st);
    const hipError_t es = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(c, e, "allocation-free count");
    if (es != hipSuccess) return hip_fail(c, es, "allocation-free count");

    float ev_ms = 0;
    c->last_event_ms =
        c->ev0 && c->ev1 && hipEventElapsedTime(&ev_ms, c->ev0, c->ev1) == hipSuccess ? (double)ev_ms : 0.0;
    auto since = [&](unsigned long long t) { return t > hs.t_start ? (double)(t - hs.t_start) / 1e5 : 0.0; };
    res->matches = hc.matches;
    res->states = hc.states;
    res->candidates = hc.candidates;
    res->alg_bytes = hc.bytes;
    res->steals = hc.steals;
    res->steps = hc.steps;
    res->ms_search = since(hs.t_end);
    c->last_ms[0] = res->ms_search;
    c->last_ms[1] = since(hs.t_work);
    c->last_ms[2] = since(hs.t_done);
    c->last_busy_ms = (double)hs.t_busy / 1e5;
    c->last_units = hs.units;
    c->last_lanes = pk.cfg.lanes;
    if (hs.bad == 1) return fail(c, SGE_E_DEVICE, "the work queue delivered an invalid task; counters are unreliable");
    if (hs.bad) return fail(c, SGE_E_DEVICE, "the lanes of a search unit disagreed on its state; counters are unreliable");
    if (hs.abort) return fail(c, SGE_E_ABORTED, "search stopped at the time limit; counters are partial");
    if (c->cap && res->states > c->cap) return fail(c, SGE_E_ABORTED, "state cap exceeded");
    return SGE_OK;
}
