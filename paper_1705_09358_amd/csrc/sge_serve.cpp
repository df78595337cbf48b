// Serving: continuous batching of pattern queries on resident targets.
//
// Targets (CSR, node records, adjacency rows, label keys) and patterns stay
// resident on the device.  A query is admitted when a slot is free and its
// device bytes (plan, domains, candidate lists) fit in the arena budget;
// otherwise submit says SGE_E_BUSY and the caller retries.  Admitted queries
// are planned (order, RI-DS domains with arc-consistency and forward
// checking) by a pool of host threads while earlier queries search, or, when
// the context plans on the device, by the plan kernel at the head of their
// launch.  A dispatcher thread packs whatever is ready into one persistent
// search launch on the first idle launch lane (one HIP stream each, with its
// own scheduler state and buffers), so queries that arrive while earlier ones
// are on the GPU start at once on another lane and run beside them.  When a
// lane's launch completes its queries' results become visible to poll and
// their slots and bytes are released.
#include <algorithm>
#include <condition_variable>
#include <deque>
#include <thread>

#include "sge_ctx.h"

using namespace sge;
using clk = std::chrono::steady_clock;

namespace sge {

struct Query {
    uint64_t ticket = 0;
    InstanceSpec spec;
    Plan plan;                    // host plan (unless planned on the device)
    std::vector<uint64_t> bits;
    InstanceOut out;
    uint64_t bytes = 0;
    bool done = false;
    double ms_prep = 0, ms_search = 0;
};

struct LaunchLane {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    LaunchBufs bufs;
    std::vector<Query *> batch;
    Pack pk;
    bool busy = false;
};

struct Server {
    sge_ctx *c = nullptr;
    uint32_t slots = 0;
    uint64_t arena = 0;
    std::mutex mu;
    std::condition_variable cv_prep, cv_disp;
    bool device_plan = false;
    std::map<uint64_t, std::unique_ptr<Query>> queries;
    uint64_t next_ticket = 1;
    uint64_t bytes_in_use = 0;
    uint32_t in_flight = 0;
    std::deque<Query *> prep_q, ready_q;
    std::vector<std::thread> preppers;
    std::thread dispatcher;
    std::vector<LaunchLane> lanes;
    bool stopping = false;
    std::string fatal;   // a device error stops the server

    void release(Query *q) {   // caller holds mu
        q->done = true;
        bytes_in_use -= q->bytes;
        in_flight--;
        // the query no longer touches its target and pattern
        const_cast<Target *>(q->spec.t)->serve_refs--;
        const_cast<Pattern *>(q->spec.p)->serve_refs--;
    }
    void prep_loop();
    void dispatch_loop();
};
void ServerDeleter::operator()(Server *s) const { delete s; }

void Server::prep_loop() {
    (void)hipSetDevice(c->device);
    for (;;) {
        Query *q;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_prep.wait(lk, [&] { return stopping || !prep_q.empty(); });
            if (prep_q.empty()) return;
            q = prep_q.front();
            prep_q.pop_front();
        }
        auto t0 = clk::now();
        std::vector<InstanceSpec> one{q->spec};
        const bool dense = choose_dense(c, one);
        build_plan(*q->spec.t, q->spec.p->g, q->spec.mode, q->spec.labelled, c->root_lo, c->root_hi, q->plan,
                   dense || q->spec.mode != SGE_RI, q->bits);
        q->ms_prep = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
        std::lock_guard<std::mutex> lk(mu);
        if (!q->plan.empty) {
            ready_q.push_back(q);
            cv_disp.notify_one();
        } else {   // an empty domain: no match, nothing to search
            release(q);
        }
    }
}

void Server::dispatch_loop() {
    (void)hipSetDevice(c->device);
    for (;;) {
        // collect finished launches
        for (LaunchLane &ln : lanes) {
            if (!ln.busy) continue;
            hipError_t e = hipEventQuery(ln.ev);
            if (e == hipErrorNotReady) continue;
            std::vector<const InstanceSpec *> sp;
            std::vector<InstanceOut *> op;
            for (Query *q : ln.batch) {
                sp.push_back(&q->spec);
                op.push_back(&q->out);
            }
            double ms = 0;
            if (e == hipSuccess) read_pack(c, ln.pk, ln.bufs, sp, op, ms);
            std::lock_guard<std::mutex> lk(mu);
            if (e != hipSuccess) fatal = std::string("search launch failed: ") + hipGetErrorString(e);
            for (Query *q : ln.batch) {
                if (e != hipSuccess) q->out.status = SGE_E_DEVICE;
                q->ms_search = ms;
                release(q);
            }
            ln.batch.clear();
            ln.busy = false;
        }
        // start a launch on an idle lane with everything that is ready
        std::vector<Query *> take;
        LaunchLane *lane = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            bool any_busy = false;
            for (LaunchLane &ln : lanes) any_busy |= ln.busy;
            if (stopping && ready_q.empty() && prep_q.empty() && !any_busy) return;
            for (LaunchLane &ln : lanes)
                if (!ln.busy) { lane = &ln; break; }
            if (lane && !ready_q.empty() && fatal.empty()) {
                while (!ready_q.empty() && take.size() < 256) {
                    take.push_back(ready_q.front());
                    ready_q.pop_front();
                }
            } else {
                // wait for work or for a launch to finish (polled)
                cv_disp.wait_for(lk, std::chrono::microseconds(any_busy ? 50 : 2000));
                continue;
            }
        }
        auto t0 = clk::now();
        std::vector<const InstanceSpec *> sp;
        std::vector<InstanceSpec> specs;
        std::vector<const Plan *> pp;
        std::vector<const std::vector<uint64_t> *> bp;
        for (Query *q : take) {
            sp.push_back(&q->spec);
            specs.push_back(q->spec);
            pp.push_back(&q->plan);
            bp.push_back(&q->bits);
        }
        bool dense = choose_dense(c, specs);
        sge_status st = device_plan ? pack_instances(c, sp, dense, 2, lane->bufs, lane->pk)
                                    : pack_host_planned(c, sp, pp, bp, dense, 2, lane->bufs, lane->pk);
        const double ms_pack = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
        for (Query *q : take) q->ms_prep += ms_pack;
        hipError_t e = hipSuccess;
        if (st == SGE_OK) {
            // a share of the device per lane, so launches of several lanes run side by side
            lane->pk.cfg.blocks = std::max(32, 2 * c->num_cus / (int)lanes.size());
            e = enqueue_pack(c, lane->pk, lane->bufs, lane->s);
            if (e == hipSuccess) e = hipEventRecord(lane->ev, lane->s);
        }
        if (st != SGE_OK || e != hipSuccess) {
            std::lock_guard<std::mutex> lk(mu);
            fatal = st != SGE_OK ? c->err : std::string("search launch failed: ") + hipGetErrorString(e);
            for (Query *q : take) {
                q->out.status = SGE_E_DEVICE;
                release(q);
            }
            continue;
        }
        lane->batch = std::move(take);
        lane->busy = true;
    }
}

}  // namespace sge

extern "C" {

// Whether a server query in flight holds the target or pattern (unloading it
// must wait until the query completes).
__attribute__((visibility("hidden"))) bool sge_serve_holds(sge_ctx *c, const Target *t, const Pattern *p) {
    if (!c || !c->server) return false;
    std::lock_guard<std::mutex> lk(c->server->mu);
    return (t && t->serve_refs) || (p && p->serve_refs);
}

__attribute__((visibility("hidden"))) void sge_serve_shutdown_internal(sge_ctx *c) {
    if (!c || !c->server) return;
    Server *sv = c->server.get();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
    }
    sv->cv_prep.notify_all();
    sv->cv_disp.notify_all();
    for (auto &t : sv->preppers) t.join();
    if (sv->dispatcher.joinable()) sv->dispatcher.join();
    for (LaunchLane &ln : sv->lanes) {
        if (ln.s) (void)hipStreamSynchronize(ln.s);
        ln.bufs.release();
        if (ln.ev) (void)hipEventDestroy(ln.ev);
        if (ln.s) (void)hipStreamDestroy(ln.s);
    }
    c->server.reset();
}

sge_status sge_serve_start(sge_ctx *c, uint32_t slots, uint64_t arena_bytes) {
    if (!c) return SGE_E_INVAL;
    if (c->server) return fail(c, SGE_E_INVAL, "server already started");
    if (slots == 0 || arena_bytes == 0) return fail(c, SGE_E_INVAL, "slots and arena_bytes must be positive");
    (void)hipSetDevice(c->device);
    c->server.reset(new Server());
    Server *sv = c->server.get();
    sv->c = c;
    sv->slots = slots;
    sv->arena = arena_bytes;
    const int nlanes = 4;
    sv->lanes.resize(nlanes);
    for (LaunchLane &ln : sv->lanes) {
        hipError_t e = hipStreamCreateWithFlags(&ln.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            sge_serve_shutdown_internal(c);
            return hip_fail(c, e, "server streams");
        }
    }
    sv->device_plan = c->plan_where == 1;
    if (!sv->device_plan) {
        const unsigned np = std::max(2u, std::min(8u, std::thread::hardware_concurrency() / 2));
        for (unsigned i = 0; i < np; i++) sv->preppers.emplace_back([sv] { sv->prep_loop(); });
    }
    sv->dispatcher = std::thread([sv] { sv->dispatch_loop(); });
    return SGE_OK;
}

sge_status sge_serve_submit(sge_ctx *c, const sge_job *job, uint64_t *ticket) {
    if (!c || !job || !ticket) return SGE_E_INVAL;
    Server *sv = c->server.get();
    if (!sv) return fail(c, SGE_E_INVAL, "server not started");
    if (job->mode < SGE_RI || job->mode > SGE_RIDS_SI_FC) return fail(c, SGE_E_INVAL, "unknown mode");
    auto it = c->targets.find(job->target);
    if (it == c->targets.end()) return fail(c, SGE_E_HANDLE, "unknown target handle");
    auto ip = c->patterns.find(job->pattern);
    if (ip == c->patterns.end()) return fail(c, SGE_E_HANDLE, "unknown pattern handle");
    auto q = std::make_unique<Query>();
    q->spec.t = it->second.get();
    q->spec.p = ip->second.get();
    q->spec.mode = job->mode;
    q->spec.labelled = job->labelled != 0;
    q->bytes = instance_device_bytes(q->spec);
    if (sv->device_plan && general_instance(q->spec))
        return fail(c, SGE_E_INVAL, "the plan kernel covers undirected graphs without edge labels");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->fatal.empty()) return fail(c, SGE_E_DEVICE, sv->fatal);
    if (sv->stopping) return fail(c, SGE_E_INVAL, "server is stopping");
    if (q->bytes > sv->arena) return fail(c, SGE_E_NOMEM, "query larger than the server's memory budget");
    if (sv->in_flight >= sv->slots || sv->bytes_in_use + q->bytes > sv->arena)
        return fail(c, SGE_E_BUSY, "no slot or memory free now");
    q->ticket = sv->next_ticket++;
    *ticket = q->ticket;
    sv->in_flight++;
    sv->bytes_in_use += q->bytes;
    it->second->serve_refs++;
    ip->second->serve_refs++;
    if (q->spec.p->g.n == 0) {   // the empty pattern has one (empty) match
        q->out.matches = 1;
        sv->release(q.get());
    } else if (sv->device_plan) {
        sv->ready_q.push_back(q.get());
        sv->cv_disp.notify_one();
    } else {
        sv->prep_q.push_back(q.get());
        sv->cv_prep.notify_one();
    }
    sv->queries[q->ticket] = std::move(q);
    return SGE_OK;
}

sge_status sge_serve_poll(sge_ctx *c, uint64_t ticket, sge_result *res) {
    if (!c || !res) return SGE_E_INVAL;
    Server *sv = c->server.get();
    if (!sv) return fail(c, SGE_E_HANDLE, "server not started");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->queries.find(ticket);
    if (it == sv->queries.end()) return fail(c, SGE_E_HANDLE, "unknown ticket");
    Query *q = it->second.get();
    if (!q->done) return SGE_E_BUSY;
    res->matches = q->out.matches;
    res->states = q->out.states;
    res->candidates = q->out.candidates;
    res->alg_bytes = q->out.bytes;
    res->steals = q->out.steals;
    res->steps = q->out.steps;
    res->ms_prep = q->ms_prep;
    res->ms_search = q->ms_search;
    sge_status st = q->out.status;
    sv->queries.erase(it);
    if (st == SGE_E_ABORTED) return fail(c, st, "state cap or time limit reached");
    if (st != SGE_OK) return fail(c, st, "query failed");
    return SGE_OK;
}

sge_status sge_serve_stop(sge_ctx *c) {
    if (!c) return SGE_E_INVAL;
    if (!c->server) return SGE_OK;
    sge_serve_shutdown_internal(c);
    return SGE_OK;
}

}  // extern "C"
