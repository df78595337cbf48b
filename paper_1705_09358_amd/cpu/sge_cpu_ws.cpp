// A multithreaded CPU baseline: the paper's own parallel search (Section 3)
// on the host cores, planned by the library's host planner.  It exists to put
// a like-for-like parallel CPU figure beside the GPU search; the GPU library
// never calls it.
//
//  * Tasks (Section 3.1) are accepted (position, target node) pairs: a
//    candidate is checked before it becomes a task, and a task carries no
//    mapping; a worker's mapping follows its own depth-first order.
//  * Work stealing with private deques (Section 3.2): a worker adds and
//    removes task groups at the front of its deque; an idle worker writes its
//    id into a random busy worker's request slot (compare-and-swap, one request
//    per worker), and that worker answers in its loop by moving the group at
//    the back of its deque, nearest the root, with the mapping prefix it needs,
//    into the thief's transfer slot.
//  * Initial distribution (Section 3.3): the root candidates are split into
//    equal contiguous shares, one per worker.
//  * Task coalescing (Section 3.4): siblings travel in groups of up to
//    `group` tasks.
//  * Termination (Section 3.5): a token passes around the ring of workers;
//    this is the Dijkstra-Feijen-van Gasteren form, with a colour per worker
//    (a worker that hands work away turns black) so that work moving behind
//    the token cannot be missed.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <random>
#include <thread>
#include <vector>

#include "sge_internal.h"

using namespace sge;

namespace {

constexpr int MAX_GROUP = 16;

struct TaskGroup {
    uint32_t depth = 0, n = 0;
    uint32_t v[MAX_GROUP];
};

struct Transfer {
    std::atomic<int> state{0};   // 0 empty, 1 task ready, 2 declined
    TaskGroup g;
    uint32_t M[KMAX];
};

struct alignas(64) WorkerShared {
    std::atomic<bool> work_available{false};
    std::atomic<int> request{-1};      // id of a worker asking this one for work
    std::atomic<bool> black{false};    // termination colour
    Transfer transfer;                 // where a victim puts this worker's stolen group
};

struct Search {
    const Target *t = nullptr;
    const Plan *pl = nullptr;
    const std::vector<uint64_t> *bits = nullptr;   // rows by position (RI-DS) or empty
    uint32_t k = 0, n = 0, W = 0;
    int nw = 1, group = 4;
    std::vector<WorkerShared> sh;
    std::atomic<int> token_at{0};
    std::atomic<bool> token_black{false};
    std::atomic<bool> done{false};
    std::atomic<uint64_t> matches{0}, states{0}, steals{0};
};

struct Worker {
    Search *S;
    int id;
    std::deque<TaskGroup> q;
    uint32_t M[KMAX];
    std::vector<uint64_t> used;
    uint64_t matches = 0, states = 0, steals = 0;
    std::mt19937 rng;
    bool probe_started = false;   // worker 0: a probe is on its way round the ring

    Worker(Search *s, int i) : S(s), id(i), used((s->n + 63) / 64, 0), rng(1705u + (unsigned)i) {}

    bool adjacent(uint32_t a, uint32_t v) const {
        const HostGraph &g = S->t->g;
        return std::binary_search(g.col.begin() + g.rp[a], g.col.begin() + g.rp[a + 1], v);
    }

    // RI's rules (and the RI-DS domain test) for candidate v at position i
    bool consistent(uint32_t i, uint32_t v) const {
        const Plan &P = *S->pl;
        const HostGraph &g = S->t->g;
        if (!S->bits->empty() && !(((*S->bits)[(size_t)i * S->W + (v >> 6)] >> (v & 63)) & 1)) return false;
        if ((used[v >> 6] >> (v & 63)) & 1) return false;
        if (P.plabel[i] != LABEL_ANY && S->t->dlab[v] != P.plabel[i]) return false;
        if (g.outdeg(v) < P.pdeg[i]) return false;
        for (uint64_t m = P.back[i]; m; m &= m - 1)
            if (!adjacent(M[__builtin_ctzll(m)], v)) return false;
        return true;
    }

    // map position i-1's last candidate done; accepted candidates of position
    // i (given M[0..i-1]) become task groups at the front, first candidate first
    void expand(uint32_t i) {
        const Plan &P = *S->pl;
        const HostGraph &g = S->t->g;
        const bool last = i + 1 == S->k;
        TaskGroup cur;
        cur.depth = i;
        std::vector<TaskGroup> made;
        auto take = [&](uint32_t v) {
            if (!consistent(i, v)) return;
            states++;
            if (last) { matches++; return; }
            cur.v[cur.n++] = v;
            if ((int)cur.n == S->group) { made.push_back(cur); cur.n = 0; }
        };
        if (P.parent[i] >= 0) {
            const uint32_t a = M[P.parent[i]];
            for (uint32_t e = g.rp[a]; e < g.rp[a + 1]; e++) take(g.col[e]);
        } else {
            for (uint32_t e = 0; e < P.list_len[i]; e++) take(P.lists[P.list_off[i] + e]);
        }
        if (cur.n) made.push_back(cur);
        for (size_t j = made.size(); j-- > 0;) q.push_front(made[j]);
    }

    // the mapping follows the deque: entering depth d drops positions >= d
    void set_depth(uint32_t d, uint32_t &depth_now) {
        while (depth_now > d) {
            depth_now--;
            used[M[depth_now] >> 6] &= ~(1ull << (M[depth_now] & 63));
        }
    }

    void answer_request() {
        WorkerShared &me = S->sh[id];
        const int thief = me.request.load(std::memory_order_acquire);
        if (thief < 0) return;
        Transfer &tr = S->sh[thief].transfer;
        if (q.empty()) {
            tr.state.store(2, std::memory_order_release);
        } else {
            // the group at the back lies nearest the root; its prefix is still ours
            tr.g = q.back();
            q.pop_back();
            std::memcpy(tr.M, M, tr.g.depth * sizeof(uint32_t));
            me.black.store(true, std::memory_order_relaxed);
            tr.state.store(1, std::memory_order_release);
        }
        me.request.store(-1, std::memory_order_release);
        me.work_available.store(!q.empty(), std::memory_order_relaxed);
    }

    // idle: pass the token on (or start / finish a probe) and ask for work
    bool idle_round(uint32_t &depth_now) {
        Search &s = *S;
        WorkerShared &me = s.sh[id];
        me.work_available.store(false, std::memory_order_relaxed);
        // decline a request that arrived meanwhile
        const int thief = me.request.load(std::memory_order_acquire);
        if (thief >= 0) {
            s.sh[thief].transfer.state.store(2, std::memory_order_release);
            me.request.store(-1, std::memory_order_release);
        }
        if (s.token_at.load(std::memory_order_acquire) == id) {
            if (id == 0) {
                if (probe_started && !s.token_black.load() && !me.black.load()) {
                    s.done.store(true, std::memory_order_release);
                    return false;
                }
                // start a probe with a white token
                probe_started = true;
                s.token_black.store(false);
                me.black.store(false);
                s.token_at.store(s.nw > 1 ? 1 : 0, std::memory_order_release);
            } else {
                if (me.black.load()) s.token_black.store(true);
                me.black.store(false);
                s.token_at.store((id + 1) % s.nw, std::memory_order_release);
            }
        }
        if (s.nw == 1) return true;
        // a request to a random worker that has work
        const int victim = (int)(rng() % (uint32_t)(s.nw - 1));
        const int v = victim >= id ? victim + 1 : victim;
        if (!s.sh[v].work_available.load(std::memory_order_relaxed)) return true;
        Transfer &tr = me.transfer;
        tr.state.store(0, std::memory_order_relaxed);
        int expect = -1;
        if (!s.sh[v].request.compare_exchange_weak(expect, id, std::memory_order_acq_rel)) return true;
        int st;
        while ((st = tr.state.load(std::memory_order_acquire)) == 0) {
            if (s.done.load(std::memory_order_acquire)) return false;
            // a worker waiting for work has none to give: decline, so that two
            // workers asking each other cannot wait on each other
            const int other = me.request.load(std::memory_order_acquire);
            if (other >= 0) {
                s.sh[other].transfer.state.store(2, std::memory_order_release);
                me.request.store(-1, std::memory_order_release);
            }
            std::this_thread::yield();
        }
        if (st == 1) {
            set_depth(0, depth_now);
            for (uint32_t i = 0; i < tr.g.depth; i++) {
                M[i] = tr.M[i];
                used[M[i] >> 6] |= 1ull << (M[i] & 63);
            }
            depth_now = tr.g.depth;
            q.push_front(tr.g);
            steals++;
        }
        return true;
    }

    void run(uint32_t root_lo, uint32_t root_hi) {
        Search &s = *S;
        const Plan &P = *s.pl;
        uint32_t depth_now = 0;   // positions 0..depth_now-1 of M are mapped (and marked used)
        // initial distribution: an equal share of the root candidates
        {
            TaskGroup cur;
            cur.depth = 0;
            std::vector<TaskGroup> made;
            for (uint32_t e = root_lo; e < root_hi; e++) {
                const uint32_t v = P.lists[P.list_off[0] + e];
                if (!consistent(0, v)) continue;
                states++;
                if (s.k == 1) { matches++; continue; }
                cur.v[cur.n++] = v;
                if ((int)cur.n == s.group) { made.push_back(cur); cur.n = 0; }
            }
            if (cur.n) made.push_back(cur);
            for (const TaskGroup &g : made) q.push_back(g);
        }
        while (!s.done.load(std::memory_order_acquire)) {
            if (q.empty()) {
                if (!idle_round(depth_now)) break;
                continue;
            }
            TaskGroup g = q.front();
            q.pop_front();
            // one task of the group now; the rest stays in front of its children
            const uint32_t v = g.v[0];
            if (g.n > 1) {
                TaskGroup rest = g;
                rest.n = g.n - 1;
                std::memmove(rest.v, g.v + 1, rest.n * sizeof(uint32_t));
                q.push_front(rest);
            }
            s.sh[id].work_available.store(!q.empty(), std::memory_order_relaxed);
            answer_request();
            set_depth(g.depth, depth_now);
            M[g.depth] = v;
            used[v >> 6] |= 1ull << (v & 63);
            depth_now = g.depth + 1;
            expand(g.depth + 1);
        }
        s.matches += matches;
        s.states += states;
        s.steals += steals;
    }
};

}  // namespace

extern "C" {

// Count the matches of a pattern in a target with `threads` workers (undirected
// graphs as in sge_load_target; mode and labelled as in sge_set_mode /
// sge_set_labelled).  counters[0..2] = matches, states, steals; *seconds = wall
// time of the parallel search (planning excluded).  Returns 0, or -1 on bad input.
int sge_cpu_count(uint32_t k, const uint32_t *p_rp, const uint32_t *p_col, const uint32_t *p_lab, uint32_t n,
                  const uint32_t *t_rp, const uint32_t *t_col, const uint32_t *t_lab, int mode, int labelled,
                  int threads, int group, uint64_t *counters, double *seconds) {
    if (!counters || !seconds || k > KMAX || threads < 1 || group < 1 || group > MAX_GROUP) return -1;
    if (mode < SGE_RI || mode > SGE_RIDS_SI_FC) return -1;
    Target t;
    if (!normalise_graph(n, t_rp, t_col, t_lab, t.g).empty()) return -1;
    HostGraph p;
    if (!normalise_graph(k, p_rp, p_col, p_lab, p).empty()) return -1;
    index_target(t);
    counters[0] = counters[1] = counters[2] = 0;
    *seconds = 0;
    if (k == 0) { counters[0] = 1; return 0; }
    Plan pl;
    std::vector<uint64_t> bits;
    build_plan(t, p, mode, labelled != 0, 0, 0xFFFFFFFFu, pl, mode != SGE_RI, bits);
    if (pl.empty) return 0;
    Search s;
    s.t = &t;
    s.pl = &pl;
    s.bits = &bits;
    s.k = k;
    s.n = n;
    s.W = t.W;
    s.nw = threads;
    s.group = group;
    s.sh = std::vector<WorkerShared>(threads);
    const uint32_t roots = pl.list_len[0];
    auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> th;
    for (int i = 0; i < threads; i++) {
        const uint32_t lo = (uint32_t)((uint64_t)roots * i / threads), hi = (uint32_t)((uint64_t)roots * (i + 1) / threads);
        th.emplace_back([&s, i, lo, hi]() {
            Worker w(&s, i);
            w.run(lo, hi);
        });
    }
    for (auto &x : th) x.join();
    *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    counters[0] = s.matches.load();
    counters[1] = s.states.load();
    counters[2] = s.steals.load();
    return 0;
}

}  // extern "C"
