// Persistent depth-first search kernels for RI / RI-DS subgraph enumeration on
// gfx950.
//
// Search unit.  A unit is a group of G lanes of a 64-lane wavefront (G = 8,
// 16, 32 or 64); a wave holds 64/G units that advance in lock-step through
// one loop, each on its own subtree.  A unit owns, in LDS, the mapping M of
// the current prefix (by order position), one frame per position and a small
// stack of accepted-but-unexplored candidates.  This is the state space of
// Section 2.2.1 traversed depth-first, with RI's candidate generation (the
// target neighbours of the mapped parent; all nodes, or the domain, for a
// node without a parent) and pruning rules in the paper's order (unused,
// label, degree, edges to mapped nodes), plus the RI-DS domain test first
// (Section 4.1).
//
// One step of a unit: pop exhausted frames; if the current frame has an
// accepted candidate left, map it and open the next position's frame; then
// evaluate the next G candidates of the current frame, one per lane, and push
// the accepted ones (at the last position, count and emit them instead).
// States are counted when a candidate is pushed (or, at the last position,
// accepted), so a candidate that did not fit in the stack is evaluated again
// later without being counted twice.
//
// Load balance.  Root candidates (position 0) are handed out in chunks from
// an atomic counter (the paper's initial distribution, Section 3.3; chunks
// play the role of task groups, Section 3.4).  Busy units donate work to a
// global queue when units are idle: the untried remainder of their shallowest
// open frame, or one accepted candidate of it -- near the root, as in the
// paper's stealing from the back of a deque (Section 3.2).  A queued task
// carries its prefix mapping, so only stolen work copies a mapping.
// Termination: `work` counts queued plus running tasks; it reaches zero only
// when no unit holds or can create work (replacing the token ring of
// Section 3.5).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sge_internal.h"

namespace sge {

namespace {

struct SearchArgs {
    const InstDesc *inst;
    const unsigned *chunk_prefix;  // ninst + 1 exclusive prefix of root chunks
    InstCounters *ctr;
    Sched *sched;
    QTask *queue;
    unsigned ninst;
    unsigned kmax, E, UW, W, unit_words;
    int donate;
    unsigned long long state_cap;
    unsigned long long limit_ticks;   // time limit in s_memrealtime ticks (100 MHz); 0 = none
};

constexpr unsigned FULL_RANGE = 0xFFFFFFFFu;
constexpr unsigned NO_TASK = 0xFFFFFFFFu;

__device__ __forceinline__ unsigned ld_rlx(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_acq(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(unsigned *p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(unsigned *p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned fadd(unsigned *p, unsigned v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned fadd_ar(unsigned *p, unsigned v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long fadd64(unsigned long long *p, unsigned long long v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_dec_if_pos(unsigned *p) {
    unsigned v = ld_rlx(p);
    while (v > 0) {
        if (__hip_atomic_compare_exchange_strong(p, &v, v - 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return true;
    }
    return false;
}
__device__ __forceinline__ void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_rel() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// Termination.  `work` counts queued plus running tasks; a root chunk is
// counted before it is claimed.  The unit whose decrement empties `work`
// checks, in this order, that every root chunk has been claimed and that
// `work` is still zero: a claim seen by the first load had already counted
// itself, so a zero after it means no task is left anywhere.
__device__ __forceinline__ void release_task(Sched *S, unsigned nchunks) {
    if (fadd(&S->work, (unsigned)-1) == 1) {
        if (ld_acq(&S->chunk_next) >= nchunks && ld_acq(&S->work) == 0) st_rel(&S->done, 1u);
    }
}

// Orders LDS accesses between lanes of one wavefront (no instruction is
// emitted beyond the compiler barrier: a wave's LDS operations execute in order).
#define WAVE_SYNC()                                               \
    do {                                                          \
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");    \
        __builtin_amdgcn_wave_barrier();                          \
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");    \
    } while (0)

__device__ __forceinline__ unsigned long long now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

template <int G>
__device__ __forceinline__ unsigned long long group_mask(unsigned long long ballot, int gbase) {
    if constexpr (G == 64) return ballot;
    else return (ballot >> gbase) & ((1ull << G) - 1);
}

// Per-unit LDS arrays.
struct UnitLds {
    unsigned *M, *MB, *MD;        // mapping by position, row start and degree of M[i]
    unsigned *cur, *end, *lb;     // frame: next candidate index, list length, list start
    unsigned *eb, *dn;            // frame: first stack entry, entries given away from the bottom
    unsigned *ev, *ebg, *edg;     // stack of accepted candidates: node, row start, degree
    unsigned *used;               // bitset of mapped target nodes
    unsigned *misc;               // group broadcast scratch
};

__device__ __forceinline__ UnitLds carve(unsigned *base, unsigned kmax, unsigned E, unsigned UW) {
    UnitLds u;
    u.M = base;
    u.MB = u.M + kmax;
    u.MD = u.MB + kmax;
    u.cur = u.MD + kmax;
    u.end = u.cur + kmax;
    u.lb = u.end + kmax;
    u.eb = u.lb + kmax;
    u.dn = u.eb + kmax;
    u.ev = u.dn + kmax;
    u.ebg = u.ev + E;
    u.edg = u.ebg + E;
    u.used = u.edg + E;
    u.misc = u.used + UW;
    return u;
}

// Per-unit LDS arrays of the dense kernel.
struct DenseLds {
    unsigned *M;                  // mapping by position
    unsigned *fc;                 // frame: number of candidates left
    unsigned long long *cand;     // frame: candidate set, kmax rows of W words
    unsigned long long *used;     // bitset of mapped target nodes (W words)
};

__host__ __device__ inline unsigned even(unsigned x) { return x + (x & 1u); }

__device__ __forceinline__ DenseLds carve_dense(unsigned *base, unsigned kmax, unsigned W) {
    DenseLds u;
    u.M = base;
    u.fc = u.M + even(kmax);
    u.cand = reinterpret_cast<unsigned long long *>(u.fc + even(kmax));
    u.used = u.cand + (size_t)kmax * W;
    return u;
}

__device__ __forceinline__ bool used_test(const unsigned *used, unsigned v) { return (used[v >> 5] >> (v & 31)) & 1u; }

// is v a target neighbour of node a (row [b, b+deg))
__device__ __forceinline__ bool adjacent(const InstDesc &d, unsigned W, unsigned a, unsigned b, unsigned deg,
                                         unsigned v) {
    if (d.adj) return (d.adj[(size_t)a * W + (v >> 6)] >> (v & 63)) & 1ull;
    unsigned lo = b, hi = b + deg;
    while (lo < hi) {
        unsigned mid = (lo + hi) >> 1;
        unsigned x = d.col[mid];
        if (x < v) lo = mid + 1;
        else hi = mid;
    }
    return lo < b + deg && d.col[lo] == v;
}

// DENSE = false: candidate lists (CSR rows) evaluated G at a time, accepted
// candidates kept on a per-unit stack.  DENSE = true: each frame holds the set
// of accepted candidates as a bitset over the target nodes; expanding a mapped
// node ANDs the parent's adjacency row, the position's domain (or label and
// degree) row, the complement of the used set and every back-edge row, one
// 64-bit word per lane, and counts the result with popcounts.
template <int G, bool DENSE>
__global__ void __launch_bounds__(256) search_kernel(SearchArgs a) {
    extern __shared__ unsigned lds[];
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const int unit = threadIdx.x / G;
    UnitLds L{};
    DenseLds D{};
    if constexpr (DENSE) {
        D = carve_dense(lds + (size_t)unit * a.unit_words, a.kmax, a.W);
        for (unsigned i = gl; i < a.W; i += G) D.used[i] = 0;
        L.M = D.M;
    } else {
        L = carve(lds + (size_t)unit * a.unit_words, a.kmax, a.E, a.UW);
        for (unsigned i = gl; i < a.UW; i += G) L.used[i] = 0;
    }
    const unsigned WS = a.W;   // LDS row stride of the dense frames

    Sched *S = a.sched;
    const unsigned nchunks = a.chunk_prefix[a.ninst];
    if (threadIdx.x == 0) atomicMin(&S->t_start, now_ticks());
    if (nchunks == 0) {   // no root candidate anywhere: nothing to search
        if (lane == 0) atomicMax(&S->t_end, now_ticks());
        return;
    }

    // unit state (identical in the G lanes of a unit)
    unsigned inst = NO_TASK, cinst = NO_TASK, lvl = 0, base = 0, etop = 0, k = 0, W = 0;
    InstDesc d{};
    const DevPlan *P = nullptr;
    unsigned long long c_states = 0, c_matches = 0, c_cands = 0, c_steals = 0;
    bool roots_done = false;
    unsigned since_donate = 0;     // steps since this unit's task began or it last gave work away
    unsigned iter = 0, backoff = 0;
    bool donate_hint = false;
    // every wave ends by the deadline, whatever the state of the search
    const unsigned long long deadline = a.limit_ticks ? now_ticks() + a.limit_ticks : ~0ull;

    auto flush = [&]() {
        if (cinst != NO_TASK && gl == 0) {
            InstCounters *c = a.ctr + cinst;
            if (c_matches) fadd64(&c->matches, c_matches);
            if (c_cands) fadd64(&c->candidates, c_cands);
            if (c_steals) fadd64(&c->steals, c_steals);
            if (c_states) {
                unsigned long long before = fadd64(&c->states, c_states);
                if (a.state_cap && before + c_states > a.state_cap)
                    __hip_atomic_store(&c->pad0, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        c_states = c_matches = c_cands = c_steals = 0;
    };
    auto inst_aborted = [&](unsigned i) -> bool {
        unsigned long long f = 0;
        if (gl == 0) f = __hip_atomic_load(&a.ctr[i].pad0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return __shfl(f, gbase) != 0;
    };
    // open the frame of position `pos` (lists follow the mapped parent)
    auto open_frame = [&](unsigned pos, unsigned lo, unsigned hi) {
        int p = P->parent[pos];
        unsigned start, len;
        if (p >= 0) { start = L.MB[p]; len = L.MD[p]; }
        else { start = P->list_off[pos]; len = P->list_len[pos]; }
        unsigned e = (hi == FULL_RANGE || hi > len) ? len : hi;
        L.cur[pos] = lo;
        L.end[pos] = e;
        L.lb[pos] = start;
        L.eb[pos] = etop;
        L.dn[pos] = 0;
    };
    // give up the current task (used bits of the mapped prefix are cleared)
    auto mark = [&](unsigned v) {
        if constexpr (DENSE) atomicOr(&D.used[v >> 6], 1ull << (v & 63));
        else atomicOr(&L.used[v >> 5], 1u << (v & 31));
    };
    auto unmark = [&](unsigned v) {
        if constexpr (DENSE) atomicAnd(&D.used[v >> 6], ~(1ull << (v & 63)));
        else atomicAnd(&L.used[v >> 5], ~(1u << (v & 31)));
    };
    // dense: take the lowest member of frame f (group-uniform result)
    auto pick_lowest = [&](unsigned f) -> unsigned {
        unsigned v = 0xFFFFFFFFu;
        for (unsigned r = 0; r * G < W; r++) {
            const unsigned w = r * G + gl;
            unsigned long long x = w < W ? D.cand[(size_t)f * WS + w] : 0ull;
            unsigned long long b = group_mask<G>(__ballot(x != 0ull), gbase);
            if (b) {
                const unsigned j = (unsigned)__builtin_ctzll(b);
                const unsigned long long xw = __shfl(x, gbase + j);
                const unsigned word = r * G + j;
                v = word * 64 + (unsigned)__builtin_ctzll(xw);
                if ((unsigned)gl == j) D.cand[(size_t)f * WS + word] = xw & (xw - 1);
                break;
            }
        }
        // a frame is only read while its count is positive; should that ever
        // disagree with its bits, stay on a valid node index
        return v == 0xFFFFFFFFu ? 0u : v;
    };
    // dense: candidates of position `pos` given M[0..pos-1]; at the last position
    // they are counted (and emitted) as matches, otherwise they become frame pos
    auto expand = [&](unsigned pos) {
        const int p = P->parent[pos];
        const unsigned mp = p >= 0 ? D.M[p] : 0u;
        const unsigned long long bmask = P->back[pos];
        const bool last = pos + 1 == k;
        unsigned cnt = 0;
        for (unsigned r = 0; r * G < W; r++) {
            const unsigned w = r * G + gl;
            if (w < W) {
                unsigned long long x = d.bits[(size_t)pos * W + w] & ~D.used[w];
                if (p >= 0) x &= d.adj[(size_t)mp * W + w];
                unsigned long long bm = bmask;
                while (bm) {   // four back-edge rows per round, loads issued together
                    const unsigned j0 = (unsigned)__builtin_ctzll(bm);
                    bm &= bm - 1;
                    const unsigned j1 = bm ? (unsigned)__builtin_ctzll(bm) : j0;
                    bm &= bm ? bm - 1 : 0ull;
                    const unsigned j2 = bm ? (unsigned)__builtin_ctzll(bm) : j0;
                    bm &= bm ? bm - 1 : 0ull;
                    const unsigned j3 = bm ? (unsigned)__builtin_ctzll(bm) : j0;
                    bm &= bm ? bm - 1 : 0ull;
                    const unsigned long long a0 = d.adj[(size_t)D.M[j0] * W + w];
                    const unsigned long long a1 = d.adj[(size_t)D.M[j1] * W + w];
                    const unsigned long long a2 = d.adj[(size_t)D.M[j2] * W + w];
                    const unsigned long long a3 = d.adj[(size_t)D.M[j3] * W + w];
                    x &= a0 & a1 & a2 & a3;
                }
                if (!last) D.cand[(size_t)pos * WS + w] = x;
                cnt += (unsigned)__popcll(x);
                if (last && d.rows) {
                    for (unsigned long long y = x; y; y &= y - 1) {
                        const unsigned v = w * 64 + (unsigned)__builtin_ctzll(y);
                        unsigned long long slot = atomicAdd(&a.ctr[inst].row_next, 1ull);
                        if (slot < d.cap_rows) {
                            uint32_t *row = d.rows + slot * k;
                            for (unsigned i = 0; i + 1 < k; i++) row[P->order[i]] = D.M[i];
                            row[P->order[k - 1]] = v;
                        }
                    }
                }
            }
        }
        for (int o = G / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
        c_states += cnt;
        if (last) c_matches += cnt;
        D.fc[pos] = last ? 0u : cnt;
    };
    auto drop_task = [&](unsigned mapped) {
        WAVE_SYNC();
        for (unsigned i = gl; i < mapped; i += G) unmark(L.M[i]);
        if (gl == 0) release_task(S, nchunks);
        inst = NO_TASK;
        etop = 0;
    };

    while (true) {
        iter++;
        const unsigned long long idle_b = __ballot(inst == NO_TASK);
        const bool wave_idle = idle_b == ~0ull;
        // ------------------------------------------------ poll the scheduler (one lane per wave)
        const bool poll = idle_b != 0 && (wave_idle || (iter & 31) == 0);
        if (poll || (iter & 63) == 0) {
            unsigned flags = 0, av = 0, cn = 0, fr = 0;
            if (lane == 0) {
                if (now_ticks() > deadline) {
                    st_rlx(&S->abort, 1u);
                    flags |= 1;
                }
                if (ld_rlx(&S->abort)) flags |= 1;
                if (ld_rlx(&S->done)) flags |= 2;
                av = ld_rlx(&S->q_avail);
                cn = ld_rlx(&S->chunk_next);
                fr = ld_rlx(&S->q_free);
            }
            flags = __shfl(flags, 0);
            av = __shfl(av, 0);
            cn = __shfl(cn, 0);
            fr = __shfl(fr, 0);
            if (flags & 1) break;                    // time limit: every wave stops
            if ((flags & 2) && wave_idle) break;     // the search is complete
            // give work away only once the roots are all claimed and the queue runs low
            donate_hint = a.donate && cn >= nchunks && av < 64 && fr > 256;
            if (poll && (av > 0 || cn < nchunks)) {
                // ---------------------------------------- task acquisition, one unit at a time
                for (int g = 0; g < 64 / G; g++) {
                    if (!(inst == NO_TASK && (lane / G) == g)) continue;
                    unsigned kind = 0, val = 0;
                    if (gl == 0) {
                        if (av > 0 && cas_dec_if_pos(&S->q_avail)) {
                            unsigned t = fadd(&S->q_head, 1);
                            unsigned slot = t % QUEUE_SLOTS;
                            kind = 1;
                            while (ld_rlx(&a.queue[slot].seq) != 2 * t + 1) {
                                __builtin_amdgcn_s_sleep(1);
                                if (now_ticks() > deadline) { kind = 0; break; }
                            }
                            fence_acq();
                            val = t;
                        } else if (!roots_done && cn < nchunks) {
                            fadd(&S->work, 1);
                            unsigned c = fadd_ar(&S->chunk_next, 1);
                            if (c < nchunks) {
                                kind = 2;
                                val = c;
                            } else {
                                roots_done = true;
                                release_task(S, nchunks);
                            }
                        }
                    }
                    kind = __shfl(kind, gbase);
                    val = __shfl(val, gbase);
                    roots_done = __shfl((int)roots_done, gbase) != 0;
                    if (kind == 0) continue;
                    unsigned ti = 0, tL = 0, tlo = 0, thi = 0;
                    if (kind == 1) {
                        QTask *q = a.queue + (val % QUEUE_SLOTS);
                        ti = q->inst;
                        tL = q->L;
                        tlo = q->lo;
                        thi = q->hi;
                        for (unsigned i = gl; i < tL; i += G) L.M[i] = q->M[i];
                        fence_rel();
                        if (gl == 0) {
                            st_rlx(&q->seq, 2 * (val + QUEUE_SLOTS));
                            fadd(&S->q_free, 1);
                        }
                    } else {
                        unsigned lo = 0, hi = a.ninst;   // largest i with prefix[i] <= val
                        if (gl == 0) {
                            while (hi - lo > 1) {
                                unsigned mid = (lo + hi) >> 1;
                                if (a.chunk_prefix[mid] <= val) lo = mid;
                                else hi = mid;
                            }
                        }
                        ti = __shfl(lo, gbase);
                        const InstDesc &dd = a.inst[ti];
                        tlo = (val - a.chunk_prefix[ti]) * dd.chunk;
                        thi = min(tlo + dd.chunk, dd.nroot);
                    }
                    // start the task
                    if (ti != cinst) {
                        flush();
                        cinst = ti;
                        d = a.inst[ti];
                        P = d.plan;
                        k = P->k;
                        W = P->W;
                    }
                    inst = ti;
                    since_donate = 0;
                    if (kind == 1) c_steals++;
                    etop = 0;
                    if (a.state_cap && inst_aborted(inst)) {   // capped instance: drop the task
                        if (gl == 0) release_task(S, nchunks);
                        inst = NO_TASK;
                        continue;
                    }
                    if constexpr (DENSE) {
                        for (unsigned i = gl; i < tL; i += G) mark(D.M[i]);
                        WAVE_SYNC();
                        base = lvl = tL;
                        if (tL == 0) {
                            // a root chunk: its list entries are the accepted candidates of position 0
                            for (unsigned w = gl; w < W; w += G) D.cand[w] = 0ull;
                            WAVE_SYNC();
                            const uint32_t *lst = d.lists + P->list_off[0] + tlo;
                            const unsigned cnt = thi - tlo;
                            for (unsigned i = gl; i < cnt; i += G) {
                                const unsigned v = lst[i];
                                atomicOr(&D.cand[v >> 6], 1ull << (v & 63));
                                if (k == 1 && d.rows) {
                                    unsigned long long slot = atomicAdd(&a.ctr[inst].row_next, 1ull);
                                    if (slot < d.cap_rows) d.rows[slot] = v;
                                }
                            }
                            c_states += cnt;
                            if (k == 1) c_matches += cnt;
                            D.fc[0] = k == 1 ? 0u : cnt;
                        } else {
                            expand(tL);
                        }
                        WAVE_SYNC();
                    } else {
                        for (unsigned i = gl; i < tL; i += G) {
                            unsigned v = L.M[i];
                            NodeRec r = d.node[v];
                            L.MB[i] = r.begin;
                            L.MD[i] = r.deg;
                            mark(v);
                        }
                        WAVE_SYNC();
                        base = lvl = tL;
                        open_frame(tL, tlo, thi);
                    }
                }
            }
        }
        if (__ballot(inst != NO_TASK) == 0) {
            // the whole wave is idle: back off before polling again
            backoff = backoff < 8 ? backoff + 1 : 8;
            for (unsigned z = 0; z < backoff; z++) __builtin_amdgcn_s_sleep(32);
            continue;
        }
        backoff = 0;
        if (inst == NO_TASK) continue;

        // ------------------------------------------------ one search step
        WAVE_SYNC();
        since_donate++;
        if constexpr (DENSE) {
            // pop exhausted frames
            bool task_done = false;
            while (true) {
                if (D.fc[lvl] > 0) break;
                if (lvl == base) { task_done = true; break; }
                lvl--;
                if (gl == 0) unmark(D.M[lvl]);
            }
            if (task_done) {
                if (c_states >= 4096) flush();
                drop_task(base);
                continue;
            }
            // map the lowest remaining candidate and expand the next position
            const unsigned v = pick_lowest(lvl);
            D.fc[lvl] = D.fc[lvl] - 1;
            D.M[lvl] = v;
            if (gl == 0) mark(v);
            WAVE_SYNC();
            expand(lvl + 1);
            if (lvl + 2 == k) {
                if (gl == 0) unmark(v);   // the last position was counted; stay on this frame
            } else {
                lvl++;
            }
        } else {
            // pop exhausted frames
            bool task_done = false;
            while (true) {
                if (etop > L.eb[lvl] + L.dn[lvl]) break;
                etop = L.eb[lvl];   // reclaim entries given away from this frame
                L.dn[lvl] = 0;
                if (L.cur[lvl] < L.end[lvl]) break;
                if (lvl == base) { task_done = true; break; }
                lvl--;
                if (gl == 0) unmark(L.M[lvl]);
            }
            if (task_done) {
                if (c_states >= 4096) flush();
                drop_task(base);
                continue;
            }
            // map the top accepted candidate and open the next frame
            if (etop > L.eb[lvl] + L.dn[lvl]) {
                etop--;
                unsigned v = L.ev[etop];
                L.M[lvl] = v;
                L.MB[lvl] = L.ebg[etop];
                L.MD[lvl] = L.edg[etop];
                if (gl == 0) mark(v);
                lvl++;
                open_frame(lvl, 0, FULL_RANGE);
            }
            // evaluate up to G candidates of the current frame
            {
                const unsigned c0 = L.cur[lvl], e = L.end[lvl], lb = L.lb[lvl];
                const unsigned idx = c0 + gl;
                bool ok = idx < e;
                const bool has_parent = P->parent[lvl] >= 0;
                unsigned v = 0;
                NodeRec r{0, 0, 0, 0};
                if (ok) {
                    v = has_parent ? d.col[lb + idx] : d.lists[lb + idx];
                    r = d.node[v];
                }
                if (ok && d.bits) ok = (d.bits[(size_t)lvl * W + (v >> 6)] >> (v & 63)) & 1ull;
                if (ok) ok = !used_test(L.used, v);
                const unsigned pl = P->plabel[lvl];
                if (ok && pl != LABEL_ANY) ok = r.label == pl;
                if (ok) ok = r.deg >= P->pdeg[lvl];
                unsigned long long bm = P->back[lvl];
                while (bm) {
                    unsigned j = (unsigned)__builtin_ctzll(bm);
                    bm &= bm - 1;
                    if (ok) ok = adjacent(d, W, L.M[j], L.MB[j], L.MD[j], v);
                }
                c_cands += min((unsigned)G, e - c0);
                unsigned long long acc = group_mask<G>(__ballot(ok), gbase);
                unsigned cnt = (unsigned)__popcll(acc);
                if (lvl + 1 == k) {
                    c_states += cnt;
                    c_matches += cnt;
                    if (d.rows && ok) {
                        unsigned long long slot = atomicAdd(&a.ctr[inst].row_next, 1ull);
                        if (slot < d.cap_rows) {
                            uint32_t *row = d.rows + slot * k;
                            for (unsigned i = 0; i + 1 < k; i++) row[P->order[i]] = L.M[i];
                            row[P->order[k - 1]] = v;
                        }
                    }
                    L.cur[lvl] = c0 + G;
                } else {
                    int room = (int)a.E - (int)etop - (int)(k - 2 - lvl);
                    unsigned take = cnt;
                    unsigned long long keep = acc;
                    unsigned ncur = c0 + G;
                    if ((int)take > room) {
                        take = (unsigned)room;
                        unsigned long long m = acc;
                        for (unsigned i = 0; i < take; i++) m &= m - 1;
                        keep = acc & ~m;                       // the first `take` accepted lanes
                        ncur = c0 + (63u - (unsigned)__clzll(keep)) + 1;
                    }
                    if ((keep >> gl) & 1ull) {
                        unsigned rank = (unsigned)__popcll(keep & ((1ull << gl) - 1));
                        L.ev[etop + rank] = v;
                        L.ebg[etop + rank] = r.begin;
                        L.edg[etop + rank] = r.deg;
                    }
                    etop += take;
                    c_states += take;
                    L.cur[lvl] = ncur;
                }
            }
        }

        // counters: flush now and then so a state cap takes effect
        if (c_states >= 8192) {
            flush();
            if (a.state_cap && inst_aborted(inst)) {
                drop_task(lvl);
                continue;
            }
        }

        // ------------------------------------------------ donation (one unit at a time)
        if (donate_hint && (iter & 15) == 0 && __ballot(since_donate >= 256) != 0) {
            for (int g = 0; g < 64 / G; g++) {
                if (!((lane / G) == g && inst != NO_TASK && since_donate >= 256)) continue;
                // shallowest frame with untried candidates or a spare accepted one
                unsigned f = base, kind = 0;
                for (; f <= lvl; f++) {
                    if constexpr (DENSE) {
                        if (D.fc[f] > (f == lvl ? 1u : 0u)) { kind = 2; break; }
                    } else {
                        if (L.cur[f] < L.end[f]) { kind = 1; break; }
                        unsigned top = f < lvl ? L.eb[f + 1] : etop;
                        unsigned live = top - (L.eb[f] + L.dn[f]);
                        if (live > (f == lvl ? 1u : 0u)) { kind = 2; break; }
                    }
                }
                if (!kind) continue;
                unsigned t = 0, okr = 0;
                if (gl == 0) {
                    if (cas_dec_if_pos(&S->q_free)) {
                        fadd(&S->work, 1);
                        t = fadd(&S->q_tail, 1);
                        okr = 1;
                        while (ld_rlx(&a.queue[t % QUEUE_SLOTS].seq) != 2 * t) {
                            __builtin_amdgcn_s_sleep(1);
                            if (now_ticks() > deadline) { okr = 0; break; }
                        }
                        fence_acq();
                    }
                }
                if (!__shfl(okr, gbase)) continue;
                t = __shfl(t, gbase);
                WAVE_SYNC();
                since_donate = 0;
                QTask *q = a.queue + (t % QUEUE_SLOTS);
                unsigned tL, tlo, thi, extra = 0;
                if constexpr (DENSE) {
                    extra = pick_lowest(f);
                    D.fc[f] = D.fc[f] - 1;
                    tL = f + 1;
                    tlo = 0;
                    thi = FULL_RANGE;
                } else if (kind == 1) {
                    unsigned c = L.cur[f], e = L.end[f];
                    unsigned mid = c + (e - c) / 2;
                    tL = f;
                    tlo = mid;
                    thi = e;
                    L.end[f] = mid;
                } else {
                    unsigned idx = L.eb[f] + L.dn[f];
                    L.dn[f] = L.dn[f] + 1;
                    extra = L.ev[idx];
                    tL = f + 1;
                    tlo = 0;
                    thi = FULL_RANGE;
                }
                for (unsigned i = gl; i < f; i += G) q->M[i] = L.M[i];
                if (kind == 2 && gl == 0) q->M[f] = extra;
                if (gl == 0) {
                    q->inst = inst;
                    q->L = tL;
                    q->lo = tlo;
                    q->hi = thi;
                }
                fence_rel();
                if (gl == 0) {
                    st_rlx(&q->seq, 2 * t + 1);
                    fadd(&S->q_avail, 1);
                }
            }
        }
    }
    flush();
    if (lane == 0) atomicMax(&S->t_end, now_ticks());
}

__global__ void reset_kernel(Sched *s, InstCounters *c, unsigned ninst, QTask *q) {
    unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned stride = gridDim.x * blockDim.x;
    if (blockIdx.x == 0) {
        unsigned *w = reinterpret_cast<unsigned *>(s);
        for (unsigned j = threadIdx.x; j < sizeof(Sched) / 4; j += blockDim.x) w[j] = 0;
        __syncthreads();
        if (threadIdx.x == 0) {
            s->q_free = QUEUE_SLOTS;
            s->t_start = ~0ull;
        }
    }
    for (unsigned j = i; j < ninst; j += stride) c[j] = InstCounters{0, 0, 0, 0, 0, 0, 0, 0};
    for (unsigned j = i; j < QUEUE_SLOTS; j += stride) q[j].seq = 2 * j;
}

template <int G, bool DENSE>
hipError_t launch_g(const SearchArgs &args, int blocks, int threads, size_t lds, hipStream_t s, int num_cus,
                    uint32_t total_chunks) {
    if (blocks <= 0) {
        // resident blocks only (a persistent grid), and no more than the root
        // chunks can keep busy before work is handed around
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, search_kernel<G, DENSE>, threads, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        int units_per_block = threads / G;
        long want = (4L * total_chunks + units_per_block - 1) / units_per_block;
        if (want < 2L * num_cus) want = 2L * num_cus;
        blocks = (int)std::min<long>((long)per_cu * num_cus, want);
    }
    hipLaunchKernelGGL((search_kernel<G, DENSE>), dim3(blocks), dim3(threads), lds, s, args);
    return hipGetLastError();
}

unsigned unit_words(const LaunchCfg &cfg) {
    if (cfg.dense) return 2 * even(cfg.kmax) + 2 * cfg.kmax * cfg.wmax + 2 * cfg.wmax;
    unsigned E = cfg.kmax + cfg.lanes;
    unsigned UW = (cfg.nmax + 31) / 32;
    return 8 * cfg.kmax + 3 * E + UW + 8;
}

// Largest block (256, 128 or 64 threads) whose units fit in 64 KiB of LDS.
int block_threads(const LaunchCfg &cfg) {
    size_t per_unit = (size_t)unit_words(cfg) * 4;
    for (int t = 256; t >= 64; t /= 2)
        if (per_unit * (t / cfg.lanes) <= 65536) return t;
    return 0;
}

}  // namespace

size_t search_lds_bytes(const LaunchCfg &cfg) {
    int t = block_threads(cfg);
    return (size_t)unit_words(cfg) * 4 * (size_t)((t ? t : 64) / cfg.lanes);
}

hipError_t launch_reset(DevWork &w, uint32_t ninst, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3(64), dim3(256), 0, s, w.sched, w.ctr, ninst, w.queue);
    return hipGetLastError();
}

hipError_t launch_search(const LaunchCfg &cfg, DevWork &w, uint32_t ninst, uint32_t total_chunks,
                         uint64_t state_cap, uint64_t time_limit_ms, hipStream_t s, int num_cus) {
    SearchArgs a{};
    a.inst = w.inst;
    a.chunk_prefix = w.chunk_prefix;
    a.ctr = w.ctr;
    a.sched = w.sched;
    a.queue = w.queue;
    a.ninst = ninst;
    a.kmax = cfg.kmax;
    a.E = cfg.kmax + cfg.lanes;
    a.UW = (cfg.nmax + 31) / 32;
    a.W = cfg.dense ? cfg.wmax : 0;
    a.unit_words = unit_words(cfg);
    a.donate = cfg.donate;
    a.state_cap = state_cap;
    a.limit_ticks = time_limit_ms * 100000ull;   // s_memrealtime runs at 100 MHz
    const int threads = block_threads(cfg);
    if (!threads) return hipErrorInvalidValue;   // one unit's LDS does not fit
    size_t lds = search_lds_bytes(cfg);
    int blocks = cfg.blocks;
    if (cfg.dense) {
        switch (cfg.lanes) {
            case 8: return launch_g<8, true>(a, blocks, threads, lds, s, num_cus, total_chunks);
            case 16: return launch_g<16, true>(a, blocks, threads, lds, s, num_cus, total_chunks);
            case 32: return launch_g<32, true>(a, blocks, threads, lds, s, num_cus, total_chunks);
            case 64: return launch_g<64, true>(a, blocks, threads, lds, s, num_cus, total_chunks);
            default: return hipErrorInvalidValue;
        }
    }
    switch (cfg.lanes) {
        case 8: return launch_g<8, false>(a, blocks, threads, lds, s, num_cus, total_chunks);
        case 16: return launch_g<16, false>(a, blocks, threads, lds, s, num_cus, total_chunks);
        case 32: return launch_g<32, false>(a, blocks, threads, lds, s, num_cus, total_chunks);
        case 64: return launch_g<64, false>(a, blocks, threads, lds, s, num_cus, total_chunks);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sge
