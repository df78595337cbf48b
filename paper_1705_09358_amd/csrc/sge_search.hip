// Persistent depth-first search kernels for RI / RI-DS subgraph enumeration on
// gfx950.
//
// Search unit.  A unit is a group of G lanes of a 64-lane wavefront (G = 8,
// 16, 32 or 64); a wave holds 64/G units that advance in lock-step through
// one loop, each on its own subtree.  The traversal is the state space of
// Section 2.2.1, depth-first, with RI's candidate generation (the target
// neighbours of the mapped parent; all nodes, or the domain, for a node
// without a parent) and pruning rules in the paper's order (unused, label,
// degree, edges to mapped nodes), plus the RI-DS domain test first
// (Section 4.1).  Two variants share the scheduling loop:
//
//  * CSR (DENSE = false).  A unit owns, in LDS, the mapping M of the current
//    prefix (by order position), one frame per position and a small stack of
//    accepted-but-unexplored candidates.  One step: pop exhausted frames; map
//    the top stacked candidate and open the next position's frame; evaluate
//    the next G candidates of the current frame, one per lane, and push the
//    accepted ones (at the last position, count and emit them instead).
//    States are counted when pushed, so a candidate that did not fit in the
//    stack is evaluated again later without being counted twice.
//  * Dense bitsets (DENSE = true).  Each frame holds the accepted candidates
//    of a position as a bitset over the target nodes; mapping the lowest
//    member and expanding the next position ANDs the parent's adjacency row,
//    the position's domain (or label and degree) row, the complement of the
//    used set and every back-edge row, one 64-bit word per lane, and counts
//    the result with popcounts.
//
// Load balance.  Root candidates (position 0) are handed out in chunks from
// an atomic counter (the paper's initial distribution, Section 3.3; chunks
// play the role of task groups, Section 3.4).  Busy units give work away to
// work-queue groups when their group runs low, near the root as in the
// paper's stealing from the back of a deque (Section 3.2), and in bulk: half
// of the untried candidates of their shallowest open frame, up to 16 of its
// accepted candidates, or (dense) half of its remaining candidate words.  A
// queued task carries its prefix mapping, so only moved work copies a
// mapping (Section 3.1).  A block's home group is blockIdx mod 8; idle units
// look at their home group first and then at the others.
//
// Termination (in place of the token ring of Section 3.5).  Each group counts,
// monotonically, the tasks given away into it and the tasks finished (root
// chunks included).  A task is created only by a unit that holds an
// unfinished task, and every creation precedes its own finish, so once all
// root chunks are claimed, reading the finished counts and then the created
// counts and finding finished = chunks + created means no task is left.
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
    unsigned donate_period;           // a unit gives work away at most once per this many of its steps
    unsigned long long state_cap;
    unsigned long long limit_ticks;   // time limit in s_memrealtime ticks (100 MHz); 0 = none
    unsigned min_blocks;              // blocks kept whatever the number of root chunks
    unsigned units_per_block;
    unsigned count_bytes;             // count the algorithmic bytes of the search (InstCounters::bytes)
    unsigned check_uniform;           // verify every step that per-unit values agree across the unit's lanes
    unsigned root_lo, root_hi;        // the first position's target-id range
};

constexpr unsigned FULL_RANGE = 0xFFFFFFFFu;
constexpr unsigned NO_TASK = 0xFFFFFFFFu;
constexpr unsigned NO_GROUP = 0xFFFFFFFFu;
// task kinds (QTask::kind)
constexpr unsigned TK_RANGE = 0;     // CSR: candidates [lo, hi) of position L; dense: expand position L
constexpr unsigned TK_ENTRIES = 1;   // CSR: `ne` accepted candidates of position L
constexpr unsigned TK_WINDOW = 2;    // dense: words [lo, hi) of position L's candidate set

__device__ __forceinline__ unsigned ld_rlx(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
// Waits until every memory operation this wave has issued is complete.
// Queue payloads and scheduler counters are read and written only with
// agent-scope atomics, which are coherent across the XCDs' L2 caches, so a
// completed store is visible to every later agent-scope load.  Ordering them
// with this wait instead of agent-scope fences keeps the L2 of the XCD intact:
// an acquire fence invalidates it and a release fence writes it back, and at
// the rate tasks move that costs the searching waves their cached graph.
__device__ __forceinline__ void vm_drain() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
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

// Timing stamps shared by every wave: read first, so that only a stamp that
// moves the value takes the atomic (thousands of waves start and exit at
// nearly the same time, and atomics on one word serialise)
__device__ __forceinline__ void stamp_min(unsigned long long *p, unsigned long long t) {
    if (t < __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(p, t);
}
__device__ __forceinline__ void stamp_max(unsigned long long *p, unsigned long long t) {
    if (t > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, t);
}

template <int G>
__device__ __forceinline__ unsigned long long group_mask(unsigned long long ballot, int gbase) {
    if constexpr (G == 64) return ballot;
    else return (ballot >> gbase) & ((1ull << G) - 1);
}

template <int G>
__device__ __forceinline__ unsigned group_sum(unsigned x) {
    for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
template <int G>
__device__ __forceinline__ unsigned long long group_sum64(unsigned long long x) {
    for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Per-unit LDS arrays of the CSR variant.
struct UnitLds {
    unsigned long long *pback;    // the current instance's plan by position: back-edge masks,
    int *ppd;                     //   parent positions (high half, -1: none) and degrees (low half),
    unsigned *plab;               //   labels (copied when the unit changes instance)
    unsigned *M, *MB, *MD;        // mapping by position, row start and degree of M[i]
    unsigned *cur, *end, *lb;     // frame: next candidate index, list length, list start
    unsigned *eb, *dn;            // frame: first stack entry, entries given away from the bottom
    unsigned *ev, *ebg, *edg;     // stack of accepted candidates: node, row start, degree
    unsigned long long *tim;      // this unit's task start, time holding tasks, last task finish
    unsigned *used;               // bitset of mapped target nodes
};

// The layout is fixed at KMAX positions and KMAX + G stack entries, so
// every array is the unit's base plus a compile-time offset: one register
// addresses all of them (immediate offsets of the LDS instructions).
template <int G>
__device__ __forceinline__ UnitLds carve(unsigned *base) {
    constexpr unsigned kmax = KMAX, E = KMAX + G;
    UnitLds u;
    u.pback = reinterpret_cast<unsigned long long *>(base);   // the unit's area starts 8-byte aligned
    u.ppd = reinterpret_cast<int *>(base + 2 * kmax);
    u.plab = base + 3 * kmax;
    u.M = base + 4 * kmax;
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
    u.tim = reinterpret_cast<unsigned long long *>(u.edg + E);   // 8-byte aligned: 12 kmax + 3 E is even
    u.used = u.edg + E + 6;
    return u;
}

// Per-unit LDS arrays of the dense variant.
struct DenseLds {
    unsigned *M;                  // mapping by position
    unsigned *fc;                 // frame: number of candidates left
    unsigned *hw;                 // frame: words at or above this index were given away
    unsigned long long *cand;     // frame: candidate set, kmax rows of W words
    unsigned long long *used;     // bitset of mapped target nodes (W words)
    unsigned long long *tim;      // this unit's task start, time holding tasks, last task finish
    unsigned *hdr;                // the header of a piece handed over by a wave-mate
};

__host__ __device__ inline unsigned even(unsigned x) { return x + (x & 1u); }

__device__ __forceinline__ DenseLds carve_dense(unsigned *base, unsigned kmax, unsigned W) {
    DenseLds u;
    u.M = base;
    u.fc = u.M + even(kmax);
    u.hw = u.fc + even(kmax);
    u.cand = reinterpret_cast<unsigned long long *>(u.hw + even(kmax));
    u.used = u.cand + (size_t)kmax * W;
    u.tim = u.used + W;
    u.hdr = reinterpret_cast<unsigned *>(u.tim + 3);
    return u;
}

__device__ __forceinline__ bool used_test(const unsigned *used, unsigned v) { return (used[v >> 5] >> (v & 31)) & 1u; }

// is v a target neighbour of node a (row [b, b+deg))
// Device memory in the global address space.  Pointers that the kernel loads
// from memory (an instance's descriptor and plan) are generic to the compiler,
// and a generic (flat) access waits on both the vector-memory and the LDS
// counters, which would hold a step's LDS work behind its outstanding loads.
template <class T>
using gp = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gp<T> glob(T *p) {
    return (gp<T>)p;
}

// 16-byte records in one load
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ NodeRec ld_node(gp<const NodeRec> p) {
    const u32x4 x = *(gp<const u32x4>)p;
    return NodeRec{x.x, x.y, x.z, x.w};
}
__device__ __forceinline__ WideEntry ld_wide(gp<const WideEntry> p) {
    const u32x4 x = *(gp<const u32x4>)p;
    return WideEntry{x.x, x.y, x.z, x.w};
}

// An instance's search descriptor with global-address-space pointers.
struct GDesc {
    gp<const uint32_t> col;
    gp<const NodeRec> node;
    gp<const WideEntry> wcol;
    gp<const uint32_t> irp, icol, elab, ielab, lmat;
    gp<const uint64_t> adj;
    gp<const DevPlan> plan;
    gp<const uint64_t> bits;
    gp<const uint32_t> lists;
    gp<uint32_t> rows;
    unsigned long long cap_rows;
};
__device__ __forceinline__ GDesc gdesc(gp<const InstDesc> s) {
    GDesc d;
    d.col = glob(s->col);
    d.node = glob(s->node);
    d.wcol = glob(s->wcol);
    d.irp = glob(s->irp);
    d.icol = glob(s->icol);
    d.elab = glob(s->elab);
    d.ielab = glob(s->ielab);
    d.lmat = glob(s->lmat);
    d.adj = glob(s->adj);
    d.plan = glob(s->plan);
    d.bits = glob(s->bits);
    d.lists = glob(s->lists);
    d.rows = glob(s->rows);
    d.cap_rows = s->cap_rows;
    return d;
}

__device__ __forceinline__ bool adjacent(const GDesc &d, unsigned W, unsigned a, unsigned b, unsigned deg,
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

// is there a target arc from the node whose out-row is [b, b+deg) to v; with
// `check`, the arc's label must be `want` (rule 4 for general graphs)
__device__ __forceinline__ bool arc_to(const GDesc &d, unsigned b, unsigned deg, unsigned v, bool check,
                                       unsigned want) {
    unsigned lo = b, hi = b + deg;
    while (lo < hi) {
        const unsigned mid = (lo + hi) >> 1;
        if (d.col[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    if (lo >= b + deg || d.col[lo] != v) return false;
    return !check || (d.elab ? d.elab[lo] : 0u) == want;
}

// GEN: the launch holds plans with PLAN_DIRECTED or PLAN_EDGE_LABELS (CSR
// only); other launches compile without those checks.
template <int G, bool DENSE, bool GEN>
__global__ void __launch_bounds__(256, DENSE ? 4 : 1) search_kernel(SearchArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned lds[];
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
        L.tim = D.tim;
    } else {
        L = carve<G>(lds + (size_t)unit * a.unit_words);
        for (unsigned i = gl; i < a.UW; i += G) L.used[i] = 0;
    }
    // the unit's timing words live in LDS (written once per task)
    if (gl < 3) L.tim[gl] = 0;
    const unsigned WS = a.W;   // LDS row stride of the dense frames

    Sched *S = a.sched;
    const unsigned nchunks = a.chunk_prefix[a.ninst];
    // blocks beyond four units per root chunk (and the minimum) have nothing to start with
    const unsigned long long want = (4ull * nchunks + a.units_per_block - 1) / a.units_per_block;
    if (blockIdx.x >= max((unsigned long long)min(gridDim.x, a.min_blocks), want)) return;
    if (threadIdx.x == 0) stamp_min(&S->t_start, now_ticks());
    if (a.count_bytes && blockIdx.x == 0) {
        // the first position's expansion, once per searched instance: dense,
        // its domain row; CSR, 5 bytes per target id of the root range (RI:
        // label and degree of every node) or 4 + 8 bytes per domain member
        // (RI-DS: the list and the domain word)
        for (unsigned j = threadIdx.x; j < a.ninst; j += blockDim.x) {
            const gp<const DevPlan> pj = glob(glob(a.inst)[j].plan);
            if (pj->empty) continue;
            unsigned long long b;
            if constexpr (DENSE) {
                b = 8ull * pj->W;
            } else if (pj->use_dom) {
                b = 12ull * pj->list_len[0];
            } else {
                const unsigned n = pj->n;
                b = 5ull * (min(a.root_hi, n) - min(a.root_lo, n));
            }
            if (b) fadd64(&a.ctr[j].bytes, b);
        }
    }
    if (nchunks == 0) {   // no root candidate anywhere: nothing to search
        if (lane == 0) stamp_max(&S->t_end, now_ticks());
        return;
    }
    const unsigned home = blockIdx.x % QUEUE_GROUPS;
    QGroup *HG = &S->grp[home];
    if (threadIdx.x == 0) fadd(&S->units, blockDim.x / G);   // every unit of the block enters the loop
    const bool checker = blockIdx.x == 0 && threadIdx.x < 64;   // the wave that detects termination

    // unit state (identical in the G lanes of a unit)
    unsigned inst = NO_TASK, cinst = NO_TASK, lvl = 0, base = 0, etop = 0, k = 0, W = 0;
    GDesc d{};
    gp<const DevPlan> P = nullptr;
    // counts not yet added to the instance's counters: 32 bits, flushed at
    // 8192 states or 2^20 steps (so no count can wrap)
    unsigned c_states = 0, c_matches = 0, c_cands = 0, c_steals = 0, c_steps = 0;
    // algorithmic bytes (counted when a.count_bytes): c_bytes per unit (the
    // same in its lanes), lane_bytes per lane (at most 2^20 steps of under
    // 600 bytes), summed over the unit at a flush
    unsigned long long c_bytes = 0;
    unsigned lane_bytes = 0;
    bool roots_done = false;
    unsigned since_donate = 0;     // steps since this unit's task began or it last gave work away
    unsigned iter = 0, backoff = 0, polls = 0;
    bool donate_hint = false;
    unsigned cn_seen = 0;          // the root chunk counter as this wave last read it
    // timing of this unit's tasks, in LDS: tim[0] start of the current task,
    // tim[1] ticks spent holding tasks, tim[2] the last task's finish
    // every wave ends by the deadline, whatever the state of the search
    const unsigned long long deadline = a.limit_ticks ? now_ticks() + a.limit_ticks : ~0ull;

    // every lane of the unit is here, so the per-lane bytes can be summed
    auto flush = [&]() {
        if (a.count_bytes) {
            c_bytes += group_sum64<G>((unsigned long long)lane_bytes);
            lane_bytes = 0;
        }
        if (cinst != NO_TASK && gl == 0) {
            InstCounters *c = a.ctr + cinst;
            if (c_bytes) fadd64(&c->bytes, c_bytes);
            if (c_matches) fadd64(&c->matches, c_matches);
            if (c_cands) fadd64(&c->candidates, c_cands);
            if (c_steals) fadd64(&c->steals, c_steals);
            if (c_steps) fadd64(&c->steps, c_steps);
            if (c_states) {
                unsigned long long before = fadd64(&c->states, c_states);
                if (a.state_cap && before + c_states > a.state_cap)
                    __hip_atomic_store(&c->pad0, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        c_states = c_matches = c_cands = c_steals = c_steps = c_bytes = 0;
    };
    auto inst_aborted = [&](unsigned i) -> bool {
        unsigned long long f = 0;
        if (gl == 0) f = __hip_atomic_load(&a.ctr[i].pad0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return __shfl(f, gbase) != 0;
    };
    // the parent position packed with the pattern degree (-1: none)
    auto parent_at = [](int ppd) -> int { return ppd >> 16; };
    // open the frame of position `pos` (lists follow the mapped parent)
    // returns the frame's end and list start (also kept in LDS)
    auto open_frame = [&](unsigned pos, unsigned lo, unsigned hi) -> uint2 {
        const int p = parent_at(L.ppd[pos]);
        unsigned start, len;
        if (p >= 0) {
            if (GEN && (P->flags & PLAN_DIRECTED) && !((P->pdir_out >> pos) & 1ull) && d.irp) {
                // the pattern arc points at the parent: its image's in-neighbours
                // (an undirected target's rows hold both directions)
                const unsigned mp = L.M[p];
                start = d.irp[mp];
                len = d.irp[mp + 1] - start;
            } else {
                start = L.MB[p];
                len = L.MD[p];
            }
        } else {
            start = P->list_off[pos];
            len = P->list_len[pos];
        }
        unsigned e = (hi == FULL_RANGE || hi > len) ? len : hi;
        L.cur[pos] = lo;
        L.end[pos] = e;
        L.lb[pos] = start;
        L.eb[pos] = etop;
        L.dn[pos] = 0;
        return make_uint2(e, start);
    };
    // the used-node set (CSR without a bitset: the mapped prefix itself)
    auto mark = [&](unsigned v) {
        if constexpr (DENSE) atomicOr(&D.used[v >> 6], 1ull << (v & 63));
        else if (a.UW) atomicOr(&L.used[v >> 5], 1u << (v & 31));
    };
    auto unmark = [&](unsigned v) {
        if constexpr (DENSE) atomicAnd(&D.used[v >> 6], ~(1ull << (v & 63)));
        else if (a.UW) atomicAnd(&L.used[v >> 5], ~(1u << (v & 31)));
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
    // dense: what a unit gives away from frame f, for the queue or a wave-mate:
    // half of the frame's remaining words above its lowest nonzero word
    // (within the words it still owns; TK_WINDOW over [tlo, thi) of position
    // f), else its lowest candidate (`extra`, mapped at position f: the
    // receiver expands position f + 1)
    auto dense_split = [&](unsigned f, unsigned &tL, unsigned &tlo, unsigned &thi, unsigned &tkind,
                           unsigned &extra) {
        const unsigned hw = D.hw[f];
        unsigned w0 = hw, nz_hi = 0;
        for (unsigned r = 0; r * G < hw; r++) {
            const unsigned w = r * G + gl;
            const bool nz = w < hw && D.cand[(size_t)f * WS + w] != 0ull;
            const unsigned long long b = group_mask<G>(__ballot(nz), gbase);
            if (b && w0 == hw) w0 = r * G + (unsigned)__builtin_ctzll(b);
        }
        for (unsigned r = 0; r * G < hw; r++) {
            const unsigned w = r * G + gl;
            if (w < hw && w > w0 && D.cand[(size_t)f * WS + w] != 0ull) nz_hi++;
        }
        nz_hi = group_sum<G>(nz_hi);
        tL = f;
        tlo = 0;
        thi = FULL_RANGE;
        tkind = TK_RANGE;
        extra = 0;
        if (nz_hi) {
            unsigned wmid = w0 + 1 + (hw - w0 - 1) / 2;
            unsigned moved = 0;
            for (unsigned r = 0; r * G < hw; r++) {
                const unsigned w = r * G + gl;
                if (w < hw && w >= wmid) moved += (unsigned)__popcll(D.cand[(size_t)f * WS + w]);
            }
            moved = group_sum<G>(moved);
            if (!moved) {
                wmid = w0 + 1;
                for (unsigned r = 0; r * G < hw; r++) {
                    const unsigned w = r * G + gl;
                    if (w < hw && w >= wmid) moved += (unsigned)__popcll(D.cand[(size_t)f * WS + w]);
                }
                moved = group_sum<G>(moved);
            }
            WAVE_SYNC();
            for (unsigned r = 0; r * G < hw; r++) {
                const unsigned w = r * G + gl;
                if (w < hw && w >= wmid) D.cand[(size_t)f * WS + w] = 0ull;
            }
            D.fc[f] = D.fc[f] - moved;
            D.hw[f] = wmid;
            tkind = TK_WINDOW;
            tlo = wmid;
            thi = hw;
        } else {
            extra = pick_lowest(f);
            D.fc[f] = D.fc[f] - 1;
            tL = f + 1;
        }
    };
    // dense: candidates of position `pos` given M[0..pos-1]; at the last position
    // they are counted (and emitted) as matches, otherwise they become frame pos.
    // `count` = false for a set that was counted by the unit that gave it away.
    auto expand = [&](unsigned pos, bool count) {
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
                if (last && count && d.rows) {
                    for (unsigned long long y = x; y; y &= y - 1) {
                        const unsigned v = w * 64 + (unsigned)__builtin_ctzll(y);
                        unsigned long long slot = atomicAdd(&a.ctr[inst].row_next, 1ull);
                        if (slot < d.cap_rows) {
                            gp<uint32_t> row = d.rows + slot * k;
                            for (unsigned i = 0; i + 1 < k; i++) row[P->order[i]] = D.M[i];
                            row[P->order[k - 1]] = v;
                        }
                    }
                }
            }
        }
        cnt = group_sum<G>(cnt);
        if (count) {
            c_states += cnt;
            if (last) c_matches += cnt;
            // one row of W words each: the position's domain (or label and
            // degree) set, the parent image's adjacency row, every back-edge row
            if (a.count_bytes) c_bytes += 8ull * W * (1u + (p >= 0 ? 1u : 0u) + (unsigned)__popcll(bmask));
        }
        D.fc[pos] = last ? 0u : cnt;
        D.hw[pos] = W;
    };
    // finish the current task (used bits of the mapped prefix are cleared)
    auto drop_task = [&](unsigned mapped) {
        WAVE_SYNC();
        for (unsigned i = gl; i < mapped; i += G) unmark(L.M[i]);
        // a unit that gave work away during the task has already waited for
        // that task's `created` count to complete
        if (gl == 0) fadd(&HG->finished, 1);
        const unsigned long long fin = now_ticks();
        if (gl == 0) {
            L.tim[1] += fin - L.tim[0];
            L.tim[2] = fin;
        }
        inst = NO_TASK;
        etop = 0;
    };

    while (true) {
        iter++;
        const unsigned long long idle_b = __ballot(inst == NO_TASK);
        const bool wave_idle = idle_b == ~0ull;
        // ------------------------------------------------ a piece for an idle wave-mate (CSR)
        // A unit whose wave-mate is idle hands it half of its shallowest
        // spare frame directly: the piece goes through LDS, not the queue,
        // and counts as a task given away (its `created` count completes
        // before the receiver can finish it).  The receiver starts it below.
        int ho_r = -1;   // the unit of this wave that receives a piece this iteration
        if constexpr (DENSE && G < 64) {
            // dense: the same split as for the queue; the header goes to the
            // receiver's header words, the prefix (and a single candidate) to its M
            if (a.donate && idle_b != 0 && !wave_idle && (iter & 3) == 0) {
                unsigned hf = 0;
                bool spare = false;
                if (inst != NO_TASK && since_donate >= HANDOFF_PERIOD) {
                    for (hf = base; hf <= lvl; hf++)
                        if (D.fc[hf] > (hf == lvl ? 1u : 0u)) { spare = true; break; }
                }
                const unsigned long long givers = __ballot(spare);
                if (givers) {
                    const int r = (int)((unsigned)__builtin_ctzll(idle_b) / G);
                    if ((lane / G) == (int)((unsigned)__builtin_ctzll(givers) / G)) {
                        DenseLds R = carve_dense(lds + (size_t)((threadIdx.x / 64) * (64 / G) + r) * a.unit_words,
                                                 a.kmax, a.W);
                        unsigned tL, tlo, thi, tkind, extra;
                        dense_split(hf, tL, tlo, thi, tkind, extra);
                        for (unsigned i = gl; i < hf; i += G) R.M[i] = D.M[i];
                        if (gl == 0) {
                            if (tkind == TK_RANGE) R.M[hf] = extra;
                            R.hdr[0] = inst;
                            R.hdr[1] = tL;
                            R.hdr[2] = tlo;
                            R.hdr[3] = thi;
                            R.hdr[4] = tkind;
                            R.hdr[5] = 0;
                            fadd(&HG->created, 1);
                        }
                        since_donate = 0;
                    }
                    vm_drain();
                    WAVE_SYNC();
                    ho_r = r;
                }
            }
        }
        if constexpr (!DENSE && G < 64) {
            if (a.donate && idle_b != 0 && !wave_idle && (iter & 3) == 0) {
                unsigned hf = 0, hkind = 0;
                if (inst != NO_TASK && since_donate >= HANDOFF_PERIOD) {
                    for (hf = base; hf <= lvl; hf++) {
                        if (L.cur[hf] < L.end[hf]) { hkind = 1; break; }
                        const unsigned top = hf < lvl ? L.eb[hf + 1] : etop;
                        if (top - (L.eb[hf] + L.dn[hf]) > (hf == lvl ? 1u : 0u)) { hkind = 2; break; }
                    }
                }
                const unsigned long long givers = __ballot(hkind != 0);
                if (givers) {
                    const int r = (int)((unsigned)__builtin_ctzll(idle_b) / G);
                    if ((lane / G) == (int)((unsigned)__builtin_ctzll(givers) / G)) {
                        UnitLds R = carve<G>(lds + (size_t)((threadIdx.x / 64) * (64 / G) + r) * a.unit_words);
                        unsigned tlo = 0, thi = FULL_RANGE, tkind = TK_RANGE, tne = 0;
                        if (hkind == 1) {
                            // the untried upper half of the frame's candidate range
                            const unsigned c = L.cur[hf], e = L.end[hf];
                            tlo = c + (e - c) / 2;
                            thi = e;
                            L.end[hf] = tlo;
                        } else {
                            // accepted candidates from the bottom of the frame, as for the queue
                            const unsigned top = hf < lvl ? L.eb[hf + 1] : etop;
                            const unsigned live = top - (L.eb[hf] + L.dn[hf]);
                            tne = hf < lvl ? (live + 1) / 2 : live / 2;
                            tne = min(min(tne, TASK_ENTRIES), a.E + hf + 3 - k);
                            const unsigned b0 = L.eb[hf] + L.dn[hf];
                            for (unsigned i = gl; i < tne; i += G) R.ev[i] = L.ev[b0 + i];
                            L.dn[hf] = L.dn[hf] + tne;
                            tkind = TK_ENTRIES;
                        }
                        for (unsigned i = gl; i < hf; i += G) R.M[i] = L.M[i];
                        if (gl == 0) {
                            // the piece's header, in the receiver's (idle) frame words
                            R.eb[0] = inst;
                            R.eb[1] = hf;
                            R.eb[2] = tlo;
                            R.eb[3] = thi;
                            R.eb[4] = tkind;
                            R.eb[5] = tne;
                            fadd(&HG->created, 1);
                        }
                        since_donate = 0;
                    }
                    vm_drain();
                    WAVE_SYNC();
                    ho_r = r;
                }
            }
        }
        // ------------------------------------------------ poll the scheduler (one lane per wave)
        const bool poll = idle_b != 0 && (wave_idle || (iter & 31) == 0);
        const bool polled = poll || (iter & 63) == 0;
        if (polled || ho_r >= 0) {
            unsigned flags = 0, src = NO_GROUP, cn = 0;
            if (lane == 0 && polled) {
                polls++;
                if (now_ticks() > deadline) {
                    st_rlx(&S->abort, 1u);
                    flags |= 1;
                }
                if (ld_rlx(&S->abort)) flags |= 1;
                if (ld_rlx(&S->done)) flags |= 2;
                cn = ld_rlx(&S->chunk_next);
                const unsigned av = ld_rlx(&HG->avail);
                const unsigned fr = ld_rlx(&HG->free);
                if (av) src = home;
                // give work away when the home group runs low (and, per unit, once
                // its own instance's root chunks are all claimed)
                if (av < 4 && fr > 32) flags |= 4;
                if (poll && !av && cn >= nchunks) {
                    for (unsigned g = 1; g < QUEUE_GROUPS && src == NO_GROUP; g++) {
                        const unsigned gg = (home + g) % QUEUE_GROUPS;
                        if (ld_rlx(&S->grp[gg].avail)) src = gg;
                    }
                    if (checker && src == NO_GROUP && wave_idle && (polls & 3) == 0) {
                        // termination check (one wave of the grid): finished counts
                        // first, then created counts.  A giver's `created` increment
                        // completes before its task is published, hence before any
                        // finish it precedes; the created counts are read only
                        // after the finished counts have arrived.
                        unsigned fin = 0, cre = 0;
                        for (unsigned g = 0; g < QUEUE_GROUPS; g++) fin += ld_rlx(&S->grp[g].finished);
                        vm_drain();
                        for (unsigned g = 0; g < QUEUE_GROUPS; g++) cre += ld_rlx(&S->grp[g].created);
                        if (fin == nchunks + cre) {
                            st_rel(&S->done, 1u);
                            atomicMax(&S->t_done, now_ticks());
                            flags |= 2;
                        }
                    }
                }
            }
            flags = __shfl(flags, 0);
            src = __shfl(src, 0);
            cn = __shfl(cn, 0);
            if (flags & 1) break;                    // time limit: every wave stops
            if ((flags & 2) && wave_idle) break;     // the search is complete
            if (polled) {
                donate_hint = a.donate && (flags & 4);
                cn_seen = max(cn_seen, cn);
            }
            if ((poll && (src != NO_GROUP || cn < nchunks)) || ho_r >= 0) {
                // ---------------------------------------- task acquisition, one unit at a time
                for (int g = 0; g < 64 / G; g++) {
                    if (!(inst == NO_TASK && (lane / G) == g)) continue;
                    unsigned kind = 0, val = 0;
                    if (g == ho_r) {
                        kind = 3;   // a piece from a wave-mate, already in this unit's LDS
                    } else if (gl == 0 && poll) {
                        if (src != NO_GROUP && cas_dec_if_pos(&S->grp[src].avail)) {
                            unsigned t = fadd(&S->grp[src].head, 1);
                            QTask *q = a.queue + src * QUEUE_GROUP_SLOTS + t % QUEUE_GROUP_SLOTS;
                            kind = 1;
                            // the payload loads below are issued after this load has
                            // returned the published sequence number
                            while (ld_rlx(&q->seq) != 2 * t + 1) {
                                __builtin_amdgcn_s_sleep(1);
                                if (now_ticks() > deadline) { kind = 0; break; }
                            }
                            val = t;
                        } else if (!roots_done && cn < nchunks) {
                            unsigned c = fadd(&S->chunk_next, 1);
                            if (c < nchunks) {
                                kind = 2;
                                val = c;
                            } else {
                                roots_done = true;
                            }
                        }
                    }
                    kind = __shfl(kind, gbase);
                    val = __shfl(val, gbase);
                    roots_done = __shfl((int)roots_done, gbase) != 0;
                    if (kind == 0) continue;
                    unsigned ti = 0, tL = 0, tlo = 0, thi = 0, tkind = TK_RANGE, tne = 0;
                    if (kind == 3) {
                        const unsigned *hd;
                        if constexpr (DENSE) hd = D.hdr;
                        else hd = L.eb;
                        ti = hd[0];
                        tL = hd[1];
                        tlo = hd[2];
                        thi = hd[3];
                        tkind = hd[4];
                        tne = hd[5];
                    } else if (kind == 1) {
                        QTask *q = a.queue + src * QUEUE_GROUP_SLOTS + val % QUEUE_GROUP_SLOTS;
                        ti = ld_rlx(&q->inst);
                        tL = ld_rlx(&q->L);
                        tlo = ld_rlx(&q->lo);
                        thi = ld_rlx(&q->hi);
                        tkind = ld_rlx(&q->kind);
                        tne = ld_rlx(&q->ne);
                        // a task is checked before any of it is used: instance, prefix
                        // length and every node it names must be in range
                        bool bad = ti >= a.ninst || tkind > TK_WINDOW || tne > TASK_ENTRIES;
                        unsigned tn = 0;
                        if (!bad) {
                            gp<const DevPlan> tp = glob(glob(a.inst)[ti].plan);
                            tn = tp->n;
                            bad = tL >= tp->k || (tkind == TK_WINDOW && (tlo > thi || thi > tp->W));
                        }
                        if (!bad) {
                            // every payload load is issued before any is used
                            // (prefix length below 64, at most TASK_ENTRIES entries)
                            bool bl = false;
                            constexpr unsigned PR = 64 / G, ER = (TASK_ENTRIES + G - 1) / G;
                            unsigned mv[PR], evv[DENSE ? 1 : ER];
#pragma unroll
                            for (unsigned r = 0; r < PR; r++) {
                                const unsigned i = r * G + gl;
                                mv[r] = i < tL ? ld_rlx(&q->M[i]) : 0u;
                            }
                            if constexpr (!DENSE) {
#pragma unroll
                                for (unsigned r = 0; r < ER; r++) {
                                    const unsigned i = r * G + gl;
                                    evv[r] = i < tne ? ld_rlx(&q->ent[i]) : 0u;
                                }
                            }
#pragma unroll
                            for (unsigned r = 0; r < PR; r++) {
                                const unsigned i = r * G + gl;
                                if (i < tL) {
                                    bl |= mv[r] >= tn;
                                    L.M[i] = mv[r];
                                }
                            }
                            if constexpr (!DENSE) {
#pragma unroll
                                for (unsigned r = 0; r < ER; r++) {
                                    const unsigned i = r * G + gl;
                                    if (i < tne) {
                                        bl |= evv[r] >= tn;
                                        L.ev[i] = evv[r];
                                    }
                                }
                            }
                            bad = group_mask<G>(__ballot(bl), gbase) != 0;
                        }
                        // the payload loads have completed (their values are in
                        // registers and LDS) before the slot is handed back
                        vm_drain();
                        WAVE_SYNC();
                        if (gl == 0) {
                            st_rlx(&q->seq, 2 * (val + QUEUE_GROUP_SLOTS));
                            fadd(&S->grp[src].free, 1);
                        }
                        if (bad) {   // reported to the host; the task counts as finished
                            if (gl == 0) {
                                st_rlx(&S->bad, 1u);
                                fadd(&HG->finished, 1);
                            }
                            continue;
                        }
                    } else if (kind == 2) {
                        unsigned lo = 0, hi = a.ninst;   // largest i with prefix[i] <= val
                        if (gl == 0) {
                            while (hi - lo > 1) {
                                unsigned mid = (lo + hi) >> 1;
                                if (a.chunk_prefix[mid] <= val) lo = mid;
                                else hi = mid;
                            }
                        }
                        ti = __shfl(lo, gbase);
                        cn_seen = max(cn_seen, val + 1);   // the counter is past the chunk just claimed
                        gp<const InstDesc> dd = glob(a.inst) + ti;
                        tlo = (val - a.chunk_prefix[ti]) * dd->chunk;
                        thi = min(tlo + dd->chunk, dd->nroot);
                    }
                    // start the task
                    if (ti != cinst) {
                        flush();
                        cinst = ti;
                        d = gdesc(glob(a.inst) + ti);
                        P = d.plan;
                        k = P->k;
                        W = P->W;
                        if constexpr (!DENSE) {
                            for (unsigned i = gl; i < k; i += G) {
                                L.pback[i] = P->back[i];
                                // pattern degrees count bits of 64-bit neighbour masks (at most 64)
                                L.ppd[i] = (int)((unsigned)P->parent[i] << 16 | min(P->pdeg[i], 0xFFFFu));
                                L.plab[i] = P->plabel[i];
                            }
                            WAVE_SYNC();
                        }
                    }
                    inst = ti;
                    if (gl == 0) L.tim[0] = now_ticks();
                    since_donate = 0;
                    if (kind != 2) c_steals++;
                    etop = 0;
                    if (a.state_cap && inst_aborted(inst)) {   // capped instance: drop the task
                        if (gl == 0) fadd(&HG->finished, 1);
                        inst = NO_TASK;
                        continue;
                    }
                    if constexpr (DENSE) {
                        for (unsigned i = gl; i < tL; i += G) mark(D.M[i]);
                        WAVE_SYNC();
                        base = lvl = tL;
                        if (kind == 2) {
                            // a root chunk: its list entries are the accepted candidates of position 0
                            for (unsigned w = gl; w < W; w += G) D.cand[w] = 0ull;
                            WAVE_SYNC();
                            gp<const uint32_t> lst = d.lists + P->list_off[0] + tlo;
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
                            D.hw[0] = W;
                        } else if (tkind == TK_WINDOW) {
                            // words [tlo, thi) of position tL's candidate set, counted by the giver
                            expand(tL, false);
                            unsigned cnt = 0;
                            for (unsigned r = 0; r * G < W; r++) {
                                const unsigned w = r * G + gl;
                                if (w < W) {
                                    unsigned long long x = D.cand[(size_t)tL * WS + w];
                                    if (w < tlo || w >= thi) x = 0ull;
                                    D.cand[(size_t)tL * WS + w] = x;
                                    cnt += (unsigned)__popcll(x);
                                }
                            }
                            D.fc[tL] = group_sum<G>(cnt);
                            D.hw[tL] = thi;
                        } else {
                            expand(tL, true);
                        }
                        WAVE_SYNC();
                    } else {
                        for (unsigned i = gl; i < tL; i += G) {
                            unsigned v = L.M[i];
                            NodeRec r = ld_node(d.node + v);
                            L.MB[i] = r.begin;
                            L.MD[i] = r.deg;
                            mark(v);
                        }
                        WAVE_SYNC();
                        base = lvl = tL;
                        if (kind != 2 && tkind == TK_ENTRIES) {
                            // accepted candidates of position tL, counted by the giver
                            open_frame(tL, 0, 0);
                            for (unsigned i = gl; i < tne; i += G) {
                                const unsigned v = L.ev[i];
                                const NodeRec r = ld_node(d.node + v);
                                L.ebg[i] = r.begin;
                                L.edg[i] = r.deg;
                            }
                            etop = tne;
                        } else {
                            open_frame(tL, tlo, thi);
                        }
                    }
                }
            }
        }
        if (__ballot(inst != NO_TASK) == 0) {
            // the whole wave is idle: back off before polling again
            // (the terminating wave keeps its polls frequent)
            const unsigned bmax = checker ? 4u : 32u;
            backoff = backoff < bmax ? backoff + 1 : bmax;
            for (unsigned z = 0; z < backoff; z++) __builtin_amdgcn_s_sleep(32);
            continue;
        }
        backoff = 0;
        if (inst == NO_TASK) continue;

        // ------------------------------------------------ one search step
        WAVE_SYNC();
        since_donate++;
        c_steps++;
        if (a.check_uniform) {
            // a unit's state is held by each of its lanes: every copy must be
            // the same (a disagreement is reported, the search goes on)
            bool diff = false;
            auto same = [&](unsigned x) { diff |= x != (unsigned)__shfl((int)x, gbase); };
            same(inst);
            same(lvl);
            same(base);
            same(etop);
            same(k);
            if constexpr (DENSE) {
                same(D.fc[lvl]);
                same(D.hw[lvl]);
                same(D.M[lvl > 0 ? lvl - 1 : 0]);
            } else {
                same(L.cur[lvl]);
                same(L.end[lvl]);
                same(L.eb[lvl]);
                same(L.dn[lvl]);
                same(L.lb[lvl]);
                same(L.M[lvl > 0 ? lvl - 1 : 0]);
            }
            if (group_mask<G>(__ballot(diff), gbase) != 0 && gl == 0) st_rlx(&S->bad, 2u);
        }
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
            expand(lvl + 1, true);
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
            // map the top accepted candidate and open the next frame (whose
            // bounds the evaluation below takes from registers, not LDS)
            unsigned c0, e, lb;
            if (etop > L.eb[lvl] + L.dn[lvl]) {
                etop--;
                unsigned v = L.ev[etop];
                L.M[lvl] = v;
                L.MB[lvl] = L.ebg[etop];
                L.MD[lvl] = L.edg[etop];
                if (gl == 0) mark(v);
                lvl++;
                const uint2 fr = open_frame(lvl, 0, FULL_RANGE);
                if (a.count_bytes) {
                    // an expansion: the bounds of the parent image's list (its ids
                    // are counted per candidate below); without a parent, the
                    // whole candidate set: 5 bytes per target node (RI) or 4 + 8
                    // per domain member (RI-DS)
                    c_bytes += parent_at(L.ppd[lvl]) >= 0 ? 8ull
                               : d.bits ? 12ull * P->list_len[lvl] : 5ull * P->n;
                }
                c0 = 0;
                e = fr.x;
                lb = fr.y;
            } else {
                c0 = L.cur[lvl];
                e = L.end[lvl];
                lb = L.lb[lvl];
            }
            // evaluate up to G candidates of the current frame
            const unsigned idx = c0 + gl;
            bool ok = idx < e;
            const bool has_parent = parent_at(L.ppd[lvl]) >= 0;
            const unsigned flags = GEN ? P->flags : 0u;
            // the pattern arc to the parent leaves the parent (pout), else it
            // points at it and candidates come from the image's in-row
            const bool pout = GEN && ((P->pdir_out >> lvl) & 1ull);
            const bool in_row = GEN && has_parent && (flags & PLAN_DIRECTED) && !pout && d.irp != nullptr;
            unsigned v = 0;
            NodeRec r{0, 0, 0, 0};
            unsigned probes = 0;      // back-edge probes of this lane's candidate, up to the first failure
            unsigned gen_extra = 0;   // general graphs: bytes of the parent-arc checks
            if (ok) {
                if (!GEN && has_parent && d.wcol) {
                    const WideEntry we = ld_wide(d.wcol + lb + idx);   // id, row start, degree, label in one load
                    v = we.v;
                    r = NodeRec{we.begin, we.deg, we.label, 0};
                } else {
                    v = has_parent ? (in_row ? d.icol[lb + idx] : d.col[lb + idx]) : d.lists[lb + idx];
                    r = ld_node(d.node + v);
                }
            }
            // the domain word needs only v, like the back-edge rows: with
            // adjacency rows it is awaited together with their first round
            const bool late_dom = (!GEN || !flags) && d.adj;
            unsigned long long dword = ~0ull;
            if (d.bits) dword = d.bits[(size_t)lvl * W + (v >> 6)];   // v is 0 for an idle lane
            // the label, degree and used tests read registers and LDS only (v
            // is 0 for an idle lane), so they are combined without branches
            const unsigned pl = L.plab[lvl];
            unsigned okb = ok ? 1u : 0u;
            if (!late_dom) okb &= (unsigned)(dword >> (v & 63)) & 1u;
            okb &= (unsigned)(pl == LABEL_ANY) | (unsigned)(r.label == pl);
            okb &= (unsigned)(r.deg >= ((unsigned)L.ppd[lvl] & 0xFFFFu));
            if (a.UW) {
                okb &= used_test(L.used, v) ? 0u : 1u;
            } else {
                // targets too large for a used bitset in LDS: v against the
                // mapped prefix (the same address in every lane: a broadcast)
                for (unsigned j = 0; j < lvl; j++) okb &= (unsigned)(L.M[j] != v);
            }
            ok = okb != 0;
            if ((!GEN || !flags) && d.adj) {
                // one adjacency-row word per back edge, four rows per round with
                // their loads issued together (every lane's address is in range:
                // v is a node id, 0 for an idle lane)
                unsigned long long bm = L.pback[lvl];
                const size_t wv = v >> 6;
                unsigned long long hit = ~0ull;
                bool alive = ok;   // this candidate's probes have not failed yet
                while (bm) {
                    const unsigned ng = min((unsigned)__popcll(bm), 4u);   // distinct rows this round
                    const unsigned j0 = (unsigned)__builtin_ctzll(bm);
                    bm &= bm - 1;
                    const unsigned j1 = bm ? (unsigned)__builtin_ctzll(bm) : j0;
                    bm &= bm ? bm - 1 : 0ull;
                    const unsigned j2 = bm ? (unsigned)__builtin_ctzll(bm) : j0;
                    bm &= bm ? bm - 1 : 0ull;
                    const unsigned j3 = bm ? (unsigned)__builtin_ctzll(bm) : j0;
                    bm &= bm ? bm - 1 : 0ull;
                    const unsigned long long a0 = d.adj[(size_t)L.M[j0] * W + wv];
                    const unsigned long long a1 = d.adj[(size_t)L.M[j1] * W + wv];
                    const unsigned long long a2 = d.adj[(size_t)L.M[j2] * W + wv];
                    const unsigned long long a3 = d.adj[(size_t)L.M[j3] * W + wv];
                    hit &= a0 & a1 & a2 & a3;
                    if (a.count_bytes) {
                        // probes in position order up to the first that fails
                        const unsigned sh = v & 63;
                        const unsigned res = (unsigned)((a0 >> sh) & 1ull) | ((unsigned)((a1 >> sh) & 1ull) << 1) |
                                             ((unsigned)((a2 >> sh) & 1ull) << 2) |
                                             ((unsigned)((a3 >> sh) & 1ull) << 3) | (0xFu << ng);
                        const unsigned f = (unsigned)__builtin_ctz(~res);   // first failure, >= ng: none
                        probes += alive ? min(f + 1, ng) : 0u;
                        alive = alive && f >= ng;
                    }
                }
                ok = ok && ((hit >> (v & 63)) & 1ull);
                if (!((dword >> (v & 63)) & 1ull)) {   // outside the domain: no check beyond it counts
                    ok = false;
                    probes = 0;
                }
            } else if (!GEN || !flags) {
                unsigned long long bm = L.pback[lvl];
                while (bm) {
                    unsigned j = (unsigned)__builtin_ctzll(bm);
                    bm &= bm - 1;
                    if (ok) {
                        probes++;
                        ok = adjacent(d, W, L.M[j], L.MB[j], L.MD[j], v);
                    }
                }
            } else if constexpr (GEN) {
                // general graphs: in-degree (r.pad), the label of the arc the
                // candidate came over, the reverse arc to the parent, and every
                // arc to an earlier position in its direction with its label
                gp<const uint32_t> lm = d.lmat;
                const bool dir = flags & PLAN_DIRECTED;
                if (ok) ok = r.pad >= P->pindeg[lvl];
                if (ok && has_parent && lm) {
                    const unsigned pp = (unsigned)parent_at(L.ppd[lvl]);
                    const unsigned tl = in_row ? (d.ielab ? d.ielab[lb + idx] : 0u) : (d.elab ? d.elab[lb + idx] : 0u);
                    gen_extra += 4;   // the label of the arc the candidate came over
                    ok = tl == (pout ? lm[pp * k + lvl] : lm[lvl * k + pp]);
                }
                if (ok && dir && has_parent && ((P->pboth >> lvl) & 1ull)) {
                    const unsigned pp = (unsigned)parent_at(L.ppd[lvl]);
                    gen_extra += 8;   // the reverse arc to the parent
                    ok = arc_to(d, r.begin, r.deg, L.M[pp], lm != nullptr, lm ? lm[lvl * k + pp] : 0u);
                }
                // earlier positions in order; for each, the arc into v, then
                // (directed) the arc out of v, up to the first that fails
                const unsigned long long bo = P->bout[lvl], bi = dir ? P->bin[lvl] : 0ull;
                for (unsigned long long bm = bo | bi; bm && ok; bm &= bm - 1) {
                    const unsigned j = (unsigned)__builtin_ctzll(bm);
                    if ((bo >> j) & 1ull) {   // M[j] -> v
                        probes++;
                        ok = arc_to(d, L.MB[j], L.MD[j], v, lm != nullptr, lm ? lm[j * k + lvl] : 0u);
                    }
                    if (ok && ((bi >> j) & 1ull)) {   // v -> M[j]
                        probes++;
                        ok = arc_to(d, r.begin, r.deg, L.M[j], lm != nullptr, lm ? lm[lvl * k + j] : 0u);
                    }
                }
            }
            c_cands += min((unsigned)G, e - c0);
            unsigned long long acc = group_mask<G>(__ballot(ok), gbase);
            unsigned cnt = (unsigned)__popcll(acc);
            // bytes of the candidates this step is done with (those past the
            // frame's new cursor are evaluated again later): with a parent, the
            // list id, 5 (RI) or 8 (RI-DS) bytes of checks, the parent-arc
            // checks and 8 per back-edge probe
            const unsigned cand_bytes = has_parent ? 4u + (d.bits ? 8u : 5u) + gen_extra + 8u * probes : 0u;
            if (lvl + 1 == k) {
                if (a.count_bytes && idx < e) lane_bytes += cand_bytes;
                c_states += cnt;
                c_matches += cnt;
                if (d.rows && ok) {
                    unsigned long long slot = atomicAdd(&a.ctr[inst].row_next, 1ull);
                    if (slot < d.cap_rows) {
                        gp<uint32_t> row = d.rows + slot * k;
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
                if (a.count_bytes && idx < e && idx < ncur) lane_bytes += cand_bytes;
            }
        }

        // counters: flush now and then so a state cap takes effect (and no
        // 32-bit count wraps)
        if (c_states >= 8192 || c_steps >= (1u << 20)) {
            flush();
            if (a.state_cap && inst_aborted(inst)) {
                drop_task(lvl);
                continue;
            }
        }

        // ------------------------------------------------ giving work away (one unit at a time)
        if (donate_hint && (iter & 7) == 0 && __ballot(since_donate >= a.donate_period) != 0) {
            for (int g = 0; g < 64 / G; g++) {
                if (!((lane / G) == g && inst != NO_TASK && since_donate >= a.donate_period)) continue;
                // while roots of this instance wait in the chunk counter, idle units take those
                if (cn_seen < a.chunk_prefix[inst + 1]) continue;
                // the shallowest frame with something to spare
                unsigned f = base, kind = 0;
                for (; f <= lvl; f++) {
                    if constexpr (DENSE) {
                        if (D.fc[f] > (f == lvl ? 1u : 0u)) { kind = 1; break; }
                    } else {
                        if (L.cur[f] < L.end[f]) { kind = 1; break; }
                        unsigned top = f < lvl ? L.eb[f + 1] : etop;
                        unsigned live = top - (L.eb[f] + L.dn[f]);
                        if (live > (f == lvl ? 1u : 0u)) { kind = 2; break; }
                    }
                }
                if (!kind) continue;
                since_donate = 0;
                unsigned t = 0, okr = 0;
                if (gl == 0) {
                    if (cas_dec_if_pos(&HG->free)) {
                        fadd(&HG->created, 1);
                        t = fadd(&HG->tail, 1);
                        okr = 1;
                        QTask *qq = a.queue + home * QUEUE_GROUP_SLOTS + t % QUEUE_GROUP_SLOTS;
                        // the slot is free once its previous payload was read; the
                        // new payload is written only after that is observed
                        while (ld_rlx(&qq->seq) != 2 * t) {
                            __builtin_amdgcn_s_sleep(1);
                            if (now_ticks() > deadline) { okr = 0; break; }
                        }
                    }
                }
                if (!__shfl(okr, gbase)) continue;
                t = __shfl(t, gbase);
                WAVE_SYNC();
                QTask *q = a.queue + home * QUEUE_GROUP_SLOTS + t % QUEUE_GROUP_SLOTS;
                unsigned tL = f, tlo = 0, thi = FULL_RANGE, tkind = TK_RANGE, tne = 0, extra = 0;
                if constexpr (DENSE) {
                    dense_split(f, tL, tlo, thi, tkind, extra);
                } else if (kind == 1) {
                    // the untried upper half of the frame's candidate range
                    unsigned c = L.cur[f], e = L.end[f];
                    unsigned mid = c + (e - c) / 2;
                    tlo = mid;
                    thi = e;
                    L.end[f] = mid;
                } else {
                    // up to TASK_ENTRIES accepted candidates from the bottom of the frame
                    unsigned top = f < lvl ? L.eb[f + 1] : etop;
                    unsigned live = top - (L.eb[f] + L.dn[f]);
                    tne = f < lvl ? (live + 1) / 2 : live / 2;
                    // the receiver holds them on its stack and still needs a slot
                    // for each deeper position: at most E - k + f + 3 of them
                    tne = min(min(tne, TASK_ENTRIES), a.E + f + 3 - k);
                    const unsigned b0 = L.eb[f] + L.dn[f];
                    for (unsigned i = gl; i < tne; i += G) st_rlx(&q->ent[i], L.ev[b0 + i]);
                    L.dn[f] = L.dn[f] + tne;
                    tkind = TK_ENTRIES;
                }
                // prefix positions taken from M (a single dense candidate carries M[f] in `extra`)
                const unsigned pre = (DENSE && tkind == TK_RANGE) ? f : tL;
                for (unsigned i = gl; i < pre; i += G) st_rlx(&q->M[i], L.M[i]);
                if (DENSE && tkind == TK_RANGE && gl == 0) st_rlx(&q->M[f], extra);
                if (gl == 0) {
                    st_rlx(&q->inst, inst);
                    st_rlx(&q->L, tL);
                    st_rlx(&q->lo, tlo);
                    st_rlx(&q->hi, thi);
                    st_rlx(&q->kind, tkind);
                    st_rlx(&q->ne, tne);
                }
                // the payload (and the `created` count taken with the ticket)
                // is complete before the task is published
                vm_drain();
                if (gl == 0) {
                    st_rlx(&q->seq, 2 * t + 1);
                    fadd(&HG->avail, 1);
                }
            }
        }
    }
    // Leaving: the units of the block combine what they still hold, so that
    // a shared word receives one atomic per block rather than one per unit
    // (thousands of units leave within microseconds of each other, mostly
    // holding the same last instance, and atomics on one word serialise).
    // Every wave of the block reaches this point (the loop is left only by
    // `break`), and the units' LDS areas are free: each unit's area (at least
    // 18 words) takes its exit record.
    if (a.count_bytes) {   // every lane is here: fold the per-lane bytes into the unit's
        c_bytes += group_sum64<G>((unsigned long long)lane_bytes);
        lane_bytes = 0;
    }
    const unsigned long long busy_ticks = L.tim[1], last_finish = L.tim[2];   // before the record covers them
    __syncthreads();
    unsigned long long *rec = reinterpret_cast<unsigned long long *>(lds + (size_t)unit * a.unit_words);
    if (gl == 0) {
        rec[0] = cinst;
        rec[1] = c_states;
        rec[2] = c_matches;
        rec[3] = c_cands;
        rec[4] = c_steals;
        rec[5] = c_steps;
        rec[6] = busy_ticks;
        rec[7] = last_finish;
        rec[8] = c_bytes;
    }
    __syncthreads();
    const unsigned nunits = blockDim.x / G;
    auto rec_of = [&](unsigned u) {
        return reinterpret_cast<const unsigned long long *>(lds + (size_t)u * a.unit_words);
    };
    if (gl == 0 && cinst != NO_TASK) {
        // the first unit holding an instance adds every later unit's counts for it
        bool first = true;
        for (unsigned u = 0; u < (unsigned)unit && first; u++) first = rec_of(u)[0] != cinst;
        if (first) {
            unsigned long long t[6] = {c_states, c_matches, c_cands, c_steals, c_steps, c_bytes};
            for (unsigned u = unit + 1; u < nunits; u++) {
                const unsigned long long *r = rec_of(u);
                if (r[0] != cinst) continue;
                for (int i = 0; i < 5; i++) t[i] += r[1 + i];
                t[5] += r[8];
            }
            InstCounters *c = a.ctr + cinst;
            if (t[5]) fadd64(&c->bytes, t[5]);
            if (t[1]) fadd64(&c->matches, t[1]);
            if (t[2]) fadd64(&c->candidates, t[2]);
            if (t[3]) fadd64(&c->steals, t[3]);
            if (t[4]) fadd64(&c->steps, t[4]);
            if (t[0]) {
                unsigned long long before = fadd64(&c->states, t[0]);
                if (a.state_cap && before + t[0] > a.state_cap)
                    __hip_atomic_store(&c->pad0, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (threadIdx.x == 0) {
        unsigned long long busy = 0, fin = 0;
        for (unsigned u = 0; u < nunits; u++) {
            busy += rec_of(u)[6];
            fin = max(fin, rec_of(u)[7]);
        }
        fadd64(&S->t_busy, busy);
        if (fin) stamp_max(&S->t_work, fin);
        stamp_max(&S->t_end, now_ticks());
    }
}

__global__ void reset_kernel(Sched *s, InstCounters *c, unsigned ninst, QTask *q) {
    unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned stride = gridDim.x * blockDim.x;
    if (blockIdx.x == 0) {
        unsigned *w = reinterpret_cast<unsigned *>(s);
        for (unsigned j = threadIdx.x; j < sizeof(Sched) / 4; j += blockDim.x) w[j] = 0;
        __syncthreads();
        if (threadIdx.x < QUEUE_GROUPS) s->grp[threadIdx.x].free = QUEUE_GROUP_SLOTS;
        if (threadIdx.x == 0) s->t_start = ~0ull;
    }
    for (unsigned j = i; j < ninst; j += stride) c[j] = InstCounters{};
    for (unsigned j = i; j < QUEUE_SLOTS; j += stride) q[j].seq = 2 * (j % QUEUE_GROUP_SLOTS);
}

template <int G, bool DENSE, bool GEN = false>
hipError_t launch_g(SearchArgs args, int blocks, int per_cu_cap, int threads, size_t lds, hipStream_t s, int num_cus) {
    if (blocks <= 0) {
        // resident blocks only (a persistent grid); the kernel trims it to
        // what the root chunks can keep busy before work is handed around
        int per_cu = 0;
        hipError_t e =
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, search_kernel<G, DENSE, GEN>, threads, lds);
        if (e != hipSuccess) return e;
        if (per_cu_cap > 0) per_cu = std::min(per_cu, per_cu_cap);
        if (per_cu < 1) per_cu = 1;
        blocks = per_cu * num_cus;
    }
    args.min_blocks = (unsigned)std::max(1, 2 * num_cus);
    args.units_per_block = (unsigned)(threads / G);
    hipLaunchKernelGGL((search_kernel<G, DENSE, GEN>), dim3(blocks), dim3(threads), lds, s, args);
    return hipGetLastError();
}

unsigned unit_words(const LaunchCfg &cfg) {
    // even: every unit's area starts 8-byte aligned; at least 18 words: the
    // area takes the unit's exit record (nine 64-bit values)
    if (cfg.dense) return std::max(18u, 3 * even(cfg.kmax) + 2 * cfg.kmax * cfg.wmax + 2 * cfg.wmax + 6 + 6);
    unsigned E = KMAX + cfg.lanes;
    unsigned UW = cfg.used_bitset ? (cfg.nmax + 31) / 32 : 0;
    return std::max(18u, even(12 * KMAX + 3 * E + 6 + UW));
}

// Largest block (256, 128 or 64 threads) whose units fit in 64 KiB of LDS.
int block_threads(const LaunchCfg &cfg) {
    size_t per_unit = (size_t)unit_words(cfg) * 4;
    for (int t = 256; t >= 64; t /= 2)
        if (per_unit * (t / cfg.lanes) <= 65536) return t;
    return 0;
}

}  // namespace

int search_block_threads(const LaunchCfg &cfg) { return block_threads(cfg); }

const void *search_kernel_fn(const LaunchCfg &cfg) {
    auto pick = [&](auto k8, auto k16, auto k32, auto k64) -> const void * {
        switch (cfg.lanes) {
            case 8: return (const void *)k8;
            case 16: return (const void *)k16;
            case 32: return (const void *)k32;
            case 64: return (const void *)k64;
            default: return nullptr;
        }
    };
    if (cfg.dense)
        return pick(search_kernel<8, true, false>, search_kernel<16, true, false>, search_kernel<32, true, false>,
                    search_kernel<64, true, false>);
    if (cfg.general)
        return pick(search_kernel<8, false, true>, search_kernel<16, false, true>, search_kernel<32, false, true>,
                    search_kernel<64, false, true>);
    return pick(search_kernel<8, false, false>, search_kernel<16, false, false>, search_kernel<32, false, false>,
                search_kernel<64, false, false>);
}

size_t search_lds_bytes(const LaunchCfg &cfg) {
    int t = block_threads(cfg);
    return (size_t)unit_words(cfg) * 4 * (size_t)((t ? t : 64) / cfg.lanes);
}

hipError_t launch_reset(DevWork &w, uint32_t ninst, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3(64), dim3(256), 0, s, w.sched, w.ctr, ninst, w.queue);
    return hipGetLastError();
}

hipError_t launch_search(const LaunchCfg &cfg, DevWork &w, uint32_t ninst, uint64_t state_cap,
                         uint64_t time_limit_ms, hipStream_t s, int num_cus) {
    SearchArgs a{};
    a.count_bytes = cfg.count_bytes ? 1u : 0u;
    a.check_uniform = cfg.check_uniform ? 1u : 0u;
    a.root_lo = cfg.root_lo;
    a.root_hi = cfg.root_hi;
    a.inst = w.inst;
    a.chunk_prefix = w.chunk_prefix;
    a.ctr = w.ctr;
    a.sched = w.sched;
    a.queue = w.queue;
    a.ninst = ninst;
    a.kmax = cfg.kmax;
    a.E = cfg.dense ? cfg.kmax + cfg.lanes : KMAX + cfg.lanes;
    a.UW = cfg.used_bitset ? (cfg.nmax + 31) / 32 : 0;
    a.W = cfg.dense ? cfg.wmax : 0;
    a.unit_words = unit_words(cfg);
    a.donate = cfg.donate != 0;
    a.donate_period = cfg.donate > 1 ? (unsigned)cfg.donate : DEFAULT_DONATE_PERIOD;
    a.state_cap = state_cap;
    a.limit_ticks = time_limit_ms * 100000ull;   // s_memrealtime runs at 100 MHz
    const int threads = block_threads(cfg);
    if (!threads) return hipErrorInvalidValue;   // one unit's LDS does not fit
    size_t lds = search_lds_bytes(cfg);
    int blocks = cfg.blocks;
    if (cfg.dense) {
        switch (cfg.lanes) {
            case 8: return launch_g<8, true>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
            case 16: return launch_g<16, true>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
            case 32: return launch_g<32, true>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
            case 64: return launch_g<64, true>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
            default: return hipErrorInvalidValue;
        }
    }
    if (cfg.general) {
        switch (cfg.lanes) {
            case 8: return launch_g<8, false, true>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
            case 16: return launch_g<16, false, true>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
            case 32: return launch_g<32, false, true>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
            case 64: return launch_g<64, false, true>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
            default: return hipErrorInvalidValue;
        }
    }
    switch (cfg.lanes) {
        case 8: return launch_g<8, false>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
        case 16: return launch_g<16, false>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
        case 32: return launch_g<32, false>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
        case 64: return launch_g<64, false>(a, blocks, cfg.per_cu, threads, lds, s, num_cus);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sge
