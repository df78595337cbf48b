// Device preparation of a batch of searches: one workgroup plans one
// instance from the resident pattern and target, then one block sets the root
// chunking of every instance.  The plan is the one the host planner
// (sge_plan.cpp) builds, step for step:
//
//  * Domains (Section 4.1): D(u) starts as the target nodes passing the label
//    and degree rules for pattern node u; lane l of a wave decides target
//    node 64 i + l for every pattern node.
//  * Arc-consistency (Section 4.1) to the greatest fixpoint.  The first round
//    (all domains still label-and-degree sets) reads the target's
//    neighbour-degree table, in the same pass that builds the domains; later
//    rounds work in support form: v stays in D(u) iff for each pattern
//    neighbour w of u some target neighbour of v lies in D(w), i.e. v lies in
//    the support set S(w), the union of the target rows of D(w).  A round
//    recomputes S(w) only for the w whose domain changed in the previous
//    round.  On targets of up to PLAN_WAVES * DT_WORDS words each lane keeps
//    its nodes' domain memberships (a 64-bit set of pattern nodes per target
//    node) in registers, the supports are kept by target node in LDS (one
//    word per node: the dirty w it supports), each list is read once per
//    round and scattered with one atomic OR per entry, and the domain rows
//    are written once at the end; otherwise S(w) is a bit row per w in LDS
//    or device memory, scattered one lane per member of D(w).
//  * Forward checking (Section 4.2.2): while a domain is a singleton {t} that
//    has not been used, t leaves every other domain.
//  * The constraint-first order (Section "RI"; singletons first and the
//    domain-size tie-break of Section 4.2.1): lane u of one wave scores
//    pattern node u, and a wave-wide maximum of the packed key
//    (w_m, w_n, degree, [-|D(u)|], -u) picks the next node.
//  * Parents and back-edges, the per-position bitsets the search reads, and
//    the candidate lists of parentless positions (compacted by a wave scan;
//    position 0 limited to the root range).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sge_internal.h"

namespace sge {

namespace {

// Workgroup size: twelve waves, so each plan's latency-bound phases spread
// over twelve waves, and two workgroups reside per CU (twenty-four waves, what
// this kernel's launches reach; the kernel is held to 80 VGPRs for it).
constexpr int PLAN_THREADS = 768;

// Neighbour-degree table columns the first arc-consistency round packs per
// target node (more distinct labels among a pattern's nodes read the table
// column by column).
constexpr uint32_t TAB_COLS = 24;

// Target words (64 nodes each) one wave keeps the domain memberships of in
// registers during arc-consistency: targets of up to PLAN_WAVES * DT_WORDS
// words take that path.
constexpr uint32_t DT_WORDS = 8;

// Device memory in the global address space: the pointers a plan request
// holds are loaded from memory, so the compiler would treat them as generic
// and emit flat accesses, whose completion counter is shared with LDS.
template <class T>
using gp = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gp<T> glob(T *p) {
    return (gp<T>)p;
}
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ NodeRec ld_node(gp<const NodeRec> p) {
    const u32x4 x = *(gp<const u32x4>)p;
    return NodeRec{x.x, x.y, x.z, x.w};
}

// dense id of a raw label among the target's increasing label keys
__device__ uint32_t label_id(gp<const uint32_t> keys, uint32_t nl, uint32_t raw) {
    uint32_t lo = 0, hi = nl;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (keys[mid] < raw) lo = mid + 1;
        else hi = mid;
    }
    return (lo < nl && keys[lo] == raw) ? lo : LABEL_NONE;
}

// Wave-wide reductions with DPP moves (register to register, no LDS round
// trip): row shifts by 1, 2, 4 and 8 leave each 16-lane row's total in its
// last lane, two row broadcasts (15: rows 1 and 3; 31: rows 2 and 3) carry
// them on, and lane 63 ends with the total of all 64 lanes.  A lane whose
// source is outside the row or the masked rows takes 0, the identity of both
// reductions (the values are unsigned).
template <class Op>
__device__ __forceinline__ uint32_t wave_reduce(uint32_t x, Op op) {
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false));   // row_shr:1
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false));   // row_shr:2
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false));   // row_shr:4
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false));   // row_shr:8
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false));   // row_bcast:15
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false));   // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
    return wave_reduce(x, [](uint32_t a, uint32_t b) { return a + b; });
}

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long x) {
    const auto o = [](uint32_t a, uint32_t b) { return a | b; };
    return ((unsigned long long)wave_reduce((uint32_t)(x >> 32), o) << 32) | wave_reduce((uint32_t)x, o);
}

// bits of word t (nodes 64t .. 64t+63) that lie in [lo, hi)
__device__ __forceinline__ unsigned long long range_mask(uint32_t t, uint32_t lo, uint32_t hi) {
    const unsigned long long base = (unsigned long long)t * 64;
    const unsigned long long a = lo > base ? lo - base : 0, b = hi < base + 64 ? (hi > base ? hi - base : 0) : 64;
    if (a >= b) return 0ull;
    const unsigned long long upto_b = b == 64 ? ~0ull : ((1ull << b) - 1);
    return upto_b & ~((1ull << a) - 1);
}

template <int PLAN_THREADS>
__global__ void __launch_bounds__(PLAN_THREADS, 6) plan_kernel(const PlanIn *reqs, uint32_t lds_words) {
    constexpr int PLAN_WAVES = PLAN_THREADS / 64;
    extern __shared__ unsigned long long s_support[];
    __shared__ unsigned long long s_nb[KMAX];
    __shared__ uint32_t s_lab[KMAX], s_deg[KMAX], s_dsize[KMAX], s_order[KMAX], s_pos[KMAX];
    __shared__ uint32_t s_bw[KMAX], s_aff[KMAX];
    __shared__ int32_t s_par[KMAX];
    __shared__ unsigned long long s_mu[KMAX], s_fix_m[KMAX];
    __shared__ uint32_t s_first[KMAX], s_fix_t[KMAX], s_nfix;
    __shared__ unsigned long long s_need[KMAX * (TAB_COLS / 8)];
    __shared__ uint32_t s_coff[TAB_COLS], s_cix[KMAX], s_ncols;   // column byte offsets in the table
    __shared__ unsigned long long s_next;
    __shared__ int s_empty;

    const PlanIn R = reqs[blockIdx.x];
    const gp<const DevPattern> pat = glob(R.pat);
    const gp<InstDesc> desc = glob(R.desc);
    const gp<uint64_t> pos_bits = glob(R.pos_bits);
    const gp<uint32_t> lists = glob(R.lists);
    const uint32_t k = pat->k, n = R.n, W = R.W;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool use_dom = R.mode != SGE_RI;
    const bool use_si = R.mode == SGE_RIDS_SI || R.mode == SGE_RIDS_SI_FC;
    const gp<const NodeRec> node = glob(desc->node);
    const gp<const uint32_t> col = glob(desc->col);
    const gp<uint64_t> D = glob(R.dom);
    const gp<DevPlan> pl = glob(R.plan);

    if ((uint32_t)tid < k) {
        s_dsize[tid] = 0;
        s_first[tid] = 0xFFFFFFFFu;
        s_nb[tid] = pat->nb[tid];
        s_deg[tid] = pat->deg[tid];
        s_lab[tid] = R.labelled ? label_id(glob(R.label_keys), R.nlabels, pat->label[tid]) : LABEL_ANY;
    }
    if (tid == 0) {
        s_empty = 0;
        s_next = 0;
    }
    __syncthreads();

    // The first arc-consistency round of RI-DS against the neighbour-degree
    // table: v keeps its place in D(u) when, for every column c (a label, or
    // "any"), its largest neighbour degree of that column reaches need(u, c),
    // the largest degree among u's pattern neighbours of that column.  Up to
    // TAB_COLS columns are read per target node, each byte clamped to 127 and
    // packed eight to a word, so one word subtraction compares eight columns
    // (no borrow crosses a byte: pattern degrees are below 128).
    bool table = use_dom && R.nbr_deg != nullptr;
    for (uint32_t u = 0; u < k; u++) table &= s_lab[u] != LABEL_NONE;   // (an absent label empties a domain anyway)
    if (table && tid == 0) {
        unsigned long long nbs = 0;   // the pattern nodes that are someone's neighbour
        for (uint32_t u = 0; u < k; u++) nbs |= s_nb[u];
        uint32_t nc = 0;
        bool fits = true;
        for (; nbs && fits; nbs &= nbs - 1) {
            const uint32_t w = (uint32_t)__builtin_ctzll(nbs);
            const uint32_t c = (s_lab[w] == LABEL_ANY ? R.nbr_cols - 1 : s_lab[w]) * R.nbr_stride;
            uint32_t x = 0;
            while (x < nc && s_coff[x] != c) x++;
            if (x == nc) {
                if (nc == TAB_COLS) fits = false;
                else s_coff[nc++] = c;
            }
            s_cix[w] = x;
            fits &= s_deg[w] < 128;
        }
        for (uint32_t x = nc; x < TAB_COLS; x++) s_coff[x] = nc ? s_coff[0] : 0;   // read, never required
        s_ncols = fits ? nc : TAB_COLS + 1;
    }
    __syncthreads();
    const bool packed = table && s_ncols <= TAB_COLS;
    if (packed && (uint32_t)tid < k) {
        for (uint32_t q = 0; q < TAB_COLS / 8; q++) s_need[tid * (TAB_COLS / 8) + q] = 0;
        for (unsigned long long m = s_nb[tid]; m; m &= m - 1) {
            const uint32_t w = (uint32_t)__builtin_ctzll(m), x = s_cix[w];
            unsigned long long &nd = s_need[tid * (TAB_COLS / 8) + (x >> 3)];
            const uint32_t sh = 8 * (x & 7), cur = (uint32_t)(nd >> sh) & 0xFFu;
            if (s_deg[w] > cur) nd = (nd & ~(0xFFull << sh)) | ((unsigned long long)s_deg[w] << sh);
        }
    }
    if (packed) __syncthreads();

    // pattern node data by lane (lane u: node u)
    const bool mine = (uint32_t)lane < k;
    const unsigned long long mynb = mine ? s_nb[lane] : 0ull;
    const uint32_t mydeg = mine ? s_deg[lane] : 0u;

    // label and degree domains, with the table round when packed; lane l of a
    // wave decides node 64 i + l
    const uint32_t ngroups = packed ? (s_ncols + 7) / 8 : 0;
    const gp<const uint8_t> tab = glob(R.nbr_deg);
    constexpr unsigned long long H = 0x8080808080808080ull;
    static_assert(TAB_COLS == 24, "three column groups");
    // node v's label, degree and (packed) table bytes, ORed with H (all H when
    // not packed or v >= n)
    auto node_facts = [&](uint32_t v, uint32_t &vl, uint32_t &vd, unsigned long long &A0, unsigned long long &A1,
                          unsigned long long &A2) {
        unsigned long long A[TAB_COLS / 8] = {};
        vl = LABEL_NONE;
        vd = 0;
        if (v < n) {
            // the offsets are read in the loop (an opaque pointer keeps the
            // compiler from hoisting all of them into registers); the loads of
            // all groups are issued before the first is used
            __attribute__((address_space(3))) const uint32_t *coff =
                (__attribute__((address_space(3))) const uint32_t *)s_coff;
            asm volatile("" : "+v"(coff));
            // one variant per group count, so that no branch separates the loads
            auto load_groups = [&](auto ng) {
                constexpr uint32_t NG = decltype(ng)::value;
                uint32_t b[NG * 8];
#pragma unroll
                for (uint32_t x = 0; x < NG * 8; x++) b[x] = tab[v + coff[x]];
#pragma unroll
                for (uint32_t x = 0; x < NG * 8; x++) A[x / 8] |= (unsigned long long)min(b[x], 127u) << (8 * (x % 8));
            };
            if (ngroups == 1) load_groups(std::integral_constant<uint32_t, 1>{});
            else if (ngroups == 2) load_groups(std::integral_constant<uint32_t, 2>{});
            else if (ngroups == 3) load_groups(std::integral_constant<uint32_t, 3>{});
            const NodeRec r = ld_node(node + v);
            vl = r.label;
            vd = r.deg;
        }
        A0 = A[0] | H;
        A1 = A[1] | H;
        A2 = A[2] | H;
    };
    // RI-DS on a target of up to PLAN_WAVES * DT_WORDS words: each lane
    // keeps, for its nodes v = 64 i + lane (i = wave + PLAN_WAVES t), dt[t] =
    // the pattern nodes whose domain holds v, in registers through the
    // arc-consistency rounds; the domain rows are written once, at the end.
    // A round reads each node's list once, so adjacency rows (ORed a word at
    // a time per member of every dirty domain) pay only on targets whose mean
    // degree exceeds 8 W
    const bool reg_ac = use_dom && (!R.rows || R.deg_mean <= 8 * W) && W <= PLAN_WAVES * DT_WORDS && W * 64 <= lds_words;
    unsigned long long dt[DT_WORDS];
    if (reg_ac) {
        unsigned long long chg = 0;   // pattern nodes the table round removed a node from
#pragma unroll
        for (uint32_t t = 0; t < DT_WORDS; t++) {
            dt[t] = 0;
            const uint32_t i = wave + t * PLAN_WAVES;
            if (i < W) {
                const uint32_t v = i * 64 + lane;
                uint32_t vl, vd;
                unsigned long long A0, A1, A2;
                node_facts(v, vl, vd, A0, A1, A2);
                const bool valid = v < n;
                unsigned long long pm = 0, qm = 0;
                for (uint32_t u = 0; u < k; u++) {
                    // (bitwise, not short-circuit: no branch per node)
                    const uint32_t lu = s_lab[u], du = s_deg[u];
                    const unsigned long long *nd = &s_need[u * (TAB_COLS / 8)];
                    const bool p = valid & ((lu == LABEL_ANY) | (vl == lu)) & (vd >= du);
                    const bool q = p & ((ngroups == 0) | (((A0 - nd[0]) & (A1 - nd[1]) & (A2 - nd[2]) & H) == H));
                    pm |= (unsigned long long)p << u;
                    qm |= (unsigned long long)q << u;
                }
                dt[t] = qm;
                chg |= pm & ~qm;
            }
        }
        if (packed) {
            chg = wave_or64(chg);
            if (lane == 0 && chg) atomicOr(&s_next, chg);
        }
    } else {
        bool first_changed = false;   // lane u: the table round removed a node from D(u)
        for (uint32_t i = wave; i < W; i += PLAN_WAVES) {
            const uint32_t v = i * 64 + lane;
            const bool valid = v < n;
            uint32_t vl, vd;
            unsigned long long A0, A1, A2;
            node_facts(v, vl, vd, A0, A1, A2);
            unsigned long long row = 0, lrow = 0;
            // the pattern node's label, degree and needs are uniform LDS reads (broadcasts)
            if (ngroups == 0) {
                for (uint32_t u = 0; u < k; u++) {
                    const uint32_t lu = s_lab[u], du = s_deg[u];
                    const bool p = valid & ((lu == LABEL_ANY) | (vl == lu)) & (vd >= du);
                    const unsigned long long b = __ballot(p);
                    if ((uint32_t)lane == u) row = b;
                }
                lrow = row;
            } else {
                for (uint32_t u = 0; u < k; u++) {
                    const uint32_t lu = s_lab[u], du = s_deg[u];
                    const unsigned long long *nd = &s_need[u * (TAB_COLS / 8)];
                    const bool p = valid & ((lu == LABEL_ANY) | (vl == lu)) & (vd >= du);
                    const bool q = p & ((((A0 - nd[0]) & (A1 - nd[1]) & (A2 - nd[2]) & H) == H));
                    const unsigned long long b = __ballot(p), bq = __ballot(q);
                    if ((uint32_t)lane == u) {
                        lrow = b;
                        row = bq;
                    }
                }
            }
            if (mine) D[(size_t)lane * W + i] = row;
            first_changed |= row != lrow;
        }
        if (packed) {
            const unsigned long long ch = __ballot(mine && first_changed);
            if (lane == 0 && ch) atomicOr(&s_next, ch);
        }
    }
    __syncthreads();

    // arc-consistency to the fixpoint.  A round takes the nodes whose domain
    // changed in the previous round in batches of B: the support sets of a
    // batch are built side by side (LDS, or device scratch for very wide
    // rows), then every pattern neighbour of a batch member is revised
    // against the supports of its neighbours in the batch.
    // the support sets live in LDS or, for very wide rows, in device memory;
    // the rounds are instantiated for each, so every access has its own
    // address space
    auto arc_consistency = [&](auto Sb, const uint32_t B, unsigned long long dirty) {
        const gp<const uint64_t> adj = glob(desc->adj);
        while (dirty) {
            if (tid == 0) s_next = 0;
            unsigned long long rest = dirty;
            while (rest) {
                unsigned long long batch = 0;
                uint32_t nbat = 0;
                for (unsigned long long r = rest; r && nbat < B; r &= r - 1, nbat++) batch |= r & (~r + 1ull);
                rest &= ~batch;
                unsigned long long aff = 0;
                for (unsigned long long m = batch; m; m &= m - 1) aff |= s_nb[__builtin_ctzll(m)];
                const uint32_t naff = (uint32_t)__popcll(aff);
                if (tid == 0) {
                    uint32_t j = 0;
                    for (unsigned long long m = batch; m; m &= m - 1) s_bw[j++] = (uint32_t)__builtin_ctzll(m);
                    j = 0;
                    for (unsigned long long m = aff; m; m &= m - 1) s_aff[j++] = (uint32_t)__builtin_ctzll(m);
                }
                for (uint32_t idx = tid; idx < nbat * W; idx += PLAN_THREADS) Sb[idx] = 0;
                __syncthreads();
                // S(w) for the batch: every target neighbour of a member of D(w)
                for (uint32_t it = wave; it < nbat * W; it += PLAN_WAVES) {
                    const uint32_t j = it / W, i = it - j * W;
                    const uint64_t word = D[(size_t)s_bw[j] * W + i];
                    const auto Sj = Sb + (size_t)j * W;
                    if (R.rows) {
                        // adjacency rows, ORed word by word (lane t: word t)
                        for (uint32_t t0 = 0; t0 < W; t0 += 64) {
                            const uint32_t t = t0 + lane;
                            unsigned long long acc = 0;
                            if (t < W) {
                                for (unsigned long long m = word; m;) {
                                    const uint32_t x0 = i * 64 + (uint32_t)__builtin_ctzll(m);
                                    m &= m - 1;
                                    const uint32_t x1 = m ? i * 64 + (uint32_t)__builtin_ctzll(m) : x0;
                                    m &= m ? m - 1 : 0ull;
                                    const uint32_t x2 = m ? i * 64 + (uint32_t)__builtin_ctzll(m) : x0;
                                    m &= m ? m - 1 : 0ull;
                                    const uint32_t x3 = m ? i * 64 + (uint32_t)__builtin_ctzll(m) : x0;
                                    m &= m ? m - 1 : 0ull;
                                    acc |= adj[(size_t)x0 * W + t] | adj[(size_t)x1 * W + t] |
                                           adj[(size_t)x2 * W + t] | adj[(size_t)x3 * W + t];
                                }
                            }
                            if (acc) __hip_atomic_fetch_or(&Sj[t], acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    } else if ((word >> lane) & 1ull) {
                        // the member's neighbour list, four entries per round
                        const NodeRec r = ld_node(node + i * 64 + lane);
                        uint32_t e = r.begin;
                        const uint32_t end = r.begin + r.deg;
                        for (; e + 4 <= end; e += 4) {
                            const uint32_t y0 = col[e], y1 = col[e + 1], y2 = col[e + 2], y3 = col[e + 3];
                            __hip_atomic_fetch_or(&Sj[y0 >> 6], 1ull << (y0 & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            __hip_atomic_fetch_or(&Sj[y1 >> 6], 1ull << (y1 & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            __hip_atomic_fetch_or(&Sj[y2 >> 6], 1ull << (y2 & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            __hip_atomic_fetch_or(&Sj[y3 >> 6], 1ull << (y3 & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        for (; e < end; e++) {
                            const uint32_t y = col[e];
                            __hip_atomic_fetch_or(&Sj[y >> 6], 1ull << (y & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                }
                __syncthreads();
                // revise the pattern neighbours of the batch
                unsigned long long changed = 0;
                for (uint32_t it = tid; it < naff * W; it += PLAN_THREADS) {
                    const uint32_t a = it / W, i = it - a * W;
                    const uint32_t u = s_aff[a];
                    unsigned long long acc = ~0ull;
                    for (unsigned long long m = s_nb[u] & batch; m; m &= m - 1) {
                        const uint32_t j = (uint32_t)__popcll(batch & ((1ull << __builtin_ctzll(m)) - 1));
                        acc &= Sb[(size_t)j * W + i];
                    }
                    const uint64_t old = D[(size_t)u * W + i], nw = old & acc;
                    if (nw != old) {
                        D[(size_t)u * W + i] = nw;
                        changed |= 1ull << u;
                    }
                }
                if (changed) atomicOr(&s_next, changed);
                __syncthreads();
            }
            dirty = s_next;
            __syncthreads();
        }
    };
    if (use_dom) {
        unsigned long long dirty = 0;   // the nodes to revise the neighbours of
        for (uint32_t u = 0; u < k; u++)
            if (s_nb[u]) dirty |= 1ull << u;
        if (packed) {
            dirty = s_next;   // the nodes the table round changed
            __syncthreads();
        }
        if (reg_ac) {
            // rounds with the supports kept by target node: T[y] bit w is set
            // when target node y has a neighbour in D(w), for the w of the
            // round's dirty set.  A round clears T, scatters the list of every
            // node in the union of those domains (lane l: its nodes, each list
            // read once for all the w whose domain holds the node), then
            // revises every pattern neighbour u of the set: v stays in D(u) iff
            // T[v] holds every dirty neighbour of u.  (Without the packed table
            // round the first round starts from every node with a neighbour,
            // which reaches the same fixpoint.)
            unsigned long long *T = s_support;
            // a node index recomputed where it is used (an opaque copy of the
            // lane): hoisted out of the unrolled loops below, the addresses of
            // all DT_WORDS words spill
            auto node_of = [&](uint32_t i) {
                uint32_t l = (uint32_t)lane;
                asm volatile("" : "+v"(l));
                return i * 64 + l;
            };
            while (dirty) {
                unsigned long long aff = 0;
                for (unsigned long long m = dirty; m; m &= m - 1) aff |= s_nb[__builtin_ctzll(m)];
                if ((uint32_t)tid < k) s_mu[tid] = s_nb[tid] & dirty;
                if (tid == 0) s_next = 0;
                for (uint32_t idx = tid; idx < W * 64; idx += PLAN_THREADS) T[idx] = 0;
                __syncthreads();
#pragma unroll
                for (uint32_t t = 0; t < DT_WORDS; t++) {
                    const uint32_t i = wave + t * PLAN_WAVES;
                    const unsigned long long mask = i < W ? dt[t] & dirty : 0ull;
                    if (mask) {   // a member of some dirty domain: node i * 64 + lane < n
                        const NodeRec r = ld_node(node + node_of(i));
                        uint32_t e = r.begin;
                        const uint32_t end = r.begin + r.deg;
                        for (; e + 4 <= end; e += 4) {
                            const uint32_t y0 = col[e], y1 = col[e + 1], y2 = col[e + 2], y3 = col[e + 3];
                            __hip_atomic_fetch_or(&T[y0], mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            __hip_atomic_fetch_or(&T[y1], mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            __hip_atomic_fetch_or(&T[y2], mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            __hip_atomic_fetch_or(&T[y3], mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        for (; e < end; e++)
                            __hip_atomic_fetch_or(&T[col[e]], mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
                __syncthreads();
                unsigned long long removed = 0;   // pattern nodes whose domain lost a node
#pragma unroll
                for (uint32_t t = 0; t < DT_WORDS; t++) {
                    const uint32_t i = wave + t * PLAN_WAVES;
                    if (i < W) {
                        const unsigned long long tv = T[node_of(i)];
                        unsigned long long fail = 0;
                        for (unsigned long long m = dt[t] & aff; m; m &= m - 1) {
                            const uint32_t u = (uint32_t)__builtin_ctzll(m);
                            const unsigned long long mu = s_mu[u];
                            if ((tv & mu) != mu) fail |= 1ull << u;
                        }
                        dt[t] &= ~fail;
                        removed |= fail;
                    }
                }
                removed = wave_or64(removed);
                if (lane == 0 && removed) atomicOr(&s_next, removed);
                __syncthreads();
                dirty = s_next;
                __syncthreads();
            }
            // the domain rows (lane u: row u of each of the wave's words) and
            // sizes; the memberships stay in LDS (T[v], for forward checking)
            // with a member of each domain
            uint32_t cnt = 0;
#pragma unroll
            for (uint32_t t = 0; t < DT_WORDS; t++) {
                const uint32_t i = wave + t * PLAN_WAVES;
                if (i < W) {
                    T[node_of(i)] = dt[t];
                    unsigned long long row = 0;
                    for (uint32_t u = 0; u < k; u++) {
                        const unsigned long long b = __ballot((dt[t] >> u) & 1ull);
                        if ((uint32_t)lane == u) row = b;
                    }
                    if (mine) {
                        D[(size_t)lane * W + i] = row;
                        cnt += (uint32_t)__popcll(row);
                        if (row) atomicMin(&s_first[lane], i * 64 + (uint32_t)__builtin_ctzll(row));
                    }
                }
            }
            if (mine && cnt) atomicAdd(&s_dsize[lane], cnt);
            __syncthreads();
        } else if (!packed && table) {
            // the first round, against the label-and-degree domains: v has a
            // neighbour in D(w) iff it has a neighbour of w's label whose
            // degree is at least w's, which the target's neighbour-degree table
            // answers; the rounds below then revise only around the domains
            // this round changed (the host planner does the same)
            const gp<const uint8_t> tab = glob(R.nbr_deg);
            const uint32_t C = R.nbr_cols;
            if (tid == 0) s_next = 0;
            __syncthreads();
            for (uint32_t it = wave; it < k * W; it += PLAN_WAVES) {
                const uint32_t u = it / W, i = it - u * W;
                const unsigned long long nbu = s_nb[u];
                if (!nbu) continue;
                const uint64_t word = D[(size_t)u * W + i];
                bool keep = (word >> lane) & 1ull;
                if (keep) {   // a member: node i * 64 + lane < n (columns by label, 64 W entries each)
                    const gp<const uint8_t> vcol = tab + i * 64 + lane;
                    for (unsigned long long m = nbu; m; m &= m - 1) {
                        const uint32_t w = (uint32_t)__builtin_ctzll(m);
                        const uint32_t cw = s_lab[w] == LABEL_ANY ? C - 1 : s_lab[w];
                        if (vcol[(size_t)cw * R.nbr_stride] < s_deg[w]) {
                            keep = false;
                            break;
                        }
                    }
                }
                const unsigned long long nw = __ballot(keep);
                if (nw != word && lane == 0) {
                    D[(size_t)u * W + i] = nw;
                    atomicOr(&s_next, 1ull << u);
                }
            }
            __syncthreads();
            dirty = s_next;
            __syncthreads();
        }
        if (!reg_ac) {
            if (W <= lds_words)
                arc_consistency(s_support, max(1u, min(k, lds_words / max(W, 1u))), dirty);
            else
                arc_consistency(glob(reinterpret_cast<unsigned long long *>(R.support)), 1u, dirty);
        }
    }

    // domain sizes (RI-DS); an empty domain leaves nothing to search
    for (uint32_t u = wave; use_dom && !reg_ac && u < k; u += PLAN_WAVES) {
        uint32_t c = 0;
        for (uint32_t i = lane; i < W; i += 64) c += (uint32_t)__popcll(D[(size_t)u * W + i]);
        c = wave_sum(c);
        if (lane == 0) s_dsize[u] = c;
    }
    __syncthreads();
    if (use_dom && tid == 0)
        for (uint32_t u = 0; u < k; u++)
            if (s_dsize[u] == 0) s_empty = 1;
    __syncthreads();

    // forward checking (one wave; lane u holds |D(u)|)
    if (R.mode == SGE_RIDS_SI_FC && !s_empty && reg_ac) {
        // with the memberships in LDS (T[v]: the pattern nodes whose domain
        // holds v), every singleton of a cascade level at once (the removals
        // of distinct members commute, and a member shared by two singletons
        // empties both): lane u of a singleton finds its member (the
        // recorded first member of D(u) unless a removal took it, then T is
        // scanned), T tells which domains lose it, and the domain words that
        // changed are rewritten from T afterwards
        unsigned long long *T = s_support;
        if (wave == 0) {
            unsigned long long done = 0;
            uint32_t mysize = (uint32_t)lane < k ? s_dsize[lane] : 0;
            bool emp = false;
            uint32_t nfix = 0;
            while (!emp) {
                const unsigned long long cand = __ballot((uint32_t)lane < k && !((done >> lane) & 1ull) && mysize == 1);
                if (!cand) break;
                done |= cand;
                const bool single = (cand >> lane) & 1ull;
                uint32_t t = single ? s_first[lane] : 0u;
                const bool none = t == 0xFFFFFFFFu;
                if (none) t = 0;   // (every T index stays in range)
                const bool lost = single && (none || !((T[t] >> lane) & 1ull));
                for (unsigned long long m = __ballot(lost); m; m &= m - 1) {   // (rare) scan for the member
                    const uint32_t u = (uint32_t)__builtin_ctzll(m);
                    uint32_t found = 0;
                    for (uint32_t i0 = 0; i0 < W * 64; i0 += 64) {
                        const unsigned long long b = __ballot((T[i0 + lane] >> u) & 1ull);
                        if (b) {
                            found = i0 + (uint32_t)__builtin_ctzll(b);
                            break;
                        }
                    }
                    if ((uint32_t)lane == u) t = found;   // (|D(u)| = 1: a member exists)
                }
                const unsigned long long lose = single ? T[t] & ~(1ull << lane) : 0ull;
                // lane w: one node less for every singleton whose member lies in D(w)
                uint32_t dec = 0;
                for (unsigned long long m = cand; m; m &= m - 1) {
                    const int u = (int)__builtin_ctzll(m);
                    const unsigned long long lu =
                        ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(lose >> 32), u) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)lose, u);
                    dec += (uint32_t)((lu >> lane) & 1ull);
                }
                mysize -= dec;
                if (single) {
                    const uint32_t f = nfix + (uint32_t)__popcll(cand & ((1ull << lane) - 1));
                    s_fix_t[f] = t;
                    s_fix_m[f] = lose;
                    T[t] = 1ull << lane;
                }
                nfix += (uint32_t)__popcll(cand);
                emp = __ballot((uint32_t)lane < k && mysize == 0) != 0ull;
            }
            if ((uint32_t)lane < k) s_dsize[lane] = mysize;
            if (lane == 0) {
                s_nfix = nfix;
                if (emp) s_empty = 1;
            }
        }
        __syncthreads();
        for (uint32_t f = wave; f < s_nfix; f += PLAN_WAVES) {
            const uint32_t i = s_fix_t[f] >> 6;
            const unsigned long long tv = T[i * 64 + lane];
            for (unsigned long long m = s_fix_m[f]; m; m &= m - 1) {
                const uint32_t w = (uint32_t)__builtin_ctzll(m);
                const unsigned long long b = __ballot((tv >> w) & 1ull);
                if (lane == 0) D[(size_t)w * W + i] = b;
            }
        }
        __syncthreads();
    } else if (R.mode == SGE_RIDS_SI_FC && !s_empty) {
        if (wave == 0) {
            unsigned long long done = 0;
            uint32_t mysize = (uint32_t)lane < k ? s_dsize[lane] : 0;
            bool emp = false;
            while (!emp) {
                const unsigned long long cand = __ballot((uint32_t)lane < k && !((done >> lane) & 1ull) && mysize == 1);
                if (!cand) break;
                const uint32_t u = (uint32_t)__builtin_ctzll(cand);
                done |= 1ull << u;
                uint32_t t = 0xFFFFFFFFu;   // the member of D(u)
                for (uint32_t i0 = 0; i0 < W; i0 += 64) {
                    const uint32_t i = i0 + lane;
                    const unsigned long long x = i < W ? D[(size_t)u * W + i] : 0ull;
                    const unsigned long long b = __ballot(x != 0ull);
                    if (b) {
                        const uint32_t j = (uint32_t)__builtin_ctzll(b);
                        const unsigned long long xw = __shfl(x, (int)j);
                        t = (i0 + j) * 64 + (uint32_t)__builtin_ctzll(xw);
                        break;
                    }
                }
                if (t != 0xFFFFFFFFu && (uint32_t)lane < k && (uint32_t)lane != u) {
                    const gp<uint64_t> pw = &D[(size_t)lane * W + (t >> 6)];
                    const uint64_t bit = 1ull << (t & 63);
                    const uint64_t x = *pw;
                    if (x & bit) {
                        *pw = x & ~bit;
                        mysize--;
                    }
                }
                emp = __ballot((uint32_t)lane < k && mysize == 0) != 0ull;
            }
            if ((uint32_t)lane < k) s_dsize[lane] = mysize;
            if (emp && lane == 0) s_empty = 1;
        }
        __syncthreads();
    }
    const bool empty = s_empty != 0;

    // the constraint-first order.  RI's depends on the pattern alone and was
    // computed when the pattern was loaded; with domains one wave scores the
    // pattern nodes (lane u: node u)
    if (!use_dom && (uint32_t)tid < k) s_order[tid] = pat->ri_order[tid];
    if (use_dom && !empty && wave == 0) {
        const uint32_t mysz = mine ? s_dsize[lane] : 0u;
        // with SI, the key holds u's rank among the domain sizes (the number
        // of pattern nodes with a smaller domain: the same order and the same
        // ties as the sizes, in six bits)
        uint32_t srank = 0;
        if (use_si)
            for (uint32_t w = 0; w < k; w++)
                srank += (uint32_t)__builtin_amdgcn_readlane((int)mysz, (int)w) < mysz ? 1u : 0u;
        unsigned long long placed = 0;
        uint32_t len = 0;
        for (unsigned long long single = __ballot(mine && mysz == 1); single; single &= single - 1) {
            const uint32_t u = (uint32_t)__builtin_ctzll(single);
            if (lane == 0) s_order[len] = u;
            len++;
            placed |= 1ull << u;
        }
        while (len < k) {
            // w_n(u) counts the placed w sharing an unplaced neighbour x with u:
            // the placed members of the union of N(x) over unplaced x in N(u).
            // Only the frontier (unplaced x with a placed neighbour) adds
            // anything; N(x) is lane x's row, read into scalar registers
            const unsigned long long front = __ballot(mine && !((placed >> lane) & 1ull) && (mynb & placed) != 0ull);
            unsigned long long two_hop = 0;
            for (unsigned long long m = front; m; m &= m - 1) {
                const int x = (int)__builtin_ctzll(m);
                const unsigned long long nx =
                    ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mynb >> 32), x) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mynb, x);
                two_hop |= nx & (0ull - ((mynb >> x) & 1ull));
            }
            uint32_t key = 0;
            if (mine && !((placed >> lane) & 1ull)) {
                const uint32_t wm = (uint32_t)__popcll(mynb & placed);
                const uint32_t wn = (uint32_t)__popcll(two_hop & placed);
                // w_m, w_n and degree are below 64; the smaller domain (a
                // larger 63 - rank) and then the lower id win the remaining ties
                key = (1u << 30) | (wm << 24) | (wn << 18) | (mydeg << 12) | ((63u - srank) << 6) | (63u - lane);
            }
            // the keys are distinct (their lowest bits are the lane), so the
            // wave-wide maximum, a wave-uniform value, names the node, which
            // keeps `placed` and the loop above scalar
            const uint32_t u = 63u - (wave_reduce(key, [](uint32_t a, uint32_t b) { return a > b ? a : b; }) & 63u);
            if (lane == 0) s_order[len] = u;
            len++;
            placed |= 1ull << u;
        }
    }
    __syncthreads();

    if (tid == 0) {
        pl->k = k;
        pl->W = W;
        pl->n = n;
        pl->use_dom = use_dom ? 1u : 0u;
        pl->labelled = R.labelled;
        pl->empty = empty ? 1u : 0u;
        pl->flags = 0;   // undirected, edge labels not compared
        if (empty) {
            pl->list_len[0] = 0;
            desc->nroot = 0;
        }
    }
    if (empty) return;

    // parents and back-edges (lane i: position i)
    if ((uint32_t)tid < k) s_pos[s_order[tid]] = (uint32_t)tid;
    __syncthreads();
    if ((uint32_t)tid < k) {
        const uint32_t u = s_order[tid];
        unsigned long long earlier = 0;
        for (unsigned long long m = s_nb[u]; m; m &= m - 1) {
            const uint32_t j = s_pos[__builtin_ctzll(m)];
            if (j < (uint32_t)tid) earlier |= 1ull << j;
        }
        const int32_t par = earlier ? (int32_t)__builtin_ctzll(earlier) : -1;
        s_par[tid] = par;
        pl->parent[tid] = par;
        pl->back[tid] = earlier ? (earlier & (earlier - 1)) : 0ull;
        pl->plabel[tid] = s_lab[u];
        pl->pdeg[tid] = s_deg[u];
        pl->order[tid] = u;
        pl->list_off[tid] = 0;
        pl->list_len[tid] = 0;
    }
    __syncthreads();

    // per-position bitsets: the domain (RI-DS) or the label/degree set (RI)
    if (pos_bits) {
        const uint32_t kw = k * W;
        for (uint32_t idx = tid; idx < kw; idx += PLAN_THREADS) {
            const uint32_t i = idx / W, t = idx - i * W;
            uint64_t x = D[(size_t)s_order[i] * W + t];
            if (i == 0) x &= range_mask(t, R.root_lo, R.root_hi);
            pos_bits[idx] = x;
        }
    }
    // candidate lists of the parentless positions, in increasing node order
    if (wave == 0) {
        uint32_t off = 0;
        for (uint32_t i = 0; i < k; i++) {
            if (s_par[i] >= 0) continue;
            const gp<const uint64_t> row = &D[(size_t)s_order[i] * W];
            const uint32_t start = off;
            for (uint32_t i0 = 0; i0 < W; i0 += 64) {
                const uint32_t t = i0 + lane;
                unsigned long long x = t < W ? row[t] : 0ull;
                if (i == 0) x &= range_mask(t, R.root_lo, R.root_hi);
                const uint32_t c = (uint32_t)__popcll(x);
                uint32_t s = c;
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(s, o);
                    if (lane >= o) s += y;
                }
                uint32_t o = off + s - c;
                for (unsigned long long y = x; y; y &= y - 1, o++)
                    if (o < R.list_cap) lists[o] = t * 64 + (uint32_t)__builtin_ctzll(y);
                off += __shfl(s, 63);
            }
            // lists fit by construction (list_cap); should they not, keep
            // every list inside the buffer
            const uint32_t len = off > R.list_cap ? (start < R.list_cap ? R.list_cap - start : 0u) : off - start;
            if (lane == 0) {
                pl->list_off[i] = start;
                pl->list_len[i] = len;
                if (i == 0) desc->nroot = len;
            }
        }
    }
}

// Root chunks of every instance and their exclusive prefix (one block).
constexpr int FIN_THREADS = 1024;

__global__ void __launch_bounds__(FIN_THREADS)
    finalize_kernel(InstDesc *desc, unsigned *prefix, uint32_t m, int policy, uint32_t root_chunk,
                    unsigned long long units) {
    __shared__ unsigned long long s_red[FIN_THREADS];
    __shared__ unsigned s_scan[FIN_THREADS];
    const int tid = threadIdx.x;
    unsigned long long t = 0;
    for (uint32_t j = tid; j < m; j += FIN_THREADS) t += desc[j].nroot;
    s_red[tid] = t;
    __syncthreads();
    for (int o = FIN_THREADS / 2; o > 0; o >>= 1) {
        if (tid < o) s_red[tid] += s_red[tid + o];
        __syncthreads();
    }
    const unsigned long long total = s_red[0];
    const unsigned long long q = total / (4ull * (units ? units : 1ull));
    const uint32_t chunk_default = q < 1 ? 1u : (q > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)q);
    // thread tid owns instances [lo, hi)
    const uint32_t per = (m + FIN_THREADS - 1) / FIN_THREADS;
    const uint32_t lo = min(m, (uint32_t)tid * per), hi = min(m, lo + per);
    unsigned local = 0;
    for (uint32_t j = lo; j < hi; j++) {
        const uint32_t nr = desc[j].nroot;
        uint32_t chunk;
        if (policy == 1) chunk = nr ? nr : 1u;
        else if (root_chunk) chunk = root_chunk;
        else chunk = chunk_default;
        const uint32_t nch = nr ? (uint32_t)(((unsigned long long)nr + chunk - 1) / chunk) : 0u;
        desc[j].chunk = chunk;
        desc[j].nchunks = nch;
        local += nch;
    }
    s_scan[tid] = local;
    __syncthreads();
    for (int o = 1; o < FIN_THREADS; o <<= 1) {   // inclusive scan
        const unsigned y = tid >= o ? s_scan[tid - o] : 0u;
        __syncthreads();
        s_scan[tid] += y;
        __syncthreads();
    }
    unsigned base = s_scan[tid] - local;
    for (uint32_t j = lo; j < hi; j++) {
        prefix[j] = base;
        base += desc[j].nchunks;
    }
    if (tid == FIN_THREADS - 1) prefix[m] = s_scan[tid];
}

}  // namespace

hipError_t launch_plan(const PlanIn *reqs, uint32_t m, uint32_t wmax, uint32_t kmax, InstDesc *desc, unsigned *chunk_prefix,
                       int policy, uint32_t root_chunk, uint64_t units, hipStream_t s) {
    if (m == 0) return hipSuccess;
    // support words: up to PLAN_LDS_WORDS (one per node of the widest target,
    // or its rows times the largest pattern, when that is smaller)
    const uint64_t w1 = std::max<uint32_t>(wmax, 1);
    const uint32_t words =
        (uint32_t)std::min<uint64_t>(std::max<uint64_t>(w1 * 64, w1 * std::max<uint32_t>(kmax, 1)), PLAN_LDS_WORDS);
    // One launch, the largest plans first (the requests come ordered by
    // estimated work).  Per-workgroup start and end stamps on the 4096-pair
    // batch (a timing build) show about 440 of the 512 resident slots busy
    // until the last requests; the largest plan takes under half the launch.
    // A split into two launches on two streams of the captured graph ran them
    // back to back; 640, 896 and 512 threads were slower than 768.
    hipLaunchKernelGGL(plan_kernel<PLAN_THREADS>, dim3(m), dim3(PLAN_THREADS), (size_t)words * 8, s, reqs, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(FIN_THREADS), 0, s, desc, chunk_prefix, m, policy, root_chunk,
                       (unsigned long long)units);
    return hipGetLastError();
}

}  // namespace sge
