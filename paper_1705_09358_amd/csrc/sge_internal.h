// Internal declarations shared by the host code and the HIP search kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "sge.h"

namespace sge {

constexpr uint32_t KMAX = 64;              // largest pattern (positions held in 64-bit masks)
constexpr uint32_t LABEL_ANY = 0xFFFFFFFEu;  // unlabelled search: every label matches
constexpr uint32_t LABEL_NONE = 0xFFFFFFFFu; // pattern label absent from the target
constexpr uint32_t QUEUE_SLOTS = 4096;     // work-queue capacity (tasks)

// ---------------------------------------------------------------- host graphs
// A graph as the host keeps it.  rp/col: the out-edges (both directions of
// every edge when undirected), sorted rows; elab: one label per col entry, or
// empty (all 0).  A directed graph also keeps its in-edges (irp/icol/ielab,
// rows sorted by source); an undirected one reads them from rp/col/elab.
struct HostGraph {
    uint32_t n = 0;
    std::vector<uint32_t> rp, col, lab;  // lab: raw labels as given (0 if none)
    std::vector<uint32_t> elab;
    std::vector<uint32_t> irp, icol, ielab;
    bool has_labels = false, directed = false;

    uint32_t outdeg(uint32_t v) const { return rp[v + 1] - rp[v]; }
    uint32_t indeg(uint32_t v) const { return directed ? irp[v + 1] - irp[v] : rp[v + 1] - rp[v]; }
    const std::vector<uint32_t> &in_rp() const { return directed ? irp : rp; }
    const std::vector<uint32_t> &in_col() const { return directed ? icol : col; }
    const std::vector<uint32_t> &in_elab() const { return directed ? ielab : elab; }
    bool has_elab() const { return !elab.empty(); }
};

// Validate and normalise CSR input: sort rows, merge duplicate entries
// (which must carry one label), reject self-loops and out-of-range ids;
// undirected input must hold both directions of every edge with one label.
// Returns an empty string on success, else the reason.
std::string normalise_graph(uint32_t n, const uint32_t *row_ptr, const uint32_t *col, const uint32_t *labels,
                            const uint32_t *edge_labels, bool directed, HostGraph &out);
inline std::string normalise_graph(uint32_t n, const uint32_t *row_ptr, const uint32_t *col, const uint32_t *labels,
                                   HostGraph &out) {
    return normalise_graph(n, row_ptr, col, labels, nullptr, false, out);
}

// Per-node record read by the search: row start and degree in the CSR, and
// the dense label id.
struct NodeRec {
    uint32_t begin, deg, label, pad;
};

// One entry of a wide CSR row: the neighbour and its node record fields.
struct WideEntry {
    uint32_t v, begin, deg, label;
};

// A target resident on the device, with the host copies the planner reads.
struct Target {
    HostGraph g;
    std::vector<uint32_t> dlab;                  // dense label id per node
    std::vector<uint32_t> label_keys;            // dense id -> raw label (increasing)
    std::vector<std::vector<uint32_t>> by_label; // dense id -> nodes
    uint32_t W = 0;                              // 64-bit words per bitset row
    uint32_t max_deg = 0;
    // nbr_deg[L * nbr_stride + v]: largest degree (saturated at 255) among
    // the neighbours of v with dense label L; column nbr_cols - 1 ignores
    // labels.  Stored by column (nbr_stride = 64 W bytes, zero padded), so a
    // domain word's 64 nodes have their entries side by side.
    // Empty when n * nbr_cols would exceed NBR_DEG_MAX_BYTES.
    std::vector<uint8_t> nbr_deg;
    uint32_t nbr_cols = 0;
    uint32_t nbr_stride = 0;
    // undirected targets: the nodes of each dense label (label_bits, one row
    // of W words per label) and of degree >= d (deg_ge, rows d = 0..63), so a
    // label-and-degree domain is one AND of two rows; empty when too large
    std::vector<uint64_t> label_bits, deg_ge;
    // device
    uint32_t *d_col = nullptr;
    NodeRec *d_node = nullptr;
    uint64_t *d_adj = nullptr;                   // n * W, or null when too large
    uint32_t *d_label_keys = nullptr;            // label_keys on the device
    WideEntry *d_wcol = nullptr;                 // undirected: per CSR entry {neighbour, its row start, degree, label}
    uint32_t *d_irp = nullptr, *d_icol = nullptr;   // directed: in-edges
    uint32_t *d_elab = nullptr, *d_ielab = nullptr; // edge labels (out, in), or null
    uint8_t *d_nbr_deg = nullptr;                // nbr_deg on the device (undirected), or null
    uint64_t dev_bytes = 0;
    uint32_t serve_refs = 0;                     // server queries in flight on it (under the server's lock)
};

// A pattern as the plan kernel reads it (resident on the device).
struct DevPattern {
    uint32_t k, ncomp;            // nodes, connected components
    uint32_t pad[2];
    uint64_t nb[KMAX];            // bit w of nb[u]: {u, w} is a pattern edge
    uint32_t label[KMAX];         // raw labels
    uint32_t deg[KMAX];
    uint32_t ri_order[KMAX];      // the RI order (pattern structure only), computed when the pattern is loaded
};

struct Pattern {
    HostGraph g;
    uint32_t ncomp = 0;
    DevPattern *d_pat = nullptr;
    uint32_t serve_refs = 0;                     // server queries in flight on it (under the server's lock)
};

// Plan flags: directions or edge labels take part in the search.
constexpr uint32_t PLAN_DIRECTED = 1u, PLAN_EDGE_LABELS = 2u;

// Search plan of one (pattern, target, mode, labelled) instance.
struct Plan {
    uint32_t k = 0, n = 0, W = 0;
    int mode = SGE_RI;
    bool labelled = true;
    bool empty = false;        // a domain became empty: no match, nothing to search
    uint32_t flags = 0;        // PLAN_DIRECTED | PLAN_EDGE_LABELS
    uint32_t order[KMAX];      // position -> pattern node
    int32_t parent[KMAX];      // position -> earlier position or -1
    uint64_t back[KMAX];       // earlier adjacent positions other than the parent
    uint64_t bout[KMAX];       // directed: earlier positions (not the parent) with an arc into this one
    uint64_t bin[KMAX];        // directed: earlier positions (not the parent) this one has an arc to
    uint64_t pdir_out = 0;     // bit i: position i's candidates are out-neighbours of its parent's image
    uint64_t pboth = 0;        // bit i: arcs both ways between position i and its parent
    uint32_t plabel[KMAX];     // dense target label id, LABEL_ANY or LABEL_NONE
    uint32_t pdeg[KMAX];       // out-degree (the degree when undirected)
    uint32_t pindeg[KMAX];     // in-degree
    std::vector<uint32_t> lmat;   // edge labels: k*k, [a*k+b] = label of arc order[a] -> order[b] or LABEL_NONE
    std::vector<uint64_t> dom_node;   // RI-DS: k * W final domains by pattern node
    std::vector<uint32_t> lists;      // candidate lists of parentless positions
    uint32_t list_off[KMAX], list_len[KMAX];
};

// Build the plan.  When want_pos_bitsets is set, `pos_bits` receives k * W
// words by position: the domain (RI-DS) or the label/degree-compatible set
// (RI), as the dense search reads them.
// The constraint-first order (Section "RI"; with domains, singletons first,
// and with SI the domain-size tie-break of Section 4.2.1): repeatedly the
// unplaced node with the most placed neighbours (w_m), then the most placed
// nodes sharing an unplaced neighbour with it (w_n), then the largest degree
// `odeg`, then (use_si) the smallest domain `dsize`, then the lowest id.
// `dsize` may be null when neither use_dom nor use_si is set.
void constraint_first_order(const uint64_t *nb, const uint32_t *odeg, const uint32_t *dsize, uint32_t k, bool use_dom,
                            bool use_si, uint32_t *order);
void build_plan(const Target &t, const HostGraph &p, int mode, bool labelled, uint32_t root_lo, uint32_t root_hi,
                Plan &plan, bool want_pos_bitsets, std::vector<uint64_t> &pos_bits);

constexpr uint64_t NBR_DEG_MAX_BYTES = 256ull << 20;
constexpr uint64_t LABEL_DEG_BITS_MAX_BYTES = 64ull << 20;

// Dense label ids of a target (fills dlab, label_keys, by_label, W, max_deg)
// and its neighbour-degree table.
void index_target(Target &t);

// ------------------------------------------------------------ device structs
// Everything one instance of the search needs, as the kernels read it.
struct DevPlan {
    uint32_t k, W, n, use_dom;
    uint32_t labelled, empty, flags, pad2;   // empty: a domain became empty (nothing to search)
    int32_t parent[KMAX];
    uint64_t back[KMAX];
    uint32_t plabel[KMAX];
    uint32_t pdeg[KMAX];                     // out-degree (the degree when undirected)
    uint32_t order[KMAX];
    uint32_t list_off[KMAX];
    uint32_t list_len[KMAX];
    // with PLAN_DIRECTED or PLAN_EDGE_LABELS (plans built on the host)
    uint32_t pindeg[KMAX];
    uint64_t bout[KMAX], bin[KMAX];
    uint64_t pdir_out, pboth;
};

struct InstDesc {
    const uint32_t *col;      // target CSR column array (out-edges)
    const NodeRec *node;      // target node records (pad = in-degree)
    const WideEntry *wcol;    // undirected target: per CSR entry {neighbour, row start, degree, label}, or null
    const uint32_t *irp;      // directed target: in-edge row starts (n+1), else null
    const uint32_t *icol;     // directed target: in-edges, rows sorted by source, else null
    const uint32_t *elab;     // target edge labels per out entry, or null (all 0)
    const uint32_t *ielab;    // target edge labels per in entry, or null
    const uint32_t *lmat;     // k*k pattern arc labels by position pair (PLAN_EDGE_LABELS), or null
    const uint64_t *adj;      // target adjacency bitsets (n*W) or null
    const DevPlan *plan;
    const uint64_t *bits;     // k*W by position: domains (CSR RI-DS) or dense-mode sets, or null
    const uint32_t *lists;    // candidate lists of parentless positions
    uint32_t *rows;           // output rows or null
    unsigned long long cap_rows;
    uint32_t nchunks;         // root chunks of this instance
    uint32_t chunk;           // root candidates per chunk
    uint32_t nroot;           // candidates of position 0
    uint32_t pad;
};

// One instance's plan request: the plan kernel turns the resident pattern
// and target into the DevPlan, the per-position bitsets and the candidate
// lists of the instance (Sections "RI" and 4), and the finalize kernel sets
// the root chunking of every instance.
struct PlanIn {
    const DevPattern *pat;
    const uint32_t *label_keys;   // the target's raw labels by dense id (increasing)
    uint32_t nlabels;
    uint32_t mode, labelled, n, W;
    uint32_t root_lo, root_hi;
    uint32_t list_cap;            // entries `lists` holds: ncomp*n + k (a singleton domain adds one)
    const uint8_t *nbr_deg;       // the target's neighbour-degree table (nbr_cols columns), or null
    uint32_t nbr_cols, nbr_stride;
    uint32_t rows;                // build support sets from adjacency rows (dense targets), not lists
    uint32_t deg_mean;            // the target's mean degree, rounded up
    InstDesc *desc;               // the instance's search descriptor (col, node read; nroot written)
    DevPlan *plan;                // written
    uint64_t *dom;                // k*W words: domains by pattern node (written)
    uint64_t *pos_bits;           // k*W words by position (written), or null
    uint32_t *lists;              // room for list_cap candidates (written)
    uint64_t *support;            // W words of scratch when W exceeds the plan kernel's LDS
};

// Per-instance device counters.  pad0: set when the instance's states
// exceeded the cap; bytes: algorithmic bytes of the search (when counted).
struct InstCounters {
    unsigned long long matches, states, candidates, steals, row_next, pad0, steps, bytes;
};

constexpr uint32_t QUEUE_GROUPS = 8;                          // work-queue groups
constexpr uint32_t QUEUE_GROUP_SLOTS = QUEUE_SLOTS / QUEUE_GROUPS;
constexpr uint32_t TASK_ENTRIES = 16;                        // accepted candidates one task can carry
constexpr uint32_t DEFAULT_DONATE_PERIOD = 32;               // steps between a unit's donations
constexpr uint32_t HANDOFF_PERIOD = 4;                        // steps before a unit hands a piece to an idle wave-mate

// Counters of one work-queue group, each on its own 128-byte line.
struct QGroup {
    unsigned int tail;         // producer tickets
    unsigned int p0[31];
    unsigned int head;         // consumer tickets
    unsigned int p1[31];
    unsigned int avail;        // published, not yet taken
    unsigned int p2[31];
    unsigned int free;         // free slots
    unsigned int p3[31];
    unsigned int created;      // tasks given away into the queues (monotonic)
    unsigned int p4[31];
    unsigned int finished;     // tasks finished, root chunks included (monotonic)
    unsigned int p5[31];
};

// Global scheduling words of one launch.
struct Sched {
    unsigned int chunk_next;   // next root chunk (flattened over instances)
    unsigned int p0[31];
    unsigned int done;         // set once every task is finished
    unsigned int abort;        // set when the launch's time limit is reached
    unsigned int bad;          // 1: a dequeued task failed validation; 2: a unit's lanes disagreed
                               // on its state (checked on request); never expected
    unsigned int units;        // units that entered the search loop
    unsigned int p1[28];
    unsigned long long t_start;  // earliest block start (s_memrealtime, 100 MHz)
    unsigned long long t_end;    // latest wave exit
    unsigned long long t_work;   // latest task finish
    unsigned long long t_done;   // when `done` was set
    unsigned long long t_busy;   // sum over units of the ticks each held a task
    unsigned long long p2[11];
    QGroup grp[QUEUE_GROUPS];
};

// One queued task: instance, prefix length L and prefix mapping M[0..L-1],
// and what of position L it covers -- by `kind`: a range [lo, hi) of its
// candidate list (hi = 0xFFFFFFFF: the whole list); `ne` accepted candidates
// in `ent` (already counted); or, dense, the words [lo, hi) of its candidate
// set (already counted).
struct QTask {
    unsigned int seq;
    unsigned int inst, L, lo, hi, kind, ne, pad;
    unsigned int M[KMAX];
    unsigned int ent[TASK_ENTRIES];
};

struct LaunchCfg {
    int lanes = 16;           // lanes per search unit
    int dense = 0;            // dense-bitset kernel
    int donate = 1;            // 0 off, 1 default period, N > 1: period of N steps
    uint32_t kmax = 0, nmax = 0, wmax = 0;
    int blocks = 0;           // 0 = fill the device
    int per_cu = 0;           // with blocks = 0: at most this many resident blocks per CU (0 = all that fit)
    int used_bitset = 1;      // CSR: a used-node bitset per unit in LDS (else the prefix is compared)
    int general = 0;          // some plan is directed or compares edge labels (CSR kernel with those checks)
    int count_bytes = 1;      // count each instance's algorithmic bytes
    int check_uniform = 0;    // verify that a unit's lanes agree on its state every step
    uint32_t root_lo = 0, root_hi = 0xFFFFFFFFu;   // the first position's target-id range
};

// Device-side work state of a context (allocated once, reused per launch).
struct DevWork {
    Sched *sched = nullptr;
    QTask *queue = nullptr;
    unsigned int *chunk_prefix = nullptr;  // per instance: exclusive prefix of chunks (ninst+1)
    size_t chunk_prefix_cap = 0;
    InstDesc *inst = nullptr;
    size_t inst_cap = 0;
    InstCounters *ctr = nullptr;
    size_t ctr_cap = 0;
};

// Plan `m` instances (one workgroup each, requests in decreasing order of
// estimated work), then set every instance's root chunks and the chunk
// prefix: `policy` 1 = one chunk per instance, else `root_chunk` candidates
// per chunk, or (0) the total roots over 4 * `units`.
hipError_t launch_plan(const PlanIn *reqs, uint32_t m, uint32_t wmax, uint32_t kmax, InstDesc *desc, unsigned *chunk_prefix,
                       int policy, uint32_t root_chunk, uint64_t units, hipStream_t s);
// LDS words of the plan kernel's support buffer (larger W uses PlanIn::support):
// 64 KB, so two plan workgroups reside per CU, and a target of up to 8192
// nodes keeps one support word per node.
constexpr uint32_t PLAN_LDS_WORDS = 8192;

// Launch one persistent search over `ninst` planned instances.  The grid is
// the resident maximum (or cfg.blocks); blocks beyond what the root chunks
// can keep busy leave at once.  Returns a HIP error code.
hipError_t launch_search(const LaunchCfg &cfg, DevWork &w, uint32_t ninst, uint64_t state_cap,
                         uint64_t time_limit_ms, hipStream_t s, int num_cus);
// Shared memory a block of the search kernel needs.
size_t search_lds_bytes(const LaunchCfg &cfg);
// Threads per block of the search kernel (256, 128 or 64; 0: one unit's LDS
// does not fit in 64 KiB).
int search_block_threads(const LaunchCfg &cfg);
// The search kernel function launch_search launches for `cfg` (to find its
// node in a captured graph).
const void *search_kernel_fn(const LaunchCfg &cfg);
// Clear the scheduling words of a launch (a fill kernel; usable in a captured graph).
hipError_t launch_reset(DevWork &w, uint32_t ninst, hipStream_t s);

}  // namespace sge
