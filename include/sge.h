/*
 * sge.h -- C ABI of the MI355X (gfx950) subgraph-enumeration library.
 *
 * The library enumerates or counts every non-induced, label-preserving
 * embedding of a pattern graph in a target graph: every injective
 * M : V_p -> V_t with lab(u) = lab(M u) (when labelled) and (M u, M w) in E_t
 * for every pattern edge (u, w) -- Kimmig, Meyerhenke, Strash, "Shared Memory
 * Parallel Subgraph Enumeration" (arXiv 1705.09358), Section 2.1, eqs. (2)-(3)
 * and the remark after them that the subgraphs are non-induced.
 *
 * The search is RI (Bonnici et al.) as the paper restates it: a depth-first
 * search over a static constraint-first order of the pattern nodes, taking the
 * candidates for each pattern node from the target neighbours of its already
 * mapped parent and pruning with four rules (unused, equal label, degree,
 * edges to mapped nodes).  RI-DS adds domains (Section 4.1): per pattern node
 * the compatible target nodes, filtered by arc-consistency.  The paper's
 * improvements (Section 4.2) are the domain-size tie-break of the order (SI)
 * and forward checking on singleton domains (FC).
 *
 * Conventions for every call:
 *  - Return value: SGE_OK (0) or a negative sge_status; the context keeps a
 *    message for the last error (sge_last_error).
 *  - Graphs are undirected and simple.  They are passed as symmetric CSR:
 *    row_ptr[n+1] (row_ptr[0] = 0, non-decreasing) and col[row_ptr[n]] with
 *    every id < n.  Rows may be unsorted and may hold duplicates (both are
 *    normalised); a self-loop or an asymmetric entry is SGE_E_INVAL.
 *  - Input arrays are host pointers, borrowed for the duration of the call
 *    and copied in.  Output buffers belong to the caller.
 *  - Handles belong to the context and die with it.
 *  - One context per host thread.  The serve calls are internally
 *    synchronised.
 *  - Pattern size k <= 64.  k = 0 has exactly one (empty) match; k > n has
 *    none.
 *  - Rows: a match is written as k uint32 values in pattern-id order,
 *    row[u] = M(u).  Rows come out in an unspecified order.
 */
#ifndef SGE_H
#define SGE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sge_status;
enum {
    SGE_OK = 0,
    SGE_E_INVAL = -1,     /* bad argument or malformed graph                          */
    SGE_E_NOMEM = -2,     /* host or device allocation failed                         */
    SGE_E_DEVICE = -3,    /* a HIP call failed (message holds the HIP error string),
                             or the search kernel rejected a malformed queued task  */
    SGE_E_OVERFLOW = -4,  /* more matches than rows given: counts are complete, the
                             first cap_rows rows are valid                             */
    SGE_E_ABORTED = -5,   /* states exceeded the cap: counters are partial            */
    SGE_E_BUSY = -6,      /* serve: not admissible now / result not ready yet         */
    SGE_E_HANDLE = -7     /* unknown target, pattern or ticket handle                 */
};

/* Search variants.  RI: Section "RI" (candidates from the parent, rules 1-4).
 * RIDS: Section 4.1 domains with arc-consistency, singleton domains first in
 * the order, roots from the first node's domain, domain test before the rules.
 * RIDS_SI: plus the domain-size tie-break of the order (Section 4.2.1).
 * RIDS_SI_FC: plus forward checking on singleton domains (Section 4.2.2). */
enum { SGE_RI = 0, SGE_RIDS = 1, SGE_RIDS_SI = 2, SGE_RIDS_SI_FC = 3 };

/* Counters of one search.
 *  matches     complete embeddings found;
 *  states      accepted (pattern node, target node) pairs, i.e. consistent
 *              partial mappings summed over their lengths -- independent of
 *              the traversal order and the parallel schedule;
 *  candidates  pairs examined (implementation-dependent, for reporting);
 *  alg_bytes   the algorithmic bytes of the search: what the method itself
 *              must read, by a per-unit model of the traversal, the
 *              numerator of the memory roofline (0 when counting is off,
 *              sge_set_count_bytes).  It depends on the instance and the
 *              kernel variant, not on the schedule.  CSR search: per
 *              expansion of a position with a parent, 8 bytes (list bounds)
 *              plus 4 per id in the parent image's neighbour list; per
 *              candidate 5 bytes (RI: label and degree) or 8 (RI-DS: a
 *              domain word); per back-edge probe 8 bytes, earliest position
 *              first, up to the first that fails (general graphs: an arc in
 *              each direction per earlier position, plus 4 bytes for the
 *              label of the arc a candidate came over and 8 for the reverse
 *              arc to the parent); a position without a parent costs 5 bytes
 *              per target node of its range (RI) or 12 per domain member
 *              (RI-DS) per expansion.  Dense-bitset search: per expansion
 *              8*ceil(n/64) bytes per row read (the domain row, the parent
 *              image's row, every back-edge row).  Rows written by
 *              sge_enumerate (4k bytes per match) are not included;
 *  steals      tasks moved between search units through the work queue;
 *  steps       search-unit steps of the launch (a step maps one candidate
 *              and/or evaluates one group of candidates), for profiling;
 *  ms_prep     host preparation time (order, parents, domains, upload);
 *  ms_search   device time of the search launch (first block start to
 *              last wave exit, device clock); for a batch or serve launch it
 *              is the whole launch's. */
typedef struct {
    uint64_t matches, states, candidates, alg_bytes, steals, steps;
    double ms_prep, ms_search;
} sge_result;

typedef struct sge_ctx sge_ctx;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (NULL = the null stream); every device operation of the context is ordered
 * on it.  *out receives the context. */
sge_status sge_create(int device, void *hip_stream, sge_ctx **out);
void sge_destroy(sge_ctx *ctx);
const char *sge_last_error(const sge_ctx *ctx);
/* Timing of the context's last count, enumerate or batch launch, from the
 * device clock, in ms since its first block started: ms[0] until the last
 * wave exited (the kernel), ms[1] until the last task finished, ms[2] until
 * termination was detected. */
sge_status sge_last_launch_timing(const sge_ctx *ctx, double *ms);
/* The search kernel of the context's last count, enumerate or batch launch
 * timed by HIP events recorded on the context's stream right before and right
 * after it (event nodes of the batch graph): *ms receives the elapsed time,
 * 0 before any launch or when the last call launched nothing. */
sge_status sge_last_kernel_ms(const sge_ctx *ctx, double *ms);
/* on = 1 (default): search launches count each instance's alg_bytes;
 * on = 0: they do not (a few instructions fewer per candidate), and
 * sge_result.alg_bytes is 0. */
sge_status sge_set_count_bytes(sge_ctx *ctx, int on);
/* on = 1: every search step also verifies that the lanes of each search unit
 * hold the same copy of the unit's state (its task, level, stack top and the
 * current frame); a disagreement makes the call return SGE_E_DEVICE (the
 * search itself runs to its end).  Off by default: a check for testing. */
sge_status sge_set_checks(sge_ctx *ctx, int on);
/* Occupancy of the same launch (the parallel search of Section 3 as run on
 * the device): *busy_unit_ms receives the sum over search units of the time
 * each held a task, *units the number of units that entered the search loop
 * (resident units the root chunks could keep busy).  busy_unit_ms / ms[0] is
 * the mean number of busy units; divided by the launch's steps it is the
 * mean duration of one step.  Both are 0 before any launch. */
sge_status sge_last_launch_occupancy(const sge_ctx *ctx, double *busy_unit_ms, uint32_t *units);

/* Load a target graph and keep it resident in device memory (CSR, per-node
 * records and, for n <= 65536, dense adjacency bitset rows).  Target size is
 * bounded only by device memory: with rows a back-edge is one 64-bit word
 * test, without them a binary search in the CSR row; a used-node bitset
 * per search unit is kept in LDS while it fits beside four waves of units,
 * and beyond that a candidate is compared with the mapped prefix instead.
 * labels: n uint32 or NULL (all nodes equivalent).  *handle receives the id. */
sge_status sge_load_target(sge_ctx *ctx, uint32_t n, const uint32_t *row_ptr, const uint32_t *col,
                           const uint32_t *labels, uint32_t *handle);
/* Unloading a target or pattern that server queries in flight still use
 * (submitted and not yet complete) is refused with SGE_E_BUSY; it succeeds
 * once they have completed (they need not have been polled). */
sge_status sge_unload_target(sge_ctx *ctx, uint32_t handle);

/* Load a pattern graph (k <= 64 nodes, same CSR conventions). */
sge_status sge_load_pattern(sge_ctx *ctx, uint32_t k, const uint32_t *row_ptr, const uint32_t *col,
                            const uint32_t *labels, uint32_t *handle);
sge_status sge_unload_pattern(sge_ctx *ctx, uint32_t handle);

/* The general graphs of Section 2.1: directed, with node and edge labels.
 * directed = 1: row_ptr/col list the out-edges (arcs) of each node; the
 * library builds the in-edges.  directed = 0: as sge_load_target (both
 * directions of every edge).  edge_labels: row_ptr[n] uint32, the label of
 * each CSR entry (an undirected edge carries one label in both directions),
 * or NULL (all 0).  Duplicate entries must carry one label (else
 * SGE_E_INVAL).  Edge labels are compared exactly when node labels are
 * (sge_set_labelled, sge_job.labelled).  A search with a directed graph on
 * either side keeps directions: rule 3 compares in- and out-degree, every
 * pattern arc must map onto a target arc of the same direction (and label);
 * the order and parents ignore directions (Section "RI").  Such searches are
 * planned on the host and run the CSR search kernel. */
sge_status sge_load_target_ex(sge_ctx *ctx, uint32_t n, const uint32_t *row_ptr, const uint32_t *col,
                              const uint32_t *labels, const uint32_t *edge_labels, int directed, uint32_t *handle);
sge_status sge_load_pattern_ex(sge_ctx *ctx, uint32_t k, const uint32_t *row_ptr, const uint32_t *col,
                               const uint32_t *labels, const uint32_t *edge_labels, int directed,
                               uint32_t *handle);

/* labelled = 0: labels are ignored (every node equivalent, Section 2.1). */
sge_status sge_set_labelled(sge_ctx *ctx, int labelled);
/* mode: SGE_RI | SGE_RIDS | SGE_RIDS_SI | SGE_RIDS_SI_FC. */
sge_status sge_set_mode(sge_ctx *ctx, int mode);
/* cap = 0: no cap.  Otherwise a search whose states exceed cap stops with
 * SGE_E_ABORTED; "exceeds" is decided on the schedule-independent count. */
sge_status sge_set_state_cap(sge_ctx *ctx, uint64_t cap);
/* Every search launch ends by this wall-clock limit (ms; 0 = none; default
 * 120000).  A launch that reaches it returns SGE_E_ABORTED with partial
 * counters. */
sge_status sge_set_time_limit(sge_ctx *ctx, uint64_t ms);
/* Restrict the first pattern node of the order to target nodes in [lo, hi)
 * (a shard of the root candidates; lo = 0, hi = UINT32_MAX restores all).
 * Counters then cover that shard only. */
sge_status sge_set_root_range(sge_ctx *ctx, uint32_t lo, uint32_t hi);

/* Count the embeddings of `pattern` in `target`. */
sge_status sge_count(sge_ctx *ctx, uint32_t target, uint32_t pattern, sge_result *res);

/* For callers that cannot allocate device or pinned memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): as
 * sge_count, with every buffer of the launch -- job descriptor, device plan,
 * domains, candidate lists, scheduler words, work queue, counters -- in one
 * static device array of 16 MiB per device (held from the library's load
 * until the process ends), and the plan made by the plan kernel.  Calls no
 * allocating routine.  The target and pattern must be loaded beforehand.
 * SGE_E_INVAL when the instance needs more than the array (about
 * 1.5 MiB + 16 k ceil(n/64) + 4 (components * n + k) bytes) or is directed
 * or compares edge labels.  Every call on a device shares that device's
 * array: calls that overlap on one device race (results undefined); calls in
 * sequence are independent (the launch clears what must start at zero). */
sge_status sge_count_noalloc(sge_ctx *ctx, uint32_t target, uint32_t pattern, sge_result *res);

/* Enumerate: as sge_count, and write up to cap_rows rows of k uint32 to
 * `rows` (host or device pointer; device memory must be on the context's
 * device).  More matches than cap_rows: SGE_E_OVERFLOW with full counts. */
sge_status sge_enumerate(sge_ctx *ctx, uint32_t target, uint32_t pattern, uint32_t *rows, uint64_t cap_rows,
                         sge_result *res);

/* ---------------------------------------------------------------- batching */
/* One (target, pattern) pair of a batch with its own mode and labelling. */
typedef struct {
    uint32_t target, pattern;
    int32_t mode, labelled;
} sge_job;

/* Search all jobs in one persistent launch (captured, with the upload of the
 * job descriptors, the plan kernel and the read-back, in one HIP graph, which
 * the context keeps and launches again while the launch shape, sizes,
 * buffers and settings are unchanged).  results[njobs] receives each job's
 * counters; the state cap of
 * the context applies per job.  Returns SGE_E_ABORTED if any job was capped
 * (its counters are partial); the others are complete. */
sge_status sge_batch_run(sge_ctx *ctx, uint32_t njobs, const sge_job *jobs, sge_result *results);

/* Batch launch policy: 0 = autotuned (default), 1 = one search unit takes a
 * whole job, 2 = jobs are split into root chunks shared by all units. */
sge_status sge_set_batch_policy(sge_ctx *ctx, int policy);

/* ----------------------------------------------------------------- serving */
/* Start the server: continuous batching of queries on the context's
 * resident targets and patterns.  Admitted queries are planned by host
 * threads (or by the plan kernel at the head of their launch when the plan
 * location is 1) and packed, whatever is ready, into one persistent search
 * launch on the first idle of four launch lanes (HIP streams with their own
 * scheduler state), so queries that arrive while others run start at once
 * beside them.  slots = maximum queries in flight; arena_bytes = device
 * memory for per-query plans and domains (admission is by this memory and by
 * free slots; a query larger than the whole arena is SGE_E_NOMEM at submit).
 * SGE_E_INVAL if the server already runs or slots or arena_bytes is 0;
 * SGE_E_DEVICE if its streams cannot be created. */
sge_status sge_serve_start(sge_ctx *ctx, uint32_t slots, uint64_t arena_bytes);
/* Submit one query (job->mode / labelled apply).  SGE_E_BUSY when no slot
 * or memory is free now.  *ticket identifies the query. */
sge_status sge_serve_submit(sge_ctx *ctx, const sge_job *job, uint64_t *ticket);
/* Poll a query: SGE_E_BUSY while it runs, else its final status with *res
 * filled and the ticket released. */
sge_status sge_serve_poll(sge_ctx *ctx, uint64_t ticket, sge_result *res);
/* Stop the server after the queries in flight complete. */
sge_status sge_serve_stop(sge_ctx *ctx);

/* ------------------------------------------------------------- inspection */
/* The host plan the library computes for a (pattern, target) pair, for
 * checking against an independent reference.  Host arrays only; no device is
 * touched.  order[k]: position -> pattern node; parent[k]: position ->
 * earlier position or -1; dom (may be NULL): k * ceil(n/64) uint64 words of
 * the final domains indexed by pattern node (unused in SGE_RI).  *empty = 1
 * when a domain became empty (no matches; order is then not written). */
sge_status sge_plan_host(uint32_t k, const uint32_t *p_row_ptr, const uint32_t *p_col, const uint32_t *p_labels,
                         uint32_t n, const uint32_t *t_row_ptr, const uint32_t *t_col, const uint32_t *t_labels,
                         int mode, int labelled, uint32_t *order, int32_t *parent, uint64_t *dom, int *empty);
/* The same for general graphs (edge labels or NULL, directed flags as in
 * sge_load_target_ex). */
sge_status sge_plan_host_ex(uint32_t k, const uint32_t *p_row_ptr, const uint32_t *p_col, const uint32_t *p_labels,
                            const uint32_t *p_edge_labels, int p_directed, uint32_t n, const uint32_t *t_row_ptr,
                            const uint32_t *t_col, const uint32_t *t_labels, const uint32_t *t_edge_labels,
                            int t_directed, int mode, int labelled, uint32_t *order, int32_t *parent, uint64_t *dom,
                            int *empty);

/* The plan the device computes for one instance, as every search launch
 * computes it before searching (domains of Section 4.1 with arc-consistency,
 * forward checking of Section 4.2.2, the order of Section "RI" with the
 * tie-break of Section 4.2.1), copied back for checking against an
 * independent reference.  Host output arrays: order[k] and parent[k] as in
 * sge_plan_host; dom (may be NULL; ignored in SGE_RI): k * ceil(n/64) uint64
 * words of the final domains by pattern node; *nroot: candidates of position
 * 0 within the context's root range.  *empty = 1 when a domain became empty
 * (order, parent and dom are then not written).  Ordered on the context's
 * stream; returns when the copy is complete. */
sge_status sge_plan_device(sge_ctx *ctx, uint32_t target, uint32_t pattern, int mode, int labelled, uint32_t *order,
                           int32_t *parent, uint64_t *dom, uint32_t *nroot, int *empty);

/* Where launches are planned: -1 = automatic (on the device for launches of
 * 64 or more instances, on the host otherwise), 0 = always on the host
 * (C++ on the calling thread, or the server's preparation threads), 1 = always
 * on the device (the plan kernel).  Both give the same plan. */
sge_status sge_set_plan_location(sge_ctx *ctx, int where);

/* Tuning knobs (for measurement): lanes per search unit (8, 16, 32 or 64;
 * 0 = automatic), root chunk size (0 = automatic), work donation (0 = off,
 * 1 = on with the default period, N > 1 = a unit gives work away at most
 * once per N of its steps), dense-bitset search (-1 = automatic, 0 = off,
 * 1 = on wherever it can run: undirected graphs without compared edge
 * labels, every target with adjacency rows -- n <= 65536 -- and a search
 * unit's k rows of ceil(n/64) words within 64 KiB of LDS; elsewhere the CSR
 * search runs, and a general graph is SGE_E_INVAL). */
sge_status sge_set_tuning(sge_ctx *ctx, int lanes_per_unit, uint32_t root_chunk, int donate, int dense);

/* Resident search blocks per compute unit (each block is four wavefronts of
 * search units, the workers of Section 3): N >= 1 launches at most N per CU,
 * 0 = automatic (as many as fit, or for batches the autotuner's choice).
 * Searches whose work sits in few deep subtrees run faster with fewer
 * resident waves; broad workloads with more.  SGE_E_INVAL outside 0..64. */
sge_status sge_set_blocks_per_cu(sge_ctx *ctx, int blocks_per_cu);

#ifdef __cplusplus
}
#endif
#endif /* SGE_H */
