/*
 * ORACLE: a plain, slow, single-threaded CPU reference for RI / RI-DS subgraph
 * enumeration (Kimmig, Meyerhenke, Strash, "Shared Memory Parallel Subgraph
 * Enumeration", arXiv 1705.09358).
 *
 * This is TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header or table
 * with the GPU library: it has its own structures and reads only the plain
 * input arrays.
 *
 * What it computes (Section 2.1, eqs. (2)-(4), non-induced as the paper states
 * after them):  every injective M : V_p -> V_t with lab(u) = lab(M u) (when
 * labelled) and (M u, M w) in E_t for every pattern edge (u, w), with equal
 * edge labels beta(u, w) = beta(M u, M w) (when labelled).  Graphs are given as
 * CSR with sorted rows, no self-loops and optional edge labels per entry: the
 * out-edges of a directed graph, or both directions of an undirected one (a
 * symmetric CSR with symmetric edge labels).  An undirected graph is the
 * directed graph with both directions of every edge.
 *
 * How (the algorithm's steps in the paper's order):
 *   1. RI-DS domains (Section 4.1): D(u) = target nodes with the label of u and
 *      degree >= deg(u); arc-consistency removes v from D(u) when some pattern
 *      edge (u, w) has no neighbour of v in D(w), repeated to a fixpoint; any
 *      empty domain means no matches.
 *   2. Forward checking on singleton domains (Section 4.2.2), RI-DS-SI-FC only.
 *   3. The constraint-first ordering (Section "RI", ordering and parent map):
 *      RI-DS places singleton-domain nodes first; then greedily the unplaced
 *      node with most neighbours in the order (w_m), ties by w_n, then degree,
 *      then (SI variants, Section 4.2.1) the smaller domain.
 *   4. The parent map: the earliest placed neighbour.
 *   5. Depth-first search (Section 2.2.1 state space; RI pruning rules 1-4;
 *      RI-DS domain test, Section 4.1): candidates for position i are the
 *      target neighbours of the parent's image, or all nodes (RI) / D(mu_i)
 *      (RI-DS) when there is no parent.
 *
 * Readings taken where the text is silent or garbled:
 *   - w_m counts neighbours *in* the order (the printed formula has a union).
 *   - The first node is the one of highest degree (the text), as the greedy
 *     key gives with an empty order.
 *   - The final tie-break is the lowest pattern node id.
 *   - w_n follows the formula: placed nodes w that share an unplaced common
 *     neighbour x with u.
 *   - Degree is the undirected degree.
 *   - The parent is the earliest *preceding* adjacent node.
 *   - Domains are sets of *target* nodes.
 *   - Arc-consistency runs to its fixpoint; forward checking then runs to its
 *     fixpoint; arc-consistency is not run again.
 *   - Singleton-domain nodes go first in ascending id; SI applies to the first
 *     greedy pick too.
 *   - k = 0 gives one (empty) match; self-loops are rejected.
 *   - Directed graphs: the order and the parents ignore directions (as the
 *     paper says for the order); degree there is |N(v)|, N(v) the nodes with
 *     an edge to or from v.  Rule 3 and the domain initialisation compare
 *     in- and out-degree separately.  A parent's candidates are its image's
 *     out-neighbours when the pattern edge leaves the parent, else its
 *     in-neighbours.  Arc-consistency asks, for a pattern edge u -> w, an
 *     out-neighbour of v in D(w) over an edge of the same label, and for
 *     w -> u an in-neighbour (the paper gives the first case; the second is
 *     its mirror).
 *   - Edge labels are compared exactly when node labels are (labelled).
 *
 * Counters: `states` = accepted (position, target) pairs (consistent prefix
 * assignments); `candidates` = pairs considered; `alg_bytes` = bytes a search
 * must read per the sparse per-unit model below; `dense_bytes` = the same for
 * a search on adjacency bitsets; `matches` = complete mappings.  Neither byte
 * count includes the rows an enumeration writes (4k bytes per match), so both
 * are the figures of a count-only search.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_RI = 0, OR_RIDS = 1, OR_RIDS_SI = 2, OR_RIDS_SI_FC = 3 };
enum { OR_OK = 0, OR_ABORTED = 2, OR_EINVAL = -1, OR_ENOMEM = -2 };

typedef struct {
    uint32_t n;
    const uint32_t *rp, *col, *lab, *elab;   /* out-edges; elab per entry, or NULL for all 0 */
    uint32_t *irp, *icol, *ielab;            /* in-edges (the transpose), built by og_index */
    int directed;
} og;

static uint32_t og_deg(const og *g, uint32_t v) { return g->rp[v + 1] - g->rp[v]; }
static uint32_t og_indeg(const og *g, uint32_t v) { return g->irp[v + 1] - g->irp[v]; }

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* index of b in the (sorted) out-list of a, or -1 */
static int64_t og_find(const og *g, uint32_t a, uint32_t b) {
    uint32_t d = og_deg(g, a);
    if (d == 0) return -1;
    const uint32_t *hit = bsearch(&b, g->col + g->rp[a], d, sizeof(uint32_t), cmp_u32);
    return hit ? (int64_t)(hit - g->col) : -1;
}

/* is there an edge a -> b */
static int og_adj(const og *g, uint32_t a, uint32_t b) { return og_find(g, a, b) >= 0; }

static uint32_t og_elab(const og *g, int64_t e) { return g->elab ? g->elab[e] : 0u; }

/* a and b are neighbours (an edge in either direction) */
static int og_nb(const og *g, uint32_t a, uint32_t b) { return og_adj(g, a, b) || og_adj(g, b, a); }

/* |N(v)|: nodes with an edge to or from v */
static uint32_t og_nbdeg(const og *g, uint32_t v) {
    uint32_t c = 0, i = g->rp[v], j = g->irp[v];
    while (i < g->rp[v + 1] || j < g->irp[v + 1]) {
        if (j >= g->irp[v + 1] || (i < g->rp[v + 1] && g->col[i] < g->icol[j])) i++;
        else if (i >= g->rp[v + 1] || g->icol[j] < g->col[i]) j++;
        else { i++; j++; }
        c++;
    }
    return c;
}

static int og_valid(const og *g) {
    for (uint32_t v = 0; v < g->n; v++) {
        if (g->rp[v + 1] < g->rp[v]) return 0;
        for (uint32_t e = g->rp[v]; e < g->rp[v + 1]; e++) {
            uint32_t w = g->col[e];
            if (w >= g->n || w == v) return 0;
            if (e > g->rp[v] && g->col[e - 1] >= w) return 0;
        }
    }
    if (!g->directed)   /* both directions of every edge, with one label */
        for (uint32_t v = 0; v < g->n; v++)
            for (uint32_t e = g->rp[v]; e < g->rp[v + 1]; e++) {
                int64_t r = og_find(g, g->col[e], v);
                if (r < 0 || og_elab(g, r) != og_elab(g, e)) return 0;
            }
    return 1;
}

/* build the in-edge lists (sorted, with their labels) */
static int og_index(og *g) {
    uint32_t n = g->n, m = g->rp[n];
    g->irp = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
    g->icol = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    g->ielab = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    if (!g->irp || !g->icol || !g->ielab) return 0;
    for (uint32_t e = 0; e < m; e++) g->irp[g->col[e] + 1]++;
    for (uint32_t v = 0; v < n; v++) g->irp[v + 1] += g->irp[v];
    uint32_t *fill = (uint32_t *)malloc(((size_t)n + 1) * sizeof(uint32_t));
    if (!fill) return 0;
    memcpy(fill, g->irp, ((size_t)n + 1) * sizeof(uint32_t));
    for (uint32_t v = 0; v < n; v++)   /* sources in increasing order: rows come out sorted */
        for (uint32_t e = g->rp[v]; e < g->rp[v + 1]; e++) {
            uint32_t w = g->col[e], at = fill[w]++;
            g->icol[at] = v;
            g->ielab[at] = og_elab(g, e);
        }
    free(fill);
    return 1;
}

static void og_free(og *g) {
    free(g->irp);
    free(g->icol);
    free(g->ielab);
    g->irp = g->icol = g->ielab = NULL;
}

typedef struct {
    og P, T;
    int mode, labelled;
    int directed;         /* either graph is directed: in-edges are checked on their own */
    uint64_t cap;
    uint32_t k, n;
    unsigned char *dom;   /* k*n, dom[u*n + v] (by pattern id); NULL in RI */
    uint32_t order[64];   /* position -> pattern node */
    int32_t parent[64];   /* position -> earlier position, or -1 */
    uint32_t M[64];       /* position -> target node */
    unsigned char *used;  /* n */
    uint64_t matches, states, candidates, alg_bytes, dense_bytes;
    uint64_t W;           /* 64-bit words of one target adjacency bitset row */
    uint32_t *rows;
    uint64_t cap_rows;
    uint32_t root_lo, root_hi;  /* first position restricted to target nodes in [lo, hi) */
    int aborted;
} oracle_t;

/* rules 2-3 of RI and the domain initialisation of RI-DS: label, out- and in-degree */
static int compat(const oracle_t *o, uint32_t u, uint32_t v) {
    if (o->labelled && o->P.lab[u] != o->T.lab[v]) return 0;
    return og_deg(&o->P, u) <= og_deg(&o->T, v) && og_indeg(&o->P, u) <= og_indeg(&o->T, v);
}

/* some target edge out of v (in-edges: into v) of label b reaches a member of D(w) */
static int supported(const oracle_t *o, uint32_t v, uint32_t w, uint32_t b, int in_edges) {
    const uint32_t *rp = in_edges ? o->T.irp : o->T.rp, *col = in_edges ? o->T.icol : o->T.col;
    for (uint32_t f = rp[v]; f < rp[v + 1]; f++) {
        if (!o->dom[(size_t)w * o->n + col[f]]) continue;
        uint32_t tb = in_edges ? o->T.ielab[f] : og_elab(&o->T, f);
        if (!o->labelled || tb == b) return 1;
    }
    return 0;
}

static uint64_t dom_size(const oracle_t *o, uint32_t u) {
    uint64_t s = 0;
    for (uint32_t v = 0; v < o->n; v++) s += o->dom[(size_t)u * o->n + v];
    return s;
}

/* Arc-consistency to its fixpoint.  Returns 1 if a domain became empty. */
static int arc_consistency(oracle_t *o) {
    int changed = 1;
    while (changed) {
        changed = 0;
        for (uint32_t u = 0; u < o->k; u++) {
            for (uint32_t v = 0; v < o->n; v++) {
                if (!o->dom[(size_t)u * o->n + v]) continue;
                int keep = 1;
                /* pattern edges u -> w need an edge v -> x, x in D(w), of the same label */
                for (uint32_t e = o->P.rp[u]; e < o->P.rp[u + 1] && keep; e++)
                    keep = supported(o, v, o->P.col[e], og_elab(&o->P, e), 0);
                /* directed: pattern edges w -> u need an edge x -> v likewise */
                if (o->directed)
                    for (uint32_t e = o->P.irp[u]; e < o->P.irp[u + 1] && keep; e++)
                        keep = supported(o, v, o->P.icol[e], o->P.ielab[e], 1);
                if (!keep) {
                    o->dom[(size_t)u * o->n + v] = 0;
                    changed = 1;
                }
            }
        }
    }
    for (uint32_t u = 0; u < o->k; u++)
        if (dom_size(o, u) == 0) return 1;
    return 0;
}

/*
 * Forward checking on singleton domains (Section 4.2.2): the target node of a
 * singleton domain is removed from every other domain; newly created
 * singletons are treated the same way until none is left.  `dom` is k*n bytes
 * (dom[u*n+v]).  Returns 1 if a domain became empty, else 0.
 */
int oracle_forward_check(uint32_t k, uint32_t n, unsigned char *dom) {
    unsigned char done[64] = {0};
    if (k > 64) return -1;
    for (;;) {
        int progressed = 0;
        for (uint32_t u = 0; u < k; u++) {
            if (done[u]) continue;
            uint64_t cnt = 0;
            uint32_t t = 0;
            for (uint32_t v = 0; v < n; v++)
                if (dom[(size_t)u * n + v]) { cnt++; t = v; }
            if (cnt == 0) return 1;
            if (cnt != 1) continue;
            done[u] = 1;
            progressed = 1;
            for (uint32_t w = 0; w < k; w++)
                if (w != u) dom[(size_t)w * n + t] = 0;
        }
        if (!progressed) break;
    }
    for (uint32_t u = 0; u < k; u++) {
        uint64_t cnt = 0;
        for (uint32_t v = 0; v < n; v++) cnt += dom[(size_t)u * n + v];
        if (cnt == 0) return 1;
    }
    return 0;
}

/* pattern neighbours, directions ignored (the order and the parents) */
static int pattern_adj(const oracle_t *o, uint32_t a, uint32_t b) { return og_nb(&o->P, a, b); }

/* The constraint-first ordering and its parent map. */
static void make_order(oracle_t *o) {
    uint32_t k = o->k;
    unsigned char placed[64] = {0};
    uint32_t len = 0;
    int use_dom = o->mode != OR_RI;
    int use_si = o->mode == OR_RIDS_SI || o->mode == OR_RIDS_SI_FC;
    uint64_t dsz[64];
    for (uint32_t u = 0; u < k; u++) dsz[u] = use_dom ? dom_size(o, u) : 0;
    if (use_dom)
        for (uint32_t u = 0; u < k; u++)
            if (dsz[u] == 1) { o->order[len++] = u; placed[u] = 1; }
    while (len < k) {
        int64_t best = -1;
        int64_t bwm = 0, bwn = 0, bdeg = 0;
        uint64_t bdom = 0;
        for (uint32_t u = 0; u < k; u++) {
            if (placed[u]) continue;
            int64_t wm = 0, wn = 0, deg = og_nbdeg(&o->P, u);
            for (uint32_t j = 0; j < len; j++)
                if (pattern_adj(o, u, o->order[j])) wm++;
            for (uint32_t j = 0; j < len; j++) {
                uint32_t w = o->order[j];
                int reach = 0;
                for (uint32_t x = 0; x < k && !reach; x++)
                    if (!placed[x] && pattern_adj(o, x, u) && pattern_adj(o, x, w)) reach = 1;
                wn += reach;
            }
            int better;
            if (best < 0) better = 1;
            else if (wm != bwm) better = wm > bwm;
            else if (wn != bwn) better = wn > bwn;
            else if (deg != bdeg) better = deg > bdeg;
            else if (use_si && dsz[u] != bdom) better = dsz[u] < bdom;
            else better = 0; /* equal key: the lower id, met first, stays */
            if (better) { best = u; bwm = wm; bwn = wn; bdeg = deg; bdom = dsz[u]; }
        }
        o->order[len++] = (uint32_t)best;
        placed[best] = 1;
    }
    for (uint32_t i = 0; i < k; i++) {
        o->parent[i] = -1;
        for (uint32_t j = 0; j < i; j++)
            if (pattern_adj(o, o->order[i], o->order[j])) { o->parent[i] = (int32_t)j; break; }
    }
}

/*
 * Algorithmic bytes.  Sparse model: 8 B for the bounds of each neighbour list
 * read plus 4 B per id in it; per candidate 5 B (RI: label byte and degree
 * word) or 8 B (RI-DS: one domain word); 8 B per back-edge probe performed (the
 * probes of a candidate stop at the first that fails).  For a parentless
 * position the candidate ids are implicit (RI) or 4 B each from the domain list
 * (RI-DS).  Dense model (a search whose target rows are bitsets of W words):
 * each expansion of a position reads W words of the domain (or label and
 * degree) row, W of the parent image's adjacency row when there is a parent,
 * and W of each earlier neighbour's row other than the parent.
 */
static uint32_t back_count(const oracle_t *o, uint32_t i) {
    uint32_t c = 0;
    for (uint32_t j = 0; j < i; j++)
        if ((int32_t)j != o->parent[i] && pattern_adj(o, o->order[i], o->order[j])) c++;
    return c;
}

static void search(oracle_t *o, uint32_t i) {
    if (o->aborted) return;
    if (i == o->k) {
        if (o->rows && o->matches < o->cap_rows) {
            uint32_t *r = o->rows + o->matches * o->k;
            for (uint32_t j = 0; j < o->k; j++) r[o->order[j]] = o->M[j];
        }
        o->matches++;
        return;
    }
    uint32_t u = o->order[i];
    int use_dom = o->mode != OR_RI;
    o->dense_bytes += 8ull * o->W * (1u + (o->parent[i] >= 0) + back_count(o, i));
    uint32_t lo, hi;
    const uint32_t *list = NULL, *labs = NULL;
    uint32_t pu = 0, pv = 0, plab = 0;
    int gen_out = 1, both = 0;
    if (o->parent[i] >= 0) {
        /* candidates: the image's out-neighbours if the pattern edge leaves
           the parent, else its in-neighbours */
        pu = o->order[o->parent[i]];
        pv = o->M[o->parent[i]];
        int64_t fe = og_find(&o->P, pu, u), re = og_find(&o->P, u, pu);
        gen_out = fe >= 0;
        both = fe >= 0 && re >= 0;
        plab = og_elab(&o->P, gen_out ? fe : re);
        if (gen_out) {
            lo = o->T.rp[pv];
            hi = o->T.rp[pv + 1];
            list = o->T.col;
            labs = o->T.elab;
        } else {
            lo = o->T.irp[pv];
            hi = o->T.irp[pv + 1];
            list = o->T.icol;
            labs = o->T.ielab;
        }
        o->alg_bytes += 8 + 4ull * (hi - lo);
    } else {
        lo = 0;
        hi = o->n;
    }
    for (uint32_t e = lo; e < hi; e++) {
        uint32_t v = list ? list[e] : e;
        if (i == 0 && (v < o->root_lo || v >= o->root_hi)) continue;   /* root shard */
        if (!list && use_dom) {
            /* parentless RI-DS position: candidates are the members of D(u) */
            if (!o->dom[(size_t)u * o->n + v]) continue;
            o->alg_bytes += 4;
        }
        o->candidates++;
        o->alg_bytes += use_dom ? 8 : 5;
        if (use_dom && !o->dom[(size_t)u * o->n + v]) continue;
        if (o->used[v]) continue;                                   /* rule 1 */
        if (o->labelled && o->P.lab[u] != o->T.lab[v]) continue;    /* rule 2 */
        if (og_deg(&o->P, u) > og_deg(&o->T, v) || og_indeg(&o->P, u) > og_indeg(&o->T, v))
            continue;                                               /* rule 3 */
        int ok = 1;                                                 /* rule 4 */
        if (list) {
            /* the parent edge used to generate v: its label; if the pattern
               has both directions, the other one too */
            if (o->labelled && (o->P.elab || o->T.elab)) {
                o->alg_bytes += 4;
                ok = (labs ? labs[e] : 0u) == plab;
            }
            if (ok && o->directed && both) {
                o->alg_bytes += 8;
                int64_t f = og_find(&o->T, v, pv);
                ok = f >= 0 && (!o->labelled || og_elab(&o->T, f) == og_elab(&o->P, og_find(&o->P, u, pu)));
            }
        }
        for (uint32_t j = 0; j < i && ok; j++) {
            if ((int32_t)j == o->parent[i]) continue;
            uint32_t w = o->order[j];
            int64_t pe = og_find(&o->P, w, u);   /* w -> u */
            if (pe >= 0) {
                o->alg_bytes += 8;
                int64_t f = og_find(&o->T, o->M[j], v);
                ok = f >= 0 && (!o->labelled || og_elab(&o->T, f) == og_elab(&o->P, pe));
            }
            if (!ok || !o->directed) continue;   /* undirected: w -> u is u -> w */
            int64_t pr = og_find(&o->P, u, w);   /* u -> w */
            if (pr >= 0) {
                o->alg_bytes += 8;
                int64_t f = og_find(&o->T, v, o->M[j]);
                ok = f >= 0 && (!o->labelled || og_elab(&o->T, f) == og_elab(&o->P, pr));
            }
        }
        if (!ok) continue;
        o->states++;
        if (o->cap && o->states > o->cap) { o->aborted = 1; return; }
        o->M[i] = v;
        o->used[v] = 1;
        search(o, i + 1);
        o->used[v] = 0;
        if (o->aborted) return;
    }
}

static void oracle_free(oracle_t *o) {
    free(o->dom);
    free(o->used);
    og_free(&o->P);
    og_free(&o->T);
}

static int oracle_setup(oracle_t *o, uint32_t k, const uint32_t *prp, const uint32_t *pcol, const uint32_t *plab,
                        const uint32_t *pelab, int pdir, uint32_t n, const uint32_t *trp, const uint32_t *tcol,
                        const uint32_t *tlab, const uint32_t *telab, int tdir, int mode, int labelled, int *empty) {
    memset(o, 0, sizeof(*o));
    if (k > 64 || mode < OR_RI || mode > OR_RIDS_SI_FC) return OR_EINVAL;
    o->P = (og){k, prp, pcol, plab, pelab, NULL, NULL, NULL, pdir != 0};
    o->T = (og){n, trp, tcol, tlab, telab, NULL, NULL, NULL, tdir != 0};
    if (!og_valid(&o->P) || !og_valid(&o->T)) return OR_EINVAL;
    if (labelled && (!plab || !tlab)) return OR_EINVAL;
    if (!og_index(&o->P) || !og_index(&o->T)) { oracle_free(o); return OR_ENOMEM; }
    o->directed = pdir || tdir;
    o->k = k;
    o->n = n;
    o->W = ((uint64_t)n + 63) / 64;
    o->mode = mode;
    o->labelled = labelled;
    o->used = (unsigned char *)calloc(n ? n : 1, 1);
    if (!o->used) return OR_ENOMEM;
    *empty = 0;
    if (mode != OR_RI && k > 0) {
        o->dom = (unsigned char *)malloc((size_t)k * (n ? n : 1));
        if (!o->dom) { oracle_free(o); return OR_ENOMEM; }
        for (uint32_t u = 0; u < k; u++)
            for (uint32_t v = 0; v < n; v++) o->dom[(size_t)u * n + v] = (unsigned char)compat(o, u, v);
        *empty = arc_consistency(o);
        if (!*empty && mode == OR_RIDS_SI_FC) *empty = oracle_forward_check(k, n, o->dom);
    }
    if (!*empty) make_order(o);
    return OR_OK;
}

/*
 * Plan only: writes order[k] (position -> pattern node), parent[k] (position
 * -> earlier position or -1) and, when dom_out is given and the mode uses
 * domains, the final domains as k*n bytes indexed by pattern node.  *empty is
 * set to 1 when a domain became empty (no matches; order is then not set).
 */
int oracle_plan_ex(uint32_t k, const uint32_t *prp, const uint32_t *pcol, const uint32_t *plab,
                   const uint32_t *pelab, int pdir, uint32_t n, const uint32_t *trp, const uint32_t *tcol,
                   const uint32_t *tlab, const uint32_t *telab, int tdir, int mode, int labelled, uint32_t *order,
                   int32_t *parent, unsigned char *dom_out, int *empty) {
    oracle_t o;
    int rc = oracle_setup(&o, k, prp, pcol, plab, pelab, pdir, n, trp, tcol, tlab, telab, tdir, mode, labelled, empty);
    if (rc != OR_OK) return rc;
    if (!*empty) {
        memcpy(order, o.order, k * sizeof(uint32_t));
        memcpy(parent, o.parent, k * sizeof(int32_t));
    }
    if (dom_out && o.dom) memcpy(dom_out, o.dom, (size_t)k * n);
    oracle_free(&o);
    return OR_OK;
}

/*
 * Full run.  counters[0..4] = matches, states, candidates, alg_bytes,
 * dense_bytes.  Rows
 * (pattern-id order) are written for the first cap_rows matches when rows is
 * given.  The first pattern node of the order is restricted to target nodes in
 * [root_lo, root_hi) (a shard of the search; 0 and UINT32_MAX for all).
 * Returns OR_OK, OR_ABORTED when states exceed state_cap (> 0), or a negative
 * error.
 */
int oracle_run_ex(uint32_t k, const uint32_t *prp, const uint32_t *pcol, const uint32_t *plab,
                  const uint32_t *pelab, int pdir, uint32_t n, const uint32_t *trp, const uint32_t *tcol,
                  const uint32_t *tlab, const uint32_t *telab, int tdir, int mode, int labelled,
                  uint64_t state_cap, uint32_t root_lo, uint32_t root_hi, uint32_t *rows, uint64_t cap_rows,
                  uint64_t *counters) {
    oracle_t o;
    int empty = 0;
    int rc = oracle_setup(&o, k, prp, pcol, plab, pelab, pdir, n, trp, tcol, tlab, telab, tdir, mode, labelled,
                          &empty);
    if (rc != OR_OK) return rc;
    o.root_lo = root_lo;
    o.root_hi = root_hi;
    o.cap = state_cap;
    o.rows = rows;
    o.cap_rows = rows ? cap_rows : 0;
    if (!empty) search(&o, 0);
    counters[0] = o.matches;
    counters[1] = o.states;
    counters[2] = o.candidates;
    counters[3] = o.alg_bytes;
    counters[4] = o.dense_bytes;
    rc = o.aborted ? OR_ABORTED : OR_OK;
    oracle_free(&o);
    return rc;
}

/* The undirected, edge-unlabelled entry points (symmetric CSR in and out). */
int oracle_plan(uint32_t k, const uint32_t *prp, const uint32_t *pcol, const uint32_t *plab,
                uint32_t n, const uint32_t *trp, const uint32_t *tcol, const uint32_t *tlab,
                int mode, int labelled, uint32_t *order, int32_t *parent, unsigned char *dom_out, int *empty) {
    return oracle_plan_ex(k, prp, pcol, plab, NULL, 0, n, trp, tcol, tlab, NULL, 0, mode, labelled, order, parent,
                          dom_out, empty);
}

int oracle_run(uint32_t k, const uint32_t *prp, const uint32_t *pcol, const uint32_t *plab,
               uint32_t n, const uint32_t *trp, const uint32_t *tcol, const uint32_t *tlab,
               int mode, int labelled, uint64_t state_cap, uint32_t root_lo, uint32_t root_hi,
               uint32_t *rows, uint64_t cap_rows, uint64_t *counters) {
    return oracle_run_ex(k, prp, pcol, plab, NULL, 0, n, trp, tcol, tlab, NULL, 0, mode, labelled, state_cap,
                         root_lo, root_hi, rows, cap_rows, counters);
}
