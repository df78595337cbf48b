// Host preparation of one search: RI-DS domains (Section 4.1), forward
// checking (Section 4.2.2), the constraint-first order with its domain-size
// tie-break (Section "RI" ordering; Section 4.2.1), parents and back-edges.
//
// Pattern neighbourhoods are 64-bit masks (k <= 64); domains are bitsets of
// ceil(n/64) words.  Arc-consistency keeps v in D(u) iff every pattern arc
// u -> w has a target arc v -> x with x in D(w), and every arc w -> u a target
// arc x -> v with x in D(w), with equal edge labels when labels are compared
// (for undirected graphs the two cases coincide).  Values are removed until
// nothing changes; every order of removals reaches the same greatest
// arc-consistent domains.  Directed graphs: the order and the parents ignore
// directions (Section "RI"); rule 3 compares in- and out-degree.
#include <algorithm>
#include <cstring>
#if defined(__SSE2__)
#include <emmintrin.h>
#endif

#include "sge_internal.h"

namespace sge {

static inline uint32_t popcount_row(const uint64_t *r, uint32_t W) {
    uint32_t c = 0;
    for (uint32_t i = 0; i < W; i++) c += (uint32_t)__builtin_popcountll(r[i]);
    return c;
}

static inline bool test_bit(const uint64_t *r, uint32_t v) { return (r[v >> 6] >> (v & 63)) & 1; }

// bit b set iff p[b] >= d, for the 64 bytes p[0..63]
static inline uint64_t bytes_at_least(const uint8_t *p, uint8_t d) {
#if defined(__SSE2__)
    const __m128i dv = _mm_set1_epi8((char)d);
    uint64_t m = 0;
    for (int q = 0; q < 4; q++) {
        const __m128i x = _mm_loadu_si128(reinterpret_cast<const __m128i *>(p + 16 * q));
        m |= (uint64_t)(uint16_t)_mm_movemask_epi8(_mm_cmpeq_epi8(_mm_max_epu8(x, dv), x)) << (16 * q);
    }
    return m;
#else
    uint64_t m = 0;
    for (int b = 0; b < 64; b++) m |= (uint64_t)(p[b] >= d) << b;
    return m;
#endif
}

void constraint_first_order(const uint64_t *nb, const uint32_t *odeg, const uint32_t *dsize, uint32_t k, bool use_dom,
                            bool use_si, uint32_t *order) {
    uint64_t placed = 0;
    uint32_t len = 0;
    if (use_dom)
        for (uint32_t u = 0; u < k; u++)
            if (dsize[u] == 1) { order[len++] = u; placed |= 1ull << u; }
    while (len < k) {
        int best = -1;
        uint32_t bwm = 0, bwn = 0, bdeg = 0, bdom = 0;
        for (uint32_t u = 0; u < k; u++) {
            if ((placed >> u) & 1) continue;
            uint32_t wm = (uint32_t)__builtin_popcountll(nb[u] & placed);
            uint32_t wn = 0;
            for (uint64_t m = placed; m; m &= m - 1) {
                uint32_t w = (uint32_t)__builtin_ctzll(m);
                if (nb[u] & nb[w] & ~placed) wn++;
            }
            const uint32_t du = use_si ? dsize[u] : 0;
            bool take;
            if (best < 0) take = true;
            else if (wm != bwm) take = wm > bwm;
            else if (wn != bwn) take = wn > bwn;
            else if (odeg[u] != bdeg) take = odeg[u] > bdeg;
            else take = use_si && du < bdom;
            if (take) { best = (int)u; bwm = wm; bwn = wn; bdeg = odeg[u]; bdom = du; }
        }
        order[len++] = (uint32_t)best;
        placed |= 1ull << best;
    }
}

void build_plan(const Target &t, const HostGraph &p, int mode, bool labelled, uint32_t root_lo, uint32_t root_hi,
                Plan &pl, bool want_pos_bits, std::vector<uint64_t> &pos_bits) {
    const HostGraph &tg = t.g;
    const uint32_t k = p.n, n = tg.n, W = t.W;
    pl.k = k;
    pl.n = n;
    pl.W = W;
    pl.mode = mode;
    pl.labelled = labelled;
    pl.empty = false;
    pl.dom_node.clear();
    pl.lists.clear();
    pl.lmat.clear();
    // directions and edge labels matter only if a graph is directed or
    // carries edge labels that are compared
    const bool directed = p.directed || tg.directed;
    const bool elabelled = labelled && (p.has_elab() || tg.has_elab());
    pl.flags = (directed ? PLAN_DIRECTED : 0u) | (elabelled ? PLAN_EDGE_LABELS : 0u);

    // pattern node data: neighbourhood (directions ignored), out-degree,
    // in-degree, degree for the order, target label id
    uint64_t nb[KMAX], outm[KMAX];
    uint32_t deg[KMAX], indeg[KMAX], odeg[KMAX], lab[KMAX];
    for (uint32_t u = 0; u < k; u++) nb[u] = outm[u] = 0;
    for (uint32_t u = 0; u < k; u++)
        for (uint32_t e = p.rp[u]; e < p.rp[u + 1]; e++) {
            outm[u] |= 1ull << p.col[e];
            nb[u] |= 1ull << p.col[e];
            nb[p.col[e]] |= 1ull << u;
        }
    for (uint32_t u = 0; u < k; u++) {
        deg[u] = p.outdeg(u);
        indeg[u] = p.indeg(u);
        odeg[u] = (uint32_t)__builtin_popcountll(nb[u]);
        if (!labelled) {
            lab[u] = LABEL_ANY;
        } else {
            lab[u] = LABEL_NONE;
            for (uint32_t id = 0; id < t.label_keys.size(); id++)
                if (t.label_keys[id] == p.lab[u]) { lab[u] = id; break; }
        }
    }
    auto tdeg_ok = [&](uint32_t u, uint32_t v) { return tg.outdeg(v) >= deg[u] && tg.indeg(v) >= indeg[u]; };
    // nodes of V_t passing the label and degree rules for pattern node u
    auto compat_nodes = [&](uint32_t u, auto &&fn) {
        if (lab[u] == LABEL_NONE) return;
        if (lab[u] == LABEL_ANY) {
            for (uint32_t v = 0; v < n; v++)
                if (tdeg_ok(u, v)) fn(v);
        } else {
            for (uint32_t v : t.by_label[lab[u]])
                if (tdeg_ok(u, v)) fn(v);
        }
    };
    // label of the pattern arc a -> b (must exist)
    auto parc = [&](uint32_t a, uint32_t b) -> uint32_t {
        if (!p.has_elab()) return 0u;
        auto it = std::lower_bound(p.col.begin() + p.rp[a], p.col.begin() + p.rp[a + 1], b);
        return p.elab[it - p.col.begin()];
    };

    const bool use_dom = mode != SGE_RI;
    std::vector<uint64_t> &D = pl.dom_node;
    uint32_t dsize[KMAX] = {0};
    if (use_dom) {
        D.assign((size_t)k * W, 0);
        if (!directed && !t.deg_ge.empty()) {
            // the label row AND the degree row (pattern degrees are below 64)
            for (uint32_t u = 0; u < k; u++) {
                if (lab[u] == LABEL_NONE) continue;
                const uint64_t *dg = &t.deg_ge[(size_t)std::min<uint32_t>(deg[u], 63) * W];
                uint64_t *d = &D[(size_t)u * W];
                if (lab[u] == LABEL_ANY) {
                    std::memcpy(d, dg, W * sizeof(uint64_t));
                } else {
                    const uint64_t *lb = &t.label_bits[(size_t)lab[u] * W];
                    for (uint32_t i = 0; i < W; i++) d[i] = dg[i] & lb[i];
                }
            }
        } else {
            for (uint32_t u = 0; u < k; u++)
                compat_nodes(u, [&](uint32_t v) { D[(size_t)u * W + (v >> 6)] |= 1ull << (v & 63); });
        }
        // arc-consistency to the fixpoint.  A round revises D(u) against the
        // pattern neighbours w whose domains changed since D(u) was last
        // revised against them (for the others every member of D(u) still has
        // its support, as D(w) is unchanged): v leaves D(u) when no target
        // neighbour of v lies in D(w).
        bool any_empty = false;
        for (uint32_t u = 0; u < k; u++) any_empty |= popcount_row(&D[(size_t)u * W], W) == 0;
        uint64_t dirty = 0;   // nodes whose domain changed since their neighbours were revised against it
        if (!any_empty && !t.nbr_deg.empty() && !directed && !elabelled) {
            // first round against the label-and-degree domains: a target node
            // has a neighbour in D(w) iff it has a neighbour of w's label whose
            // degree is at least w's, which the target's table answers
            // (one pass over D(u) per pattern neighbour w, reading w's column
            // 64 nodes at a time; pattern degrees are below 64)
            // Pattern nodes sharing a (label column, degree) key share the
            // row "has a neighbour of that label with at least that degree":
            // each word of a key's row is computed once, when a domain of a
            // pattern neighbour first needs it (words a domain no longer
            // holds are skipped, as before), and then reused.
            const uint32_t C = t.nbr_cols;
            uint32_t key_of[KMAX], nkeys = 0;
            uint64_t keys[KMAX];
            for (uint32_t w = 0; w < k; w++) {
                const uint64_t key = ((uint64_t)(lab[w] == LABEL_ANY ? C - 1 : lab[w]) << 8) | std::min<uint32_t>(deg[w], 255);
                uint32_t j = 0;
                while (j < nkeys && keys[j] != key) j++;
                if (j == nkeys) keys[nkeys++] = key;
                key_of[w] = j;
            }
            const uint32_t WB = (W + 63) / 64;   // words of the per-key "computed" bitmaps
            std::vector<uint64_t> rows((size_t)nkeys * W), done((size_t)nkeys * WB, 0);
            for (uint32_t u = 0; u < k; u++) {
                if (!nb[u]) continue;
                uint64_t *d = &D[(size_t)u * W];
                for (uint64_t m = nb[u]; m; m &= m - 1) {
                    const uint32_t w = (uint32_t)__builtin_ctzll(m);
                    const uint32_t j = key_of[w];
                    uint64_t *row = &rows[(size_t)j * W];
                    uint64_t *dn = &done[(size_t)j * WB];
                    const uint8_t *cl = &t.nbr_deg[(size_t)(keys[j] >> 8) * t.nbr_stride];
                    const uint8_t dmin = (uint8_t)(keys[j] & 0xFF);
                    for (uint32_t i = 0; i < W; i++) {
                        if (!d[i]) continue;
                        if (!((dn[i >> 6] >> (i & 63)) & 1)) {
                            row[i] = bytes_at_least(cl + (size_t)i * 64, dmin);
                            dn[i >> 6] |= 1ull << (i & 63);
                        }
                        const uint64_t keep = d[i] & row[i];
                        if (keep != d[i]) {
                            d[i] = keep;
                            dirty |= 1ull << u;
                        }
                    }
                }
            }
        } else if (!any_empty) {
            for (uint32_t u = 0; u < k; u++)
                if (nb[u]) dirty |= 1ull << u;
        }
        const std::vector<uint32_t> &irp = tg.in_rp(), &icol = tg.in_col(), &ielab = tg.in_elab();
        // a target arc out of v (in: into v) of label b reaching a member of D(w)
        auto supported = [&](uint32_t v, const uint64_t *dw, bool in, uint32_t b) {
            const std::vector<uint32_t> &rp = in ? irp : tg.rp, &cl = in ? icol : tg.col;
            const std::vector<uint32_t> &el = in ? ielab : tg.elab;
            for (uint32_t e = rp[v]; e < rp[v + 1]; e++)
                if (test_bit(dw, cl[e]) && (!elabelled || (el.empty() ? 0u : el[e]) == b)) return true;
            return false;
        };
        if (!directed && !elabelled) {
            // undirected, no edge labels compared: a round builds, for each w
            // whose domain changed, the support set S(w) (every target
            // neighbour of a member of D(w)) and intersects the domains of
            // w's pattern neighbours with it
            std::vector<uint64_t> S(W);
            while (dirty) {
                uint64_t next = 0;
                for (uint64_t mw = dirty; mw; mw &= mw - 1) {
                    const uint32_t w = (uint32_t)__builtin_ctzll(mw);
                    std::fill(S.begin(), S.end(), 0ull);
                    const uint64_t *dw = &D[(size_t)w * W];
                    for (uint32_t i = 0; i < W; i++)
                        for (uint64_t bits = dw[i]; bits; bits &= bits - 1) {
                            const uint32_t x = i * 64 + (uint32_t)__builtin_ctzll(bits);
                            for (uint32_t e = tg.rp[x]; e < tg.rp[x + 1]; e++) {
                                const uint32_t y = tg.col[e];
                                S[y >> 6] |= 1ull << (y & 63);
                            }
                        }
                    for (uint64_t mu = nb[w]; mu; mu &= mu - 1) {
                        const uint32_t u = (uint32_t)__builtin_ctzll(mu);
                        uint64_t *d = &D[(size_t)u * W];
                        uint64_t diff = 0;
                        for (uint32_t i = 0; i < W; i++) {
                            const uint64_t x = d[i] & S[i];
                            diff |= x ^ d[i];
                            d[i] = x;
                        }
                        if (diff) next |= 1ull << u;
                    }
                }
                dirty = next;
            }
        }
        while (dirty) {
            uint64_t next = 0;
            for (uint32_t u = 0; u < k; u++) {
                const uint64_t ws = nb[u] & dirty;
                if (!ws) continue;
                uint64_t *d = &D[(size_t)u * W];
                for (uint32_t i = 0; i < W; i++) {
                    for (uint64_t bits = d[i]; bits; bits &= bits - 1) {
                        const uint32_t v = i * 64 + (uint32_t)__builtin_ctzll(bits);
                        for (uint64_t m = ws; m; m &= m - 1) {
                            const uint32_t w = (uint32_t)__builtin_ctzll(m);
                            const uint64_t *dw = &D[(size_t)w * W];
                            bool sup;
                            if (!directed) {
                                sup = supported(v, dw, false, elabelled ? parc(u, w) : 0u);
                            } else {
                                sup = true;
                                if ((outm[u] >> w) & 1) sup = supported(v, dw, false, elabelled ? parc(u, w) : 0u);
                                if (sup && ((outm[w] >> u) & 1)) sup = supported(v, dw, true, elabelled ? parc(w, u) : 0u);
                            }
                            if (!sup) {
                                d[i] &= ~(1ull << (v & 63));
                                next |= 1ull << u;
                                break;
                            }
                        }
                    }
                }
            }
            dirty = next;
        }
        for (uint32_t u = 0; u < k; u++) {
            dsize[u] = popcount_row(&D[(size_t)u * W], W);
            if (!dsize[u]) pl.empty = true;
        }
        if (!pl.empty && mode == SGE_RIDS_SI_FC) {
            // forward checking: a singleton's node leaves every other domain,
            // repeated for singletons this creates
            uint64_t done = 0;
            for (bool progress = true; progress && !pl.empty;) {
                progress = false;
                for (uint32_t u = 0; u < k && !pl.empty; u++) {
                    if (((done >> u) & 1) || dsize[u] != 1) continue;
                    done |= 1ull << u;
                    progress = true;
                    const uint64_t *du = &D[(size_t)u * W];
                    uint32_t word = 0;
                    while (!du[word]) word++;
                    uint64_t bit = du[word];
                    for (uint32_t w = 0; w < k; w++) {
                        if (w == u) continue;
                        uint64_t &x = D[(size_t)w * W + word];
                        if (x & bit) {
                            x &= ~bit;
                            if (--dsize[w] == 0) pl.empty = true;
                        }
                    }
                }
            }
        }
    }
    if (pl.empty) return;

    // constraint-first order
    const bool use_si = mode == SGE_RIDS_SI || mode == SGE_RIDS_SI_FC;
    constraint_first_order(nb, odeg, dsize, k, use_dom, use_si, pl.order);

    uint32_t pos_of[KMAX];
    for (uint32_t i = 0; i < k; i++) pos_of[pl.order[i]] = i;
    pl.pdir_out = pl.pboth = 0;
    if (elabelled) {
        // edge labels by position pair: lmat[a * k + b] = label of arc order[a] -> order[b]
        pl.lmat.assign((size_t)k * k, LABEL_NONE);
        for (uint32_t a = 0; a < k; a++)
            for (uint32_t e = p.rp[pl.order[a]]; e < p.rp[pl.order[a] + 1]; e++)
                pl.lmat[(size_t)a * k + pos_of[p.col[e]]] = p.elab.empty() ? 0u : p.elab[e];
    }
    for (uint32_t i = 0; i < k; i++) {
        uint32_t u = pl.order[i];
        uint64_t earlier = 0;
        for (uint64_t m = nb[u]; m; m &= m - 1) {
            uint32_t j = pos_of[__builtin_ctzll(m)];
            if (j < i) earlier |= 1ull << j;
        }
        pl.parent[i] = earlier ? (int32_t)__builtin_ctzll(earlier) : -1;
        pl.back[i] = earlier ? (earlier & (earlier - 1)) : 0;
        pl.plabel[i] = lab[u];
        pl.pdeg[i] = deg[u];
        pl.pindeg[i] = indeg[u];
        // directed: which earlier positions have an arc into u, which an arc
        // from u; the parent's candidates follow the arc parent -> u if there
        // is one, else u -> parent
        pl.bout[i] = pl.bin[i] = 0;
        for (uint64_t m = earlier; m; m &= m - 1) {
            const uint32_t j = (uint32_t)__builtin_ctzll(m), w = pl.order[j];
            if ((outm[w] >> u) & 1) pl.bout[i] |= 1ull << j;
            if ((outm[u] >> w) & 1) pl.bin[i] |= 1ull << j;
        }
        if (pl.parent[i] >= 0) {
            const uint64_t pb = 1ull << pl.parent[i];
            if (pl.bout[i] & pb) pl.pdir_out |= 1ull << i;
            if ((pl.bout[i] & pb) && (pl.bin[i] & pb)) pl.pboth |= 1ull << i;
            pl.bout[i] &= ~pb;
            pl.bin[i] &= ~pb;
        }
        pl.list_off[i] = pl.list_len[i] = 0;
        if (pl.parent[i] >= 0) continue;
        // parentless position: candidates are V_t (RI) or D(u) (RI-DS), here
        // pre-filtered by the label and degree rules, which every candidate
        // must pass anyway; the first position is limited to [root_lo, root_hi)
        uint32_t lo = i == 0 ? root_lo : 0, hi = i == 0 ? root_hi : 0xFFFFFFFFu;
        pl.list_off[i] = (uint32_t)pl.lists.size();
        if (use_dom) {
            const uint64_t *d = &D[(size_t)u * W];
            for (uint32_t w = 0; w < W; w++)
                for (uint64_t bits = d[w]; bits; bits &= bits - 1) {
                    uint32_t v = w * 64 + (uint32_t)__builtin_ctzll(bits);
                    if (v >= lo && v < hi) pl.lists.push_back(v);
                }
        } else {
            std::vector<uint32_t> tmp;
            compat_nodes(u, [&](uint32_t v) { if (v >= lo && v < hi) tmp.push_back(v); });
            std::sort(tmp.begin(), tmp.end());
            pl.lists.insert(pl.lists.end(), tmp.begin(), tmp.end());
        }
        pl.list_len[i] = (uint32_t)pl.lists.size() - pl.list_off[i];
    }

    if (want_pos_bits) {
        pos_bits.assign((size_t)k * W, 0);
        for (uint32_t i = 0; i < k; i++) {
            uint64_t *dst = &pos_bits[(size_t)i * W];
            uint32_t u = pl.order[i];
            if (use_dom) {
                std::memcpy(dst, &D[(size_t)u * W], W * sizeof(uint64_t));
            } else {
                compat_nodes(u, [&](uint32_t v) { dst[v >> 6] |= 1ull << (v & 63); });
            }
            if (i == 0 && (root_lo > 0 || root_hi < n)) {
                for (uint32_t v = 0; v < n; v++)
                    if (v < root_lo || v >= root_hi) dst[v >> 6] &= ~(1ull << (v & 63));
            }
        }
    }
}

}  // namespace sge
