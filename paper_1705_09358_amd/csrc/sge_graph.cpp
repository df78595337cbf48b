// Graph ingest: validation and normalisation of symmetric CSR input, and the
// per-target label index the planner reads.  Graphs are undirected and simple
// (Section 2.1 with undirected edges); labels are compared for equality only.
#include <algorithm>
#include <unordered_map>

#include "sge_internal.h"

namespace sge {

std::string normalise_graph(uint32_t n, const uint32_t *row_ptr, const uint32_t *col, const uint32_t *labels,
                            HostGraph &out) {
    if (!row_ptr) return "row_ptr is NULL";
    if (row_ptr[0] != 0) return "row_ptr[0] must be 0";
    for (uint32_t v = 0; v < n; v++)
        if (row_ptr[v + 1] < row_ptr[v]) return "row_ptr is decreasing at node " + std::to_string(v);
    uint64_t m = row_ptr[n];
    if (m && !col) return "col is NULL";
    if (m > 0xFFFFFFF0ull) return "too many adjacency entries";
    out.n = n;
    out.rp.assign(n + 1, 0);
    out.col.clear();
    out.col.reserve(m);
    std::vector<uint32_t> row;
    for (uint32_t v = 0; v < n; v++) {
        row.assign(col + row_ptr[v], col + row_ptr[v + 1]);
        for (uint32_t w : row) {
            if (w >= n) return "neighbour id out of range at node " + std::to_string(v);
            if (w == v) return "self-loop at node " + std::to_string(v);
        }
        std::sort(row.begin(), row.end());
        row.erase(std::unique(row.begin(), row.end()), row.end());
        out.col.insert(out.col.end(), row.begin(), row.end());
        out.rp[v + 1] = (uint32_t)out.col.size();
    }
    // symmetry: every (v, w) needs (w, v)
    for (uint32_t v = 0; v < n; v++) {
        for (uint32_t e = out.rp[v]; e < out.rp[v + 1]; e++) {
            uint32_t w = out.col[e];
            if (!std::binary_search(out.col.begin() + out.rp[w], out.col.begin() + out.rp[w + 1], v))
                return "asymmetric adjacency: " + std::to_string(v) + " -> " + std::to_string(w) +
                       " has no reverse entry";
        }
    }
    out.has_labels = labels != nullptr;
    out.lab.assign(n, 0);
    if (labels) std::copy(labels, labels + n, out.lab.begin());
    return "";
}

void index_target(Target &t) {
    const HostGraph &g = t.g;
    // dense label ids in increasing order of the raw labels, so that a raw
    // label's id is its rank among label_keys (found by binary search)
    t.label_keys.assign(g.lab.begin(), g.lab.end());
    std::sort(t.label_keys.begin(), t.label_keys.end());
    t.label_keys.erase(std::unique(t.label_keys.begin(), t.label_keys.end()), t.label_keys.end());
    t.dlab.resize(g.n);
    t.by_label.assign(t.label_keys.size(), {});
    for (uint32_t v = 0; v < g.n; v++) {
        const uint32_t id =
            (uint32_t)(std::lower_bound(t.label_keys.begin(), t.label_keys.end(), g.lab[v]) - t.label_keys.begin());
        t.dlab[v] = id;
        t.by_label[id].push_back(v);
    }
    t.W = (g.n + 63) / 64;
    t.max_deg = 0;
    for (uint32_t v = 0; v < g.n; v++) t.max_deg = std::max(t.max_deg, g.rp[v + 1] - g.rp[v]);
    // the first arc-consistency round reads, for a candidate v and a pattern
    // neighbour of label L and degree d, whether v has a neighbour of label L
    // and degree >= d (pattern degrees are below 64, so 255 saturates safely)
    t.nbr_deg.clear();
    t.nbr_cols = (uint32_t)t.label_keys.size() + 1;
    if ((uint64_t)g.n * t.nbr_cols <= NBR_DEG_MAX_BYTES) {
        const uint32_t C = t.nbr_cols;
        t.nbr_deg.assign((size_t)g.n * C, 0);
        for (uint32_t v = 0; v < g.n; v++) {
            uint8_t *row = &t.nbr_deg[(size_t)v * C];
            for (uint32_t e = g.rp[v]; e < g.rp[v + 1]; e++) {
                const uint32_t x = g.col[e];
                const uint8_t dx = (uint8_t)std::min<uint32_t>(g.rp[x + 1] - g.rp[x], 255);
                row[t.dlab[x]] = std::max(row[t.dlab[x]], dx);
                row[C - 1] = std::max(row[C - 1], dx);
            }
        }
    }
}

}  // namespace sge
