// Graph ingest: validation and normalisation of CSR input, and the per-target
// label index the planner reads.  Graphs are simple (Section 2.1), directed or
// undirected (both directions of every edge), with node and optional edge
// labels compared for equality only.
#include <algorithm>
#include <unordered_map>

#include "sge_internal.h"

namespace sge {

std::string normalise_graph(uint32_t n, const uint32_t *row_ptr, const uint32_t *col, const uint32_t *labels,
                            const uint32_t *edge_labels, bool directed, HostGraph &out) {
    if (!row_ptr) return "row_ptr is NULL";
    if (row_ptr[0] != 0) return "row_ptr[0] must be 0";
    for (uint32_t v = 0; v < n; v++)
        if (row_ptr[v + 1] < row_ptr[v]) return "row_ptr is decreasing at node " + std::to_string(v);
    uint64_t m = row_ptr[n];
    if (m && !col) return "col is NULL";
    if (m > 0xFFFFFFF0ull) return "too many adjacency entries";
    out = HostGraph{};
    out.n = n;
    out.directed = directed;
    out.rp.assign(n + 1, 0);
    out.col.reserve(m);
    if (edge_labels) out.elab.reserve(m);
    std::vector<std::pair<uint32_t, uint32_t>> row;   // (neighbour, edge label)
    for (uint32_t v = 0; v < n; v++) {
        row.clear();
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            const uint32_t w = col[e];
            if (w >= n) return "neighbour id out of range at node " + std::to_string(v);
            if (w == v) return "self-loop at node " + std::to_string(v);
            row.emplace_back(w, edge_labels ? edge_labels[e] : 0u);
        }
        std::sort(row.begin(), row.end());
        for (size_t i = 0; i < row.size(); i++) {
            if (i && row[i].first == row[i - 1].first) {
                if (row[i].second != row[i - 1].second)
                    return "edge " + std::to_string(v) + " -> " + std::to_string(row[i].first) +
                           " given twice with different labels";
                continue;
            }
            out.col.push_back(row[i].first);
            if (edge_labels) out.elab.push_back(row[i].second);
        }
        out.rp[v + 1] = (uint32_t)out.col.size();
    }
    if (!directed) {
        // every (v, w) needs (w, v), with the same label
        for (uint32_t v = 0; v < n; v++) {
            for (uint32_t e = out.rp[v]; e < out.rp[v + 1]; e++) {
                const uint32_t w = out.col[e];
                auto b = out.col.begin() + out.rp[w], en = out.col.begin() + out.rp[w + 1];
                auto it = std::lower_bound(b, en, v);
                if (it == en || *it != v)
                    return "asymmetric adjacency: " + std::to_string(v) + " -> " + std::to_string(w) +
                           " has no reverse entry";
                if (edge_labels && out.elab[it - out.col.begin()] != out.elab[e])
                    return "undirected edge " + std::to_string(v) + " - " + std::to_string(w) +
                           " has different labels in its two directions";
            }
        }
    } else {
        // in-edges: the transpose, rows sorted by source
        out.irp.assign(n + 1, 0);
        for (uint32_t w : out.col) out.irp[w + 1]++;
        for (uint32_t v = 0; v < n; v++) out.irp[v + 1] += out.irp[v];
        out.icol.resize(out.col.size());
        if (edge_labels) out.ielab.resize(out.col.size());
        std::vector<uint32_t> fill(out.irp.begin(), out.irp.end() - 1);
        for (uint32_t v = 0; v < n; v++)
            for (uint32_t e = out.rp[v]; e < out.rp[v + 1]; e++) {
                const uint32_t at = fill[out.col[e]]++;
                out.icol[at] = v;
                if (edge_labels) out.ielab[at] = out.elab[e];
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
    t.label_bits.clear();
    t.deg_ge.clear();
    if (!g.directed && ((uint64_t)t.label_keys.size() + 64) * t.W * 8 <= LABEL_DEG_BITS_MAX_BYTES) {
        t.label_bits.assign((size_t)t.label_keys.size() * t.W, 0);
        t.deg_ge.assign((size_t)64 * t.W, 0);
        for (uint32_t v = 0; v < g.n; v++) {
            const uint64_t bit = 1ull << (v & 63);
            t.label_bits[(size_t)t.dlab[v] * t.W + (v >> 6)] |= bit;
            const uint32_t dv = std::min<uint32_t>(g.rp[v + 1] - g.rp[v], 63);
            for (uint32_t d = 0; d <= dv; d++) t.deg_ge[(size_t)d * t.W + (v >> 6)] |= bit;
        }
    }
    // the first arc-consistency round reads, for a candidate v and a pattern
    // neighbour of label L and degree d, whether v has a neighbour of label L
    // and degree >= d (pattern degrees are below 64, so 255 saturates safely)
    t.nbr_deg.clear();
    t.nbr_cols = (uint32_t)t.label_keys.size() + 1;
    t.nbr_stride = t.W * 64;   // columns padded to whole 64-node words (zeros)
    if ((uint64_t)t.nbr_stride * t.nbr_cols <= NBR_DEG_MAX_BYTES) {
        const uint32_t C = t.nbr_cols;
        t.nbr_deg.assign((size_t)t.nbr_stride * C, 0);
        uint8_t *any = &t.nbr_deg[(size_t)(C - 1) * t.nbr_stride];
        for (uint32_t v = 0; v < g.n; v++) {
            for (uint32_t e = g.rp[v]; e < g.rp[v + 1]; e++) {
                const uint32_t x = g.col[e];
                const uint8_t dx = (uint8_t)std::min<uint32_t>(g.rp[x + 1] - g.rp[x], 255);
                uint8_t &byl = t.nbr_deg[(size_t)t.dlab[x] * t.nbr_stride + v];
                byl = std::max(byl, dx);
                any[v] = std::max(any[v], dx);
            }
        }
    }
}

}  // namespace sge
