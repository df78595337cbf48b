/*
 * Synthetic protein-contact-like target graphs: a confined 3-D self-avoiding
 * walk whose nodes are joined when they lie closer than a contact cutoff.
 *
 * This file is an input generator only.  It holds none of the subgraph
 * enumeration method; it is shared by the tests, the benchmark and the
 * oracle harness as the source of seeded workloads.
 *
 * Random numbers: xoshiro256** (Blackman and Vigna, "Scrambled linear
 * pseudorandom number generators", 2018) seeded through splitmix64, both
 * written from their published definitions.  The 64-bit seed is drawn by
 * the Python side from numpy's PCG64 stream.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; } xo_state;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t xo_next(xo_state *st) {
    uint64_t *s = st->s;
    uint64_t r = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return r;
}

/* uniform double in [0,1) from the top 53 bits */
static double xo_unif(xo_state *st) { return (double)(xo_next(st) >> 11) * (1.0 / 9007199254740992.0); }

typedef struct {
    int nc;          /* cells per axis */
    double lo, cell; /* grid origin and cell edge */
    int32_t *head;   /* nc^3 list heads (-1 = empty) */
    int32_t *next;   /* per node */
} grid;

static int cell_of(const grid *g, double v) {
    int c = (int)floor((v - g->lo) / g->cell);
    if (c < 0) c = 0;
    if (c >= g->nc) c = g->nc - 1;
    return c;
}

static int grid_init(grid *g, double half_extent, double cell, uint32_t n) {
    g->cell = cell;
    g->lo = -half_extent;
    g->nc = (int)ceil(2.0 * half_extent / cell) + 1;
    size_t ncell = (size_t)g->nc * g->nc * g->nc;
    g->head = (int32_t *)malloc(ncell * sizeof(int32_t));
    g->next = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
    if (!g->head || !g->next) { free(g->head); free(g->next); return -1; }
    for (size_t i = 0; i < ncell; i++) g->head[i] = -1;
    return 0;
}

static void grid_free(grid *g) { free(g->head); free(g->next); }

static size_t cell_index(const grid *g, int cx, int cy, int cz) {
    return ((size_t)cx * g->nc + cy) * g->nc + cz;
}

/*
 * Confined self-avoiding walk of n points.  Step length `step`; a proposed
 * point is rejected if it leaves the ball of radius `radius` or comes closer
 * than `excl` to any point other than its predecessor.  Up to `max_tries`
 * directions (uniform on the sphere) are tried per step; when all fail the
 * walk retracts its last point and continues.  Returns 0, or -1 when the walk
 * retracts more than `max_retract` times in total (the caller redraws).
 */
int synth_saw(uint32_t n, double step, double excl, double radius, uint64_t seed,
              int max_tries, int64_t max_retract, double *xyz) {
    if (n == 0) return 0;
    xo_state st;
    uint64_t sm = seed;
    for (int i = 0; i < 4; i++) st.s[i] = splitmix64(&sm);
    grid g;
    if (grid_init(&g, radius + step, excl, n) != 0) return -2;
    xyz[0] = xyz[1] = xyz[2] = 0.0;
    int cx = cell_of(&g, 0.0);
    g.next[0] = -1;
    g.head[cell_index(&g, cx, cx, cx)] = 0;
    uint32_t cur = 1;
    int64_t retracts = 0;
    const double excl2 = excl * excl, rad2 = radius * radius;
    while (cur < n) {
        const double *pv = xyz + 3 * (size_t)(cur - 1);
        int placed = 0;
        for (int t = 0; t < max_tries && !placed; t++) {
            double z = 2.0 * xo_unif(&st) - 1.0;
            double ph = 6.283185307179586 * xo_unif(&st);
            double r = sqrt(1.0 - z * z);
            double p[3] = {pv[0] + step * r * cos(ph), pv[1] + step * r * sin(ph), pv[2] + step * z};
            if (p[0] * p[0] + p[1] * p[1] + p[2] * p[2] > rad2) continue;
            int c0 = cell_of(&g, p[0]), c1 = cell_of(&g, p[1]), c2 = cell_of(&g, p[2]);
            int clash = 0;
            for (int a = c0 - 1; a <= c0 + 1 && !clash; a++) {
                if (a < 0 || a >= g.nc) continue;
                for (int b = c1 - 1; b <= c1 + 1 && !clash; b++) {
                    if (b < 0 || b >= g.nc) continue;
                    for (int c = c2 - 1; c <= c2 + 1 && !clash; c++) {
                        if (c < 0 || c >= g.nc) continue;
                        for (int32_t j = g.head[cell_index(&g, a, b, c)]; j >= 0; j = g.next[j]) {
                            if ((uint32_t)j == cur - 1) continue;
                            const double *q = xyz + 3 * (size_t)j;
                            double dx = q[0] - p[0], dy = q[1] - p[1], dz = q[2] - p[2];
                            if (dx * dx + dy * dy + dz * dz < excl2) { clash = 1; break; }
                        }
                    }
                }
            }
            if (clash) continue;
            double *o = xyz + 3 * (size_t)cur;
            o[0] = p[0]; o[1] = p[1]; o[2] = p[2];
            size_t ci = cell_index(&g, c0, c1, c2);
            g.next[cur] = g.head[ci];
            g.head[ci] = (int32_t)cur;
            cur++;
            placed = 1;
        }
        if (!placed) {
            if (++retracts > max_retract || cur <= 1) { grid_free(&g); return -1; }
            /* the newest point is the head of its cell's list */
            const double *q = xyz + 3 * (size_t)(cur - 1);
            size_t ci = cell_index(&g, cell_of(&g, q[0]), cell_of(&g, q[1]), cell_of(&g, q[2]));
            g.head[ci] = g.next[cur - 1];
            cur--;
        }
    }
    grid_free(&g);
    return 0;
}

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Contact graph: undirected edge {i,j} (i != j) when |x_i - x_j| < cutoff.
 * With col == NULL only the degrees are computed: row_ptr[0..n] is filled and
 * the number of adjacency entries (twice the edge count) is returned.  With
 * col given (of that size) the sorted rows are written.  Returns -1 on
 * allocation failure.
 */
int64_t synth_contacts(uint32_t n, const double *xyz, double cutoff, uint32_t *row_ptr, uint32_t *col) {
    if (n == 0) { row_ptr[0] = 0; return 0; }
    double ext = 0.0;
    for (size_t i = 0; i < 3 * (size_t)n; i++) ext = fmax(ext, fabs(xyz[i]));
    grid g;
    if (grid_init(&g, ext + cutoff, cutoff, n) != 0) return -1;
    for (uint32_t i = 0; i < n; i++) {
        const double *p = xyz + 3 * (size_t)i;
        size_t ci = cell_index(&g, cell_of(&g, p[0]), cell_of(&g, p[1]), cell_of(&g, p[2]));
        g.next[i] = g.head[ci];
        g.head[ci] = (int32_t)i;
    }
    const double c2 = cutoff * cutoff;
    uint32_t *fill = NULL;
    if (col) {
        fill = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
        if (!fill) { grid_free(&g); return -1; }
        for (uint32_t i = 0; i < n; i++) fill[i] = row_ptr[i];
    }
    int64_t total = 0;
    for (uint32_t i = 0; i < n; i++) {
        const double *p = xyz + 3 * (size_t)i;
        int c0 = cell_of(&g, p[0]), c1 = cell_of(&g, p[1]), c2i = cell_of(&g, p[2]);
        uint32_t deg = 0;
        for (int a = c0 - 1; a <= c0 + 1; a++) {
            if (a < 0 || a >= g.nc) continue;
            for (int b = c1 - 1; b <= c1 + 1; b++) {
                if (b < 0 || b >= g.nc) continue;
                for (int c = c2i - 1; c <= c2i + 1; c++) {
                    if (c < 0 || c >= g.nc) continue;
                    for (int32_t j = g.head[cell_index(&g, a, b, c)]; j >= 0; j = g.next[j]) {
                        if ((uint32_t)j == i) continue;
                        const double *q = xyz + 3 * (size_t)j;
                        double dx = q[0] - p[0], dy = q[1] - p[1], dz = q[2] - p[2];
                        if (dx * dx + dy * dy + dz * dz < c2) {
                            if (col) col[fill[i]++] = (uint32_t)j;
                            deg++;
                        }
                    }
                }
            }
        }
        if (!col) row_ptr[i + 1] = deg;
        total += deg;
    }
    if (!col) {
        row_ptr[0] = 0;
        for (uint32_t i = 0; i < n; i++) row_ptr[i + 1] += row_ptr[i];
    } else {
        for (uint32_t i = 0; i < n; i++)
            qsort(col + row_ptr[i], row_ptr[i + 1] - row_ptr[i], sizeof(uint32_t), cmp_u32);
        free(fill);
    }
    grid_free(&g);
    return total;
}
