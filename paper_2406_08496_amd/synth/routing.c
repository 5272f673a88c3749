/*
 * Shortest-time routing for the synthetic demand generator.
 *
 * The simulated method takes routed demand as input: every trip arrives with
 * its full route (a contiguous edge sequence) already chosen (paper, Section
 * 3.1, data layout, vehicle data).  This helper produces those routes for the
 * seeded stand-in instances.  It contains none of the simulation arithmetic.
 *
 * Route rule: static shortest travel time, edge weight w_e = length_e / v0_e in
 * fp64.  For every destination d a backward Dijkstra gives dist(u -> d) and the
 * next edge out of every node u.  Among equally short choices the lower edge
 * id is kept, so the result does not depend on heap order or thread count.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC routing.c -o _routing.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct {
    double key;
    int32_t node;
} heap_item;

typedef struct {
    heap_item *a;
    int64_t n, cap;
} heap;

static int heap_push(heap *h, double key, int32_t node) {
    if (h->n == h->cap) {
        int64_t nc = h->cap ? h->cap * 2 : 1024;
        heap_item *na = (heap_item *)realloc(h->a, (size_t)nc * sizeof(heap_item));
        if (!na) return -1;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->n++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p].key <= key) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].key = key;
    h->a[i].node = node;
    return 0;
}

static heap_item heap_pop(heap *h) {
    heap_item top = h->a[0];
    heap_item last = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1;
        if (l >= h->n) break;
        int64_t r = l + 1;
        int64_t c = (r < h->n && h->a[r].key < h->a[l].key) ? r : l;
        if (h->a[c].key >= last.key) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->n > 0) h->a[i] = last;
    return top;
}

/*
 * next_edge[d * n_nodes + u] = edge to take at node u toward dest_nodes[d]
 * (-1 at the destination itself and at nodes that cannot reach it).
 * in_off/in_edges: CSR of incoming edges per node (any order).
 * Returns 0, or -1 on allocation failure.
 */
int synth_route_trees(int32_t n_nodes, int32_t n_edges, const int32_t *src,
                      const int32_t *dst, const double *weight,
                      const int64_t *in_off, const int32_t *in_edges,
                      int32_t n_dest, const int32_t *dest_nodes,
                      int32_t *next_edge) {
    int failed = 0;
    (void)n_edges;
    (void)dst;
#pragma omp parallel
    {
        double *dist = (double *)malloc((size_t)n_nodes * sizeof(double));
        uint8_t *done = (uint8_t *)malloc((size_t)n_nodes);
        heap h = {0, 0, 0};
        if (!dist || !done) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int32_t d = 0; d < n_dest; d++) {
            if (!dist || !done) continue;
            int32_t *nx = next_edge + (int64_t)d * n_nodes;
            for (int32_t u = 0; u < n_nodes; u++) {
                dist[u] = INFINITY;
                done[u] = 0;
                nx[u] = -1;
            }
            int32_t t = dest_nodes[d];
            dist[t] = 0.0;
            h.n = 0;
            if (heap_push(&h, 0.0, t)) { failed = 1; continue; }
            while (h.n > 0) {
                heap_item it = heap_pop(&h);
                int32_t y = it.node;
                if (done[y]) continue;
                done[y] = 1;
                for (int64_t j = in_off[y]; j < in_off[y + 1]; j++) {
                    int32_t e = in_edges[j];
                    int32_t x = src[e];
                    if (done[x]) continue;
                    double cand = dist[y] + weight[e];
                    if (cand < dist[x] || (cand == dist[x] && e < nx[x])) {
                        dist[x] = cand;
                        nx[x] = e;
                        if (heap_push(&h, cand, x)) { failed = 1; break; }
                    }
                }
            }
        }
        free(dist);
        free(done);
        free(h.a);
    }
    return failed ? -1 : 0;
}

/*
 * Route length (edge count) of each trip origin -> dest_nodes[dest_idx].
 * Returns -1 if some trip cannot reach its destination or origin == dest.
 */
int synth_route_lengths(int32_t n_nodes, const int32_t *dst,
                        const int32_t *next_edge, const int32_t *dest_nodes,
                        int64_t n_trips, const int32_t *origin,
                        const int32_t *dest_idx, int32_t *out_len) {
    int bad = 0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_trips; i++) {
        const int32_t *nx = next_edge + (int64_t)dest_idx[i] * n_nodes;
        int32_t t = dest_nodes[dest_idx[i]];
        int32_t u = origin[i];
        int32_t len = 0;
        while (u != t) {
            int32_t e = nx[u];
            if (e < 0 || len > n_nodes) { len = -1; break; }
            u = dst[e];
            len++;
        }
        if (len <= 0) bad = 1;
        out_len[i] = len;
    }
    return bad ? -1 : 0;
}

/* Writes each trip's edge sequence at route_off[i] .. route_off[i+1]. */
void synth_route_fill(int32_t n_nodes, const int32_t *dst,
                      const int32_t *next_edge, const int32_t *dest_nodes,
                      int64_t n_trips, const int32_t *origin,
                      const int32_t *dest_idx, const int64_t *route_off,
                      int32_t *route_edges) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_trips; i++) {
        const int32_t *nx = next_edge + (int64_t)dest_idx[i] * n_nodes;
        int32_t t = dest_nodes[dest_idx[i]];
        int32_t u = origin[i];
        int64_t p = route_off[i];
        while (u != t) {
            int32_t e = nx[u];
            route_edges[p++] = e;
            u = dst[e];
        }
    }
}
