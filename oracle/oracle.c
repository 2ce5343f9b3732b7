/*
 * CPU oracle for the superstep engine -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library.  The device library never links, calls or
 * includes it, and this file includes nothing from the device library.
 *
 * What it computes is one superstep of the paper's vertex-program template
 * (Section "Algorithm Template": MSGGen produces a message per edge from the
 * source vertex, MSGMerge combines the messages bound for one destination,
 * MSGApply folds the combined message into the vertex state), executed in the
 * BSP order Gen -> Merge -> Apply (Section "PowerGraph", which contrasts it
 * with GAS order).  Messages of one iteration have no data dependencies on
 * each other (Section "Pipeline Shuffling", Pipeline Parallelism paragraph),
 * so every message of superstep k is generated from the state as it stood at
 * the start of superstep k (Jacobi semantics).
 *
 * The three algorithms are the ones the evaluation runs (Section "Setup"):
 * PageRank, Bellman-Ford SSSP and label propagation (read as min-label
 * connected components).  The paper gives no formulas for them; the readings
 * used are:
 *   PageRank  x0 = 1/V; D = sum of x over vertices with out-degree 0;
 *             x'[v] = (1-d)/V + d * (sum_{u->v} x[u]/outdeg(u) + D/V).
 *   PPR       as PageRank with the teleport term and the dangling mass D sent
 *             to the seed s only; x0 = e_s.
 *   SSSP      dist[s] = 0, others INF = 0xFFFFFFFF; F1 = {s}; a vertex in
 *             F_k sends sat_add(dist[u], w) along each out-edge; the merge is
 *             min; F_{k+1} = vertices whose distance strictly decreased.
 *   CC        label[v] = global id of v; F1 = vertices with an edge; labels
 *             travel along both directions of every edge; merge is min.
 *   LP        (second reading of "label propagation", with the evaluation's
 *             15-iteration cap) labels start at the global id; every vertex
 *             takes the most frequent label among its distinct neighbours,
 *             the smallest on a tie (or_lp).
 * Everything runs in plain loops over the edge list, with PageRank in double
 * precision.  The functions above the "OpenMP timing mode" line are the
 * single-threaded reference.  The functions below it run the same
 * supersteps on all host cores and exist only to time the CPU baseline;
 * a CPU test pins them bitwise to the reference (integer minima are order
 * free; PageRank sums each destination's messages in the same edge order).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_INF 0xFFFFFFFFu

static inline uint32_t sat_add_u32(uint32_t a, uint32_t b)
{
    uint64_t s = (uint64_t)a + (uint64_t)b;
    return s > OR_INF ? OR_INF : (uint32_t)s;
}

/* Out-degree of every vertex from the edge list. */
void or_out_degree(int64_t V, int64_t E, const int32_t *src, int32_t *deg)
{
    memset(deg, 0, (size_t)V * sizeof(int32_t));
    for (int64_t e = 0; e < E; e++) deg[src[e]]++;
}

/*
 * One PageRank superstep (template order Gen -> Merge -> Apply).
 *   Gen:   each edge u->v carries x[u] / outdeg(u).
 *   Merge: acc[v] = sum of the messages bound for v (edge-list order).
 *   Apply: x'[v] = (1-d)/V + d * (acc[v] + D/V), D = dangling mass.
 * x_next must not alias x.
 */
void or_pr_superstep(int64_t V, int64_t E, const int32_t *src, const int32_t *dst,
                     const int32_t *deg, double d, const double *x, double *x_next)
{
    double D = 0.0;
    for (int64_t u = 0; u < V; u++)
        if (deg[u] == 0) D += x[u];
    for (int64_t v = 0; v < V; v++) x_next[v] = 0.0;
    for (int64_t e = 0; e < E; e++) {
        int32_t u = src[e];
        x_next[dst[e]] += x[u] / (double)deg[u];
    }
    double base = (1.0 - d) / (double)V;
    for (int64_t v = 0; v < V; v++) x_next[v] = base + d * (x_next[v] + D / (double)V);
}

/*
 * One personalised-PageRank superstep for seed s: the same Gen and Merge;
 * Apply sends the teleport (1-d) and the dangling mass D to the seed only:
 *   x'[v] = (1-d)*[v==s] + d * (acc[v] + D*[v==s]).
 */
void or_ppr_superstep(int64_t V, int64_t E, const int32_t *src, const int32_t *dst,
                      const int32_t *deg, double d, int32_t s, const double *x, double *x_next)
{
    double D = 0.0;
    for (int64_t u = 0; u < V; u++)
        if (deg[u] == 0) D += x[u];
    for (int64_t v = 0; v < V; v++) x_next[v] = 0.0;
    for (int64_t e = 0; e < E; e++) {
        int32_t u = src[e];
        x_next[dst[e]] += x[u] / (double)deg[u];
    }
    for (int64_t v = 0; v < V; v++) x_next[v] = d * x_next[v];
    x_next[s] += (1.0 - d) + d * D;
}

/*
 * One min-combine superstep shared by SSSP and CC (Jacobi):
 *   Gen:   every edge (u, v) with u in the frontier carries
 *          sat_add(state[u], w) (SSSP) or state[u] (CC, w == NULL).
 *          With `both_dirs` the edge also carries state[v] to u
 *          (CC treats edges as undirected).
 *   Merge: min over the messages bound for a vertex.
 *   Apply: state'[v] = min(state[v], merged); v joins the next frontier
 *          iff state'[v] < state[v].
 * Messages read `state` (start of superstep) and are folded into
 * `state_next`, so no message sees a value produced in the same superstep.
 * Returns |F_{k+1}|; *edges_out receives the number of messages generated.
 */
int64_t or_min_superstep(int64_t V, int64_t E, const int32_t *src, const int32_t *dst,
                         const uint32_t *w, int both_dirs, const uint32_t *state,
                         const uint8_t *front, uint32_t *state_next, uint8_t *front_next,
                         int64_t *edges_out)
{
    int64_t msgs = 0;
    memcpy(state_next, state, (size_t)V * sizeof(uint32_t));
    for (int64_t e = 0; e < E; e++) {
        int32_t u = src[e], v = dst[e];
        if (front[u]) {
            uint32_t m = w ? sat_add_u32(state[u], w[e]) : state[u];
            if (m < state_next[v]) state_next[v] = m;
            msgs++;
        }
        if (both_dirs && front[v]) {
            uint32_t m = state[v];
            if (m < state_next[u]) state_next[u] = m;
            msgs++;
        }
    }
    int64_t changed = 0;
    for (int64_t v = 0; v < V; v++) {
        front_next[v] = state_next[v] < state[v];
        changed += front_next[v];
    }
    if (edges_out) *edges_out = msgs;
    return changed;
}

/*
 * SSSP to convergence by repeated supersteps (Section "Iteration Control":
 * iterate until no vertex changes).  dist: V outputs.  Per superstep k
 * (0-based) the optional arrays receive |F_k|, the messages generated and
 * |F_{k+1}|.  Returns the number of supersteps K including the last one that
 * changed nothing, or -1 if max_steps was reached first (dist then holds the
 * state after max_steps supersteps), or -2 on allocation failure.
 */
int64_t or_sssp(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, const uint32_t *w,
                int32_t s, int64_t max_steps, uint32_t *dist,
                int64_t *front_size, int64_t *edges, int64_t *changed)
{
    uint32_t *nd = (uint32_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(uint32_t));
    uint8_t *f = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    uint8_t *nf = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    if (!nd || !f || !nf) { free(nd); free(f); free(nf); return -2; }
    for (int64_t v = 0; v < V; v++) dist[v] = OR_INF;
    int64_t fs = 0;
    if (s >= 0 && s < V) { dist[s] = 0; f[s] = 1; fs = 1; }
    int64_t k = 0, K = -1;
    while (k < max_steps) {
        int64_t ef = 0;
        int64_t c = or_min_superstep(V, E, src, dst, w, 0, dist, f, nd, nf, &ef);
        if (front_size) front_size[k] = fs;
        if (edges) edges[k] = ef;
        if (changed) changed[k] = c;
        memcpy(dist, nd, (size_t)V * sizeof(uint32_t));
        uint8_t *t = f; f = nf; nf = t;
        fs = c;
        k++;
        if (c == 0) { K = k; break; }
    }
    free(nd); free(f); free(nf);
    return K;
}

/*
 * Min-label connected components to convergence.  label[v] starts at the
 * global id (l2g[v], or v when l2g is NULL); F1 = vertices with at least one
 * edge.  Same return convention as or_sssp.
 */
int64_t or_cc(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, const int32_t *l2g,
              int64_t max_steps, uint32_t *label,
              int64_t *front_size, int64_t *edges, int64_t *changed)
{
    uint32_t *nl = (uint32_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(uint32_t));
    uint8_t *f = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    uint8_t *nf = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    if (!nl || !f || !nf) { free(nl); free(f); free(nf); return -2; }
    for (int64_t v = 0; v < V; v++) label[v] = l2g ? (uint32_t)l2g[v] : (uint32_t)v;
    for (int64_t e = 0; e < E; e++) { f[src[e]] = 1; f[dst[e]] = 1; }
    int64_t fs = 0;
    for (int64_t v = 0; v < V; v++) fs += f[v];
    int64_t k = 0, K = -1;
    while (k < max_steps) {
        int64_t ef = 0;
        int64_t c = or_min_superstep(V, E, src, dst, NULL, 1, label, f, nl, nf, &ef);
        if (front_size) front_size[k] = fs;
        if (edges) edges[k] = ef;
        if (changed) changed[k] = c;
        memcpy(label, nl, (size_t)V * sizeof(uint32_t));
        uint8_t *t = f; f = nf; nf = t;
        fs = c;
        k++;
        if (c == 0) { K = k; break; }
    }
    free(nl); free(f); free(nf);
    return K;
}

/*
 * Sync set (Section "Synchronization Caching", lazy uploading; Section
 * "Synchronization Skipping"): a vertex is uploaded only when another node
 * needs it (remote[v] != 0) and its value differs from the copy last
 * uploaded (bitwise); only its final value is sent.  Emits (gid, value) in
 * ascending local id order, which is ascending gid because local ids follow
 * global order.  Returns the count; an empty set means the synchronisation
 * of this iteration can be skipped.  `synced` is updated to the uploaded
 * values.
 */
int64_t or_delta(int64_t V, const uint8_t *remote, const int32_t *l2g, const uint32_t *now,
                 uint32_t *synced, int32_t *gid_out, uint32_t *val_out)
{
    int64_t n = 0;
    for (int64_t v = 0; v < V; v++) {
        if (!remote[v] || now[v] == synced[v]) continue;
        gid_out[n] = l2g ? l2g[v] : (int32_t)v;
        val_out[n] = now[v];
        synced[v] = now[v];
        n++;
    }
    return n;
}

/*
 * Label propagation in its community-detection form (the "LP" of Section
 * "Setup", which the evaluation caps at 15 iterations; NEXT-3 reading):
 *   labels start at the global id (l2g[v], or v);
 *   Gen:   every edge carries the label of each endpoint to the other
 *          (edges are undirected; self-loops carry nothing; a neighbour
 *          joined to v by several edges counts once);
 *   Merge: the multiset of labels arriving at v;
 *   Apply: v takes the label that arrives most often, the smallest of the
 *          most frequent ones on a tie; a vertex without neighbours keeps
 *          its label.  Messages read the labels of the start of the
 *          iteration (Jacobi), like every other superstep here.
 * or_sym_adjacency builds the deduplicated neighbour lists once (rows in
 * ascending vertex order, each row ascending); or_lp_superstep runs one
 * iteration on them and returns the number of vertices whose label changed.
 */
static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : x > y;
}

/* Returns the number of neighbour entries (nb_out needs room for 2E); -2 on
 * allocation failure.  rp_out has V+1 entries. */
int64_t or_sym_adjacency(int64_t V, int64_t E, const int32_t *src, const int32_t *dst,
                         int64_t *rp_out, int32_t *nb_out)
{
    uint64_t *pairs = (uint64_t *)malloc((size_t)(2 * E > 0 ? 2 * E : 1) * sizeof(uint64_t));
    if (!pairs) return -2;
    int64_t n = 0;
    for (int64_t e = 0; e < E; e++) {
        uint64_t u = (uint32_t)src[e], v = (uint32_t)dst[e];
        if (u == v) continue;
        pairs[n++] = (u << 32) | v;
        pairs[n++] = (v << 32) | u;
    }
    qsort(pairs, (size_t)n, sizeof(uint64_t), cmp_u64);
    for (int64_t v = 0; v <= V; v++) rp_out[v] = 0;
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        if (i > 0 && pairs[i] == pairs[i - 1]) continue;
        int64_t u = (int64_t)(pairs[i] >> 32);
        nb_out[m++] = (int32_t)(pairs[i] & 0xFFFFFFFFu);
        rp_out[u + 1]++;
    }
    for (int64_t v = 0; v < V; v++) rp_out[v + 1] += rp_out[v];
    free(pairs);
    return m;
}

int64_t or_lp_superstep(int64_t V, const int64_t *rp, const int32_t *nb, const uint32_t *label,
                        uint32_t *label_next)
{
    int64_t maxd = 0;
    for (int64_t v = 0; v < V; v++)
        if (rp[v + 1] - rp[v] > maxd) maxd = rp[v + 1] - rp[v];
    uint32_t *tmp = (uint32_t *)malloc((size_t)(maxd > 0 ? maxd : 1) * sizeof(uint32_t));
    if (!tmp) return -2;
    int64_t changed = 0;
    for (int64_t v = 0; v < V; v++) {
        int64_t d = rp[v + 1] - rp[v];
        if (d == 0) {
            label_next[v] = label[v];
            continue;
        }
        for (int64_t i = 0; i < d; i++) tmp[i] = label[nb[rp[v] + i]];
        qsort(tmp, (size_t)d, sizeof(uint32_t), cmp_u32);
        /* runs of equal labels in ascending order: the first longest run
         * holds the smallest of the most frequent labels */
        uint32_t best = tmp[0];
        int64_t best_n = 0, run = 0;
        for (int64_t i = 0; i < d; i++) {
            run = (i > 0 && tmp[i] == tmp[i - 1]) ? run + 1 : 1;
            if (run > best_n) {
                best_n = run;
                best = tmp[i];
            }
        }
        label_next[v] = best;
        changed += best != label[v];
    }
    free(tmp);
    return changed;
}

/*
 * LP for at most max_steps iterations, stopping after the first iteration
 * that changes nothing (counted).  label: V outputs; changed[k] (optional)
 * receives iteration k's changed count.  Returns the iterations run when the
 * last one changed nothing, -1 when max_steps ran and labels still moved
 * (label then holds the state after max_steps), -2 on allocation failure.
 */
int64_t or_lp(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, const int32_t *l2g,
              int64_t max_steps, uint32_t *label, int64_t *changed)
{
    int64_t *rp = (int64_t *)malloc((size_t)(V + 1) * sizeof(int64_t));
    int32_t *nb = (int32_t *)malloc((size_t)(2 * E > 0 ? 2 * E : 1) * sizeof(int32_t));
    uint32_t *nl = (uint32_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(uint32_t));
    if (!rp || !nb || !nl || or_sym_adjacency(V, E, src, dst, rp, nb) < 0) {
        free(rp); free(nb); free(nl);
        return -2;
    }
    for (int64_t v = 0; v < V; v++) label[v] = l2g ? (uint32_t)l2g[v] : (uint32_t)v;
    int64_t K = -1;
    for (int64_t k = 0; k < max_steps; k++) {
        int64_t c = or_lp_superstep(V, rp, nb, label, nl);
        if (c < 0) { K = -2; break; }
        if (changed) changed[k] = c;
        memcpy(label, nl, (size_t)V * sizeof(uint32_t));
        if (c == 0) { K = k + 1; break; }
    }
    free(rp); free(nb); free(nl);
    return K;
}

/* ------------------------------------------------------------------------
 * Independent pins.  These reach the same answers by different algorithms
 * and are used only to check the functions above.
 * ------------------------------------------------------------------------ */

/*
 * Binary-heap Dijkstra.  With hops == NULL it returns exact shortest
 * distances (unreachable -> INF).  With hops != NULL it orders paths
 * lexicographically by (distance, number of edges), by running on the
 * composite weight w * 2^26 + 1, and also returns for every vertex the
 * fewest edges among its shortest paths (-1 when unreachable).  Requires
 * V < 2^26 in that mode.
 */
int or_dijkstra(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, const uint32_t *w,
                int32_t s, uint32_t *dist, int32_t *hops)
{
    const int HB = 26;
    int64_t *rp = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
    int32_t *adj = (int32_t *)malloc((size_t)(E > 0 ? E : 1) * sizeof(int32_t));
    uint64_t *aw = (uint64_t *)malloc((size_t)(E > 0 ? E : 1) * sizeof(uint64_t));
    uint64_t *d = (uint64_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(uint64_t));
    uint8_t *done = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    int64_t *pos = (int64_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(int64_t));
    int64_t hcap = E + 1;
    uint64_t *hk = (uint64_t *)malloc((size_t)hcap * sizeof(uint64_t));
    int32_t *hv = (int32_t *)malloc((size_t)hcap * sizeof(int32_t));
    int rc = 0;
    if (!rp || !adj || !aw || !d || !done || !pos || !hk || !hv) { rc = -2; goto out; }
    if (hops && V >= ((int64_t)1 << HB)) { rc = -1; goto out; }
    for (int64_t e = 0; e < E; e++) rp[src[e] + 1]++;
    for (int64_t v = 0; v < V; v++) rp[v + 1] += rp[v];
    for (int64_t v = 0; v < V; v++) pos[v] = rp[v];
    for (int64_t e = 0; e < E; e++) {
        int64_t p = pos[src[e]]++;
        adj[p] = dst[e];
        aw[p] = hops ? (((uint64_t)w[e] << HB) + 1) : (uint64_t)w[e];
    }
    for (int64_t v = 0; v < V; v++) d[v] = UINT64_MAX;
    int64_t hn = 0;
    if (s >= 0 && s < V) { d[s] = 0; hk[0] = 0; hv[0] = s; hn = 1; }
    while (hn > 0) {
        uint64_t key = hk[0];
        int32_t u = hv[0];
        hn--;
        if (hn > 0) {  /* move the last element to the root and sift it down */
            uint64_t lk = hk[hn];
            int32_t lv = hv[hn];
            int64_t i = 0;
            for (;;) {
                int64_t c = 2 * i + 1;
                if (c >= hn) break;
                if (c + 1 < hn && hk[c + 1] < hk[c]) c++;
                if (hk[c] >= lk) break;
                hk[i] = hk[c]; hv[i] = hv[c]; i = c;
            }
            hk[i] = lk; hv[i] = lv;
        }
        if (done[u] || key != d[u]) continue;
        done[u] = 1;
        for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
            int32_t v = adj[p];
            uint64_t nd = key + aw[p];
            if (nd >= d[v]) continue;
            d[v] = nd;
            if (hn == hcap) {
                int64_t nc = hcap * 2;
                uint64_t *k2 = (uint64_t *)realloc(hk, (size_t)nc * sizeof(uint64_t));
                if (!k2) { rc = -2; goto out; }
                hk = k2;
                int32_t *v2 = (int32_t *)realloc(hv, (size_t)nc * sizeof(int32_t));
                if (!v2) { rc = -2; goto out; }
                hv = v2;
                hcap = nc;
            }
            int64_t i = hn++;  /* sift up */
            while (i > 0) {
                int64_t p2 = (i - 1) / 2;
                if (hk[p2] <= nd) break;
                hk[i] = hk[p2]; hv[i] = hv[p2]; i = p2;
            }
            hk[i] = nd; hv[i] = v;
        }
    }
    for (int64_t v = 0; v < V; v++) {
        uint64_t x = d[v];
        if (x == UINT64_MAX) {
            dist[v] = OR_INF;
            if (hops) hops[v] = -1;
            continue;
        }
        uint64_t dv = hops ? (x >> HB) : x;
        dist[v] = dv > (uint64_t)OR_INF ? OR_INF : (uint32_t)dv;
        if (hops) hops[v] = (int32_t)(x & (((uint64_t)1 << HB) - 1));
    }
out:
    free(rp); free(adj); free(aw); free(d); free(done); free(pos); free(hk); free(hv);
    return rc;
}

/*
 * Undirected BFS from the smallest vertex of every component (vertices are
 * scanned in increasing id; an unvisited vertex is the smallest of its
 * component).  hop[v] = edges from v to that smallest vertex.  Returns the
 * maximum hop over all vertices, or -2 on allocation failure.
 */
int64_t or_cc_hops(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, int32_t *hop)
{
    int64_t *rp = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
    int32_t *adj = (int32_t *)malloc((size_t)(2 * E > 0 ? 2 * E : 1) * sizeof(int32_t));
    int64_t *pos = (int64_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(int64_t));
    int32_t *q = (int32_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(int32_t));
    if (!rp || !adj || !pos || !q) { free(rp); free(adj); free(pos); free(q); return -2; }
    for (int64_t e = 0; e < E; e++) { rp[src[e] + 1]++; rp[dst[e] + 1]++; }
    for (int64_t v = 0; v < V; v++) rp[v + 1] += rp[v];
    for (int64_t v = 0; v < V; v++) pos[v] = rp[v];
    for (int64_t e = 0; e < E; e++) { adj[pos[src[e]]++] = dst[e]; adj[pos[dst[e]]++] = src[e]; }
    for (int64_t v = 0; v < V; v++) hop[v] = -1;
    int64_t maxh = 0;
    for (int64_t r = 0; r < V; r++) {
        if (hop[r] >= 0) continue;
        int64_t qh = 0, qt = 0;
        hop[r] = 0;
        q[qt++] = (int32_t)r;
        while (qh < qt) {
            int32_t u = q[qh++];
            for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
                int32_t v = adj[p];
                if (hop[v] >= 0) continue;
                hop[v] = hop[u] + 1;
                if (hop[v] > maxh) maxh = hop[v];
                q[qt++] = v;
            }
        }
    }
    free(rp); free(adj); free(pos); free(q);
    return maxh;
}

/* Union-find (path halving, union by smaller root id): min id per component
 * over undirected edges; label[v] = min over the component of gid. */
int or_union_find_min(int64_t V, int64_t E, const int32_t *src, const int32_t *dst,
                      const int32_t *l2g, uint32_t *label)
{
    int64_t *par = (int64_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(int64_t));
    if (!par) return -2;
    for (int64_t v = 0; v < V; v++) par[v] = v;
    for (int64_t e = 0; e < E; e++) {
        int64_t a = src[e], b = dst[e];
        while (par[a] != a) { par[a] = par[par[a]]; a = par[a]; }
        while (par[b] != b) { par[b] = par[par[b]]; b = par[b]; }
        if (a == b) continue;
        if (a < b) par[b] = a; else par[a] = b;
    }
    uint32_t *best = (uint32_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(uint32_t));
    if (!best) { free(par); return -2; }
    for (int64_t v = 0; v < V; v++) best[v] = OR_INF;
    for (int64_t v = 0; v < V; v++) {
        int64_t r = v;
        while (par[r] != r) r = par[r];
        par[v] = r;
        uint32_t g = l2g ? (uint32_t)l2g[v] : (uint32_t)v;
        if (g < best[r]) best[r] = g;
    }
    for (int64_t v = 0; v < V; v++) label[v] = best[par[v]];
    free(par); free(best);
    return 0;
}

/* ------------------------------------------------------------------------
 * OpenMP timing mode.  Same supersteps as the reference functions above,
 * spread over `nthreads` host threads (0 = the OpenMP default).
 * ------------------------------------------------------------------------ */

static void set_threads(int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

/* Atomic minimum on a 32-bit word (compare-and-swap loop). */
static inline void atomic_min_u32(uint32_t *p, uint32_t x)
{
    uint32_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (x < cur && !__atomic_compare_exchange_n(p, &cur, x, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
    }
}

/*
 * The min superstep of or_min_superstep with the edge loop split over
 * threads.  Each message is folded with an atomic minimum, so the merged
 * value is the same whatever the order (min is exact and commutative).
 */
static int64_t min_superstep_omp(int64_t V, int64_t E, const int32_t *src, const int32_t *dst,
                                 const uint32_t *w, int both_dirs, const uint32_t *state,
                                 const uint8_t *front, uint32_t *state_next, uint8_t *front_next,
                                 int64_t *edges_out)
{
    int64_t msgs = 0, changed = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < V; v++) state_next[v] = state[v];
    #pragma omp parallel for schedule(static, 65536) reduction(+:msgs)
    for (int64_t e = 0; e < E; e++) {
        int32_t u = src[e], v = dst[e];
        if (front[u]) {
            atomic_min_u32(&state_next[v], w ? sat_add_u32(state[u], w[e]) : state[u]);
            msgs++;
        }
        if (both_dirs && front[v]) {
            atomic_min_u32(&state_next[u], state[v]);
            msgs++;
        }
    }
    #pragma omp parallel for schedule(static) reduction(+:changed)
    for (int64_t v = 0; v < V; v++) {
        front_next[v] = state_next[v] < state[v];
        changed += front_next[v];
    }
    if (edges_out) *edges_out = msgs;
    return changed;
}

/* or_sssp / or_cc on all threads: same arguments and return convention.
 * Takes ownership of the frontier buffer f (frees it). */
static int64_t min_run_omp(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, const uint32_t *w,
                           int both_dirs, int64_t max_steps, uint32_t *state, uint8_t *f,
                           int64_t *front_size, int64_t *edges, int64_t *changed)
{
    uint32_t *ns = (uint32_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(uint32_t));
    uint8_t *nf = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    if (!ns || !nf) { free(ns); free(nf); return -2; }
    int64_t fs = 0;
    for (int64_t v = 0; v < V; v++) fs += f[v];
    int64_t k = 0, K = -1;
    while (k < max_steps) {
        int64_t ef = 0;
        int64_t c = min_superstep_omp(V, E, src, dst, w, both_dirs, state, f, ns, nf, &ef);
        if (front_size) front_size[k] = fs;
        if (edges) edges[k] = ef;
        if (changed) changed[k] = c;
        memcpy(state, ns, (size_t)V * sizeof(uint32_t));
        uint8_t *t = f; f = nf; nf = t;
        fs = c;
        k++;
        if (c == 0) { K = k; break; }
    }
    free(ns);
    free(f);
    free(nf);
    return K;
}

int64_t or_sssp_omp(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, const uint32_t *w,
                    int32_t s, int64_t max_steps, uint32_t *dist,
                    int64_t *front_size, int64_t *edges, int64_t *changed, int nthreads)
{
    set_threads(nthreads);
    uint8_t *f = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    if (!f) return -2;
    for (int64_t v = 0; v < V; v++) dist[v] = OR_INF;
    if (s >= 0 && s < V) { dist[s] = 0; f[s] = 1; }
    return min_run_omp(V, E, src, dst, w, 0, max_steps, dist, f, front_size, edges, changed);
}

int64_t or_cc_omp(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, const int32_t *l2g,
                  int64_t max_steps, uint32_t *label,
                  int64_t *front_size, int64_t *edges, int64_t *changed, int nthreads)
{
    set_threads(nthreads);
    uint8_t *f = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    if (!f) return -2;
    for (int64_t v = 0; v < V; v++) label[v] = l2g ? (uint32_t)l2g[v] : (uint32_t)v;
    for (int64_t e = 0; e < E; e++) { f[src[e]] = 1; f[dst[e]] = 1; }
    return min_run_omp(V, E, src, dst, NULL, 1, max_steps, label, f, front_size, edges, changed);
}

/*
 * Destination-major copy of the edge list for the PageRank timing mode: a
 * stable counting sort by destination, so each destination lists its
 * messages in edge-list order, the order in which or_pr_superstep adds them.
 * in_rp[V+1] and in_src[E] are caller buffers.
 */
void or_in_edges(int64_t V, int64_t E, const int32_t *src, const int32_t *dst,
                 int64_t *in_rp, int32_t *in_src)
{
    memset(in_rp, 0, (size_t)(V + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < E; e++) in_rp[dst[e] + 1]++;
    for (int64_t v = 0; v < V; v++) in_rp[v + 1] += in_rp[v];
    int64_t *pos = (int64_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(int64_t));
    for (int64_t v = 0; v < V; v++) pos[v] = in_rp[v];
    for (int64_t e = 0; e < E; e++) in_src[pos[dst[e]]++] = src[e];
    free(pos);
}

/*
 * or_pr_superstep (ppr_seed < 0) or or_ppr_superstep (ppr_seed = s) with
 * the merge pulled per destination over the in-edges from or_in_edges and
 * split over threads.  Each destination adds its messages in edge-list
 * order starting from 0.0, exactly as the reference's edge loop does, and
 * the dangling mass is summed over vertices in ascending order on one
 * thread, so the result is bitwise the reference's.
 */
void or_pr_superstep_omp(int64_t V, const int64_t *in_rp, const int32_t *in_src, const int32_t *deg,
                         double d, int32_t ppr_seed, const double *x, double *x_next, int nthreads)
{
    set_threads(nthreads);
    double D = 0.0;
    for (int64_t u = 0; u < V; u++)
        if (deg[u] == 0) D += x[u];
    double base = (1.0 - d) / (double)V;
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < V; v++) {
        double acc = 0.0;
        for (int64_t i = in_rp[v]; i < in_rp[v + 1]; i++) {
            int32_t u = in_src[i];
            acc += x[u] / (double)deg[u];
        }
        x_next[v] = ppr_seed < 0 ? base + d * (acc + D / (double)V) : d * acc;
    }
    if (ppr_seed >= 0) x_next[ppr_seed] += (1.0 - d) + d * D;
}

/* B independent single-source SSSP runs (reference or_sssp, one per
 * thread): dist is [B x V] (lane b at b*V), K[b] its superstep count. */
void or_sssp_many(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, const uint32_t *w,
                  const int32_t *sources, int32_t B, uint32_t *dist, int64_t *K, int nthreads)
{
    set_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t b = 0; b < B; b++)
        K[b] = or_sssp(V, E, src, dst, w, sources[b], V + 2, dist + (size_t)b * (size_t)V, NULL, NULL, NULL);
}

/* B Dijkstra runs (or_dijkstra, one per thread); same layout. */
void or_dijkstra_many(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, const uint32_t *w,
                      const int32_t *sources, int32_t B, uint32_t *dist, int nthreads)
{
    set_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t b = 0; b < B; b++)
        or_dijkstra(V, E, src, dst, w, sources[b], dist + (size_t)b * (size_t)V, NULL);
}

/* B independent personalised-PageRank runs of T reference supersteps
 * (or_ppr_superstep, one lane per thread): x is [B x V] (lane b at b*V). */
int or_ppr_many(int64_t V, int64_t E, const int32_t *src, const int32_t *dst, const int32_t *deg,
                double d, const int32_t *seeds, int32_t B, int32_t T, double *x, int nthreads)
{
    set_threads(nthreads);
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:bad)
    for (int32_t b = 0; b < B; b++) {
        double *cur = x + (size_t)b * (size_t)V;
        double *tmp = (double *)malloc((size_t)(V > 0 ? V : 1) * sizeof(double));
        if (!tmp) { bad = 1; continue; }
        for (int64_t v = 0; v < V; v++) cur[v] = 0.0;
        cur[seeds[b]] = 1.0;
        for (int32_t t = 0; t < T; t++) {
            or_ppr_superstep(V, E, src, dst, deg, d, seeds[b], cur, tmp);
            memcpy(cur, tmp, (size_t)V * sizeof(double));
        }
        free(tmp);
    }
    return bad ? -2 : 0;
}

/* Threads the OpenMP mode uses for nthreads = 0. */
int or_max_threads(void) { return omp_get_max_threads(); }
