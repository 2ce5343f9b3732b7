/*
 * Seeded synthetic input generator: R-MAT directed graphs, per-edge weights,
 * and a hash vertex-cut into parts.
 *
 * This file produces INPUTS only.  It holds none of the graph algorithms'
 * arithmetic and is shared by the CPU oracle and the device library purely as
 * the source of test and benchmark graphs.
 *
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): each edge picks, at every
 * one of `scale` bit levels (most significant first), one of four quadrants
 * with probabilities (a, b, c, d); quadrant a sets neither bit, b sets the
 * destination bit, c sets the source bit, d sets both.  No noise and no vertex
 * permutation are applied, so vertex 0 is the densest corner.
 *
 * Randomness is counter based (SplitMix64, Steele, Lea, Flood, OOPSLA 2014):
 * the draw for edge i and level pair j is a pure function of (seed, i, j), so
 * generation is order free and parallel, and any subset of edges can be
 * regenerated independently.
 *
 * Self-loops are dropped and duplicate (u, v) pairs are merged.  The weight of
 * an edge depends only on (seed, u, v): w = 1 + H(u, v) mod 255, uniform in
 * [1, 255].  The hash vertex-cut assigns edge (u, v) to part H'(u, v) mod P;
 * a vertex's replicas are the parts holding at least one of its edges and its
 * master is one replica chosen by a hash of v.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static inline uint64_t sm64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

/* Salts separating the independent random streams drawn from one seed. */
#define SALT_EDGE   0x5EED0001ULL
#define SALT_WEIGHT 0x5EED0002ULL
#define SALT_PART   0x5EED0003ULL
#define SALT_MASTER 0x5EED0004ULL

static inline uint64_t edge_key(uint64_t seedmix, int scale, int64_t i,
                                uint32_t ta, uint32_t tab, uint32_t tabc)
{
    uint64_t src = 0, dst = 0;
    for (int lv = 0; lv < scale; lv += 2) {
        uint64_t r = sm64(seedmix ^ (((uint64_t)i << 5) | (uint64_t)(lv >> 1)));
        for (int h = 0; h < 2 && lv + h < scale; h++) {
            uint32_t x = h ? (uint32_t)(r >> 32) : (uint32_t)r;
            uint64_t sb, db;
            if (x < ta)        { sb = 0; db = 0; }
            else if (x < tab)  { sb = 0; db = 1; }
            else if (x < tabc) { sb = 1; db = 0; }
            else               { sb = 1; db = 1; }
            src = (src << 1) | sb;
            dst = (dst << 1) | db;
        }
    }
    return (src << scale) | dst;
}

static void thresholds(double a, double b, double c, uint32_t *ta, uint32_t *tab, uint32_t *tabc)
{
    const double two32 = 4294967296.0;
    double x;
    x = a * two32;           *ta   = x >= two32 ? 0xFFFFFFFFu : (uint32_t)x;
    x = (a + b) * two32;     *tab  = x >= two32 ? 0xFFFFFFFFu : (uint32_t)x;
    x = (a + b + c) * two32; *tabc = x >= two32 ? 0xFFFFFFFFu : (uint32_t)x;
}

/* Parallel LSD radix sort of 64-bit keys on their low `key_bits` bits. */
static void radix_sort_u64(uint64_t *a, uint64_t *tmp, int64_t n, int key_bits)
{
    enum { RB = 11, NB = 1 << RB };
    int maxt = omp_get_max_threads();
    int64_t *hist = (int64_t *)malloc((size_t)maxt * NB * sizeof(int64_t));
    int passes = (key_bits + RB - 1) / RB;
    uint64_t *src = a, *dst = tmp;
    for (int p = 0; p < passes; p++) {
        int shift = p * RB;
        #pragma omp parallel
        {
            int t = omp_get_thread_num(), nt = omp_get_num_threads();
            int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
            int64_t *h = hist + (int64_t)t * NB;
            memset(h, 0, NB * sizeof(int64_t));
            for (int64_t i = lo; i < hi; i++) h[(src[i] >> shift) & (NB - 1)]++;
            #pragma omp barrier
            #pragma omp single
            {
                int64_t sum = 0;
                for (int d = 0; d < NB; d++)
                    for (int tt = 0; tt < nt; tt++) {
                        int64_t c = hist[(int64_t)tt * NB + d];
                        hist[(int64_t)tt * NB + d] = sum;
                        sum += c;
                    }
            }
            for (int64_t i = lo; i < hi; i++) {
                uint64_t k = src[i];
                dst[h[(k >> shift) & (NB - 1)]++] = k;
            }
        }
        uint64_t *s = src; src = dst; dst = s;
    }
    if (src != a) memcpy(a, src, (size_t)n * sizeof(uint64_t));
    free(hist);
}

/* Drops self-loops and duplicates from sorted keys, in place; returns new n. */
static int64_t unique_no_loops(uint64_t *k, int64_t n, int scale)
{
    uint64_t mask = (scale >= 32) ? ~0ULL : ((1ULL << scale) - 1);
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        uint64_t x = k[i];
        if ((x >> scale) == (x & mask)) continue;
        if (m > 0 && k[m - 1] == x) continue;
        k[m++] = x;
    }
    return m;
}

static inline uint32_t edge_weight(uint64_t wmix, uint64_t u, uint64_t v)
{
    return 1u + (uint32_t)(sm64(((u << 32) | v) ^ wmix) % 255u);
}

/* Sorted unique keys -> CSR (row_ptr has V+1 entries) plus weights. */
static void keys_to_csr(const uint64_t *k, int64_t E, int scale, int64_t V, uint64_t wmix,
                        int32_t *row_ptr, int32_t *col, uint32_t *w)
{
    uint64_t mask = (1ULL << scale) - 1;
    memset(row_ptr, 0, (size_t)(V + 1) * sizeof(int32_t));
    for (int64_t i = 0; i < E; i++) row_ptr[(k[i] >> scale) + 1]++;
    for (int64_t v = 0; v < V; v++) row_ptr[v + 1] += row_ptr[v];
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < E; i++) {
        uint64_t u = k[i] >> scale, d = k[i] & mask;
        col[i] = (int32_t)d;
        if (w) w[i] = edge_weight(wmix, u, d);
    }
}

/*
 * Whole R-MAT graph as CSR.  E_raw edges are drawn, then self-loops and
 * duplicates are removed.  row_ptr: V+1 = 2^scale + 1 entries; col and w:
 * capacity E_raw.  Returns the number of kept edges, or -1 on bad arguments
 * or allocation failure.
 */
int64_t gen_rmat_csr(int scale, int64_t E_raw, double a, double b, double c, uint64_t seed,
                     int32_t *row_ptr, int32_t *col, uint32_t *w)
{
    if (scale < 1 || scale > 30 || E_raw < 0) return -1;
    int64_t V = (int64_t)1 << scale;
    uint32_t ta, tab, tabc;
    thresholds(a, b, c, &ta, &tab, &tabc);
    uint64_t emix = sm64(seed ^ SALT_EDGE), wmix = sm64(seed ^ SALT_WEIGHT);
    uint64_t *k = (uint64_t *)malloc((size_t)(E_raw > 0 ? E_raw : 1) * sizeof(uint64_t));
    uint64_t *t = (uint64_t *)malloc((size_t)(E_raw > 0 ? E_raw : 1) * sizeof(uint64_t));
    if (!k || !t) { free(k); free(t); return -1; }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < E_raw; i++) k[i] = edge_key(emix, scale, i, ta, tab, tabc);
    radix_sort_u64(k, t, E_raw, 2 * scale);
    free(t);
    int64_t E = unique_no_loops(k, E_raw, scale);
    keys_to_csr(k, E, scale, V, wmix, row_ptr, col, w);
    free(k);
    return E;
}

/*
 * One part of a hash vertex-cut of an R-MAT graph.  Every raw edge is drawn
 * once; self-loops are dropped; edge (u, v) belongs to part H(u, v) mod
 * nparts.  Duplicates hash to the same part, so they are merged inside it.
 *
 * The part's local vertex ids are the sorted global ids of the endpoints of
 * its kept edges (l2g ascending).  flags per local vertex:
 *   bit0 master     : this part is v's master (one replica chosen by hash)
 *   bit1 remote_out : v has an out-edge in another part
 *   bit2 remote_any : v has any edge (in or out) in another part
 *
 * The output arrays are allocated here with malloc (row_ptr V+1, col, w: E,
 * l2g, flags: V) and released with gen_free.  Returns 0, or -1 on bad
 * arguments or allocation failure.
 */
int gen_rmat_part(int scale, int64_t E_raw, double a, double b, double c, uint64_t seed,
                  int nparts, int part, int64_t *V_out, int64_t *E_out,
                  int32_t **row_ptr_out, int32_t **col_out, uint32_t **w_out,
                  int32_t **l2g_out, uint8_t **flags_out)
{
    if (scale < 1 || scale > 30 || E_raw < 0 || nparts < 1 || nparts > 8 || part < 0 || part >= nparts)
        return -1;
    int64_t V = (int64_t)1 << scale;
    uint32_t ta, tab, tabc;
    thresholds(a, b, c, &ta, &tab, &tabc);
    uint64_t emix = sm64(seed ^ SALT_EDGE), wmix = sm64(seed ^ SALT_WEIGHT);
    uint64_t pmix = sm64(seed ^ SALT_PART), mmix = sm64(seed ^ SALT_MASTER);
    uint64_t vmask = (1ULL << scale) - 1;

    uint8_t *rep_out = (uint8_t *)calloc((size_t)V, 1);
    uint8_t *rep_any = (uint8_t *)calloc((size_t)V, 1);
    int maxt = omp_get_max_threads();
    uint64_t **buf = (uint64_t **)calloc((size_t)maxt, sizeof(uint64_t *));
    int64_t *len = (int64_t *)calloc((size_t)maxt + 1, sizeof(int64_t));
    int failed = 0;
    if (!rep_out || !rep_any || !buf || !len) failed = 1;
    if (!failed) {
        #pragma omp parallel
        {
            int th = omp_get_thread_num(), nt = omp_get_num_threads();
            int64_t lo = E_raw * th / nt, hi = E_raw * (th + 1) / nt;
            int64_t cap = (hi - lo) / nparts + 1024, n = 0;
            uint64_t *mine = (uint64_t *)malloc((size_t)cap * sizeof(uint64_t));
            for (int64_t i = lo; i < hi && mine; i++) {
                uint64_t key = edge_key(emix, scale, i, ta, tab, tabc);
                uint64_t u = key >> scale, v = key & vmask;
                if (u == v) continue;
                int p = (int)(sm64(((u << 32) | v) ^ pmix) % (uint64_t)nparts);
                uint8_t bit = (uint8_t)(1u << p);
                if (!(__atomic_load_n(&rep_out[u], __ATOMIC_RELAXED) & bit)) __atomic_fetch_or(&rep_out[u], bit, __ATOMIC_RELAXED);
                if (!(__atomic_load_n(&rep_any[u], __ATOMIC_RELAXED) & bit)) __atomic_fetch_or(&rep_any[u], bit, __ATOMIC_RELAXED);
                if (!(__atomic_load_n(&rep_any[v], __ATOMIC_RELAXED) & bit)) __atomic_fetch_or(&rep_any[v], bit, __ATOMIC_RELAXED);
                if (p != part) continue;
                if (n == cap) {
                    cap = cap * 2;
                    uint64_t *g = (uint64_t *)realloc(mine, (size_t)cap * sizeof(uint64_t));
                    if (!g) { free(mine); mine = NULL; break; }
                    mine = g;
                }
                mine[n++] = key;
            }
            buf[th] = mine;
            len[th + 1] = mine ? n : -1;
        }
        for (int t = 0; t < maxt; t++) if (len[t + 1] < 0) failed = 1;
    }
    int64_t kept = 0;
    for (int t = 0; t < maxt && !failed; t++) kept += len[t + 1];
    uint64_t *k = failed ? NULL : (uint64_t *)malloc((size_t)(kept > 0 ? kept : 1) * sizeof(uint64_t));
    uint64_t *tmp = failed ? NULL : (uint64_t *)malloc((size_t)(kept > 0 ? kept : 1) * sizeof(uint64_t));
    if (!k || !tmp) failed = 1;
    if (!failed) {
        int64_t pos = 0;
        for (int t = 0; t < maxt; t++) {
            if (buf[t] && len[t + 1] > 0) memcpy(k + pos, buf[t], (size_t)len[t + 1] * sizeof(uint64_t));
            if (len[t + 1] > 0) pos += len[t + 1];
        }
    }
    if (buf) for (int t = 0; t < maxt; t++) free(buf[t]);
    free(buf); free(len);
    if (failed) { free(rep_out); free(rep_any); free(k); free(tmp); return -1; }
    /* Sorting makes the result independent of the collection order. */
    radix_sort_u64(k, tmp, kept, 2 * scale);
    free(tmp);
    int64_t E = unique_no_loops(k, kept, scale);

    uint8_t *present = (uint8_t *)calloc((size_t)V, 1);
    int32_t *g2l = (int32_t *)malloc((size_t)V * sizeof(int32_t));
    if (!present || !g2l) { free(rep_out); free(rep_any); free(k); free(present); free(g2l); return -1; }
    for (int64_t i = 0; i < E; i++) { present[k[i] >> scale] = 1; present[k[i] & vmask] = 1; }
    int64_t Vp = 0;
    for (int64_t v = 0; v < V; v++) g2l[v] = present[v] ? (int32_t)Vp++ : -1;
    free(present);
    int32_t *row_ptr = (int32_t *)calloc((size_t)Vp + 1, sizeof(int32_t));
    int32_t *col = (int32_t *)malloc((size_t)(E > 0 ? E : 1) * sizeof(int32_t));
    uint32_t *w = (uint32_t *)malloc((size_t)(E > 0 ? E : 1) * sizeof(uint32_t));
    int32_t *l2g = (int32_t *)malloc((size_t)(Vp > 0 ? Vp : 1) * sizeof(int32_t));
    uint8_t *flags = (uint8_t *)malloc((size_t)(Vp > 0 ? Vp : 1));
    if (!row_ptr || !col || !w || !l2g || !flags) {
        free(rep_out); free(rep_any); free(k); free(g2l);
        free(row_ptr); free(col); free(w); free(l2g); free(flags);
        return -1;
    }
    uint8_t self = (uint8_t)(1u << part);
    for (int64_t i = 0; i < E; i++) row_ptr[g2l[k[i] >> scale] + 1]++;
    for (int64_t x = 0; x < Vp; x++) row_ptr[x + 1] += row_ptr[x];
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < E; i++) {
        uint64_t u = k[i] >> scale, v = k[i] & vmask;
        col[i] = g2l[v];
        w[i] = edge_weight(wmix, u, v);
    }
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < V; v++) {
        int32_t lv = g2l[v];
        if (lv < 0) continue;
        l2g[lv] = (int32_t)v;
        uint8_t any = rep_any[v];
        int nrep = __builtin_popcount(any);
        int pick = (int)(sm64((uint64_t)v ^ mmix) % (uint64_t)nrep);
        int master = -1;
        for (int p = 0, seen = 0; p < nparts; p++)
            if (any & (1u << p)) { if (seen == pick) { master = p; break; } seen++; }
        uint8_t f = 0;
        if (master == part) f |= 1;
        if (rep_out[v] & (uint8_t)~self) f |= 2;
        if (any & (uint8_t)~self) f |= 4;
        flags[lv] = f;
    }
    free(rep_out); free(rep_any); free(k); free(g2l);
    *V_out = Vp; *E_out = E;
    *row_ptr_out = row_ptr; *col_out = col; *w_out = w; *l2g_out = l2g; *flags_out = flags;
    return 0;
}

void gen_free(void *p) { free(p); }

/* Level-0 quadrant counts of the first n raw edges (for distribution checks). */
void gen_rmat_quadrants(int scale, int64_t n, double a, double b, double c, uint64_t seed, int64_t out[4])
{
    uint32_t ta, tab, tabc;
    thresholds(a, b, c, &ta, &tab, &tabc);
    uint64_t emix = sm64(seed ^ SALT_EDGE);
    int64_t q0 = 0, q1 = 0, q2 = 0, q3 = 0;
    #pragma omp parallel for schedule(static) reduction(+ : q0, q1, q2, q3)
    for (int64_t i = 0; i < n; i++) {
        uint64_t key = edge_key(emix, scale, i, ta, tab, tabc);
        int sb = (int)((key >> (2 * scale - 1)) & 1), db = (int)((key >> (scale - 1)) & 1);
        int q = sb * 2 + db;
        if (q == 0) q0++; else if (q == 1) q1++; else if (q == 2) q2++; else q3++;
    }
    out[0] = q0; out[1] = q1; out[2] = q2; out[3] = q3;
}
