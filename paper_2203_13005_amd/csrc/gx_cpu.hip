// The CPU daemon: the same superstep on host threads, for a heterogeneous
// worker set in which CPUs and GPUs hold parts of one graph (Section
// "Beyond-Iteration Optimization: Workload Balancing": accelerators of
// different computation capacity 1/c_j; the evaluation's "CPU+GraphX" and
// "CPU+PowerGraph" daemons run the template on CPU threads).  Host code
// only: no kernel, no device memory.
//
// A superstep is the template's Jacobi step on the part's out-CSR (SSSP) or
// symmetric adjacency (CC): every active vertex sends the value it held at
// the superstep's start along its edges (sat_add(value, w) for SSSP), a
// destination keeps the minimum (compare-and-swap), and a vertex whose value
// fell joins the next frontier and the set of changes not yet synchronised.
// Minima do not depend on the threads' interleaving, so the result is
// deterministic.  The sync set and its receiving side follow the device
// engine's gx_sync_delta (GX_DELTA_ALL) / gx_apply_delta, on host buffers.
//
// gx_balance_split implements Lemma "minmaxcidi": d_j = D (1/c_j) / sum_i 1/c_i.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "gx_internal.h"

using namespace gx;

namespace {

template <class F>
void run_threads(int nthreads, int64_t n, F &&f) {
    nthreads = (int)std::max<int64_t>(1, std::min<int64_t>(nthreads, (n + 4095) / 4096));
    if (nthreads <= 1) {
        f(0, (int64_t)0, n);
        return;
    }
    std::vector<std::thread> ts;
    for (int t = 0; t < nthreads; t++)
        ts.emplace_back([&, t] { f(t, n * t / nthreads, n * (t + 1) / nthreads); });
    for (auto &t : ts) t.join();
}

inline uint32_t sat_add_host(uint32_t a, uint32_t b) {
    const uint64_t s = (uint64_t)a + b;
    return s > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)s;
}

// atomic minimum on a plain word; true if this call lowered it
inline bool fetch_min(uint32_t *p, uint32_t v) {
    uint32_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (v < cur)
        if (__atomic_compare_exchange_n(p, &cur, v, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) return true;
    return false;
}

}  // namespace

struct gx_cpu {
    int32_t algo = GX_SSSP;
    int64_t V = 0;
    int threads = 1;
    std::vector<int32_t> rp, col;  // SSSP: out-CSR; CC: symmetric adjacency
    std::vector<uint32_t> w;
    std::vector<int32_t> l2g;
    std::vector<uint8_t> remote;  // another part needs the vertex (empty: every vertex)
    std::vector<uint32_t> val;
    std::vector<uint8_t> dirty, mark;
    std::vector<int32_t> front;  // active vertices of the next superstep (ascending)
    int64_t k = 0;
};

extern "C" gx_status gx_cpu_create(const gx_graph_desc *d, int32_t algo, int32_t source, int32_t threads,
                                   gx_cpu **out) {
    clear_error();
    GX_REQUIRE(out, GX_EINVAL, "out is NULL");
    *out = nullptr;
    GX_REQUIRE(d, GX_EINVAL, "desc is NULL");
    GX_REQUIRE(algo == GX_SSSP || algo == GX_CC, GX_EINVAL, "the CPU daemon runs SSSP and CC");
    GX_REQUIRE(d->V >= 0 && d->V < (int64_t(1) << 31) && d->E >= 0 && d->E < (int64_t(1) << 30), GX_EINVAL,
               "V / E out of range");
    GX_REQUIRE(d->V == 0 || (d->row_ptr && (d->col || d->E == 0)), GX_EINVAL, "CSR arrays are NULL");
    GX_REQUIRE(algo != GX_SSSP || d->w || d->E == 0, GX_EINVAL, "SSSP needs weights");
    GX_REQUIRE(algo != GX_SSSP || (source >= -1 && source < d->V), GX_EINVAL, "source out of [-1, V)");
    GX_REQUIRE(threads >= 0, GX_EINVAL, "threads < 0");
    if (d->V > 0) {
        GX_REQUIRE(d->row_ptr[0] == 0 && d->row_ptr[d->V] == d->E, GX_EINVAL, "row_ptr does not span E");
        for (int64_t v = 0; v < d->V; v++) GX_REQUIRE(d->row_ptr[v + 1] >= d->row_ptr[v], GX_EINVAL, "row_ptr decreases");
        for (int64_t e = 0; e < d->E; e++) GX_REQUIRE((uint32_t)d->col[e] < (uint32_t)d->V, GX_EINVAL, "col out of range");
    }
    gx_cpu *c = new (std::nothrow) gx_cpu();
    GX_REQUIRE(c, GX_ENOMEM, "host allocation failed");
    try {
        c->algo = algo;
        c->V = d->V;
        c->threads = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
        const int64_t V = d->V;
        if (algo == GX_SSSP) {
            c->rp.assign(d->row_ptr, d->row_ptr + V + 1);
            c->col.assign(d->col, d->col + d->E);
            c->w.assign(d->w, d->w + d->E);
        } else {  // symmetric, deduplicated, no self-loops
            std::vector<uint64_t> pairs;
            pairs.reserve(2 * (size_t)d->E);
            for (int64_t u = 0; u < V; u++)
                for (int32_t e = d->row_ptr[u]; e < d->row_ptr[u + 1]; e++) {
                    const uint64_t v = (uint32_t)d->col[e];
                    if ((uint64_t)u == v) continue;
                    pairs.push_back((uint64_t)u << 32 | v);
                    pairs.push_back(v << 32 | (uint64_t)u);
                }
            std::sort(pairs.begin(), pairs.end());
            pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
            c->rp.assign(V + 1, 0);
            c->col.resize(pairs.size());
            for (size_t i = 0; i < pairs.size(); i++) {
                c->rp[(pairs[i] >> 32) + 1]++;
                c->col[i] = (int32_t)(uint32_t)pairs[i];
            }
            for (int64_t v = 0; v < V; v++) c->rp[v + 1] += c->rp[v];
        }
        if (d->l2g) c->l2g.assign(d->l2g, d->l2g + V);
        if (d->flags) {  // SSSP: an out-edge elsewhere; CC: any edge elsewhere (as the device engine)
            const uint8_t bit = algo == GX_SSSP ? GX_FLAG_REMOTE_OUT : GX_FLAG_REMOTE_ANY;
            c->remote.resize((size_t)V);
            for (int64_t v = 0; v < V; v++) c->remote[(size_t)v] = (d->flags[v] & bit) != 0;
        }
        c->val.assign((size_t)V, 0xFFFFFFFFu);
        c->dirty.assign((size_t)V, 0);
        c->mark.assign((size_t)V, 0);
        if (algo == GX_SSSP) {
            if (source >= 0) {
                c->val[source] = 0;
                c->front.push_back(source);
            }
        } else {
            for (int64_t v = 0; v < V; v++) {
                c->val[v] = d->l2g ? (uint32_t)d->l2g[v] : (uint32_t)v;
                if (c->rp[v + 1] > c->rp[v]) c->front.push_back((int32_t)v);
            }
        }
    } catch (const std::bad_alloc &) {
        delete c;
        set_error("host allocation failed");
        return GX_ENOMEM;
    }
    *out = c;
    return GX_OK;
}

extern "C" gx_status gx_cpu_superstep(gx_cpu *c, gx_step_stats *stats) {
    clear_error();
    GX_REQUIRE(c, GX_EINVAL, "handle is NULL");
    const int64_t n = (int64_t)c->front.size();
    // the values the active vertices send: those of the superstep's start
    std::vector<uint32_t> sendv((size_t)n);
    for (int64_t i = 0; i < n; i++) sendv[(size_t)i] = c->val[(size_t)c->front[(size_t)i]];
    std::vector<std::vector<int32_t>> lowered((size_t)c->threads);
    std::vector<int64_t> msgs((size_t)c->threads, 0);
    const bool weighted = c->algo == GX_SSSP;
    uint32_t *val = c->val.data();
    uint8_t *mark = c->mark.data();
    run_threads(c->threads, n, [&](int t, int64_t lo, int64_t hi) {
        auto &mine = lowered[(size_t)t];
        int64_t m = 0;
        for (int64_t i = lo; i < hi; i++) {
            const int32_t u = c->front[(size_t)i];
            const uint32_t x = sendv[(size_t)i];
            for (int32_t e = c->rp[u]; e < c->rp[u + 1]; e++) {
                const uint32_t cand = weighted ? sat_add_host(x, c->w[e]) : x;
                const int32_t v = c->col[e];
                m++;
                if (fetch_min(&val[v], cand) && __atomic_exchange_n(&mark[v], (uint8_t)1, __ATOMIC_RELAXED) == 0)
                    mine.push_back(v);  // the first thread to lower v lists it
            }
        }
        msgs[(size_t)t] = m;
    });
    std::vector<int32_t> next;
    for (auto &l : lowered) next.insert(next.end(), l.begin(), l.end());
    std::sort(next.begin(), next.end());
    for (int32_t v : next) {
        mark[v] = 0;
        c->dirty[v] = 1;
    }
    if (stats) {
        *stats = gx_step_stats{};
        stats->frontier = n;
        for (int64_t m : msgs) stats->edges += m;
        stats->changed = (int64_t)next.size();
    }
    c->front.swap(next);
    c->k++;
    return GX_OK;
}

extern "C" gx_status gx_cpu_sync_delta(gx_cpu *c, int32_t *gid, uint32_t *val, uint32_t cap, uint32_t *count) {
    clear_error();
    GX_REQUIRE(c && count, GX_EINVAL, "NULL argument");
    GX_REQUIRE(cap == 0 || (gid && val), GX_EINVAL, "output buffers are NULL");
    const bool all = c->remote.empty();
    uint32_t n = 0;
    for (int64_t v = 0; v < c->V; v++) n += c->dirty[(size_t)v] && (all || c->remote[(size_t)v]);
    *count = n;
    if (n > cap) {
        set_error("sync set has %u entries, capacity %u", n, cap);
        return GX_ENOMEM;
    }
    uint32_t i = 0;
    for (int64_t v = 0; v < c->V; v++)
        if (c->dirty[(size_t)v] && !(all || c->remote[(size_t)v])) {
            c->dirty[(size_t)v] = 0;  // nobody else needs it
        } else if (c->dirty[(size_t)v]) {
            gid[i] = c->l2g.empty() ? (int32_t)v : c->l2g[(size_t)v];
            val[i] = c->val[(size_t)v];
            c->dirty[(size_t)v] = 0;
            i++;
        }
    return GX_OK;
}

extern "C" gx_status gx_cpu_apply_delta(gx_cpu *c, const int32_t *gid, const uint32_t *val, uint32_t n,
                                        int64_t *active_next) {
    clear_error();
    GX_REQUIRE(c, GX_EINVAL, "handle is NULL");
    GX_REQUIRE(n == 0 || (gid && val), GX_EINVAL, "input buffers are NULL");
    std::vector<int32_t> add;
    for (uint32_t i = 0; i < n; i++) {
        int64_t x;
        if (c->l2g.empty()) {
            if (gid[i] < 0 || gid[i] >= c->V) continue;
            x = gid[i];
        } else {
            auto it = std::lower_bound(c->l2g.begin(), c->l2g.end(), gid[i]);
            if (it == c->l2g.end() || *it != gid[i]) continue;
            x = it - c->l2g.begin();
        }
        if (val[i] < c->val[(size_t)x]) {  // a lowered replica is active next (not dirty: the sender sent it)
            c->val[(size_t)x] = val[i];
            add.push_back((int32_t)x);
        }
    }
    if (!add.empty()) {
        add.insert(add.end(), c->front.begin(), c->front.end());
        std::sort(add.begin(), add.end());
        add.erase(std::unique(add.begin(), add.end()), add.end());
        c->front.swap(add);
    }
    if (active_next) *active_next = (int64_t)c->front.size();
    return GX_OK;
}

extern "C" gx_status gx_cpu_values(gx_cpu *c, const uint32_t **values) {
    clear_error();
    GX_REQUIRE(c && values, GX_EINVAL, "NULL argument");
    *values = c->val.data();
    return GX_OK;
}

extern "C" gx_status gx_cpu_free(gx_cpu *c) {
    clear_error();
    delete c;
    return GX_OK;
}

extern "C" gx_status gx_balance_split(const double *c, int32_t m, double D, double *d_out) {
    clear_error();
    GX_REQUIRE(c && d_out && m >= 1, GX_EINVAL, "NULL argument or m < 1");
    GX_REQUIRE(D >= 0, GX_EINVAL, "D < 0");
    double cap = 0.0;
    for (int32_t j = 0; j < m; j++) {
        GX_REQUIRE(c[j] > 0 && std::isfinite(c[j]), GX_EINVAL, "c[%d] must be positive and finite", j);
        cap += 1.0 / c[j];
    }
    for (int32_t j = 0; j < m; j++) d_out[j] = D * (1.0 / c[j]) / cap;
    return GX_OK;
}
