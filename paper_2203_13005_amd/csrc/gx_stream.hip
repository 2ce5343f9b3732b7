// Streamed supersteps (out-of-core): the edge triplets stay in pinned host
// memory and every superstep streams them through the device in blocks,
// following Section "Intra-Iteration Optimization: Pipeline Shuffling".
//
// Device block buffers play the n-, c- and u-blocks of the paper's pipeline
// (Algorithms "Pipeline Shuffle - Daemon Side" / "Agent Side"): block i is
// downloaded into buffer i mod R on a copy stream, computed there on the
// compute stream, and its results uploaded from the same buffer on a third
// stream, so the download of block i+1, the computation of block i and the
// upload of block i-1 overlap, and the roles rotate over the buffers without
// copying data between them.  R = 3 is the paper's rotation; a deeper ring
// (up to GX_STREAM_RING_MAX) lets a download start before the upload three
// blocks back has finished, which hides the latency between the streams.  Events order the stages: a
// download waits for the upload that last used its buffer, a computation
// for its download, an upload for its computation.
//
// What a block computes is the template's MSGGen and MSGMerge for its
// triplets (Section "Algorithm Template"): triplet (u, v, w) carries
// sat_add(snap[u], w) (SSSP; CC carries snap[u]) when u is active, INF
// otherwise; the message is merged into v by an integer minimum and written
// back into the triplet's result slot, which the upload returns to the host
// (the triplet is "the carrier of output").  Vertex state stays resident;
// snap holds the values of the superstep's start (Jacobi), and a vertex that
// a message lowers joins the next frontier.  Each superstep ends with the
// changed count.
//
// Block size: gx_pipeline_plan evaluates Lemma "bSizeSelection" (Section
// "Block Size Selection") for measured per-entity costs k1 (download), k2
// (compute), k3 (upload) and the per-call constant a, and picks between the
// floor and ceiling of the optimal block count by the time model itself.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "gx_device.h"
#include "gx_internal.h"

using namespace gx;

namespace {

constexpr int ST_BLOCK = 256;

struct StCounters {
    unsigned long long messages;  // triplets whose source was active
    unsigned long long changed;   // vertices in the next frontier
    unsigned long long pad[14];
};

__global__ __launch_bounds__(ST_BLOCK) void k_st_init(uint32_t *val, uint8_t *f0, uint8_t *f1, const int32_t *l2g,
                                                      const uint8_t *has_edge, int64_t V, int32_t cc, int32_t source) {
    const int64_t v = (int64_t)blockIdx.x * ST_BLOCK + threadIdx.x;
    if (v >= V) return;
    if (cc) {
        val[v] = l2g ? (uint32_t)l2g[v] : (uint32_t)v;
        f0[v] = has_edge[v];
    } else {
        val[v] = v == source ? 0u : INF;
        f0[v] = v == source;
    }
    f1[v] = 0;
}

__global__ __launch_bounds__(ST_BLOCK) void k_st_begin(const uint32_t *__restrict__ val, uint32_t *__restrict__ snap,
                                                       uint8_t *__restrict__ next, int64_t V, StCounters *c) {
    const int64_t v = (int64_t)blockIdx.x * ST_BLOCK + threadIdx.x;
    if (v == 0) *c = StCounters{};
    if (v >= V) return;
    snap[v] = val[v];
    next[v] = 0;
}

// A block holds its triplets packed: (u, v, w) (SSSP, tw = 3) or (u, v)
// (CC, tw = 2), so one copy downloads it.
__global__ __launch_bounds__(ST_BLOCK) void k_st_relax(const uint32_t *__restrict__ trip, int tw, uint32_t n,
                                                       const uint32_t *__restrict__ snap,
                                                       const uint8_t *__restrict__ front, uint32_t *__restrict__ val,
                                                       uint8_t *__restrict__ next, uint32_t *__restrict__ msg,
                                                       StCounters *c) {
    __shared__ unsigned long long s_c[ST_BLOCK / 64];
    const uint32_t i = blockIdx.x * ST_BLOCK + threadIdx.x;
    unsigned act = 0;
    if (i < n) {
        const uint32_t *t = trip + (size_t)i * tw;
        const uint32_t u = t[0], v = t[1];
        uint32_t m = INF;
        if (front[u]) {
            act = 1;
            m = tw == 3 ? sat_add(snap[u], t[2]) : snap[u];
            if (m < val[v]) {
                atomicMin(&val[v], m);
                next[v] = 1;
            }
        }
        msg[i] = m;
    }
    const unsigned long long t = block_sum<unsigned long long>((unsigned long long)act, s_c);
    if (threadIdx.x == 0 && t) atomicAdd(&c->messages, t);
}

__global__ __launch_bounds__(ST_BLOCK) void k_st_end(const uint8_t *__restrict__ next, int64_t V, StCounters *c) {
    __shared__ unsigned long long s_c[ST_BLOCK / 64];
    const int64_t v = (int64_t)blockIdx.x * ST_BLOCK + threadIdx.x;
    const unsigned x = v < V ? (unsigned)(next[v] != 0) : 0u;
    const unsigned long long t = block_sum<unsigned long long>((unsigned long long)x, s_c);
    if (threadIdx.x == 0 && t) atomicAdd(&c->changed, t);
}

template <class T>
unsigned blocks_of(T n) {
    return (unsigned)std::max<T>(1, (n + ST_BLOCK - 1) / ST_BLOCK);
}

// Eq. "PipelineTimeSimplied2": time of s blocks of b = d / s entities.
double pipeline_time(double k1, double k2, double k3, double a, double d, double s) {
    const double b = d / s;
    const double tn = k1 * b, tc = a + k2 * b, tu = k3 * b;
    return tn + std::max(tn, tc) + (s - 2) * std::max(tn, std::max(tc, tu)) + std::max(tc, tu) + tu;
}

}  // namespace

struct gx_stream {
    int32_t algo = GX_SSSP;
    int64_t V = 0, E = 0;  // E: triplets (CC: both directions of every distinct undirected edge)
    int32_t source = -1;
    uint64_t bmax = 0;
    int device = 0;
    bool dev_error = false;
    int ring = 3;   // device block buffers (the n-, c- and u-blocks rotate over them)
    int tw = 3;     // words per triplet
    // pinned host memory: the packed triplets and the uploaded results
    uint32_t *h_trip = nullptr, *h_msg = nullptr;
    std::vector<int32_t> l2g;
    std::vector<uint8_t> has_edge;
    // device
    uint32_t *val = nullptr, *snap = nullptr;
    uint8_t *front[2] = {nullptr, nullptr};
    int32_t *d_l2g = nullptr;
    uint8_t *d_has_edge = nullptr;
    StCounters *cnt = nullptr;
    uint32_t *b_trip[GX_STREAM_RING_MAX] = {}, *b_msg[GX_STREAM_RING_MAX] = {};
    int64_t k = 0;
    hipStream_t s_copy = nullptr, s_comp = nullptr, s_up = nullptr;
    hipEvent_t ev_n[GX_STREAM_RING_MAX] = {}, ev_c[GX_STREAM_RING_MAX] = {}, ev_u[GX_STREAM_RING_MAX] = {};
    std::vector<hipEvent_t> tev;  // timing events of the serial form
    StCounters *h_cnt = nullptr;  // pinned
    ~gx_stream() {
        for (hipStream_t s : {s_copy, s_comp, s_up})
            if (s) (void)hipStreamSynchronize(s);
        for (int i = 0; i < GX_STREAM_RING_MAX; i++)
            for (hipEvent_t e : {ev_n[i], ev_c[i], ev_u[i]})
                if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : tev) (void)hipEventDestroy(e);
        for (hipStream_t s : {s_copy, s_comp, s_up})
            if (s) (void)hipStreamDestroy(s);
        for (void *p : {(void *)h_trip, (void *)h_msg, (void *)h_cnt})
            if (p) (void)hipHostFree(p);
    }
};

static size_t stream_layout(int64_t V, uint64_t bmax, int ring, bool weighted, bool partitioned, Carver &c,
                            gx_stream *s) {
    s->val = c.take<uint32_t>(V);
    s->snap = c.take<uint32_t>(V);
    s->front[0] = c.take<uint8_t>(V);
    s->front[1] = c.take<uint8_t>(V);
    s->d_has_edge = c.take<uint8_t>(V);
    s->d_l2g = partitioned ? c.take<int32_t>(V) : nullptr;
    s->cnt = c.take<StCounters>(1);
    for (int i = 0; i < ring; i++) {
        s->b_trip[i] = c.take<uint32_t>(bmax * (weighted ? 3 : 2));
        s->b_msg[i] = c.take<uint32_t>(bmax);
    }
    return c.used;
}

// Triplets of the description: SSSP the out-edges (u, v, w) in CSR order; CC
// both directions of every distinct undirected edge, self-loops dropped, in
// (u, v) order.
static void host_triplets(const gx_graph_desc *d, int32_t algo, std::vector<uint32_t> &src,
                          std::vector<uint32_t> &dst, std::vector<uint32_t> &w) {
    const int64_t V = d->V;
    if (algo == GX_SSSP) {
        src.resize(d->E);
        dst.resize(d->E);
        w.resize(d->E);
        for (int64_t u = 0; u < V; u++)
            for (int32_t e = d->row_ptr[u]; e < d->row_ptr[u + 1]; e++) {
                src[e] = (uint32_t)u;
                dst[e] = (uint32_t)d->col[e];
                w[e] = d->w[e];
            }
        return;
    }
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
    src.resize(pairs.size());
    dst.resize(pairs.size());
    for (size_t i = 0; i < pairs.size(); i++) {
        src[i] = (uint32_t)(pairs[i] >> 32);
        dst[i] = (uint32_t)pairs[i];
    }
    w.clear();
}

static int64_t triplet_count(const gx_graph_desc *d, int32_t algo) {
    if (algo == GX_SSSP) return d->E;
    std::vector<uint32_t> s, t, w;
    host_triplets(d, algo, s, t, w);
    return (int64_t)s.size();
}

static gx_status check_desc(const gx_graph_desc *d, int32_t algo, uint64_t bmax, int ring) {
    GX_REQUIRE(ring >= 3 && ring <= GX_STREAM_RING_MAX, GX_EINVAL, "ring %d out of [3, %d]", ring,
               GX_STREAM_RING_MAX);
    GX_REQUIRE(d, GX_EINVAL, "desc is NULL");
    GX_REQUIRE(algo == GX_SSSP || algo == GX_CC, GX_EINVAL, "streamed supersteps serve SSSP and CC");
    GX_REQUIRE(d->V >= 0 && d->V < (int64_t(1) << 31) && d->E >= 0 && d->E < (int64_t(1) << 31), GX_EINVAL,
               "V / E out of range");
    GX_REQUIRE(d->V == 0 || (d->row_ptr && (d->col || d->E == 0)), GX_EINVAL, "CSR arrays are NULL");
    GX_REQUIRE(algo != GX_SSSP || d->w || d->E == 0, GX_EINVAL, "SSSP needs weights");
    GX_REQUIRE(bmax >= 1 && bmax < (uint64_t(1) << 31), GX_EINVAL, "block_edges_max out of [1, 2^31)");
    if (d->V > 0) {
        GX_REQUIRE(d->row_ptr[0] == 0 && d->row_ptr[d->V] == d->E, GX_EINVAL, "row_ptr does not span E");
        for (int64_t v = 0; v < d->V; v++)
            GX_REQUIRE(d->row_ptr[v + 1] >= d->row_ptr[v], GX_EINVAL, "row_ptr decreases");
        for (int64_t e = 0; e < d->E; e++)
            GX_REQUIRE((uint32_t)d->col[e] < (uint32_t)d->V, GX_EINVAL, "col out of range");
    }
    return GX_OK;
}

#define ST_CHECK(expr)                                                                                   \
    do {                                                                                                 \
        hipError_t _e = (expr);                                                                          \
        if (_e != hipSuccess) {                                                                          \
            set_error("%s failed: %s", #expr, hipGetErrorString(_e));                                   \
            s->dev_error = true;                                                                         \
            return GX_EDEVICE;                                                                           \
        }                                                                                                \
    } while (0)

extern "C" gx_status gx_stream_bytes(const gx_graph_desc *desc, int32_t algo, uint64_t block_edges_max, int32_t ring,
                                     size_t *bytes) {
    clear_error();
    GX_REQUIRE(bytes, GX_EINVAL, "bytes is NULL");
    gx_status st = check_desc(desc, algo, block_edges_max, ring);
    if (st != GX_OK) return st;
    Carver c(nullptr, 0);
    gx_stream tmp;
    *bytes = stream_layout(desc->V, block_edges_max, ring, algo == GX_SSSP, desc->l2g != nullptr, c, &tmp);
    return GX_OK;
}

extern "C" gx_status gx_stream_create(const gx_graph_desc *desc, int32_t algo, int32_t source, void *dev_arena,
                                      size_t arena_bytes, uint64_t block_edges_max, int32_t ring, gx_stream **out) {
    clear_error();
    GX_REQUIRE(out, GX_EINVAL, "out is NULL");
    *out = nullptr;
    gx_status st = check_desc(desc, algo, block_edges_max, ring);
    if (st != GX_OK) return st;
    GX_REQUIRE(algo != GX_SSSP || (source >= -1 && source < desc->V), GX_EINVAL, "source out of [-1, V)");
    GX_REQUIRE(dev_arena && reinterpret_cast<uintptr_t>(dev_arena) % ALIGN == 0, GX_EINVAL,
               "dev_arena NULL or not 256-byte aligned");
    {
        Carver m(nullptr, 0);
        gx_stream tmp;
        size_t need = stream_layout(desc->V, block_edges_max, ring, algo == GX_SSSP, desc->l2g != nullptr, m, &tmp);
        GX_REQUIRE(need <= arena_bytes, GX_ENOMEM, "arena too small: need %zu bytes, have %zu", need, arena_bytes);
    }
    std::vector<uint32_t> src, dst, w;
    try {
        host_triplets(desc, algo, src, dst, w);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed while building the triplets");
        return GX_ENOMEM;
    }
    gx_stream *s = new (std::nothrow) gx_stream();
    GX_REQUIRE(s, GX_ENOMEM, "host allocation failed");
    s->algo = algo;
    s->V = desc->V;
    s->E = (int64_t)src.size();
    s->source = source;
    s->bmax = block_edges_max;
    s->ring = ring;
    s->tw = algo == GX_SSSP ? 3 : 2;
    if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
    Carver c(dev_arena, arena_bytes);
    stream_layout(desc->V, block_edges_max, ring, algo == GX_SSSP, desc->l2g != nullptr, c, s);
    auto fail = [&](gx_status code) {
        delete s;
        return code;
    };
    const size_t nb = (size_t)std::max<int64_t>(1, s->E) * 4;
    if (hipHostMalloc((void **)&s->h_trip, nb * s->tw, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&s->h_msg, nb, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&s->h_cnt, sizeof(StCounters), hipHostMallocDefault) != hipSuccess) {
        set_error("pinned host allocation of %zu bytes failed", nb * (s->tw + 1));
        return fail(GX_ENOMEM);
    }
    for (int64_t i = 0; i < s->E; i++) {
        uint32_t *t = s->h_trip + (size_t)i * s->tw;
        t[0] = src[(size_t)i];
        t[1] = dst[(size_t)i];
        if (s->tw == 3) t[2] = w[(size_t)i];
    }
    s->has_edge.assign((size_t)std::max<int64_t>(1, s->V), 0);
    for (int64_t i = 0; i < s->E; i++) s->has_edge[src[(size_t)i]] = 1;
    if (desc->l2g) s->l2g.assign(desc->l2g, desc->l2g + desc->V);
    for (hipStream_t *p : {&s->s_copy, &s->s_comp, &s->s_up})
        if (hipStreamCreateWithFlags(p, hipStreamNonBlocking) != hipSuccess) {
            set_error("stream creation failed");
            return fail(GX_EDEVICE);
        }
    for (int i = 0; i < s->ring; i++)
        for (hipEvent_t *e : {&s->ev_n[i], &s->ev_c[i], &s->ev_u[i]})
            if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
                set_error("event creation failed");
                return fail(GX_EDEVICE);
            }
    if (s->V > 0) {
        if (s->d_l2g && hipMemcpy(s->d_l2g, s->l2g.data(), (size_t)s->V * 4, hipMemcpyHostToDevice) != hipSuccess) {
            set_error("upload of l2g failed");
            return fail(GX_EDEVICE);
        }
        if (hipMemcpy(s->d_has_edge, s->has_edge.data(), (size_t)s->V, hipMemcpyHostToDevice) != hipSuccess) {
            set_error("upload of the edge flags failed");
            return fail(GX_EDEVICE);
        }
    }
    const gx_status r = gx_stream_reset(s);
    if (r != GX_OK) return fail(r);
    *out = s;
    return GX_OK;
}

extern "C" gx_status gx_stream_reset(gx_stream *s) {
    clear_error();
    GX_REQUIRE(s, GX_EINVAL, "stream handle is NULL");
    GX_REQUIRE(!s->dev_error, GX_EDEVICE, "sticky device error");
    s->k = 0;
    if (s->V > 0)
        hipLaunchKernelGGL(k_st_init, dim3(blocks_of<int64_t>(s->V)), dim3(ST_BLOCK), 0, s->s_comp, s->val,
                           s->front[0], s->front[1], s->d_l2g, s->d_has_edge, s->V, (int)(s->algo == GX_CC),
                           s->source);
    ST_CHECK(hipGetLastError());
    ST_CHECK(hipStreamSynchronize(s->s_comp));
    return GX_OK;
}

extern "C" gx_status gx_stream_superstep(gx_stream *s, uint64_t block_edges, uint32_t mode, gx_stream_stats *out) {
    clear_error();
    GX_REQUIRE(s, GX_EINVAL, "stream handle is NULL");
    GX_REQUIRE(!s->dev_error, GX_EDEVICE, "sticky device error");
    GX_REQUIRE(block_edges >= 1 && block_edges <= s->bmax, GX_EINVAL, "block_edges %llu out of [1, %llu]",
               (unsigned long long)block_edges, (unsigned long long)s->bmax);
    GX_REQUIRE(mode == GX_STREAM_PIPELINED || mode == GX_STREAM_SERIAL, GX_EINVAL, "mode %u invalid", mode);
    gx_stream_stats st{};
    const auto t0 = std::chrono::steady_clock::now();
    const int cur = (int)(s->k & 1);
    const uint8_t *front = s->front[cur];
    uint8_t *next = s->front[cur ^ 1];
    const int64_t nblocks = (s->E + (int64_t)block_edges - 1) / (int64_t)block_edges;
    if (s->V > 0)
        hipLaunchKernelGGL(k_st_begin, dim3(blocks_of<int64_t>(s->V)), dim3(ST_BLOCK), 0, s->s_comp, s->val,
                           s->snap, next, s->V, s->cnt);
    ST_CHECK(hipGetLastError());
    const bool serial = mode == GX_STREAM_SERIAL;
    if (serial) {
        const size_t need = (size_t)nblocks * 3 + 1;
        while (s->tev.size() < need) {
            hipEvent_t e;
            ST_CHECK(hipEventCreate(&e));
            s->tev.push_back(e);
        }
        if (nblocks > 0) ST_CHECK(hipEventRecord(s->tev[0], s->s_comp));
    }
    for (int64_t i = 0; i < nblocks; i++) {
        const int64_t e0 = i * (int64_t)block_edges;
        const uint32_t n = (uint32_t)std::min<int64_t>((int64_t)block_edges, s->E - e0);
        const int b = serial ? 0 : (int)(i % s->ring);
        hipStream_t sn = serial ? s->s_comp : s->s_copy, sc = s->s_comp, su = serial ? s->s_comp : s->s_up;
        // n-block: download block i (the upload that last used this buffer is done)
        if (!serial && i >= s->ring) ST_CHECK(hipStreamWaitEvent(sn, s->ev_u[b], 0));
        ST_CHECK(hipMemcpyAsync(s->b_trip[b], s->h_trip + (size_t)e0 * s->tw, (size_t)n * 4 * s->tw,
                                hipMemcpyHostToDevice, sn));
        if (serial) ST_CHECK(hipEventRecord(s->tev[3 * i + 1], sn));
        else ST_CHECK(hipEventRecord(s->ev_n[b], sn));
        // c-block: compute it
        if (!serial) ST_CHECK(hipStreamWaitEvent(sc, s->ev_n[b], 0));
        hipLaunchKernelGGL(k_st_relax, dim3(blocks_of<uint32_t>(n)), dim3(ST_BLOCK), 0, sc, s->b_trip[b], s->tw, n,
                           s->snap, front, s->val, next, s->b_msg[b], s->cnt);
        ST_CHECK(hipGetLastError());
        if (serial) ST_CHECK(hipEventRecord(s->tev[3 * i + 2], sc));
        else ST_CHECK(hipEventRecord(s->ev_c[b], sc));
        // u-block: upload its results
        if (!serial) ST_CHECK(hipStreamWaitEvent(su, s->ev_c[b], 0));
        ST_CHECK(hipMemcpyAsync(s->h_msg + e0, s->b_msg[b], (size_t)n * 4, hipMemcpyDeviceToHost, su));
        if (serial) ST_CHECK(hipEventRecord(s->tev[3 * i + 3], su));
        else ST_CHECK(hipEventRecord(s->ev_u[b], su));
    }
    if (s->V > 0) {
        hipLaunchKernelGGL(k_st_end, dim3(blocks_of<int64_t>(s->V)), dim3(ST_BLOCK), 0, s->s_comp, next, s->V, s->cnt);
        ST_CHECK(hipGetLastError());
        ST_CHECK(hipMemcpyAsync(s->h_cnt, s->cnt, sizeof(StCounters), hipMemcpyDeviceToHost, s->s_comp));
    }
    ST_CHECK(hipStreamSynchronize(s->s_comp));
    ST_CHECK(hipStreamSynchronize(s->s_up));
    ST_CHECK(hipStreamSynchronize(s->s_copy));
    st.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (serial)
        for (int64_t i = 0; i < nblocks; i++) {
            float a = 0, b = 0, c = 0;
            ST_CHECK(hipEventElapsedTime(&a, s->tev[3 * i], s->tev[3 * i + 1]));
            ST_CHECK(hipEventElapsedTime(&b, s->tev[3 * i + 1], s->tev[3 * i + 2]));
            ST_CHECK(hipEventElapsedTime(&c, s->tev[3 * i + 2], s->tev[3 * i + 3]));
            st.download_ms += a;
            st.compute_ms += b;
            st.upload_ms += c;
        }
    st.blocks = nblocks;
    st.triplets = s->E;
    st.messages = s->V > 0 ? (int64_t)s->h_cnt->messages : 0;
    st.changed = s->V > 0 ? (int64_t)s->h_cnt->changed : 0;
    s->k++;
    if (out) *out = st;
    return GX_OK;
}

extern "C" gx_status gx_stream_values(gx_stream *s, void **dev_values, void **dev_frontier) {
    clear_error();
    GX_REQUIRE(s, GX_EINVAL, "stream handle is NULL");
    if (dev_values) *dev_values = s->val;
    if (dev_frontier) *dev_frontier = s->front[s->k & 1];
    return GX_OK;
}

extern "C" gx_status gx_stream_results(gx_stream *s, const uint32_t **host_results, int64_t *n) {
    clear_error();
    GX_REQUIRE(s && host_results && n, GX_EINVAL, "NULL argument");
    *host_results = s->h_msg;
    *n = s->E;
    return GX_OK;
}

extern "C" gx_status gx_stream_free(gx_stream *s) {
    clear_error();
    delete s;
    return GX_OK;
}

extern "C" gx_status gx_pipeline_time(const gx_pipeline_coef *k, double d, double s, double *T) {
    clear_error();
    GX_REQUIRE(k && T, GX_EINVAL, "NULL argument");
    GX_REQUIRE(d >= 2 && s >= 2 && s <= d, GX_EINVAL, "the model needs 2 <= s <= d");
    *T = pipeline_time(k->k1, k->k2, k->k3, k->a, d, s);
    return GX_OK;
}

extern "C" gx_status gx_pipeline_plan(const gx_pipeline_coef *k, int64_t d, int64_t *blocks, double *block_size,
                                      double *T) {
    clear_error();
    GX_REQUIRE(k && blocks, GX_EINVAL, "NULL argument");
    GX_REQUIRE(d >= 2, GX_EINVAL, "d = %lld: the pipeline needs at least 2 entities", (long long)d);
    GX_REQUIRE(k->k1 >= 0 && k->k2 >= 0 && k->k3 >= 0 && k->a >= 0 && k->k1 + k->k3 > 0, GX_EINVAL,
               "coefficients must be non-negative with k1 + k3 > 0");
    const double D = (double)d, k1 = k->k1, k2 = k->k2, k3 = k->k3, a = k->a;
    const double Q = std::sqrt(a * D / (k1 + k3));
    // the Lemma: when the download (upload) cost per entity is the largest,
    // the block that just keeps the computation hidden, a / (k1 - k2)
    // (a / (k3 - k2)), unless Q is smaller; otherwise Q
    double b = Q;
    if (k1 >= k2 && k1 >= k3 && k1 > k2) {
        const double bb = a / (k1 - k2);
        if (bb < Q) b = bb;
    } else if (k3 >= k1 && k3 >= k2 && k3 > k2) {
        const double bb = a / (k3 - k2);
        if (bb < Q) b = bb;
    }
    // integer block counts: the floor and the ceiling of d / b, by the model
    const double s_opt = b > 0 ? D / b : D;
    int64_t best = 2;
    double bestT = INFINITY;
    for (double sc : {std::floor(s_opt), std::ceil(s_opt)}) {
        const int64_t si = std::min<int64_t>(d, std::max<int64_t>(2, (int64_t)sc));
        const double t = pipeline_time(k1, k2, k3, a, D, (double)si);
        if (t < bestT) {
            bestT = t;
            best = si;
        }
    }
    *blocks = best;
    if (block_size) *block_size = D / (double)best;
    if (T) *T = bestT;
    return GX_OK;
}
