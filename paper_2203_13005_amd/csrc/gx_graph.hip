// Graph ingestion: host validation, host packaging of the device images, and
// block-streamed host-to-device transfer through three rotating pinned
// buffers (the n/c/u block rotation of Section "Pipeline Shuffling": while
// block i is in flight on the copy stream, block i+1 is packaged into the
// next buffer; pointers rotate instead of data being copied between stages).
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <functional>
#include <map>
#include <mutex>
#include <memory>
#include <thread>
#include <tuple>

#include "gx_internal.h"

namespace gx {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }

int device_cus(int device) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0) n = 256;
    return n;
}

int occupancy_per_cu(const void *kernel, int block) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, int>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_tuple(dev, kernel, block);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    cache[key] = per_cu;
    return per_cu;
}

// Host threads kept for the packaging passes (a load runs hundreds of them,
// one per 16 MiB block, and starting threads for each would cost more than
// the pass).  One pass at a time; a pass started from inside a pass, or
// while another load holds the workers, runs on the calling thread.
class HostWorkers {
  public:
    static HostWorkers &get() {
        static HostWorkers w;
        return w;
    }
    unsigned size() const { return (unsigned)workers_.size() + 1; }
    // Runs job(t) for t = 0 .. size()-1, share 0 on the calling thread; false
    // (nothing run) when the workers are busy.
    bool run(const std::function<void(unsigned)> &job) {
        std::unique_lock<std::mutex> busy(pass_, std::try_to_lock);
        if (!busy.owns_lock() || in_pass_) return false;
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &job;
            left_ = (unsigned)workers_.size();
            gen_++;
        }
        cv_.notify_all();
        in_pass_ = true;
        job(0);
        in_pass_ = false;
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [this] { return left_ == 0; });
        job_ = nullptr;
        return true;
    }
    ~HostWorkers() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            gen_++;
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
    }

  private:
    HostWorkers() {
        const unsigned n = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        for (unsigned t = 1; t < n; t++) workers_.emplace_back([this, t] { loop(t); });
    }
    void loop(unsigned t) {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            cv_.wait(lk, [&] { return gen_ != seen; });
            seen = gen_;
            if (stop_) return;
            const std::function<void(unsigned)> *job = job_;
            lk.unlock();
            in_pass_ = true;
            (*job)(t);
            in_pass_ = false;
            lk.lock();
            if (--left_ == 0) done_.notify_all();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex pass_, mu_;
    std::condition_variable cv_, done_;
    const std::function<void(unsigned)> *job_ = nullptr;
    unsigned left_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
    static thread_local bool in_pass_;
};
thread_local bool HostWorkers::in_pass_ = false;

template <class F>
static void parallel_for(int64_t n, F f, int64_t serial_below = 65536) {
    HostWorkers &w = HostWorkers::get();
    const unsigned nt = w.size();
    if (n < serial_below || nt == 1) {
        f(0, n);
        return;
    }
    const std::function<void(unsigned)> job = [&](unsigned t) { f(n * t / nt, n * (t + 1) / nt); };
    if (!w.run(job)) f(0, n);
}

// Host images built from the description before upload.
// Vectors whose elements start uninitialised (resize leaves them as they
// are): the edge-sized images are written in full by parallel passes, so a
// value fill on one thread first would only cost time.
template <class T>
struct NoInit : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInit<U>;
    };
    NoInit() = default;
    template <class U>
    NoInit(const NoInit<U> &) {}
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        if constexpr (sizeof...(A) == 0) ::new ((void *)p) U;
        else ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
template <class T>
using EdgeVec = std::vector<T, NoInit<T>>;

struct HostImages {
    std::vector<int32_t> in_rp, outdeg, tile_row, pr_slot;
    EdgeVec<int32_t> in_col, pr_src;
    EdgeVec<uint32_t> in_w;
    std::vector<int32_t> sym_rp;
    EdgeVec<int32_t> sym_col;
    EdgeVec<uint2> pull_w, pull_sym;
    std::vector<uint4> pull_w_units, pull_sym_units;
    PullSlices pull_w_off{}, pull_sym_off{};
    std::vector<uint32_t> rem_out, rem_any, master, master_rep;
};

static gx_status validate(const gx_graph_desc *d) {
    GX_REQUIRE(d, GX_EINVAL, "desc is NULL");
    GX_REQUIRE(d->V >= 0 && d->V < (int64_t(1) << 31) - 64, GX_EINVAL, "V=%lld out of range", (long long)d->V);
    GX_REQUIRE(d->E >= 0 && d->E < (int64_t(1) << 31) - PR_TILE_MAX, GX_EINVAL, "E=%lld out of range",
               (long long)d->E);
    GX_REQUIRE(d->pr_tile_edges == 0 || d->pr_tile_edges == 256 || d->pr_tile_edges == 512 ||
                   d->pr_tile_edges == 1024 || d->pr_tile_edges == 2048,
               GX_EINVAL, "pr_tile_edges=%u not 0, 256, 512, 1024 or 2048", d->pr_tile_edges);
    GX_REQUIRE(d->needs != 0 && (d->needs & ~7u) == 0, GX_EINVAL, "needs=%u invalid", d->needs);
    // the symmetric image holds up to two entries per directed edge, indexed by int32 row pointers
    GX_REQUIRE(!(d->needs & GX_NEED_SYM) || 2 * d->E <= (int64_t)INT32_MAX - PULL_VT * 64, GX_EINVAL,
               "E=%lld too large for the symmetric (CC) image: 2E must stay below 2^31", (long long)d->E);
    GX_REQUIRE(d->row_ptr || d->V == 0, GX_EINVAL, "row_ptr is NULL");
    GX_REQUIRE(d->col || d->E == 0, GX_EINVAL, "col is NULL");
    GX_REQUIRE(!(d->needs & GX_NEED_OUT) || d->w || d->E == 0, GX_EINVAL, "weights required for GX_NEED_OUT");
    if (d->V == 0) {
        GX_REQUIRE(d->E == 0, GX_EINVAL, "E > 0 with V == 0");
        return GX_OK;
    }
    GX_REQUIRE(d->row_ptr[0] == 0, GX_EINVAL, "row_ptr[0] != 0");
    GX_REQUIRE(d->row_ptr[d->V] == d->E, GX_EINVAL, "row_ptr[V]=%d != E=%lld", d->row_ptr[d->V], (long long)d->E);
    for (int64_t v = 0; v < d->V; v++)
        GX_REQUIRE(d->row_ptr[v + 1] >= d->row_ptr[v], GX_EINVAL, "row_ptr decreases at %lld", (long long)v);
    std::atomic<int64_t> badpos{INT64_MAX};  // the first column out of range, over the host threads
    parallel_for(d->E, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; e++)
            if ((uint32_t)d->col[e] >= (uint32_t)d->V) {
                int64_t cur = badpos.load();
                while (e < cur && !badpos.compare_exchange_weak(cur, e)) {
                }
                return;
            }
    });
    const int64_t bp = badpos.load();
    GX_REQUIRE(bp == INT64_MAX, GX_EINVAL, "col[%lld]=%d out of [0,V)", (long long)bp,
               bp == INT64_MAX ? 0 : d->col[bp]);
    GX_REQUIRE((d->V_global == 0) == (d->outdeg_global == nullptr), GX_EINVAL,
               "V_global and outdeg_global come together");
    if (d->outdeg_global) {
        GX_REQUIRE(d->V_global >= d->V && d->V_global < (int64_t(1) << 31), GX_EINVAL, "V_global=%lld out of range",
                   (long long)d->V_global);
        for (int64_t v = 0; v < d->V; v++)
            GX_REQUIRE(d->outdeg_global[v] >= d->row_ptr[v + 1] - d->row_ptr[v], GX_EINVAL,
                       "outdeg_global[%lld] below the local out-degree", (long long)v);
    }
    if (d->l2g) {
        GX_REQUIRE(d->l2g[0] >= 0, GX_EINVAL, "l2g[0] negative");
        for (int64_t v = 1; v < d->V; v++)
            GX_REQUIRE(d->l2g[v] > d->l2g[v - 1], GX_EINVAL, "l2g not strictly ascending at %lld", (long long)v);
    }
    return GX_OK;
}

static unsigned host_threads() { return std::max(1u, std::min(16u, std::thread::hardware_concurrency())); }

// Stable counting sort of the edges by destination: in-rows list their
// sources in ascending order, the same result as one sequential pass.  The
// destinations are cut into buckets of equal vertex ranges; the edges, in
// source order, are cut into one chunk per thread.  Each thread counts its
// chunk's edges per bucket, the counts are laid out bucket by bucket and
// chunk by chunk (so a bucket keeps the chunks' source order), each thread
// copies its chunk's edges to their buckets, and the buckets, handed out
// one at a time, are sorted by destination with a counting sort of their
// own.  Every edge is read a bounded number of times whatever the thread
// count.
static void build_in_csr(const gx_graph_desc *d, HostImages &h) {
    const int64_t V = d->V, E = d->E;
    h.in_rp.assign(V + 1, 0);
    h.in_col.resize(E);
    const bool wts = d->w && (d->needs & GX_NEED_OUT);
    if (wts) h.in_w.resize(E);
    if (E == 0) return;
    const unsigned nt = E < 4096 ? 1u : host_threads();
    const int64_t NB = std::max<int64_t>(1, std::min<int64_t>(256, V / 64));  // destination buckets
    const int64_t span = (V + NB - 1) / NB;                                    // vertices per bucket
    // source-ordered edge chunks: chunk t holds the out-rows of sources [src_cut[t], src_cut[t+1])
    std::vector<int64_t> src_cut(nt + 1, V);
    src_cut[0] = 0;
    for (unsigned t = 1; t < nt; t++)
        src_cut[t] = std::upper_bound(d->row_ptr, d->row_ptr + V, (int32_t)(E * t / nt)) - d->row_ptr - 1;
    for (unsigned t = 1; t <= nt; t++) src_cut[t] = std::max(src_cut[t], src_cut[t - 1]);
    std::vector<int64_t> cnt((size_t)nt * NB, 0);  // [chunk][bucket]
    auto run = [&](auto &&body) {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; t++) th.emplace_back([&, t] { body(t); });
        for (auto &x : th) x.join();
    };
    run([&](unsigned t) {
        int64_t *c = cnt.data() + (size_t)t * NB;
        for (int64_t e = d->row_ptr[src_cut[t]]; e < d->row_ptr[src_cut[t + 1]]; e++) c[d->col[e] / span]++;
    });
    // offsets: bucket-major, then chunk order inside a bucket
    std::vector<int64_t> boff(NB + 1, 0);
    std::vector<int64_t> off((size_t)nt * NB);
    int64_t acc = 0;
    for (int64_t bk = 0; bk < NB; bk++) {
        boff[bk] = acc;
        for (unsigned t = 0; t < nt; t++) {
            off[(size_t)t * NB + bk] = acc;
            acc += cnt[(size_t)t * NB + bk];
        }
    }
    boff[NB] = acc;
    // edges grouped by bucket: (destination, source[, weight])
    std::unique_ptr<int32_t[]> bdst(new int32_t[E]), bsrc(new int32_t[E]);  // (no zero fill)
    std::unique_ptr<uint32_t[]> bw(wts ? new uint32_t[E] : nullptr);
    run([&](unsigned t) {
        int64_t *o = off.data() + (size_t)t * NB;
        for (int64_t u = src_cut[t]; u < src_cut[t + 1]; u++)
            for (int32_t e = d->row_ptr[u]; e < d->row_ptr[u + 1]; e++) {
                const int32_t v = d->col[e];
                const int64_t p = o[v / span]++;
                bdst[p] = v;
                bsrc[p] = (int32_t)u;
                if (wts) bw[p] = d->w[e];
            }
    });
    // each bucket: counting sort by destination (stable), row pointers of its range
    std::atomic<int64_t> next{0};
    run([&](unsigned) {
        std::vector<int32_t> pos;
        for (int64_t bk; (bk = next.fetch_add(1)) < NB;) {
            const int64_t vlo = bk * span, vhi = std::min<int64_t>(V, vlo + span);
            if (vlo >= vhi) continue;
            const int64_t e0 = boff[bk], e1 = boff[bk + 1];
            pos.assign((size_t)(vhi - vlo) + 1, 0);
            for (int64_t i = e0; i < e1; i++) pos[bdst[i] - vlo + 1]++;
            for (int64_t j = 0; j < vhi - vlo; j++) {  // pos[j]: first slot of destination vlo + j
                pos[j + 1] += pos[j];
                h.in_rp[vlo + j + 1] = (int32_t)(e0 + pos[j + 1]);
            }
            for (int64_t i = e0; i < e1; i++) {
                const int64_t p = e0 + pos[bdst[i] - vlo]++;
                h.in_col[p] = bsrc[i];
                if (wts) h.in_w[p] = bw[i];
            }
        }
    });
}

// PageRank contribution slots: the PR_HOT vertices with the most out-edges
// (ties by id) take slots 0.. in that order, the others follow in id order,
// so the gathers of hub contributions fall on a few cache lines.
static void build_pr_slots(const gx_graph_desc *d, HostImages &h) {
    const int64_t V = d->V, E = d->E;
    const int64_t K = std::min<int64_t>(V, PR_HOT);
    std::vector<int32_t> ids(V);
    for (int64_t v = 0; v < V; v++) ids[v] = (int32_t)v;
    auto deg = [d](int32_t v) { return d->row_ptr[v + 1] - d->row_ptr[v]; };
    auto hotter = [&](int32_t a, int32_t b) { return deg(a) != deg(b) ? deg(a) > deg(b) : a < b; };
    std::partial_sort(ids.begin(), ids.begin() + K, ids.end(), hotter);
    h.pr_slot.assign(V, -1);
    for (int64_t i = 0; i < K; i++) h.pr_slot[ids[i]] = (int32_t)i;
    int64_t next = K;
    for (int64_t v = 0; v < V; v++)
        if (h.pr_slot[v] < 0) h.pr_slot[v] = (int32_t)next++;
    h.pr_src.resize(E);
    parallel_for(E, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; e++) h.pr_src[e] = h.pr_slot[h.in_col[e]];
    });
}

// Pull tiles: tile t covers edges [t*T, (t+1)*T) of a CSR and owns the rows
// whose first edge position falls in that range (the last tile also owns the
// rows starting at E).
static int64_t ntiles_for(int64_t E, int64_t T) { return std::max<int64_t>(1, (E + T - 1) / T); }

// PageRank tile size: the caller's choice, else the largest size up to 1024
// that still gives 2048 tiles (eight per CU), else the smallest.  (2048-edge
// tiles measured 3% slower on the scale-25 partition and 8% slower on R-MAT
// scale 20 than 1024, and 0.6% faster on R-MAT scale 22.)
static int32_t pr_tile_for(const gx_graph_desc *d) {
    if (d->pr_tile_edges) return (int32_t)d->pr_tile_edges;
    for (int32_t T = PR_TILE_MAX / 2; T > PR_BLOCK; T /= 2)
        if (ntiles_for(d->E, T) >= 2048) return T;
    return PR_BLOCK;
}

static void build_tiles(const std::vector<int32_t> &rp, std::vector<int32_t> &tile_row, int64_t T) {
    int64_t V = (int64_t)rp.size() - 1, E = rp.back();
    int64_t nt = ntiles_for(E, T);
    tile_row.resize(nt + 1);
    for (int64_t t = 0; t < nt; t++)
        tile_row[t] = (int32_t)(std::lower_bound(rp.begin(), rp.end() - 1, (int32_t)(t * T)) - rp.begin());
    tile_row[0] = 0;
    tile_row[nt] = (int32_t)V;
}

// Pull records from a CSR over destinations (rows) listing sources in
// ascending order.  Destinations are taken in blocks of
// 2^PULL_SLICE_SHIFT and dealt to PULL_SLICES * S bins greedily, heaviest
// in-edge count first, each to the lightest bin so far (degree skew would
// otherwise pile most edges onto one bin).  Bin j belongs to XCD slice
// j mod PULL_SLICES; S is chosen so a bin's destination values fit
// PULL_BIN_BYTES, and an XCD sweeps its S bins one after another.  Within a
// bin the records are grouped by source band, keeping the (destination,
// source) order of the CSR inside a group; every group is padded to whole
// PULL_VT records with sentinels (destination PULL_SENTINEL) and cut into
// units of at most PULL_UNIT records.  Weighted records are
// {dst, (src mod PULL_BAND) << 8 | w}: the unit names the band, so a source
// takes 12 bits and any vertex count fits; with `w` null they are {dst, src}
// (sentinel source: the band base).
static void build_pull(const std::vector<int32_t> &rp, const int32_t *src, const uint32_t *w,
                       EdgeVec<uint2> &out, std::vector<uint4> &units, PullSlices &sl) {
    const int64_t V = (int64_t)rp.size() - 1;
    const int64_t nb = (V >> PULL_BAND_BITS) + 1;
    const int64_t nbin = pull_bins(V), S = nbin / PULL_SLICES;
    const int64_t nblk = (V + (1 << PULL_SLICE_SHIFT) - 1) >> PULL_SLICE_SHIFT;
    std::vector<int64_t> bcnt((size_t)nblk, 0);
    for (int64_t v = 0; v < V; v++) bcnt[v >> PULL_SLICE_SHIFT] += rp[v + 1] - rp[v];
    std::vector<int64_t> order((size_t)nblk);
    for (int64_t i = 0; i < nblk; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return bcnt[a] > bcnt[b]; });
    // group index of block b's bin: slices are contiguous, their bins in order
    std::vector<int32_t> group((size_t)nblk, 0);
    std::vector<int64_t> load((size_t)nbin, 0);
    for (int64_t b : order) {
        int64_t j = 0;
        for (int64_t y = 1; y < nbin; y++)
            if (load[y] < load[j]) j = y;
        load[j] += bcnt[b];
        group[b] = (int32_t)((j % PULL_SLICES) * S + j / PULL_SLICES);
    }
    const int64_t ng = nbin * nb;
    std::vector<int64_t> cnt((size_t)ng, 0);
    // one thread per slice: it owns the groups of its bins, so the counts and
    // the fill below need no shared counters
    auto per_slice = [&](auto &&body) {
        std::vector<std::thread> th;
        for (int x = 0; x < PULL_SLICES; x++)
            th.emplace_back([&, x] {
                const int64_t glo = x * S, ghi = (x + 1) * S;
                for (int64_t v = 0; v < V; v++) {
                    const int64_t gb = group[v >> PULL_SLICE_SHIFT];
                    if (gb >= glo && gb < ghi) body(v, gb * nb);
                }
            });
        for (auto &t : th) t.join();
    };
    per_slice([&](int64_t v, int64_t g0) {
        for (int32_t e = rp[v]; e < rp[v + 1]; e++) cnt[g0 + (src[e] >> PULL_BAND_BITS)]++;
    });
    std::vector<int64_t> pos((size_t)ng + 1, 0);
    for (int64_t g = 0; g < ng; g++) pos[g + 1] = pos[g] + (cnt[g] + PULL_VT - 1) / PULL_VT * PULL_VT;
    out.resize((size_t)pos[ng]);  // every slot is written below: a record or a sentinel
    for (int64_t g = 0; g < ng; g++) {  // sentinels: a source inside their band, weight 0
        const uint32_t bb = (uint32_t)((g % nb) << PULL_BAND_BITS);
        for (int64_t i = pos[g] + cnt[g]; i < pos[g + 1]; i++) out[i] = make_uint2(PULL_SENTINEL, w ? 0u : bb);
    }
    std::vector<int64_t> fill(pos.begin(), pos.end() - 1);
    per_slice([&](int64_t v, int64_t g0) {
        for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
            const uint32_t u = (uint32_t)src[e];
            out[fill[g0 + (u >> PULL_BAND_BITS)]++] =
                make_uint2((uint32_t)v, w ? (((u & (PULL_BAND - 1)) << 8) | w[e]) : u);
        }
    });
    units.clear();
    for (int x = 0; x < PULL_SLICES; x++) {
        sl.uoff[x] = (int64_t)units.size();
        for (int64_t g = x * S * nb; g < (x + 1) * S * nb; g++)
            for (int64_t s0 = pos[g]; s0 < pos[g + 1]; s0 += PULL_UNIT)
                units.push_back(make_uint4((uint32_t)s0, (uint32_t)std::min<int64_t>(PULL_UNIT, pos[g + 1] - s0),
                                           (uint32_t)((g % nb) << PULL_BAND_BITS), 0u));
    }
    sl.uoff[PULL_SLICES] = (int64_t)units.size();
}

static bool banded_weights_fit(const gx_graph_desc *d) {
    std::atomic<bool> ok{true};
    parallel_for(d->E, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; e++)
            if (d->w[e] > 255u) {
                ok = false;
                return;
            }
    });
    return ok;
}

// Symmetric adjacency: sorted union of out- and in-neighbours, self
// excluded, duplicates removed (needs the in-CSR).
static void build_sym(const gx_graph_desc *d, HostImages &h) {
    int64_t V = d->V;
    const int32_t *orp = d->row_ptr, *oc = d->col;
    const int32_t *irp = h.in_rp.data(), *ic = h.in_col.data();
    auto merge_row = [&](int64_t u, int32_t *out) -> int32_t {
        int32_t a = orp[u], ae = orp[u + 1], b = irp[u], be = irp[u + 1], n = 0, last = -1;
        while (a < ae || b < be) {
            int32_t x;
            if (b >= be || (a < ae && oc[a] <= ic[b])) x = oc[a++];
            else x = ic[b++];
            if (x == (int32_t)u || x == last) continue;
            if (out) out[n] = x;
            n++;
            last = x;
        }
        return n;
    };
    h.sym_rp.assign(V + 1, 0);
    parallel_for(V, [&](int64_t lo, int64_t hi) {
        for (int64_t u = lo; u < hi; u++) h.sym_rp[u + 1] = merge_row(u, nullptr);
    });
    for (int64_t v = 0; v < V; v++) h.sym_rp[v + 1] += h.sym_rp[v];
    h.sym_col.resize(h.sym_rp[V]);
    parallel_for(V, [&](int64_t lo, int64_t hi) {
        for (int64_t u = lo; u < hi; u++) merge_row(u, h.sym_col.data() + h.sym_rp[u]);
    });
}

static void build_flags(const gx_graph_desc *d, int32_t W, HostImages &h) {
    h.rem_out.assign(W, 0);
    h.rem_any.assign(W, 0);
    h.master.assign(W, 0);
    h.master_rep.assign(W, 0);
    if (!d->flags) return;
    for (int64_t v = 0; v < d->V; v++) {
        uint32_t bit = 1u << (v & 31);
        const uint8_t f = d->flags[v];
        if (f & GX_FLAG_REMOTE_OUT) h.rem_out[v >> 5] |= bit;
        if (f & GX_FLAG_REMOTE_ANY) h.rem_any[v >> 5] |= bit;
        if (f & GX_FLAG_MASTER) h.master[v >> 5] |= bit;
        if ((f & GX_FLAG_MASTER) && (f & GX_FLAG_REMOTE_ANY)) h.master_rep[v >> 5] |= bit;
    }
}

// Device layout; with a measuring Carver it only sizes the arena.  E_sym
// must be known for the symmetric image (computed by the caller).
static void layout(const gx_graph_desc *desc, int64_t E_sym, Carver &c, DevGraph *d) {
    int64_t V = desc->V, E = desc->E;
    d->V = V;
    d->E = E;
    d->E_sym = E_sym;
    d->W = (int32_t)((V + 31) / 32);
    if (desc->needs & GX_NEED_OUT) {
        d->out_rp = c.take<int32_t>(V + 1);
        d->out_adj = c.take<uint2>(E);
    }
    if (desc->needs & (GX_NEED_IN | GX_NEED_OUT)) {
        d->in_rp = c.take<int32_t>(V + 1);
        d->pr_tile = pr_tile_for(desc);
        d->pr_ntiles = (int32_t)ntiles_for(E, d->pr_tile);
        d->pr_tile_row = c.take<int32_t>(d->pr_ntiles + 1);
    }
    if (desc->needs & GX_NEED_IN) {
        d->in_col = c.take<int32_t>(E);
        d->outdeg = c.take<int32_t>(V);
        d->pr_src = c.take<int32_t>(E);
        d->pr_slot = c.take<int32_t>(V);
    }
    if ((desc->needs & GX_NEED_OUT) && (desc->E == 0 || banded_weights_fit(desc))) {
        d->pull_w = c.take<uint2>(pull_rec_cap(V, E));
        d->pull_w_units = c.take<uint4>(pull_unit_cap(V, E));
    }
    if (desc->needs & GX_NEED_SYM) {
        d->sym_rp = c.take<int32_t>(V + 1);
        d->sym_col = c.take<int32_t>(E_sym);
        d->pull_sym = c.take<uint2>(pull_rec_cap(V, E_sym));
        d->pull_sym_units = c.take<uint4>(pull_unit_cap(V, E_sym));
    }
    if (desc->l2g) d->l2g = c.take<int32_t>(V);
    if (desc->outdeg_global) {
        d->outdeg_g = c.take<int32_t>(V);
        d->V_global = desc->V_global;
    }
    if (desc->flags) {
        d->remote_out = c.take<uint32_t>(d->W);
        d->remote_any = c.take<uint32_t>(d->W);
        d->master = c.take<uint32_t>(d->W);
        d->master_rep = c.take<uint32_t>(d->W);
    }
}

// Upper bound of the symmetric image without building it: every directed
// edge contributes at most two neighbour entries.
static int64_t sym_bound(const gx_graph_desc *d) { return 2 * d->E; }

// Streams byte ranges produced by `fill` to device memory in fixed blocks
// through three rotating pinned buffers on a dedicated copy stream.
struct Uploader {
    static constexpr size_t BLOCK = size_t(16) << 20;
    hipStream_t copy = nullptr;
    void *buf[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    uint64_t idx = 0;
    hipError_t err = hipSuccess;

    hipError_t open() {
        if ((err = hipStreamCreateWithFlags(&copy, hipStreamNonBlocking)) != hipSuccess) return err;
        for (int i = 0; i < 3; i++) {
            if ((err = hipHostMalloc(&buf[i], BLOCK, hipHostMallocDefault)) != hipSuccess) return err;
            if ((err = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming)) != hipSuccess) return err;
        }
        return hipSuccess;
    }
    hipError_t put(void *dev, size_t bytes, const std::function<void(char *, size_t, size_t)> &fill) {
        for (size_t off = 0; off < bytes && err == hipSuccess; off += BLOCK) {
            size_t n = std::min(BLOCK, bytes - off);
            int b = (int)(idx++ % 3);
            if ((err = hipEventSynchronize(ev[b])) != hipSuccess) break;  // buffer b free again
            fill(static_cast<char *>(buf[b]), off, n);                     // package block (host)
            if ((err = hipMemcpyAsync(static_cast<char *>(dev) + off, buf[b], n, hipMemcpyHostToDevice, copy)) !=
                hipSuccess)
                break;
            err = hipEventRecord(ev[b], copy);
        }
        return err;
    }
    hipError_t put_array(void *dev, const void *host, size_t bytes) {
        return put(dev, bytes, [host](char *dst, size_t off, size_t n) {  // copied in 1 MiB pieces on the host threads
            const int64_t pieces = (int64_t)((n + (size_t(1) << 20) - 1) >> 20);
            parallel_for(
                pieces,
                [&](int64_t lo, int64_t hi) {
                    for (int64_t i = lo; i < hi; i++) {
                        const size_t a = (size_t)i << 20, len = std::min(n - a, size_t(1) << 20);
                        std::memcpy(dst + a, static_cast<const char *>(host) + off + a, len);
                    }
                },
                2);
        });
    }
    hipError_t finish(hipStream_t user) {
        hipEvent_t done = nullptr;
        if (err == hipSuccess) err = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        if (err == hipSuccess) err = hipEventRecord(done, copy);
        if (err == hipSuccess) err = hipStreamWaitEvent(user, done, 0);
        if (err == hipSuccess) err = hipStreamSynchronize(copy);
        if (done) (void)hipEventDestroy(done);
        return err;
    }
    ~Uploader() {
        if (copy) (void)hipStreamSynchronize(copy);
        for (int i = 0; i < 3; i++) {
            if (ev[i]) (void)hipEventDestroy(ev[i]);
            if (buf[i]) (void)hipHostFree(buf[i]);
        }
        if (copy) (void)hipStreamDestroy(copy);
    }
};

}  // namespace gx

using namespace gx;

extern "C" const char *gx_last_error(void) { return g_err.c_str(); }
extern "C" const char *gx_version(void) { return "gx 0.1 (gfx950)"; }

extern "C" gx_status gx_graph_bytes(const gx_graph_desc *desc, size_t *arena_bytes) {
    clear_error();
    GX_REQUIRE(arena_bytes, GX_EINVAL, "arena_bytes is NULL");
    gx_status st = validate(desc);
    if (st != GX_OK) return st;
    Carver c(nullptr, 0);
    DevGraph d;
    layout(desc, sym_bound(desc), c, &d);
    *arena_bytes = c.used;
    return GX_OK;
}

extern "C" gx_status gx_graph_load(const gx_graph_desc *desc, void *dev_arena, size_t arena_bytes, void *stream,
                                   gx_graph **out) {
    clear_error();
    GX_REQUIRE(out, GX_EINVAL, "out is NULL");
    *out = nullptr;
    gx_status st = validate(desc);
    if (st != GX_OK) return st;
    GX_REQUIRE(dev_arena || arena_bytes == 0, GX_EINVAL, "dev_arena is NULL");
    GX_REQUIRE(reinterpret_cast<uintptr_t>(dev_arena) % ALIGN == 0, GX_EINVAL, "dev_arena not 256-byte aligned");
    {
        Carver m(nullptr, 0);
        DevGraph tmp;
        layout(desc, sym_bound(desc), m, &tmp);
        GX_REQUIRE(m.used <= arena_bytes, GX_ENOMEM, "arena too small: need %zu bytes, have %zu", m.used, arena_bytes);
    }

    HostImages h;
    int32_t W = (int32_t)((desc->V + 31) / 32);
    try {
        build_in_csr(desc, h);
        build_tiles(h.in_rp, h.tile_row, pr_tile_for(desc));
        if (desc->needs & GX_NEED_IN) build_pr_slots(desc, h);
        if ((desc->needs & GX_NEED_OUT) && (desc->E == 0 || banded_weights_fit(desc)))
            build_pull(h.in_rp, h.in_col.data(), h.in_w.data(), h.pull_w, h.pull_w_units, h.pull_w_off);
        if (desc->needs & GX_NEED_SYM) {
            build_sym(desc, h);
            build_pull(h.sym_rp, h.sym_col.data(), nullptr, h.pull_sym, h.pull_sym_units, h.pull_sym_off);
        }
        build_flags(desc, W, h);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed while packaging the graph");
        return GX_ENOMEM;
    } catch (const std::exception &ex) {
        set_error("graph packaging failed: %s", ex.what());
        return GX_EINVAL;
    }

    gx_graph *g = new (std::nothrow) gx_graph();
    GX_REQUIRE(g, GX_ENOMEM, "host allocation failed");
    Carver c(dev_arena, arena_bytes);
    layout(desc, (int64_t)h.sym_col.size(), c, &g->d);
    g->d.pull_w_off = h.pull_w_off;
    g->d.pull_sym_off = h.pull_sym_off;
    for (const uint4 &u : h.pull_w_units) g->pull_w_recs.push_back(u.y);
    for (const uint4 &u : h.pull_sym_units) g->pull_sym_recs.push_back(u.y);
    g->needs = desc->needs;
    g->arena = dev_arena;
    g->arena_bytes = arena_bytes;
    if (hipGetDevice(&g->device) != hipSuccess) g->device = 0;
    g->num_cus = device_cus(g->device);
    g->host_outdeg.resize(desc->V);
    for (int64_t v = 0; v < desc->V; v++) g->host_outdeg[v] = desc->row_ptr[v + 1] - desc->row_ptr[v];
    if (!h.sym_rp.empty()) {
        g->host_symdeg.resize(desc->V);
        for (int64_t v = 0; v < desc->V; v++) g->host_symdeg[v] = h.sym_rp[v + 1] - h.sym_rp[v];
    }

    hipStream_t s = static_cast<hipStream_t>(stream);
    Uploader up;
    hipError_t e = up.open();
    const DevGraph &d = g->d;
    int64_t V = desc->V, E = desc->E;
    if (e == hipSuccess && d.out_rp) e = up.put_array((void *)d.out_rp, desc->row_ptr, (V + 1) * 4);
    if (e == hipSuccess && d.out_adj) {
        const int32_t *col = desc->col;
        const uint32_t *w = desc->w;
        // Package (destination, weight) pairs block by block.
        e = up.put((void *)d.out_adj, E * sizeof(uint2), [col, w](char *dst, size_t off, size_t n) {
            uint2 *o = reinterpret_cast<uint2 *>(dst);
            const size_t e0 = off / sizeof(uint2), cnt = n / sizeof(uint2);
            parallel_for((int64_t)cnt, [&](int64_t lo, int64_t hi) {
                for (int64_t i = lo; i < hi; i++) o[i] = make_uint2((uint32_t)col[e0 + i], w[e0 + i]);
            });
        });
    }
    if (e == hipSuccess && d.in_rp) {
        e = up.put_array((void *)d.in_rp, h.in_rp.data(), (V + 1) * 4);
        if (e == hipSuccess) e = up.put_array((void *)d.pr_tile_row, h.tile_row.data(), h.tile_row.size() * 4);
    }
    if (e == hipSuccess && d.in_col) {
        e = up.put_array((void *)d.in_col, h.in_col.data(), E * 4);
        if (e == hipSuccess) e = up.put_array((void *)d.outdeg, g->host_outdeg.data(), V * 4);
        if (e == hipSuccess) e = up.put_array((void *)d.pr_src, h.pr_src.data(), E * 4);
        if (e == hipSuccess) e = up.put_array((void *)d.pr_slot, h.pr_slot.data(), V * 4);
    }
    if (e == hipSuccess && d.pull_w) {
        e = up.put_array((void *)d.pull_w, h.pull_w.data(), h.pull_w.size() * sizeof(uint2));
        if (e == hipSuccess)
            e = up.put_array((void *)d.pull_w_units, h.pull_w_units.data(), h.pull_w_units.size() * sizeof(uint4));
    }
    if (e == hipSuccess && d.sym_rp) {
        e = up.put_array((void *)d.sym_rp, h.sym_rp.data(), (V + 1) * 4);
        if (e == hipSuccess) e = up.put_array((void *)d.sym_col, h.sym_col.data(), h.sym_col.size() * 4);
        if (e == hipSuccess)
            e = up.put_array((void *)d.pull_sym, h.pull_sym.data(), h.pull_sym.size() * sizeof(uint2));
        if (e == hipSuccess)
            e = up.put_array((void *)d.pull_sym_units, h.pull_sym_units.data(),
                             h.pull_sym_units.size() * sizeof(uint4));
    }
    if (e == hipSuccess && d.l2g) e = up.put_array((void *)d.l2g, desc->l2g, V * 4);
    if (e == hipSuccess && d.outdeg_g) e = up.put_array((void *)d.outdeg_g, desc->outdeg_global, V * 4);
    if (e == hipSuccess && d.remote_out) {
        e = up.put_array((void *)d.remote_out, h.rem_out.data(), (size_t)W * 4);
        if (e == hipSuccess) e = up.put_array((void *)d.remote_any, h.rem_any.data(), (size_t)W * 4);
        if (e == hipSuccess) e = up.put_array((void *)d.master, h.master.data(), (size_t)W * 4);
        if (e == hipSuccess) e = up.put_array((void *)d.master_rep, h.master_rep.data(), (size_t)W * 4);
    }
    if (e == hipSuccess) e = up.finish(s);
    if (e != hipSuccess) {
        set_error("graph upload failed: %s", hipGetErrorString(e));
        delete g;
        return GX_EDEVICE;
    }
    *out = g;
    return GX_OK;
}

extern "C" gx_status gx_graph_free(gx_graph *g) {
    clear_error();
    delete g;
    return GX_OK;
}

extern "C" gx_status gx_graph_info(const gx_graph *g, int64_t *V, int64_t *E, uint32_t *needs) {
    clear_error();
    GX_REQUIRE(g, GX_EINVAL, "graph is NULL");
    if (V) *V = g->d.V;
    if (E) *E = g->d.E;
    if (needs) *needs = g->needs;
    return GX_OK;
}
