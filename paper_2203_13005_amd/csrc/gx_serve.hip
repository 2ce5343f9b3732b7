// Serving: continuous batching of SSSP and personalised-PageRank queries over
// graphs kept resident in HBM.
//
// A scheduler thread owns per-(graph, algorithm) lane pools.  Each pool is a
// [V x B] batched state (the lanes of the batched engine) with its own
// stream.  A pool advances in epochs of a few supersteps; between epochs
// (superstep boundaries) the scheduler retires lanes whose query is done --
// SSSP when the lane activated nothing in a superstep, PPR after its
// iterations -- copies their column to the caller's buffer, and admits
// queued queries into free lanes.  New pools are created only while the
// device budget allows (first-fit inside the caller's arena); idle empty
// pools are evicted to make room.  Pools on different streams overlap on the
// GPU, so pool epochs use ordinary launches (no grid-wide co-residency is
// assumed).  Every lane's arithmetic is independent of the other lanes, so a
// query's answer is the same alone and in the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "gx_batch.h"
#include "gx_device.h"
#include "gx_internal.h"

using namespace gx;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SQuery {
    int64_t id;
    int32_t graph, algo, source;
    void *result;
    double t_submit = 0, t_start = 0, t_done = 0;
    int64_t steps = 0;
    int32_t status = GX_OK;
};

// First-fit allocator over the server arena (256-byte granules).
struct ArenaAlloc {
    char *base = nullptr;
    size_t cap = 0;
    std::map<size_t, size_t> free_;  // offset -> size
    void init(void *b, size_t c) {
        base = static_cast<char *>(b);
        size_t off = (ALIGN - reinterpret_cast<uintptr_t>(b) % ALIGN) % ALIGN;
        cap = c > off ? c - off : 0;
        base += off;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    // First fit, skipping free ranges that overlap [skip_off, skip_off + skip_len).
    void *alloc(size_t n, size_t skip_off = 0, size_t skip_len = 0) {
        n = align_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            if (skip_len && it->first < skip_off + skip_len && skip_off < it->first + it->second) continue;
            size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > n) free_[off + n] = sz - n;
            return base + off;
        }
        return nullptr;
    }
    void release(void *p, size_t n) {
        n = align_up(n);
        size_t off = static_cast<char *>(p) - base;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Pool {
    int32_t graph = -1, algo = -1;
    gx_graph *g = nullptr;
    uint32_t B = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *mem = nullptr;
    size_t bytes = 0;
    double t_ready = 0;     // when it last became idle (created, or its epoch ended)
    bool draining = false;  // takes no new queries, so that it empties and its memory can go to a waiting pair
    // SSSP
    uint32_t *D = nullptr;
    BsWork bw{};
    uint32_t *lane_cnt = nullptr;
    // PPR
    BpWork pw{};
    // result staging: a finished lane is copied into a free slot (device, then
    // pinned host memory) on the pool's stream, and the completion thread
    // hands it to the caller once the copy's event has fired, so no copy is
    // waited for while the scheduler holds the lock
    static constexpr int SLOTS = 4;
    uint32_t *stage[SLOTS] = {};
    uint32_t *host_stage[SLOTS] = {};  // pinned, V words each
    hipEvent_t stage_ev[SLOTS] = {};
    bool stage_busy[SLOTS] = {};
    int pending = 0;                   // copies handed to the completion thread, not yet delivered
    uint32_t *host_cnt = nullptr;      // pinned: SSSP epoch x B activation counts; PPR seeds and ends
    size_t stage_bytes = 0, cnt_bytes = 0;
    std::vector<int64_t> lane_q;     // query id per lane, -1 = free
    std::vector<int64_t> lane_age;   // supersteps since the lane joined
    std::vector<int64_t> lane_done;  // finished, waiting for a staging slot: supersteps it took (-1 = running)
    std::vector<int32_t> seeds;      // PPR seed per lane (-1 = free)
    std::vector<uint32_t> ends;      // PPR: first superstep the lane no longer runs (mod 2^32)
    uint32_t k = 0;                  // supersteps run (buffer parity)
    bool in_flight = false;
    uint32_t epoch_len = 0;
    int occupied() const {
        int n = 0;
        for (auto q : lane_q) n += q >= 0;
        return n;
    }
};

size_t pool_bytes(const gx_graph *g, int32_t algo, uint32_t B, uint32_t epoch_max) {
    Carver c(nullptr, 0);
    const DevGraph &d = g->d;
    if (algo == GX_SSSP) {
        c.take<uint32_t>((size_t)d.V * B);
        BsWork w;
        bs_layout(d, B, c, &w);
        c.take<uint32_t>((size_t)epoch_max * B);
    } else {
        BpWork w;
        bp_layout(d, B, c, &w);
    }
    for (int i = 0; i < Pool::SLOTS; i++) c.take<uint32_t>(d.V);
    return c.used;
}

struct Delivery {  // a result on its way to the caller
    Pool *pool;
    int slot;
    gx_query_result r;
    void *result;
    int64_t V;
};

}  // namespace

struct gx_server {
    gx_server_config cfg{};
    ArenaAlloc arena;
    std::vector<gx_graph *> graphs;
    std::vector<std::unique_ptr<Pool>> pools;
    std::deque<SQuery> queue;
    std::map<int64_t, SQuery> running;
    std::vector<gx_query_result> completed;
    // Pinned host buffers of pools that went away, by size, for the next
    // pools (allocating pinned memory costs milliseconds, paid under the
    // scheduler's lock); at most PINNED_KEEP bytes are kept.
    static constexpr size_t PINNED_KEEP = size_t(1) << 30;
    std::multimap<size_t, void *> pinned_free;
    size_t pinned_kept = 0;
    void *pinned_take(size_t bytes) {
        auto it = pinned_free.find(bytes);
        if (it != pinned_free.end()) {
            void *p = it->second;
            pinned_free.erase(it);
            pinned_kept -= bytes;
            return p;
        }
        void *p = nullptr;
        return hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess ? p : nullptr;
    }
    void pinned_give(void *p, size_t bytes) {
        if (!p) return;
        if (pinned_kept + bytes > PINNED_KEEP) {
            (void)hipHostFree(p);
            return;
        }
        pinned_free.emplace(bytes, p);
        pinned_kept += bytes;
    }

    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_deliver;
    std::thread worker, deliverer;
    std::deque<Delivery> deliveries;
    bool stop = false, stop_delivery = false;
    int64_t next_id = 1;
    std::string fatal;
    int grid = 0;
    // the one pair that may carve a new pool while the arena has no room
    // for it; pools chosen to make room for it drain meanwhile
    bool reserved = false;
    int32_t res_graph = -1, res_algo = -1;
    size_t res_off = 0, res_len = 0;  // the stretch drained for it (other pools stay out)

    ~gx_server() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_work.notify_all();
        if (worker.joinable()) worker.join();
        {
            std::lock_guard<std::mutex> lk(mu);
            stop_delivery = true;
        }
        cv_deliver.notify_all();
        if (deliverer.joinable()) deliverer.join();
        for (auto &p : pools) destroy_pool(*p, false);
        for (auto &f : pinned_free) (void)hipHostFree(f.second);
    }

    // Completion thread: waits for each staged copy, copies it into the
    // caller's buffer and publishes the result.
    void deliver() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            cv_deliver.wait(lk, [this] { return stop_delivery || !deliveries.empty(); });
            if (deliveries.empty()) break;
            Delivery dv = deliveries.front();
            deliveries.pop_front();
            lk.unlock();
            hipError_t e = hipEventSynchronize(dv.pool->stage_ev[dv.slot]);
            if (e == hipSuccess) std::memcpy(dv.result, dv.pool->host_stage[dv.slot], (size_t)dv.V * 4);
            dv.r.done_s = now_s();
            if (e != hipSuccess) dv.r.status = GX_EDEVICE;
            lk.lock();
            dv.pool->stage_busy[dv.slot] = false;
            dv.pool->pending--;
            completed.push_back(dv.r);
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }

    void destroy_pool(Pool &p, bool give_back) {
        if (p.stream) (void)hipStreamSynchronize(p.stream);
        if (p.done) (void)hipEventDestroy(p.done);
        for (int i = 0; i < Pool::SLOTS; i++) {
            if (p.stage_ev[i]) (void)hipEventDestroy(p.stage_ev[i]);
            pinned_give(p.host_stage[i], p.stage_bytes);
            p.stage_ev[i] = nullptr;
            p.host_stage[i] = nullptr;
        }
        if (p.stream) (void)hipStreamDestroy(p.stream);
        pinned_give(p.host_cnt, p.cnt_bytes);
        if (give_back && p.mem) arena.release(p.mem, p.bytes);
        p.stream = nullptr;
        p.done = nullptr;
        p.host_cnt = nullptr;
        p.mem = nullptr;
    }

    uint32_t epoch_max(int32_t algo) const { return algo == GX_SSSP ? cfg.sssp_epoch_supersteps : cfg.epoch_supersteps; }

    // Creates a pool for (graph, algo) inside the budget; nullptr if it does not fit.
    // (skip: keep out of the stretch drained for another pair's reservation)
    Pool *create_pool(int32_t graph, int32_t algo, uint32_t B, bool skip = false) {
        gx_graph *g = graphs[graph];
        size_t bytes = pool_bytes(g, algo, B, epoch_max(algo));
        const size_t so = skip ? res_off : 0, sl = skip ? res_len : 0;
        void *mem = arena.alloc(bytes, so, sl);
        if (!mem) {  // evict idle empty pools, then retry
            for (size_t i = 0; i < pools.size();) {
                Pool &p = *pools[i];
                if (!p.in_flight && p.occupied() == 0 && p.pending == 0) {
                    destroy_pool(p, true);
                    pools.erase(pools.begin() + i);
                } else {
                    i++;
                }
            }
            mem = arena.alloc(bytes, so, sl);
            if (!mem) return nullptr;
        }
        auto p = std::make_unique<Pool>();
        p->graph = graph;
        p->algo = algo;
        p->g = g;
        p->B = B;
        p->mem = mem;
        p->bytes = bytes;
        p->t_ready = now_s();
        p->lane_q.assign(B, -1);
        p->lane_age.assign(B, 0);
        p->lane_done.assign(B, -1);
        p->seeds.assign(B, -1);
        p->ends.assign(B, 0u);
        const DevGraph &d = g->d;
        Carver c(mem, bytes);
        p->cnt_bytes = std::max<size_t>((size_t)epoch_max(algo), 2) * B * 4;
        p->stage_bytes = std::max<size_t>(4, d.V * 4);
        bool ok = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&p->done, hipEventDisableTiming) == hipSuccess &&
                  (p->host_cnt = static_cast<uint32_t *>(pinned_take(p->cnt_bytes))) != nullptr;
        for (int i = 0; i < Pool::SLOTS && ok; i++)
            ok = hipEventCreateWithFlags(&p->stage_ev[i], hipEventDisableTiming) == hipSuccess &&
                 (p->host_stage[i] = static_cast<uint32_t *>(pinned_take(p->stage_bytes))) != nullptr;
        if (algo == GX_SSSP) {
            p->D = c.take<uint32_t>((size_t)d.V * B);
            bs_layout(d, B, c, &p->bw);
            p->lane_cnt = c.take<uint32_t>((size_t)epoch_max(algo) * B);
        } else {
            bp_layout(d, B, c, &p->pw);
        }
        for (int i = 0; i < Pool::SLOTS; i++) p->stage[i] = c.take<uint32_t>(d.V);
        if (ok) {
            hipStream_t s = p->stream;
            if (algo == GX_SSSP) {
                const size_t VG = (size_t)d.V * (B / 32);
                ok = hipMemsetAsync(p->D, 0xFF, (size_t)d.V * B * 4, s) == hipSuccess &&
                     hipMemsetAsync(p->bw.M[0], 0, VG * 4, s) == hipSuccess &&
                     hipMemsetAsync(p->bw.M[1], 0, VG * 4, s) == hipSuccess &&
                     hipMemsetAsync(p->bw.ctl, 0, sizeof(BsCtl), s) == hipSuccess;
            } else {
                const size_t n = (size_t)d.V * B * 4;
                ok = hipMemsetAsync(p->pw.x[0], 0, n, s) == hipSuccess &&
                     hipMemsetAsync(p->pw.x[1], 0, n, s) == hipSuccess &&
                     hipMemsetAsync(p->pw.c[0], 0, n, s) == hipSuccess &&
                     hipMemsetAsync(p->pw.c[1], 0, n, s) == hipSuccess &&
                     hipMemsetAsync(p->pw.D[0], 0, B * 8, s) == hipSuccess &&
                     hipMemsetAsync(p->pw.D[1], 0, B * 8, s) == hipSuccess &&
                     hipMemsetAsync(p->pw.seed, 0xFF, B * 4, s) == hipSuccess &&
                     bp_make_tiles(d.in_rp, d.V, p->pw.ntiles, p->pw.trow, s) == hipSuccess;
            }
            ok = ok && hipStreamSynchronize(s) == hipSuccess;
        }
        if (!ok) {
            destroy_pool(*p, true);
            fatal = "pool creation failed (HIP error)";
            return nullptr;
        }
        pools.push_back(std::move(p));
        return pools.back().get();
    }

    BsArgs bs_args(Pool &p) {
        const DevGraph &d = p.g->d;
        BsArgs a{};
        a.rp = d.out_rp;
        a.adj = d.out_adj;
        a.V = d.V;
        a.B = p.B;
        a.l0 = 0;
        a.G = p.B / 32;
        a.D = p.D;
        a.M[0] = p.bw.M[0];
        a.M[1] = p.bw.M[1];
        a.list = p.bw.list;
        a.S = p.bw.S;
        a.tile_start = p.bw.tile_start;
        a.ctl = p.bw.ctl;
        a.max_steps = 1;
        a.lane_cnt = p.lane_cnt;
        a.stop_when_idle = 0;
        return a;
    }

    BpArgs bp_args(Pool &p) {
        const DevGraph &d = p.g->d;
        BpArgs a{};
        a.in_rp = d.in_rp;
        a.in_col = d.in_col;
        a.outdeg = d.outdeg;
        a.trow = p.pw.trow;
        a.ntiles = p.pw.ntiles;
        a.V = d.V;
        a.E = d.E;
        a.B = p.B;
        a.Bw = p.B;
        a.d = cfg.damping;
        a.seed = p.pw.seed;
        a.end = p.pw.end;
        a.x[0] = p.pw.x[0];
        a.x[1] = p.pw.x[1];
        a.c[0] = p.pw.c[0];
        a.c[1] = p.pw.c[1];
        a.head = p.pw.head;
        a.tailp = p.pw.tailp;
        a.dsum = p.pw.dsum;
        a.dpart = p.pw.dpart;
        a.D[0] = p.pw.D[0];
        a.D[1] = p.pw.D[1];
        a.spill = p.pw.spill;
        return a;
    }

    bool admit(Pool &p, SQuery &q, uint32_t lane) {
        const DevGraph &d = p.g->d;
        hipError_t e;
        if (p.algo == GX_SSSP) {
            e = bs_lane_reset(p.D, p.bw.M[p.k & 1], p.bw.M[(p.k + 1) & 1], d.V, p.B, p.B / 32, lane, q.source,
                              p.stream);
        } else {
            // the lane runs supersteps k .. k + iterations - 1; its seed and end
            // reach the device with the next epoch's lane table
            p.seeds[lane] = q.source;
            p.ends[lane] = p.k + (uint32_t)cfg.ppr_iters;
            e = bp_lane_reset(p.pw.x[p.k & 1], p.pw.c[p.k & 1], p.pw.D[p.k & 1], d.outdeg, d.V, p.B, lane, q.source,
                              p.stream);
        }
        if (e != hipSuccess) return false;
        p.lane_q[lane] = q.id;
        p.lane_age[lane] = 0;
        q.t_start = now_s();
        running[q.id] = q;
        return true;
    }

    // A finished lane's column goes to a free staging slot on the pool's
    // stream (later work on the stream is ordered after the copy, so the lane
    // is free at once); without a free slot the lane waits, finished, for the
    // next pass of the scheduler (it changes no more: an SSSP lane that
    // activated nothing stays idle, a PPR lane past its end is frozen).
    bool retire(Pool &p, uint32_t lane, int64_t steps) {
        const DevGraph &d = p.g->d;
        auto it = running.find(p.lane_q[lane]);
        if (it == running.end()) return true;
        int slot = -1;
        for (int i = 0; i < Pool::SLOTS; i++)
            if (!p.stage_busy[i]) {
                slot = i;
                break;
            }
        if (slot < 0) {
            p.lane_done[lane] = steps;
            return false;
        }
        SQuery &q = it->second;
        // a PPR lane froze after its last superstep: its values are in x[end & 1]
        const uint32_t *tile =
            p.algo == GX_SSSP ? p.D : reinterpret_cast<const uint32_t *>(p.pw.x[p.ends[lane] & 1]);
        hipError_t e = lane_extract(tile, d.V, p.B, lane, p.stage[slot], p.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(p.host_stage[slot], p.stage[slot], d.V * 4, hipMemcpyDeviceToHost, p.stream);
        if (e == hipSuccess) e = hipEventRecord(p.stage_ev[slot], p.stream);
        q.status = e == hipSuccess ? GX_OK : GX_EDEVICE;
        q.steps = steps;
        Delivery dv{&p, slot, {q.id, q.graph, q.algo, q.source, q.status, q.t_submit, q.t_start, 0.0, q.steps},
                    q.result, d.V};
        if (e != hipSuccess) {  // nothing in flight for this slot: publish the failure now
            dv.r.done_s = now_s();
            completed.push_back(dv.r);
            cv_done.notify_all();
        } else {
            p.stage_busy[slot] = true;
            p.pending++;
            deliveries.push_back(dv);
            cv_deliver.notify_all();
        }
        running.erase(it);
        p.lane_q[lane] = -1;
        p.seeds[lane] = -1;
        p.lane_done[lane] = -1;
        return true;
    }

    void retire_waiting() {
        for (auto &pp : pools) {
            Pool &p = *pp;
            if (p.in_flight) continue;
            for (uint32_t b = 0; b < p.B; b++)
                if (p.lane_q[b] >= 0 && p.lane_done[b] >= 0 && !retire(p, b, p.lane_done[b])) break;
        }
    }

    void finish_epoch(Pool &p) {
        p.in_flight = false;
        p.t_ready = now_s();
        const uint32_t B = p.B;
        if (p.algo == GX_SSSP) {
            for (uint32_t b = 0; b < B; b++) {
                if (p.lane_q[b] < 0 || p.lane_done[b] >= 0) continue;
                int64_t conv = -1;
                for (uint32_t it = 0; it < p.epoch_len; it++)
                    if (p.host_cnt[(size_t)it * B + b] == 0) {
                        conv = it;
                        break;
                    }
                if (conv >= 0) {
                    retire(p, b, p.lane_age[b] + conv + 1);
                } else {
                    p.lane_age[b] += p.epoch_len;
                }
            }
        } else {
            for (uint32_t b = 0; b < B; b++) {
                if (p.lane_q[b] < 0 || p.lane_done[b] >= 0) continue;
                p.lane_age[b] += p.epoch_len;
                if ((int32_t)(p.ends[b] - p.k) <= 0) retire(p, b, (int64_t)cfg.ppr_iters);
            }
        }
    }

    bool launch_epoch(Pool &p) {
        if (p.algo == GX_SSSP) {
            p.epoch_len = epoch_max(GX_SSSP);
            if (hipMemsetAsync(p.lane_cnt, 0, (size_t)p.epoch_len * p.B * 4, p.stream) != hipSuccess) return false;
            BsArgs a = bs_args(p);
            for (uint32_t it = 0; it < p.epoch_len; it++)
                if (bs_launch_superstep(a, p.k + it, it, grid, p.stream) != hipSuccess) return false;
            if (hipMemcpyAsync(p.host_cnt, p.lane_cnt, (size_t)p.epoch_len * p.B * 4, hipMemcpyDeviceToHost,
                               p.stream) != hipSuccess)
                return false;
        } else {
            // Lanes that reach their end inside the epoch freeze on the device;
            // the epoch runs until the last lane's end or the epoch limit.
            int64_t left = 1;
            for (uint32_t b = 0; b < p.B; b++)
                if (p.lane_q[b] >= 0) left = std::max<int64_t>(left, (int32_t)(p.ends[b] - p.k));
            p.epoch_len = (uint32_t)std::min<int64_t>(left, epoch_max(GX_PPR));
            int32_t *lt = reinterpret_cast<int32_t *>(p.host_cnt);  // idle pool: the last epoch's copies are done
            for (uint32_t b = 0; b < p.B; b++) {
                lt[b] = p.lane_q[b] >= 0 ? p.seeds[b] : -1;
                lt[p.B + b] = (int32_t)p.ends[b];
            }
            if (hipMemcpyAsync(p.pw.seed, lt, (size_t)p.B * 8, hipMemcpyHostToDevice, p.stream) != hipSuccess)
                return false;
            BpArgs a = bp_args(p);
            // only the occupied prefix of lanes (lowest free lanes are taken first)
            uint32_t hi = 0;
            for (uint32_t b = 0; b < p.B; b++)
                if (p.lane_q[b] >= 0) hi = b + 1;
            a.Bw = std::min<uint32_t>(p.B, (hi + 15) / 16 * 16);
            for (uint32_t it = 0; it < p.epoch_len; it++)
                if (bp_launch_superstep(a, p.k + it, grid, p.stream) != hipSuccess) return false;
        }
        p.k += p.epoch_len;
        if (hipEventRecord(p.done, p.stream) != hipSuccess) return false;
        p.in_flight = true;
        return true;
    }

    // Lanes for a new pool of a pair: enough for the pair's waiting queries,
    // in multiples of 32, at most lanes_per_pool (a pair with steady demand
    // adds pools; one with little demand holds little memory).
    uint32_t pool_lanes(int32_t graph, int32_t algo) const {
        uint32_t n = 0;
        for (auto &q : queue) n += q.graph == graph && q.algo == algo;
        return std::min<uint32_t>(cfg.lanes_per_pool, std::max<uint32_t>(32, (n + 31) / 32 * 32));
    }

    // Picks the contiguous stretch of the arena, made of free ranges and
    // pools, that can hold `need` bytes at the least cost (lanes running
    // plus queries waiting for the pools it covers) and drains its pools.
    void plan_room(size_t need) {
        struct Seg {
            size_t off, len;
            int64_t cost;
            Pool *pool;
        };
        std::vector<Seg> seg;
        for (auto &f : arena.free_) seg.push_back({f.first, f.second, 0, nullptr});
        for (auto &pp : pools) {
            Pool &p = *pp;
            int64_t cost = 0;
            if (!p.draining) {
                cost = p.occupied();
                for (auto &q : queue) cost += q.graph == p.graph && q.algo == p.algo;
            }
            seg.push_back({(size_t)(static_cast<char *>(p.mem) - arena.base), align_up(p.bytes), cost, &p});
        }
        std::sort(seg.begin(), seg.end(), [](const Seg &x, const Seg &y) { return x.off < y.off; });
        size_t best_i = 0, best_j = 0;
        int64_t best_cost = -1;
        for (size_t i = 0; i < seg.size(); i++) {
            size_t len = 0;
            int64_t cost = 0;
            for (size_t j = i; j < seg.size(); j++) {
                if (j > i && seg[j].off != seg[j - 1].off + seg[j - 1].len) break;  // not contiguous
                len += seg[j].len;
                cost += seg[j].cost;
                if (len >= need) {
                    if (best_cost < 0 || cost < best_cost) {
                        best_cost = cost;
                        best_i = i;
                        best_j = j;
                    }
                    break;
                }
            }
        }
        if (best_cost < 0) return;
        res_off = seg[best_i].off;
        res_len = seg[best_j].off + seg[best_j].len - res_off;
        for (size_t j = best_i; j <= best_j; j++)
            if (seg[j].pool) seg[j].pool->draining = true;
    }

    // Admission in arrival order.  A query joins a pool of its (graph,
    // algorithm) that has a free lane, at an epoch boundary (it waits while
    // that pool is mid-epoch).  A pair with no pool gets a new one carved from
    // the arena after evicting pools that are idle and empty.  When even that
    // leaves no room, the pair takes the reservation: the cheapest stretch of
    // the arena that would hold its pool is drained (its pools admit nothing
    // more, finish what they run and are then evicted), and until the
    // reserving pair has its own pool other pairs carve theirs only outside
    // that stretch, so that steady traffic to the resident pairs or small
    // pools filling the holes cannot starve a pair.
    void admit_queued() {
        for (size_t i = 0; i < pools.size();) {  // drained pools leave at once
            Pool &p = *pools[i];
            if (p.draining && !p.in_flight && p.occupied() == 0 && p.pending == 0) {
                destroy_pool(p, true);
                pools.erase(pools.begin() + i);
            } else {
                i++;
            }
        }
        for (size_t i = 0; i < queue.size();) {
            SQuery &q = queue[i];
            Pool *target = nullptr;
            uint32_t lane = 0;
            bool live_pool = false, wait_boundary = false;
            for (auto &pp : pools) {
                Pool &p = *pp;
                if (p.graph != q.graph || p.algo != q.algo || p.draining) continue;
                live_pool = true;
                int free_lane = -1;
                for (uint32_t b = 0; b < p.B; b++)
                    if (p.lane_q[b] < 0) {
                        free_lane = (int)b;
                        break;
                    }
                if (free_lane < 0) continue;
                if (p.in_flight) {
                    wait_boundary = true;
                    continue;
                }
                target = &p;
                lane = (uint32_t)free_lane;
                break;
            }
            bool draining_pool = false;
            for (auto &pp : pools) draining_pool |= pp->graph == q.graph && pp->algo == q.algo && pp->draining;
            const bool mine = reserved && res_graph == q.graph && res_algo == q.algo;
            // a pair whose pools all drain waits for their eviction; while another
            // pair holds the reservation, new pools keep out of its stretch
            if (!target && !wait_boundary && (live_pool || !draining_pool || mine)) {
                const bool skip = reserved && !mine;
                const uint32_t B = pool_lanes(q.graph, q.algo);
                target = create_pool(q.graph, q.algo, B, skip);
                if (!target && B > 32) target = create_pool(q.graph, q.algo, 32, skip);
                if (target && mine) {
                    reserved = false;
                    res_len = 0;
                }
                if (!target && !live_pool && !reserved) {
                    reserved = true;
                    res_graph = q.graph;
                    res_algo = q.algo;
                    res_len = 0;
                    plan_room(align_up(pool_bytes(graphs[q.graph], q.algo, 32, epoch_max(q.algo))));
                }
            }
            if (target && admit(*target, q, lane)) {
                queue.erase(queue.begin() + i);
                continue;
            }
            i++;
        }
    }

    int device = 0;

    void run() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            bool any_flight = false;
            for (auto &pp : pools) {
                Pool &p = *pp;
                if (p.in_flight && hipEventQuery(p.done) == hipSuccess) finish_epoch(p);
            }
            retire_waiting();
            admit_queued();
            // Idle pools launch SSSP first, then in the order they became idle.
            // An SSSP epoch is a few cheap supersteps, a PPR epoch whole-graph
            // pulls, and epochs that share a hardware queue run in order: with
            // few running slots (max_pools near the hardware queue count) the
            // order chosen here is the order the GPU runs them in, so short
            // queries pass long ones instead of queueing behind them.
            int flying = 0;
            std::vector<Pool *> ready;
            for (auto &pp : pools) {
                flying += pp->in_flight;
                if (!pp->in_flight && pp->occupied() > 0) ready.push_back(pp.get());
            }
            std::sort(ready.begin(), ready.end(), [](const Pool *x, const Pool *y) {
                if ((x->algo == GX_SSSP) != (y->algo == GX_SSSP)) return x->algo == GX_SSSP;
                return x->t_ready < y->t_ready;
            });
            for (Pool *p : ready) {
                if (flying >= (int)cfg.max_pools) break;
                if (launch_epoch(*p)) flying++;
                else fatal = "epoch launch failed";
            }
            for (auto &pp : pools) any_flight |= pp->in_flight;
            if (stop && !any_flight) break;
            if (!any_flight && queue.empty()) {
                cv_work.wait_for(lk, std::chrono::milliseconds(5));
            } else {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            }
        }
    }
};

extern "C" gx_status gx_server_bytes_per_lane(const gx_graph *g, int32_t algo, size_t *bytes) {
    clear_error();
    GX_REQUIRE(g && bytes, GX_EINVAL, "NULL argument");
    GX_REQUIRE(algo == GX_SSSP || algo == GX_PPR, GX_EINVAL, "algo must be GX_SSSP or GX_PPR");
    *bytes = (pool_bytes(g, algo, 64, 8) + 63) / 64;
    return GX_OK;
}

extern "C" gx_status gx_server_create(const gx_server_config *cfg, gx_server **out) {
    clear_error();
    GX_REQUIRE(cfg && out, GX_EINVAL, "NULL argument");
    GX_REQUIRE(cfg->dev_arena && cfg->arena_bytes > 0, GX_EINVAL, "server needs a device arena");
    gx_server_config c = *cfg;
    if (c.lanes_per_pool == 0) c.lanes_per_pool = 64;
    if (c.max_pools == 0) c.max_pools = 4;
    if (c.epoch_supersteps == 0) c.epoch_supersteps = 4;
    if (c.sssp_epoch_supersteps == 0) c.sssp_epoch_supersteps = 16;
    if (c.damping == 0.f) c.damping = 0.85f;
    if (c.ppr_iters == 0) c.ppr_iters = 50;
    GX_REQUIRE(c.lanes_per_pool % 32 == 0 && c.lanes_per_pool <= 256, GX_EINVAL,
               "lanes_per_pool must be a multiple of 32 up to 256");
    GX_REQUIRE(c.epoch_supersteps <= 64 && c.sssp_epoch_supersteps <= 64, GX_EINVAL,
               "epoch_supersteps and sssp_epoch_supersteps must be <= 64");
    GX_REQUIRE(c.damping > 0.f && c.damping < 1.f, GX_EINVAL, "damping out of (0,1)");
    gx_server *s = new (std::nothrow) gx_server();
    GX_REQUIRE(s, GX_ENOMEM, "host allocation failed");
    s->cfg = c;
    s->arena.init(c.dev_arena, c.arena_bytes);
    int dev = 0;
    (void)hipGetDevice(&dev);
    s->device = dev;
    s->grid = device_cus(dev) * 2;
    s->worker = std::thread([s] { s->run(); });
    s->deliverer = std::thread([s] { s->deliver(); });
    *out = s;
    return GX_OK;
}

extern "C" gx_status gx_server_add_graph(gx_server *s, gx_graph *g, int32_t *graph_id) {
    clear_error();
    GX_REQUIRE(s && g && graph_id, GX_EINVAL, "NULL argument");
    GX_REQUIRE((g->needs & (GX_NEED_OUT | GX_NEED_IN)) == (GX_NEED_OUT | GX_NEED_IN), GX_EINVAL,
               "serving needs graphs loaded with GX_NEED_OUT | GX_NEED_IN");
    std::lock_guard<std::mutex> lk(s->mu);
    s->graphs.push_back(g);
    *graph_id = (int32_t)s->graphs.size() - 1;
    return GX_OK;
}

extern "C" gx_status gx_server_submit(gx_server *s, int32_t graph_id, int32_t algo, int32_t source, void *result,
                                      int64_t *id) {
    clear_error();
    GX_REQUIRE(s && result && id, GX_EINVAL, "NULL argument");
    GX_REQUIRE(algo == GX_SSSP || algo == GX_PPR, GX_EINVAL, "algo must be GX_SSSP or GX_PPR");
    std::lock_guard<std::mutex> lk(s->mu);
    GX_REQUIRE(graph_id >= 0 && graph_id < (int32_t)s->graphs.size(), GX_ENOTFOUND, "unknown graph %d", graph_id);
    gx_graph *g = s->graphs[graph_id];
    GX_REQUIRE(source >= 0 && source < g->d.V, GX_EINVAL, "source %d out of [0,V)", source);
    const size_t need = align_up(pool_bytes(g, algo, 32, algo == GX_SSSP ? s->cfg.sssp_epoch_supersteps
                                                                        : s->cfg.epoch_supersteps));
    GX_REQUIRE(need <= s->arena.cap, GX_ENOMEM, "a 32-lane pool needs %zu bytes, the budget is %zu", need,
               s->arena.cap);
    GX_REQUIRE(s->fatal.empty(), GX_EDEVICE, "server failed: %s", s->fatal.c_str());
    SQuery q;
    q.id = s->next_id++;
    q.graph = graph_id;
    q.algo = algo;
    q.source = source;
    q.result = result;
    q.t_submit = now_s();
    s->queue.push_back(q);
    *id = q.id;
    s->cv_work.notify_all();
    return GX_OK;
}

extern "C" gx_status gx_server_poll(gx_server *s, gx_query_result *out, uint32_t cap, uint32_t *n, int32_t wait_ms) {
    clear_error();
    GX_REQUIRE(s && n && (out || cap == 0), GX_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->completed.empty() && wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [s] { return !s->completed.empty(); });
    uint32_t m = (uint32_t)std::min<size_t>(cap, s->completed.size());
    for (uint32_t i = 0; i < m; i++) out[i] = s->completed[i];
    s->completed.erase(s->completed.begin(), s->completed.begin() + m);
    *n = m;
    GX_REQUIRE(s->fatal.empty(), GX_EDEVICE, "server failed: %s", s->fatal.c_str());
    return GX_OK;
}

extern "C" gx_status gx_server_pending(gx_server *s, int64_t *n) {
    clear_error();
    GX_REQUIRE(s && n, GX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *n = (int64_t)(s->queue.size() + s->running.size() + s->deliveries.size());
    return GX_OK;
}

extern "C" gx_status gx_server_destroy(gx_server *s) {
    clear_error();
    delete s;
    return GX_OK;
}
