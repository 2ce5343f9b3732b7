// Internal declarations of the gx engine (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "gx.h"

namespace gx {

constexpr uint32_t INF = 0xFFFFFFFFu;
constexpr size_t ALIGN = 256;

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
void clear_error();

#define GX_CHECK_HIP(expr, handle)                                                       \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess) {                                                          \
            ::gx::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e),        \
                            __FILE__, __LINE__);                                         \
            if (handle) (handle)->dev_error = true;                                      \
            return GX_EDEVICE;                                                           \
        }                                                                                \
    } while (0)

#define GX_REQUIRE(cond, code, ...)        \
    do {                                   \
        if (!(cond)) {                     \
            ::gx::set_error(__VA_ARGS__);  \
            return (code);                 \
        }                                  \
    } while (0)

inline size_t align_up(size_t x, size_t a = ALIGN) { return (x + a - 1) / a * a; }

// Bump allocator over a caller-owned device arena.
struct Carver {
    char *base;
    size_t cap, used = 0;
    bool measure_only;
    Carver(void *b, size_t c) : base(static_cast<char *>(b)), cap(c), measure_only(b == nullptr) {}
    template <class T>
    T *take(size_t count) {
        size_t off = used;
        used = align_up(used + count * sizeof(T) + (count == 0 ? 1 : 0));
        return measure_only ? nullptr : reinterpret_cast<T *>(base + off);
    }
    bool fits() const { return used <= cap; }
};

// ---------------------------------------------------------------- graph
// Edge tile of the PageRank pull (in-edges per workgroup tile): PR_BLOCK
// threads times 1, 2, 4 or 8 edges, chosen per graph at load.
constexpr int PR_BLOCK = 256;
// Contribution slots of the hottest sources, contiguous at the front: 2 MiB
// of fp32, which a workgroup's L2 keeps while the in-edges stream past (on
// R-MAT graphs they are the sources of about 70% of the in-edges).
constexpr int64_t PR_HOT = int64_t(1) << 19;
constexpr int PR_TILE_MAX = PR_BLOCK * 8;
// Records of the SSSP / CC pull.  Destinations are dealt to PULL_SLICES
// slices in blocks of 2^PULL_SLICE_SHIFT vertices, balanced by in-edge
// count; a slice is a sequence of bins of at most PULL_BIN_BYTES of
// destination values; a bin's records are grouped by source band
// (source >> PULL_BAND_BITS) and ordered by (destination, source) inside a
// group.  Groups are padded to whole PULL_VT records with sentinels and cut
// into work units of at most PULL_UNIT records.  The workgroups of a pull
// take the units of the slice of the XCD they run on (slice x belongs to XCD
// x of the 8), so each XCD's L2 holds one bin's destination values, and a
// unit's band of source snapshots (PULL_BAND words) is staged in LDS.
constexpr int PULL_SLICES = 8;
constexpr int PULL_SLICE_SHIFT = 6;
constexpr int64_t PULL_BIN_BYTES = int64_t(2) << 20;  // destination values an XCD sweeps at a time
constexpr int PULL_BAND_BITS = 13;  // 8192 sources: 32 KB of snapshots in LDS
constexpr int PULL_BAND = 1 << PULL_BAND_BITS;
constexpr int PULL_VT = 8;       // records per thread and group padding
constexpr int PULL_UNIT = 8192;  // records per work unit at most (a multiple of PULL_VT)
constexpr uint32_t PULL_SENTINEL = 0xFFFFFFFFu;  // destination of a padding record
struct PullSlices {
    int64_t uoff[PULL_SLICES + 1];  // slice x owns work units uoff[x] .. uoff[x+1]-1
};
// Capacity of the record array and of the unit table (upper bounds, known
// before the layout is built).
inline int64_t pull_bins(int64_t V) {
    return PULL_SLICES *
           std::max<int64_t>(1, (V * 4 + PULL_SLICES * PULL_BIN_BYTES - 1) / (PULL_SLICES * PULL_BIN_BYTES));
}
inline int64_t pull_groups(int64_t V) { return pull_bins(V) * ((V >> PULL_BAND_BITS) + 1); }
inline int64_t pull_rec_cap(int64_t V, int64_t E) { return E + (PULL_VT - 1) * pull_groups(V) + PULL_VT; }
inline int64_t pull_unit_cap(int64_t V, int64_t E) { return pull_rec_cap(V, E) / PULL_UNIT + pull_groups(V) + 1; }

// Label propagation: vertices are grouped by the number of distinct
// neighbours d.  Classes 0..4 take d <= 4, 8, 16, 32, 64 and run as lane
// groups of that width; class 5 (d <= LP_MID_MAX) runs one workgroup per
// vertex with a hash table of labels in LDS; class 6 (hubs) counts in hash
// tables in device memory, cut into chunks of LP_HUB_CHUNK neighbours.
constexpr int LP_CLASSES = 7;
constexpr int LP_MID_MAX = 2048;
constexpr int LP_MID_SLOTS = 4096;   // LDS table of the mid class (load at most 1/2)
constexpr int LP_HUB_CHUNK = 8192;
constexpr uint32_t LP_NONE = 0xFFFFFFFFu;

struct DevGraph {
    int64_t V = 0, E = 0, E_sym = 0;
    int32_t W = 0;                 // bitmap words: ceil(V / 32)
    // out-CSR (SSSP push): row_ptr + interleaved (dst, weight)
    const int32_t *out_rp = nullptr;
    const uint2 *out_adj = nullptr;
    // in-CSR: sources only (PageRank pull) and interleaved (source, weight)
    // (SSSP pull); out-degree; equal in-edge tiles shared by both pulls
    const int32_t *in_rp = nullptr;
    const int32_t *in_col = nullptr;
    const int32_t *outdeg = nullptr;
    // PageRank contributions live in slots: the PR_HOT sources with the most
    // out-edges first (by out-degree, then id), every other vertex after them
    // in id order.  pr_src = the slot of each in-edge's source, pr_slot = the
    // slot of each vertex.
    const int32_t *pr_src = nullptr;
    const int32_t *pr_slot = nullptr;
    int32_t pr_tile = PR_TILE_MAX;  // in-edges per PageRank tile
    int32_t pr_ntiles = 0;
    const int32_t *pr_tile_row = nullptr;  // [pr_ntiles + 1]
    // sliced, banded in-edge records for the SSSP pull:
    // {dst, (src mod PULL_BAND) << 8 | w} (padded to whole PULL_VT groups);
    // null when a weight exceeds 255 (the engine then only pushes)
    const uint2 *pull_w = nullptr;
    const uint4 *pull_w_units = nullptr;  // {first record, records, band base, 0}
    PullSlices pull_w_off{};
    // symmetric adjacency (CC push and pull) and its equal edge tiles
    const int32_t *sym_rp = nullptr;
    const int32_t *sym_col = nullptr;
    // sliced, banded symmetric records for the CC pull: {dst, src}
    const uint2 *pull_sym = nullptr;
    const uint4 *pull_sym_units = nullptr;
    PullSlices pull_sym_off{};
    // partition metadata
    const int32_t *l2g = nullptr;          // nullptr = identity
    const uint32_t *remote_out = nullptr;  // bitmaps of W words (nullptr = none remote)
    const uint32_t *remote_any = nullptr;
    const uint32_t *master = nullptr;      // this part holds the master copy
    const uint32_t *master_rep = nullptr;  // ... of a vertex another part holds a replica of
    // PageRank exchanged between the parts: out-degrees in the whole graph
    const int32_t *outdeg_g = nullptr;
    int64_t V_global = 0;
};

}  // namespace gx

struct gx_graph {
    gx::DevGraph d;
    uint32_t needs = 0;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    int device = 0;
    int num_cus = 0;
    bool dev_error = false;
    std::vector<int32_t> host_outdeg;  // out-degree (host copy, for sources and stats)
    std::vector<int32_t> host_symdeg;  // distinct neighbours (with GX_NEED_SYM; label propagation classes)
    std::vector<uint32_t> pull_w_recs, pull_sym_recs;  // records of each pull unit (sizes fix-up regions)
    // supersteps of the last converged SSSP / CC run on this graph: the size
    // of the next run's first speculative group (solves on one graph tend to
    // need similar superstep counts)
    std::atomic<uint32_t> last_supersteps[2] = {0u, 0u};
    // PageRank runs replayed as HIP graphs: n supersteps from ring slot `slot`
    // (which also fixes the buffer parity) of a state laid out in `mem` with
    // damping `damping`; a state re-created in the same memory finds its graph
    // again.  Captured on `cap_stream`; the oldest entry goes past PR_GRAPHS.
    struct PrGraph {
        const void *mem;
        double damping;
        int64_t slot;
        uint32_t n;
        hipGraphExec_t exec;
    };
    static constexpr size_t PR_GRAPHS = 8;
    std::mutex pr_mu;
    std::vector<PrGraph> pr_graphs;
    hipStream_t cap_stream = nullptr;
    ~gx_graph() {
        for (auto &e : pr_graphs) (void)hipGraphExecDestroy(e.exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace gx {

// Host-side build + upload of the device images (gx_graph.hip).
gx_status graph_layout(const gx_graph_desc *desc, Carver &c, DevGraph *d);

// Per-superstep statistics slot kept in device memory.
// The compaction's workgroups each add to `list` and to `frontier`; adds to
// one address serialise, so the two counters live on different 128-byte
// lines and do not queue behind each other.
struct DevStep {
    unsigned long long list;      // (entries << 32) | edges, via one 64-bit add per workgroup
    unsigned long long changed;   // PageRank changed values
    unsigned long long pad;       // 1 when the superstep pulled
    unsigned long long rot_mixed; // pull: 1 when its workgroups saw different XCD rotations
    unsigned long long spare0[12];
    unsigned long long frontier;  // |F_k|
    unsigned long long spare1[15];
};
static_assert(sizeof(DevStep) == 256, "DevStep spans two 128-byte lines");
constexpr int STEP_RING = 4096;

// Tiles of the push relaxation (active out-edges per workgroup tile).
constexpr int PUSH_BLOCK = 256;
constexpr int PUSH_VT = 8;
constexpr int PUSH_TILE = PUSH_BLOCK * PUSH_VT;

int device_cus(int device);

// Workgroups per CU the occupancy query reports for (kernel, block size) on
// the current device; cached, because the query is slow.
int occupancy_per_cu(const void *kernel, int block);

}  // namespace gx

// Engine state of one algorithm run on a graph (gx_plain.hip, gx_lp.hip).
struct gx_state {
    gx_graph *g = nullptr;
    gx_params p{};
    int64_t k = 0;
    bool dev_error = false;
    int relax_grid = 0;   // persistent grid of the relaxation kernel
    uint32_t xcd_shift = 0;  // added to the XCD a workgroup is expected on (non-zero only to exercise the check)
    uint2 *fix = nullptr;         // fix-up regions, fix_cap entries per relaxation workgroup
    uint32_t *fixn = nullptr;     // entries recorded per workgroup
    uint32_t fix_cap = 0;
    // SSSP / CC
    uint32_t *val = nullptr;
    uint8_t *front8[2] = {nullptr, nullptr};  // frontier byte maps: A_k lives in front8[k & 1]
    uint8_t *dirty8 = nullptr;                // changed since the last sync (byte per vertex)
    uint4 *list = nullptr;
    uint32_t *tile_start = nullptr;
    uint32_t *snap = nullptr;      // start-of-superstep values of active vertices (pull)
    uint32_t pull_edges = 0xFFFFFFFFu;
    // PageRank
    float *x[2] = {nullptr, nullptr};
    float *contrib[2] = {nullptr, nullptr};
    uint32_t *synced = nullptr;
    double *head = nullptr, *tailp = nullptr;
    int32_t *spill_row = nullptr;
    double *dpart = nullptr;
    uint32_t *cpart = nullptr;   // per-tile changed counts (PageRank)
    double *Dval = nullptr;
    int pr_fix_grid = 1;              // workgroups of k_pr_fix
    double *fix_d = nullptr;          // their dangling-mass partials
    unsigned long long *fix_c = nullptr;  // and changed counts
    uint32_t *fix_done = nullptr;     // workgroups finished (the last resets it)
    void *mem = nullptr;              // the caller's state buffer (keys the graph's replay cache)
    // label propagation: lab[k & 1] holds the labels at the start of superstep k
    uint32_t *lab[2] = {nullptr, nullptr};
    uint32_t *lp_list = nullptr;              // vertices with neighbours, grouped by degree class
    int64_t lp_off[gx::LP_CLASSES + 1] = {};  // class c owns lp_list[lp_off[c] .. lp_off[c + 1])
    uint4 *lp_chunks = nullptr;               // hub edge chunks {hub index, first entry, end entry, 0}
    int64_t lp_nchunks = 0;
    uint2 *lp_hub = nullptr;                  // per hub {first table slot, slots (a power of two)}
    uint2 *lp_tab = nullptr;                  // hub tables {label, count}; label LP_NONE = free
    int64_t lp_tab_slots = 0;
    // separate template calls (gx_params.phases): merged messages per vertex,
    // the index of the pending map in front8, and what is waiting
    uint32_t *acc = nullptr;         // SSSP / CC: min of the merged messages (INF = none)
    double *acc_d = nullptr;         // PageRank: sum of the merged messages
    uint8_t *junk8 = nullptr;        // marks the relaxation makes against the accumulator (never read)
    double *Dscratch = nullptr;      // dangling-mass slot the merge's fix-up writes (never read)
    gx::DevStep *ph_steps = nullptr; // counter slots the merge's fix-up writes (never read)
    int ph_p = 0;                    // front8[ph_p] collects the vertices the next MSGGen sends from
    double D_host = 0.0;             // staging of gx_dangling_set (lives as long as the state)
    bool ph_msgs = false, ph_merged = false;
    // shared
    gx::DevStep *steps = nullptr;
    uint32_t *blk_cnt = nullptr;
    uint32_t *delta_total = nullptr;
    int delta_blocks = 0;
    // edge-kernel timing
    std::vector<hipEvent_t> ev_pool;
    struct Pending {
        int64_t k;
        hipEvent_t a, b;
    };
    std::vector<Pending> ev_pending;
    double kernel_ms = 0;
    int64_t kernel_launches = 0;
    gx::DevStep *host_steps = nullptr;  // pinned, HOST_STEPS entries (from a process-wide pool)
    ~gx_state();
};

namespace gx {
// Label propagation (gx_lp.hip): state layout (also sizes the arena with a
// measuring Carver), initialisation (synchronises `hs`), one superstep.
size_t lp_layout(gx_graph *g, Carver &c, gx_state *s);
gx_status lp_init(gx_state *s, hipStream_t hs);
void lp_enqueue(gx_state *s, hipStream_t hs, DevStep *step, DevStep *next);
int64_t lp_active(const gx_state *s);
}  // namespace gx
