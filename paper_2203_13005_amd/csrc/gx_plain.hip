// One worker's superstep engine: PageRank (pull), Bellman-Ford SSSP and
// min-label CC (frontier push), the lazy-upload sync set, and iteration
// control.
//
// A superstep is the algorithm template MSGGen -> MSGMerge -> MSGApply of
// Section "Algorithm Template", in BSP order.  Messages of one superstep
// are generated from the state at its start (no dependency between the
// edge triplets of one iteration, Section "Pipeline Shuffling"), so the
// frontier compaction stores a snapshot of every active vertex's value.
//
// SSSP / CC superstep k (A_k = vertices active in superstep k), one
// launch of k_relax that runs one of two forms:
//   push      : every workgroup tile relaxes exactly PUSH_TILE active
//               out-edges: Gen = snapshot (+ weight), Merge + Apply =
//               integer atomicMin on the destination, filtered by a plain
//               read; a candidate that passes marks the destination in the
//               next frontier (a plain, idempotent byte store; the next
//               compaction carries the marks into the dirty map).
//   pull      : for large frontiers instead: one streaming sweep over all
//               in-edge records, grouped by source band so the gathered
//               snapshots are staged in LDS, 64 consecutive records per
//               wave; improving candidates are stored plainly and recorded,
//               and k_fixup re-applies the ones a racing store overwrote.
//               The device picks push or pull from the frontier's out-edge
//               count; no host round trip.
//   k_compact : frontier byte map A_{k+1} -> active list of (edge offset,
//               CSR base, snapshot) for active vertices with out-edges; one
//               64-bit atomic per workgroup reserves list slots and edge
//               offsets; every PUSH_TILE-edge tile records the entry where it
//               starts; |A_{k+1}| is the count of vertices superstep k changed.
//               It runs after the relaxation, so the next superstep's form
//               is known on the device when its launch starts.
//               The frontier stands in for the paper's synchronisation
//               skipping (Section "Synchronization Skipping") and the equal
//               edge tiles for its fixed-size edge blocks (Section "Data Flows
//               & Management") under the balanced objective of Section
//               "Workload Balancing".
// PageRank superstep:
//   k_pr_pull : equal in-edge tiles; contributions are gathered into LDS and
//               summed per destination row in a fixed order; rows that
//               cross a tile boundary leave fixed partials.
//   k_pr_fix  : completes the crossing rows (each by one thread, in tile
//               order) and reduces the dangling mass for the next superstep:
//               per-workgroup partials, then the last workgroup to finish
//               sums them in workgroup order.  No floating-point atomics:
//               results are bitwise reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <mutex>

#include "gx_device.h"
#include "gx_internal.h"

using namespace gx;


static void pool_return(hipEvent_t e);
static void host_steps_return(gx::DevStep *p);

gx_state::~gx_state() {
    for (auto e : ev_pool) pool_return(e);
    for (auto &pr : ev_pending) {
        pool_return(pr.a);
        pool_return(pr.b);
    }
    if (host_steps) host_steps_return(host_steps);
}

namespace {

// ------------------------------------------------------------ SSSP / CC

__global__ __launch_bounds__(256) void k_min_init(uint32_t *val, uint8_t *f0, uint8_t *f1, uint8_t *dirty,
                                                  const int32_t *l2g, const int32_t *rp, int64_t V, int32_t algo,
                                                  int32_t source, DevStep *step0) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *step0 = DevStep{};
    if (i < V) {
        uint32_t x;
        uint8_t f;
        if (algo == GX_CC) {
            x = l2g ? (uint32_t)l2g[i] : (uint32_t)i;
            f = rp[i + 1] > rp[i];
        } else {
            x = (i == source) ? 0u : INF;
            f = i == source;
        }
        val[i] = x;
        f0[i] = f;
        f1[i] = 0;
        dirty[i] = 0;
    }
}

// Frontier byte map -> active list.  Each thread takes CVT consecutive
// vertices: one 16-byte load of their frontier bytes (and one 16-byte store
// clearing the byte map the next relaxation fills, which held A_{k-1}); a
// thread with an active vertex loads its CVT+1 row pointers and CVT values
// as whole vectors, so no load waits on another.  A workgroup covers
// CBLOCK*CVT vertices and issues two counter atomics (list, |A|).  Active
// vertices with out-edges get a list entry (edge offset, CSR base,
// snapshot, vertex) and the tiles that start inside an entry's edges record
// it.  When the next superstep may pull (snap_all), threads with an active
// vertex also store their vertices' values as snapshots (the pull stages
// them with the frontier map and treats inactive sources as INF).  |A_{k+1}|
// is the number of vertices superstep k changed.
constexpr int CVT = 16;
// Threads per compaction workgroup: each workgroup makes one list
// reservation (an add with return on a single counter, which serialises
// across workgroups), so fewer, larger workgroups shorten that chain.
constexpr int CBLOCK = 1024;

__global__ __launch_bounds__(CBLOCK) void k_compact(const uint8_t *__restrict__ front, uint8_t *__restrict__ front_clear,
                                                 const int32_t *__restrict__ rp, const uint32_t *__restrict__ val,
                                                 uint32_t *__restrict__ snap, int64_t V,
                                                 uint4 *__restrict__ list, uint32_t *__restrict__ tile_start,
                                                 DevStep *__restrict__ step, DevStep *__restrict__ next_step,
                                                 int snap_all, const DevStep *__restrict__ prev,
                                                 uint8_t *__restrict__ dirty, uint32_t pull_edges) {
    __shared__ unsigned long long s_scan[CBLOCK / 64];
    __shared__ unsigned long long s_base;
    __shared__ int s_nf[CBLOCK / 64];
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) *next_step = DevStep{};
    // The previous superstep had no active vertex: nothing was relaxed, the
    // map read here is still the cleared one and the map cleared here is
    // empty, so A_{k+1} is empty without a sweep (its counters stay zero).
    if (prev != nullptr && prev->frontier == 0) return;
    const int64_t u0 = ((int64_t)blockIdx.x * CBLOCK + tid) * CVT;
    uint32_t actmask = 0;
    if (u0 < V) {  // byte maps are padded to whole 32-vertex words: the 16 bytes at u0 exist
        const uint4 f = *reinterpret_cast<const uint4 *>(front + u0);
        *reinterpret_cast<uint4 *>(front_clear + u0) = make_uint4(0u, 0u, 0u, 0u);
        if (dirty != nullptr && (f.x | f.y | f.z | f.w)) {  // changed vertices become dirty here
            uint4 *d4 = reinterpret_cast<uint4 *>(dirty + u0);
            const uint4 d = *d4;
            *d4 = make_uint4(d.x | f.x, d.y | f.y, d.z | f.z, d.w | f.w);
        }
        const uint32_t fw[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int b = 0; b < 4; b++)
                if ((fw[q] >> (8 * b)) & 0xFFu) actmask |= 1u << (4 * q + b);
        if (V - u0 < CVT) actmask &= (1u << (V - u0)) - 1u;  // padding bytes are no vertices
    }
    if (!__syncthreads_or(actmask != 0)) return;
    int32_t r[CVT + 1];
    uint32_t x[CVT];
#pragma unroll
    for (int i = 0; i < CVT; i++) {
        r[i] = 0;
        x[i] = 0;
    }
    r[CVT] = 0;
    if (actmask) {
        if (u0 + CVT <= V) {  // rows u0 .. u0+CVT of the V+1 row pointers
            const int4 *r4 = reinterpret_cast<const int4 *>(rp + u0);
            const uint4 *x4 = reinterpret_cast<const uint4 *>(val + u0);
#pragma unroll
            for (int q = 0; q < CVT / 4; q++) {
                const int4 a = r4[q];
                const uint4 b = x4[q];
                r[4 * q] = a.x, r[4 * q + 1] = a.y, r[4 * q + 2] = a.z, r[4 * q + 3] = a.w;
                x[4 * q] = b.x, x[4 * q + 1] = b.y, x[4 * q + 2] = b.z, x[4 * q + 3] = b.w;
            }
            r[CVT] = rp[u0 + CVT];
        } else {
#pragma unroll
            for (int i = 0; i < CVT; i++) {
                if (u0 + i < V) x[i] = val[u0 + i];
                if (u0 + i <= V) r[i] = rp[u0 + i];
            }
        }
    }
    // Snapshots for the pull: a thread with an active vertex stores the values
    // of all its CVT vertices (the pull masks inactive sources with the
    // frontier map, so whatever an inactive entry holds is never used).
    if (snap_all && actmask) {
        if (u0 + CVT <= V) {
            uint4 *s4 = reinterpret_cast<uint4 *>(snap + u0);
#pragma unroll
            for (int q = 0; q < CVT / 4; q++) s4[q] = make_uint4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
        } else {
#pragma unroll
            for (int i = 0; i < CVT; i++)
                if (u0 + i < V) snap[u0 + i] = x[i];
        }
    }
    uint32_t cnt = 0, edges = 0;
#pragma unroll
    for (int i = 0; i < CVT; i++) {
        const int32_t dg = r[i + 1] - r[i];
        if (((actmask >> i) & 1u) && dg > 0) {
            cnt++;
            edges += (uint32_t)dg;
        }
    }
    unsigned long long mine = ((unsigned long long)cnt << 32) | edges, total;
    unsigned long long pre = block_excl_scan_u64(mine, &total, s_scan);
    int nf = __popc(actmask);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nf += __shfl_down(nf, o, 64);
    if ((tid & 63) == 0) s_nf[tid >> 6] = nf;
    if (tid == 0) s_base = total ? atomicAdd(&step->list, total) : 0ull;
    __syncthreads();
    if (tid == 0) {
        int nfb = 0;
#pragma unroll
        for (int w = 0; w < CBLOCK / 64; w++) nfb += s_nf[w];
        atomicAdd(&step->frontier, (unsigned long long)nfb);
    }
    // The out-edges counted up to this workgroup are a lower bound of the
    // frontier's: once it reaches pull_edges the next superstep pulls and
    // never reads the list, so the rest of the workgroups skip writing it.
    if ((uint32_t)(s_base + total) >= pull_edges) return;
    unsigned long long pos = s_base + pre;
#pragma unroll
    for (int i = 0; i < CVT; i++) {
        const int32_t dg = r[i + 1] - r[i];
        if (!((actmask >> i) & 1u) || dg <= 0) continue;
        const int64_t u = u0 + i;
        const uint32_t idx = (uint32_t)(pos >> 32), off = (uint32_t)pos;
        list[idx] = make_uint4(off, (uint32_t)(r[i] - (int32_t)off), x[i], (uint32_t)u);
        const uint32_t t0 = (off + PUSH_TILE - 1) / PUSH_TILE, t1 = (off + (uint32_t)dg - 1) / PUSH_TILE;
        for (uint32_t t = t0; t <= t1; t++) tile_start[t] = idx;
        pos += (1ull << 32) + (uint32_t)dg;
    }
}

// Relaxes the active out-edges, PUSH_TILE per workgroup tile (persistent
// grid; the tile count comes from the compaction's counter).
struct PushLds {
    uint32_t base[PUSH_TILE + 1];
    uint32_t snap[PUSH_TILE + 1];
    int32_t own[PUSH_TILE];
    int32_t red[4];
};

// Where a pulling workgroup's improving candidates go.  A candidate below a
// value read during the superstep is below the destination's start value
// (values only fall), so the destination changes whatever else lands: it is
// marked in the next frontier, its value is set with a plain store, and the
// pair (destination, candidate) is appended to the workgroup's fix-up
// region.  Plain stores racing on one destination may leave a larger
// candidate; the fix-up kernel then re-applies every recorded candidate
// still below the stored value with an atomic minimum.  Min atomics cost
// several times a plain store here.  This is sound because every writer of
// a destination in the pull runs on the XCD that owns the destination's
// slice (one L2 sees all of its plain stores) and the fix-up is a later
// launch; regions are sized for every record a workgroup can meet, so no
// candidate bypasses them (plain stores and atomics on one word in one
// kernel would not be ordered).
// A relaxation workgroup leaves its fix-up count in the low bits of its word
// and, from a pull, the XCD rotation it saw in the top three.
constexpr int FIX_ROT_SHIFT = 29;

struct FixRegion {
    uint2 *ent;        // this workgroup's region
    uint32_t cap;      // its capacity
    uint32_t *count;   // LDS: candidates offered so far
};

template <int N>
__device__ __forceinline__ void apply_hits(const uint32_t (&dst)[N], const uint32_t (&m)[N], uint32_t hits,
                                           uint32_t *__restrict__ val, uint8_t *__restrict__ front_next,
                                           const FixRegion &fr) {
    // one LDS reservation per wave: lane-ordered, contiguous entries
    const int lane = threadIdx.x & 63;
    const uint32_t cnt = (uint32_t)__popc(hits);
    uint32_t incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    const uint32_t total = __shfl(incl, 63, 64);
    uint32_t base = 0;
    if (lane == 63 && total) base = atomicAdd(fr.count, total);
    base = __shfl(base, 63, 64);
    uint32_t pos = base + incl - cnt;
#pragma unroll
    for (int i = 0; i < N; i++) {
        if ((hits >> i) & 1u) {
            if (pos < fr.cap) {
                fr.ent[pos] = make_uint2(dst[i], m[i]);
                val[dst[i]] = m[i];
            } else {
                atomicMin(&val[dst[i]], m[i]);
            }
            front_next[dst[i]] = 1;
            pos++;
        }
    }
}

template <bool WEIGHTED>
__device__ __forceinline__ void push_body(const uint4 *__restrict__ list, const uint32_t *__restrict__ tile_start,
                                          const void *__restrict__ adj, uint32_t *__restrict__ val,
                                          uint8_t *__restrict__ front_next, unsigned long long le, PushLds &lds) {
    uint32_t *s_base = lds.base;
    uint32_t *s_snap = lds.snap;
    int32_t *s_own = lds.own;
    int32_t *s_red = lds.red;
    const int tid = threadIdx.x;
    const uint32_t L = (uint32_t)(le >> 32), EF = (uint32_t)le;
    const uint32_t ntiles = (EF + PUSH_TILE - 1) / PUSH_TILE;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t e0 = t * PUSH_TILE;
        const int n = (int)min((uint32_t)PUSH_TILE, EF - e0);
        const uint32_t s0 = tile_start[t];
        const uint32_t s1 = (t + 1 < ntiles) ? tile_start[t + 1] : L - 1;
        const int m = (int)(s1 - s0) + 1;
        for (int p = tid; p < n; p += PUSH_BLOCK) s_own[p] = 0;
        __syncthreads();
        for (int i = tid; i < m; i += PUSH_BLOCK) {
            uint4 en = list[s0 + i];
            s_base[i] = en.y + e0;  // CSR index of the tile's edge p is s_base[j] + p
            s_snap[i] = en.z;
            uint32_t rel = en.x - e0;
            if (i > 0 && rel < (uint32_t)n) s_own[rel] = i;
        }
        __syncthreads();
        block_max_scan<PUSH_VT>(s_own, n, s_red);
        // Batched memory access: every load is unconditional (slots past the
        // tile's end repeat its last edge and are dropped at the end), so the
        // thread issues all its edge loads, then all destination reads, with
        // one wait each and no load behind another edge's atomic.
        uint32_t idx[PUSH_VT], sv[PUSH_VT];
#pragma unroll
        for (int i = 0; i < PUSH_VT; i++) {
            const int p = min(tid + i * PUSH_BLOCK, n - 1);
            const int j = s_own[p];
            idx[i] = s_base[j] + (uint32_t)p;
            sv[i] = s_snap[j];
        }
        uint32_t dst[PUSH_VT], cand[PUSH_VT], cur[PUSH_VT];
#pragma unroll
        for (int i = 0; i < PUSH_VT; i++) {
            if (WEIGHTED) {
                const uint2 a = static_cast<const uint2 *>(adj)[idx[i]];
                dst[i] = a.x;
                cand[i] = a.y;
            } else {
                dst[i] = (uint32_t) static_cast<const int32_t *>(adj)[idx[i]];
            }
        }
#pragma unroll
        for (int i = 0; i < PUSH_VT; i++) cur[i] = val[dst[i]];
#pragma unroll
        for (int i = 0; i < PUSH_VT; i++) {
            cand[i] = WEIGHTED ? sat_add(sv[i], cand[i]) : sv[i];
            if (tid + i * PUSH_BLOCK >= n) cand[i] = INF;
        }
        // A candidate below a value read during this superstep is below the
        // destination's start-of-superstep value (values only fall), so the
        // destination changes in this superstep whichever atomic lands last:
        // mark it with an idempotent plain store and let the atomic go
        // without waiting for its result.  (Destinations here are written
        // from every XCD, so the merge stays an atomic minimum.)
#pragma unroll
        for (int i = 0; i < PUSH_VT; i++) {
            if (cand[i] < cur[i]) {
                atomicMin(&val[dst[i]], cand[i]);
                front_next[dst[i]] = 1;
            }
        }
        __syncthreads();
    }
}

// Pull form of the same superstep, for large frontiers.  The in-edges are
// stored as records {dst, (src mod PULL_BAND) << 8 | w} (CC: {dst, src}) in
// work units of one destination slice and one band of PULL_BAND sources
// (layout built at load).  A workgroup takes the units of the slice of the
// XCD it runs on (the j-th workgroup of an XCD takes units j, j + grid/8,
// ...), so each XCD's L2 holds its slice's destination values and every
// writer of a destination shares that L2.  A unit's band of
// snapshots is staged in LDS, INF where the frontier map A_k says the source
// is inactive, so a record's gather is an LDS read.  The 64 lanes of a wave
// take 64 consecutive records (destinations in ascending order), so lanes
// whose destinations share a cache line make one memory request between
// them: the destination reads, one per record, are what bounds the pull,
// and wider bands make consecutive records' destinations denser.  A record
// without a candidate (inactive source or padding) reads nothing: the
// destination reads are buffer loads whose offset for such lanes lies past
// the buffer, which fetches nothing and returns 0.  Lanes holding the same
// destination each apply their candidate; the fix-up pass leaves the
// minimum.  Runs only when the frontier's out-edges reach pull_edges (V * 4
// must fit the 32-bit buffer range; the host enables the pull only then).
template <bool WEIGHTED>
__device__ __forceinline__ void pull_body(const uint2 *__restrict__ rec, const uint4 *__restrict__ units,
                                          const PullSlices &sl, int64_t V, const uint32_t *__restrict__ snap,
                                          const uint8_t *__restrict__ front_cur, uint32_t *__restrict__ val,
                                          uint8_t *__restrict__ front_next, DevStep *__restrict__ step,
                                          uint32_t *__restrict__ s_snap, const FixRegion &fr, uint32_t xcd_shift,
                                          uint32_t *rot) {
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) step->pad = 1;
    const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc(val, (short)0, (int)(uint32_t)(V * 4), 0x00020000);
    // The workgroup takes the slice of the XCD it runs on, so every writer of
    // a destination shares one L2.  The hardware deals a launch's workgroups
    // to the XCDs in turn, from XCD r for workgroup 0 (r has been seen to
    // differ between launches), so workgroup b runs on XCD (b + r) mod 8 and
    // is the (b / 8)-th of its XCD (the grid is a multiple of 8).  Each
    // workgroup leaves the r it saw beside its fix-up count, and the fix-up
    // pass flags the superstep if the workgroups of one launch saw more than
    // one.  (xcd_shift, zero outside tests, offsets the odd workgroups' XCD
    // to exercise that check.)
    const uint32_t xr = (xcc_id() + ((blockIdx.x & 1u) ? xcd_shift : 0u)) % PULL_SLICES;
    *rot = (xr + PULL_SLICES - blockIdx.x % PULL_SLICES) % PULL_SLICES;
    const int x = (int)xr;
    const int64_t nblk = gridDim.x / PULL_SLICES;
    for (int64_t ui = sl.uoff[x] + blockIdx.x / PULL_SLICES; ui < sl.uoff[x + 1]; ui += nblk) {
        const uint4 un = units[ui];
        const uint32_t start = un.x, cnt = un.y, bb = un.z;
        __syncthreads();  // the previous unit's gathers are done
        // the band's snapshots, INF where the source is not in A_k
        if ((int64_t)bb + PULL_BAND <= V) {
            const uint4 *s4 = reinterpret_cast<const uint4 *>(snap + bb);
            const uint32_t *f4 = reinterpret_cast<const uint32_t *>(front_cur + bb);
            uint4 sv[PULL_BAND / 4 / 256];
            uint32_t fv[PULL_BAND / 4 / 256];
#pragma unroll
            for (int q = 0; q < PULL_BAND / 4 / 256; q++) {
                sv[q] = s4[q * 256 + tid];
                fv[q] = f4[q * 256 + tid];
            }
#pragma unroll
            for (int q = 0; q < PULL_BAND / 4 / 256; q++)
                reinterpret_cast<uint4 *>(s_snap)[q * 256 + tid] =
                    make_uint4(fv[q] & 0xFFu ? sv[q].x : INF, fv[q] & 0xFF00u ? sv[q].y : INF,
                               fv[q] & 0xFF0000u ? sv[q].z : INF, fv[q] & 0xFF000000u ? sv[q].w : INF);
        } else {  // the last band ends at V
            for (int i = tid; i < PULL_BAND; i += 256) s_snap[i] = bb + i < V && front_cur[bb + i] ? snap[bb + i] : INF;
        }
        __syncthreads();
        // every lane runs every chunk (the hits' reservation is a wave-wide
        // scan); lanes past the unit's end load its first record and offer nothing
        for (uint32_t c0 = start; c0 < start + cnt; c0 += 256 * PULL_VT) {
            uint32_t dst[PULL_VT], src[PULL_VT], m[PULL_VT], cur[PULL_VT];
#pragma unroll
            for (int i = 0; i < PULL_VT; i++) {  // record c0 + 256 i + tid; past the unit: no candidate
                const uint32_t e = c0 + (uint32_t)i * 256 + (uint32_t)tid;
                const bool in = e < start + cnt;
                const uint2 q = rec[in ? e : start];
                dst[i] = in ? q.x : PULL_SENTINEL;
                src[i] = q.y;
            }
#pragma unroll
            for (int i = 0; i < PULL_VT; i++) {
                const uint32_t sv = s_snap[(WEIGHTED ? (src[i] >> 8) : (src[i] - bb)) & (PULL_BAND - 1)];
                m[i] = WEIGHTED ? sat_add(sv, src[i] & 0xFFu) : sv;
                if (dst[i] == PULL_SENTINEL) m[i] = INF;
            }
            // one batched read of the destinations (only records with a
            // candidate fetch), then the compares and the merge
#pragma unroll
            for (int i = 0; i < PULL_VT; i++)
                cur[i] = __builtin_amdgcn_raw_buffer_load_b32(vrs, m[i] != INF ? dst[i] * 4u : 0x80000000u, 0, 0);
            __builtin_amdgcn_sched_barrier(0);  // every read above is issued before the first compare
            uint32_t hits = 0;
#pragma unroll
            for (int i = 0; i < PULL_VT; i++) hits |= (uint32_t)(m[i] < cur[i]) << i;
            apply_hits<PULL_VT>(dst, m, hits, val, front_next, fr);
        }
    }
}

// One launch per superstep: the frontier's edge count, known on the device
// after the compaction, picks the form (a second, idle launch would cost a
// dispatch and a sweep of exiting workgroups every superstep).
struct PullArgs {
    const uint2 *rec;
    const uint4 *units;
    PullSlices sl;
};
union RelaxLds {
    PushLds push;
    uint32_t pull_snap[PULL_BAND];
};

template <bool WEIGHTED>
__global__ __launch_bounds__(256) void k_relax(const uint4 *__restrict__ list, const uint32_t *__restrict__ tile_start,
                                               const void *__restrict__ adj, PullArgs pa, int64_t V,
                                               const uint32_t *__restrict__ snap, uint32_t *__restrict__ val,
                                               const uint8_t *__restrict__ front_cur, uint8_t *__restrict__ front_next,
                                               DevStep *__restrict__ step, uint32_t pull_edges,
                                               uint2 *__restrict__ fix, uint32_t *__restrict__ fixn, uint32_t fix_cap,
                                               uint32_t xcd_shift) {
    __shared__ RelaxLds lds;
    __shared__ uint32_t s_fixn;
    if (threadIdx.x == 0) s_fixn = 0;
    __syncthreads();
    const FixRegion fr{fix + (size_t)blockIdx.x * fix_cap, fix_cap, &s_fixn};
    const unsigned long long le = step->list;
    uint32_t rot = 0;
    if ((uint32_t)le >= pull_edges) {
        pull_body<WEIGHTED>(pa.rec, pa.units, pa.sl, V, snap, front_cur, val, front_next, step, lds.pull_snap, fr,
                            xcd_shift, &rot);
    } else {
        push_body<WEIGHTED>(list, tile_start, adj, val, front_next, le, lds.push);
    }
    __syncthreads();
    if (threadIdx.x == 0) fixn[blockIdx.x] = min(s_fixn, fix_cap) | (rot << FIX_ROT_SHIFT);
}

// The relaxation's fix-up: workgroup b re-applies the recorded candidates of
// relaxation workgroup b that are still below the stored value (a separate
// launch: the relaxation's stores are visible to every XCD by then), and
// flags the superstep if relaxation workgroup b saw another XCD rotation
// than workgroup 0 (a push leaves rotation 0 everywhere).
__global__ __launch_bounds__(256) void k_fixup(const uint2 *__restrict__ fix, const uint32_t *__restrict__ fixn,
                                               uint32_t fix_cap, uint32_t *__restrict__ val, DevStep *__restrict__ step) {
    const uint32_t w = fixn[blockIdx.x];
    if (threadIdx.x == 0 && (w >> FIX_ROT_SHIFT) != (fixn[0] >> FIX_ROT_SHIFT)) step->rot_mixed = 1ull;
    const uint32_t n = w & ((1u << FIX_ROT_SHIFT) - 1u);
    const uint2 *e = fix + (size_t)blockIdx.x * fix_cap;
    for (uint32_t i = threadIdx.x; i < n; i += 256) {
        const uint2 q = e[i];
        if (q.y < val[q.x]) atomicMin(&val[q.x], q.y);
    }
}

// ------------------------------------------------------------ PageRank

__global__ __launch_bounds__(256) void k_pr_init(float *x, float *contrib, uint32_t *synced,
                                                 const int32_t *__restrict__ outdeg, const int32_t *__restrict__ slot,
                                                 int64_t V, float x0, double *dpart, DevStep *step0) {
    __shared__ double s_d[4];
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0) *step0 = DevStep{};
    double dl = 0.0;
    if (v < V) {
        int od = outdeg[v];
        x[v] = x0;
        synced[v] = __float_as_uint(x0);
        contrib[slot[v]] = od > 0 ? x0 / (float)od : 0.0f;
        if (od == 0) dl = (double)x0;
    }
    double t = block_sum<double>(dl, s_d);
    if (threadIdx.x == 0) dpart[blockIdx.x] = t;
}

// Single workgroup: D = sum of n partials in a fixed order.
__global__ __launch_bounds__(1024) void k_reduce_D(const double *__restrict__ part, int n, double *D) {
    __shared__ double s_d[16];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a += part[i];
    double t = block_sum<double>(a, s_d);
    if (threadIdx.x == 0) *D = t;
}

struct PrApply {
    double base, d, dD;  // x' = base + d * acc + dD, with dD = d * D / V
    const int32_t *outdeg;
    const float *x_in;
    float *x_out, *c_out;
    const int32_t *slot;  // contribution slot of each vertex (hottest sources first)
    static constexpr bool kRows = true;  // the pull stages outdeg, slot and x_in of its rows in LDS
    __device__ __forceinline__ void load_row(int32_t r, int32_t &od, int32_t &sl, float &xi) const {
        od = outdeg[r];
        sl = slot[r];
        xi = x_in[r];
    }
    __device__ __forceinline__ void row(int32_t r, double acc, int32_t od, int32_t sl, float xi, double &dsum,
                                        int &chg) const {
        float xn = (float)(base + d * acc + dD);
        x_out[r] = xn;
        c_out[sl] = od > 0 ? xn / (float)od : 0.0f;
        if (od == 0) dsum += (double)xn;
        chg += __float_as_uint(xn) != __float_as_uint(xi);
    }
    __device__ __forceinline__ void operator()(int32_t r, double acc, double &dsum, int &chg) const {
        row(r, acc, outdeg[r], slot[r], x_in[r], dsum, chg);
    }
};

// The merge alone (separate template calls): the combined messages of a row
// are stored; what is applied happens later.
struct PrStore {
    double d, dD;  // (unused)
    double *acc;
    static constexpr bool kRows = false;
    __device__ __forceinline__ void load_row(int32_t, int32_t &, int32_t &, float &) const {}
    __device__ __forceinline__ void row(int32_t r, double total, int32_t, int32_t, float, double &, int &) const {
        acc[r] = total;
    }
    __device__ __forceinline__ void operator()(int32_t r, double total, double &, int &) const { acc[r] = total; }
};

template <int VT, class AP>
__global__ __launch_bounds__(PR_BLOCK) void k_pr_pull(const int32_t *__restrict__ in_rp,
                                                      const int32_t *__restrict__ in_col,
                                                      const int32_t *__restrict__ tile_row, int64_t E,
                                                      const float *__restrict__ c_in, AP ap,
                                                      const double *__restrict__ Dp, double inv_V,
                                                      double *__restrict__ head, double *__restrict__ tailp,
                                                      int32_t *__restrict__ spill_row, double *__restrict__ dpart,
                                                      uint32_t *__restrict__ cpart) {
    constexpr int TILE = PR_BLOCK * VT;
    constexpr int RPT = 2;                    // rows per thread whose data is staged in LDS
    constexpr int ROWS = RPT * PR_BLOCK;
    __shared__ float s_val[TILE];
    __shared__ int32_t s_own[TILE];
    __shared__ double s_last[PR_BLOCK];
    __shared__ double s_wy[PR_BLOCK / 64];
    __shared__ int s_wf[PR_BLOCK / 64];
    __shared__ int32_t s_red[4];
    __shared__ double s_d[4];
    __shared__ unsigned long long s_c[4];
    __shared__ int32_t s_re[ROWS];            // end of row r_lo + i (in_rp[r + 1])
    __shared__ int32_t s_od[AP::kRows ? ROWS : 1], s_sl[AP::kRows ? ROWS : 1];
    __shared__ float s_xi[AP::kRows ? ROWS : 1];
    const int tid = threadIdx.x;
    const int32_t t = blockIdx.x;
    const int64_t e0 = (int64_t)t * TILE;
    const int n = (int)max((int64_t)0, min((int64_t)TILE, E - e0));
    const int32_t r_lo = tile_row[t], r_hi = tile_row[t + 1];
    ap.dD = ap.d * (*Dp) * inv_V;
    if (tid == 0) spill_row[t] = -1;
    // Every load that depends only on the tile is issued at once: the edges'
    // sources, the row pointers of the tile's first ROWS rows and what the
    // apply reads of them; then the gathers of the contributions.
    int32_t u[VT];
    float cv[VT];
    int32_t ra[RPT], rb[RPT], od[RPT], sl[RPT];
    float xi[RPT];
#pragma unroll
    for (int i = 0; i < VT; i++)  // (the in-edges stream by once: kept out of the caches' way)
        u[i] = n > 0 ? __builtin_nontemporal_load(&in_col[e0 + min(tid + i * PR_BLOCK, n - 1)]) : 0;
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int32_t r = r_lo + tid + k * PR_BLOCK;
        ra[k] = rb[k] = 0;
        od[k] = sl[k] = 0;
        xi[k] = 0.f;
        if (r < r_hi) {
            ra[k] = in_rp[r];
            rb[k] = in_rp[r + 1];
            ap.load_row(r, od[k], sl[k], xi[k]);
        }
    }
#pragma unroll
    for (int i = 0; i < VT; i++) cv[i] = n > 0 ? c_in[u[i]] : 0.f;
#pragma unroll
    for (int i = 0; i < VT; i++) {
        const int p = tid + i * PR_BLOCK;
        if (p < n) {
            s_val[p] = cv[i];
            s_own[p] = 0;
        }
    }
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int i = tid + k * PR_BLOCK;
        if (r_lo + i < r_hi) {
            s_re[i] = rb[k];
            if (AP::kRows) {
                s_od[i] = od[k];
                s_sl[i] = sl[k];
                s_xi[i] = xi[k];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int32_t r = r_lo + tid + k * PR_BLOCK;
        if (r < r_hi && rb[k] > ra[k]) s_own[ra[k] - e0] = r - r_lo + 1;
    }
    for (int32_t r = r_lo + ROWS + tid; r < r_hi; r += PR_BLOCK) {  // rows past the staged ones
        int32_t a = in_rp[r], b = in_rp[r + 1];
        if (b > a) s_own[a - e0] = r - r_lo + 1;
    }
    __syncthreads();
    block_max_scan<VT>(s_own, n, s_red);

    // a row's apply, from its staged data when it has some
    auto apply_row = [&](int32_t r, double total, double &dsum, int &chg) {
        const int i = r - r_lo;
        if (i < ROWS)
            ap.row(r, total, s_od[AP::kRows ? i : 0], s_sl[AP::kRows ? i : 0], s_xi[AP::kRows ? i : 0], dsum, chg);
        else
            ap(r, total, dsum, chg);
    };
    auto row_end = [&](int32_t r) { return r - r_lo < ROWS ? s_re[r - r_lo] : in_rp[r + 1]; };

    // Per-thread contiguous chunk: sequential sums per destination row.
    double dsum = 0.0;
    int chg = 0;
    const int c0 = tid * VT, c1 = min(c0 + VT, n);
    int own = -1;
    bool started = false, first = true;
    double sum = 0.0, first_sum = 0.0;
    int first_own = -1;
    bool defer_first = false, defer_ends_tile = false;
    auto finish = [&](int o, double total, bool ends_tile) {
        if (o == 0) {
            head[t] = total;  // row continued from an earlier tile
            return;
        }
        int32_t r = r_lo + o - 1;
        if (ends_tile && row_end(r) > e0 + n) {
            tailp[t] = total;  // row continues into later tiles
            spill_row[t] = r;
            return;
        }
        apply_row(r, total, dsum, chg);
    };
    for (int p = c0; p < c1; p++) {
        int o = s_own[p];
        if (o != own) {
            if (own >= 0) {  // run `own` ended at p-1 inside this chunk
                if (first && !started) {
                    defer_first = true;
                    first_sum = sum;
                    first_own = own;
                } else {
                    finish(own, sum, false);
                }
                first = false;
            }
            own = o;
            sum = 0.0;
            started = (p == 0) ? (o != 0) : (p > c0 || s_own[p - 1] != o);
        }
        sum += (double)s_val[p];
    }
    bool last_ends_here = false;
    if (own >= 0) {
        last_ends_here = (c1 == n) || (s_own[c1] != own);
        if (last_ends_here) {
            if (first && !started) {
                defer_first = true;
                defer_ends_tile = (c1 == n);
                first_sum = sum;
                first_own = own;
            } else {
                finish(own, sum, c1 == n);
            }
        }
    }
    // Pieces of rows that run past a chunk: an inclusive segmented scan over
    // the threads, a segment starting at the thread where a row's trailing
    // piece starts (or where a row ends).  Fixed order: a shuffle scan inside
    // each wave, then the wave totals folded in wave order; a deferred first
    // piece then adds the scan value of the thread before it.
    {
        double y = (own >= 0 && !last_ends_here) ? sum : 0.0;
        int f = (own < 0 || started || last_ends_here) ? 1 : 0;
        const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double yp = __shfl_up(y, d, 64);
            const int fp = __shfl_up(f, d, 64);
            if (lane >= d) {
                if (!f) y = yp + y;
                f |= fp;
            }
        }
        if (lane == 63) {
            s_wy[wv] = y;
            s_wf[wv] = f;
        }
        __syncthreads();
        if (!f) {
            double c = 0.0;
            for (int v = 0; v < wv; v++) c = s_wf[v] ? s_wy[v] : c + s_wy[v];
            y = c + y;
        }
        s_last[tid] = y;
    }
    __syncthreads();
    if (defer_first) finish(first_own, tid > 0 ? first_sum + s_last[tid - 1] : first_sum, defer_ends_tile);
    // Rows of this tile without in-edges.
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int32_t r = r_lo + tid + k * PR_BLOCK;
        if (r < r_hi && rb[k] == ra[k]) apply_row(r, 0.0, dsum, chg);
    }
    for (int32_t r = r_lo + ROWS + tid; r < r_hi; r += PR_BLOCK)
        if (in_rp[r + 1] == in_rp[r]) ap(r, 0.0, dsum, chg);
    double td = block_sum<double>(dsum, s_d);
    unsigned long long tc = block_sum<unsigned long long>((unsigned long long)chg, s_c);
    if (tid == 0) {  // per-tile partials, summed by k_pr_fix (no atomics on one shared counter)
        dpart[t] = td;
        cpart[t] = (uint32_t)tc;
    }
}

// Completes the rows that cross tile boundaries (each by one thread, adding
// the row's partials in tile order) and reduces the dangling mass of the new
// ranks for the next superstep: every workgroup leaves its partial sums, and
// the last one to finish adds them up in workgroup order, so the result does
// not depend on timing.  The kernel boundary makes every pull workgroup's
// partials visible here; *Dp (the old mass) is read by every workgroup
// before the last one overwrites it.
constexpr int PR_FIX_BLOCK = 256;
constexpr int PR_FIX_MAX_GRID = 1024;

template <class AP>
__global__ __launch_bounds__(PR_FIX_BLOCK) void k_pr_fix(const int32_t *__restrict__ in_rp, int32_t ntiles,
                                                         int32_t tile, const double *__restrict__ head,
                                                         const double *__restrict__ tailp,
                                                         const int32_t *__restrict__ spill_row,
                                                         const double *__restrict__ dpart,
                                                         const uint32_t *__restrict__ cpart, AP ap, double *Dp,
                                                         double inv_V, DevStep *__restrict__ step,
                                                         DevStep *__restrict__ next_step, double *fix_d,
                                                         unsigned long long *fix_c, uint32_t *fix_done) {
    __shared__ double s_d[PR_FIX_BLOCK / 64];
    __shared__ unsigned long long s_c[PR_FIX_BLOCK / 64];
    __shared__ int s_last;
    ap.dD = ap.d * (*Dp) * inv_V;
    double dsum = 0.0;
    int chg = 0;
    unsigned long long csum = 0;
    for (int32_t t = blockIdx.x * PR_FIX_BLOCK + threadIdx.x; t < ntiles; t += gridDim.x * PR_FIX_BLOCK) {
        const int32_t r = spill_row[t];
        if (r >= 0) {
            double total = tailp[t];
            const int32_t t_end = (in_rp[r + 1] - 1) / tile;
            for (int32_t t2 = t + 1; t2 <= t_end; t2++) total += head[t2];
            ap(r, total, dsum, chg);
        }
        dsum += dpart[t];
        csum += cpart[t];
    }
    const double td = block_sum<double>(dsum, s_d);
    const unsigned long long tc = block_sum<unsigned long long>(csum + (unsigned long long)chg, s_c);
    if (threadIdx.x == 0) {
        fix_d[blockIdx.x] = td;
        fix_c[blockIdx.x] = tc;
        // release this workgroup's partials; acquire the others' if last
        const uint32_t before = __hip_atomic_fetch_add(fix_done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = before == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    double d = 0.0;
    unsigned long long c = 0;
    for (uint32_t b = threadIdx.x; b < gridDim.x; b += PR_FIX_BLOCK) {
        d += fix_d[b];
        c += fix_c[b];
    }
    const double D = block_sum<double>(d, s_d);
    const unsigned long long C = block_sum<unsigned long long>(c, s_c);
    if (threadIdx.x == 0) {
        *Dp = D;  // dangling mass of x_{t+1}
        step->changed = C;
        step->frontier = 0;
        *next_step = DevStep{};
        *fix_done = 0;  // for the next superstep (after this kernel ends)
    }
}

// ------------------------------------------------------------ PageRank across the parts of a vertex-cut

__device__ __forceinline__ bool bit_of(const uint32_t *bm, int64_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }

// Replicas this part sends its merged messages for: held elsewhere too, the
// master elsewhere, and with at least one in-edge here (else the sum is 0).
__device__ __forceinline__ uint32_t partial_word(int32_t w, int64_t V, const uint32_t *remote_any,
                                                 const uint32_t *master, const int32_t *in_rp) {
    const uint32_t valid = (int64_t)(w + 1) * 32 <= V ? 0xFFFFFFFFu : ((1u << (V - (int64_t)w * 32)) - 1u);
    const uint32_t cand = remote_any[w] & ~master[w] & valid;
    uint32_t out = 0;
    for (uint32_t m = cand; m; m &= m - 1) {
        const int b = __ffs(m) - 1;
        const int64_t v = (int64_t)w * 32 + b;
        if (in_rp[v + 1] > in_rp[v]) out |= 1u << b;
    }
    return out;
}

__global__ __launch_bounds__(256) void k_part_count(int32_t W, int64_t V, const uint32_t *remote_any,
                                                    const uint32_t *master, const int32_t *in_rp, uint32_t *blk_cnt) {
    __shared__ unsigned long long s[4];
    const int32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t c = w < W ? __popc(partial_word(w, V, remote_any, master, in_rp)) : 0u;
    const unsigned long long t = block_sum<unsigned long long>(c, s);
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = (uint32_t)t;
}

// (gid, merged sum) of the selected replicas in ascending gid; positions from
// the block counts as in the sync set.
__global__ __launch_bounds__(256) void k_part_emit(int32_t W, int64_t V, const uint32_t *remote_any,
                                                   const uint32_t *master, const int32_t *in_rp,
                                                   const int32_t *l2g, const double *__restrict__ acc,
                                                   const uint32_t *__restrict__ blk_cnt, int nblk, uint32_t cap,
                                                   int32_t *gid_out, double *val_out, uint32_t *total_out) {
    __shared__ unsigned long long s_scan[4];
    __shared__ unsigned long long s_pre[4], s_all[4];
    const int tid = threadIdx.x;
    unsigned long long pre = 0, all_ = 0;
    for (int b = tid; b < nblk; b += blockDim.x) {
        const unsigned long long c = blk_cnt[b];
        all_ += c;
        if (b < (int)blockIdx.x) pre += c;
    }
    {
        const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            pre += __shfl_down(pre, o, 64);
            all_ += __shfl_down(all_, o, 64);
        }
        if (lane == 0) {
            s_pre[wid] = pre;
            s_all[wid] = all_;
        }
        __syncthreads();
        pre = s_pre[0] + s_pre[1] + s_pre[2] + s_pre[3];
        all_ = s_all[0] + s_all[1] + s_all[2] + s_all[3];
        __syncthreads();
    }
    if (blockIdx.x == 0 && tid == 0) *total_out = (uint32_t)all_;
    const int32_t w = blockIdx.x * blockDim.x + tid;
    const uint32_t bits = w < W ? partial_word(w, V, remote_any, master, in_rp) : 0u;
    unsigned long long tot;
    unsigned long long pos = pre + block_excl_scan_u64(__popc(bits), &tot, s_scan);
    for (uint32_t m = bits; m; m &= m - 1) {
        const int64_t v = (int64_t)w * 32 + __ffs(m) - 1;
        if (pos < cap) {
            gid_out[pos] = l2g[v];
            val_out[pos] = acc[v];
        }
        pos++;
    }
}

__device__ __forceinline__ int64_t local_of(const int32_t *__restrict__ l2g, int64_t V, int32_t g) {
    int64_t lo = 0, hi = V;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (l2g[mid] < g) lo = mid + 1;
        else hi = mid;
    }
    return (lo < V && l2g[lo] == g) ? lo : -1;
}

// A master adds another part's merged sum for it (one pair per vertex per
// call; the caller orders the calls, so the sum's order is fixed).
__global__ __launch_bounds__(256) void k_part_add(const int32_t *__restrict__ gid, const double *__restrict__ vals,
                                                  uint32_t n, const int32_t *__restrict__ l2g, int64_t V,
                                                  const uint32_t *__restrict__ master, double *__restrict__ acc) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t x = local_of(l2g, V, gid[i]);
    if (x >= 0 && bit_of(master, x)) acc[x] += vals[i];
}

// A replica takes its master's new rank.
__global__ __launch_bounds__(256) void k_replica_set(const int32_t *__restrict__ gid, const uint32_t *__restrict__ vals,
                                                     uint32_t n, const int32_t *__restrict__ l2g, int64_t V,
                                                     const uint32_t *__restrict__ master, uint32_t *__restrict__ x) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t v = local_of(l2g, V, gid[i]);
    if (v >= 0 && !bit_of(master, v)) x[v] = vals[i];
}

// ------------------------------------------------------------ sync set

__device__ __forceinline__ uint32_t delta_word(int32_t w, int64_t V, const uint32_t *remote, bool all,
                                               const uint8_t *dirty, const uint32_t *vals,
                                               const uint32_t *synced) {
    uint32_t valid = (int64_t)(w + 1) * 32 <= V ? 0xFFFFFFFFu : ((1u << (V - (int64_t)w * 32)) - 1u);
    uint32_t mask = (all ? 0xFFFFFFFFu : (remote ? remote[w] : 0u)) & valid;
    if (!mask) return 0;
    if (dirty) {
        uint32_t bits = 0;
        const uint32_t *d4 = reinterpret_cast<const uint32_t *>(dirty + (int64_t)w * 32);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const uint32_t x = d4[q];
            bits |= (uint32_t)((x & 0xFFu) != 0) << (4 * q) | (uint32_t)((x & 0xFF00u) != 0) << (4 * q + 1) |
                    (uint32_t)((x & 0xFF0000u) != 0) << (4 * q + 2) | (uint32_t)((x & 0xFF000000u) != 0) << (4 * q + 3);
        }
        return bits & mask;
    }
    uint32_t out = 0;
    for (uint32_t m = mask; m; m &= m - 1) {
        int b = __ffs(m) - 1;
        int64_t v = (int64_t)w * 32 + b;
        if (vals[v] != synced[v]) out |= 1u << b;
    }
    return out;
}

__global__ __launch_bounds__(256) void k_delta_count(int32_t W, int64_t V, const uint32_t *remote, int all,
                                                     const uint8_t *dirty, const uint32_t *vals,
                                                     const uint32_t *synced, uint32_t *blk_cnt) {
    __shared__ unsigned long long s[4];
    int32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t c = w < W ? __popc(delta_word(w, V, remote, all, dirty, vals, synced)) : 0u;
    unsigned long long t = block_sum<unsigned long long>(c, s);
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = (uint32_t)t;
}

__global__ __launch_bounds__(256) void k_delta_emit(int32_t W, int64_t V, const uint32_t *remote, int all,
                                                    uint8_t *dirty, const uint32_t *vals, uint32_t *synced,
                                                    const int32_t *l2g, const uint32_t *__restrict__ blk_cnt,
                                                    int nblk, uint32_t cap, int32_t *gid_out, uint32_t *val_out,
                                                    uint32_t *total_out) {
    __shared__ unsigned long long s_scan[4];
    __shared__ unsigned long long s_pre[4], s_all[4];
    const int tid = threadIdx.x;
    unsigned long long pre = 0, all_ = 0;
    for (int b = tid; b < nblk; b += blockDim.x) {
        unsigned long long c = blk_cnt[b];
        all_ += c;
        if (b < (int)blockIdx.x) pre += c;
    }
    // block sums of pre / all (same tree for every block: identical totals)
    {
        const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            pre += __shfl_down(pre, o, 64);
            all_ += __shfl_down(all_, o, 64);
        }
        if (lane == 0) {
            s_pre[wid] = pre;
            s_all[wid] = all_;
        }
        __syncthreads();
        pre = s_pre[0] + s_pre[1] + s_pre[2] + s_pre[3];
        all_ = s_all[0] + s_all[1] + s_all[2] + s_all[3];
        __syncthreads();
    }
    if (blockIdx.x == 0 && tid == 0) *total_out = (uint32_t)all_;
    const bool commit = all_ <= cap;
    int32_t w = blockIdx.x * blockDim.x + tid;
    uint32_t bits = w < W ? delta_word(w, V, remote, all, dirty, vals, synced) : 0u;
    unsigned long long tot;
    unsigned long long pos = pre + block_excl_scan_u64(__popc(bits), &tot, s_scan);
    for (uint32_t m = bits; m; m &= m - 1) {
        int64_t v = (int64_t)w * 32 + __ffs(m) - 1;
        if (pos < cap) {
            gid_out[pos] = l2g ? l2g[v] : (int32_t)v;
            val_out[pos] = vals[v];
        }
        pos++;
        if (commit && synced) synced[v] = vals[v];
    }
    if (commit && dirty && w < W) {  // the dirty bytes of this word's vertices are cleared
        uint32_t *d4 = reinterpret_cast<uint32_t *>(dirty + (int64_t)w * 32);
#pragma unroll
        for (int q = 0; q < 8; q++) d4[q] = 0u;
    }
}

// Receiving side of the sync set: values other parts emitted for vertices
// this part holds (global id -> local id by binary search in the ascending
// l2g map; ids it does not hold are ignored) are merged by integer min; a
// replica whose value falls becomes active in the next superstep.
__global__ __launch_bounds__(256) void k_apply_delta(const int32_t *__restrict__ gid,
                                                     const uint32_t *__restrict__ vals, uint32_t n,
                                                     const int32_t *__restrict__ l2g, int64_t V,
                                                     uint32_t *__restrict__ val, uint8_t *__restrict__ front_next) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t g = gid[i];
    int64_t x;
    if (l2g) {
        int64_t lo = 0, hi = V;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (l2g[mid] < g) lo = mid + 1;
            else hi = mid;
        }
        if (lo >= V || l2g[lo] != g) return;
        x = lo;
    } else {
        if (g < 0 || g >= V) return;
        x = g;
    }
    const uint32_t v = vals[i];
    if (v < val[x]) {  // below the value before the merge: the replica changes
        atomicMin(&val[x], v);
        front_next[x] = 1;
    }
}

__global__ void k_zero_step(DevStep *step) { *step = DevStep{}; }
__global__ void k_set_u32(uint32_t *p, uint32_t v) { *p = v; }

// ------------------------------------------------------------ separate template calls

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// MSGApply of SSSP / CC: a vertex whose merged message is below its value
// takes it, and is marked for the next MSGGen and for the sync set; the
// accumulator is reset for the next merge.
__global__ __launch_bounds__(256) void k_ph_apply(uint32_t *__restrict__ acc, uint32_t *__restrict__ val,
                                                  uint8_t *__restrict__ pend, uint8_t *__restrict__ dirty, int64_t V,
                                                  DevStep *step) {
    __shared__ unsigned long long s_c[4];
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned c = 0;
    if (v < V) {
        const uint32_t a = acc[v];
        if (a != INF) {
            acc[v] = INF;
            if (a < val[v]) {
                val[v] = a;
                pend[v] = 1;
                dirty[v] = 1;
                c = 1;
            }
        }
    }
    const unsigned long long t = block_sum<unsigned long long>((unsigned long long)c, s_c);
    if (threadIdx.x == 0 && t) atomicAdd(&step->changed, t);
}

// MSGGen of PageRank: every vertex's message x[u]/outdeg(u) and the
// dangling mass (per-workgroup partials, summed in order by k_reduce_D).
// (master != NULL: a part of a vertex-cut; only its masters' dangling mass
// counts, every other part counts its own masters)
__global__ __launch_bounds__(256) void k_ph_pr_gen(const float *__restrict__ x, const int32_t *__restrict__ outdeg,
                                                   const int32_t *__restrict__ slot, float *__restrict__ contrib,
                                                   int64_t V, double *dpart, const uint32_t *__restrict__ master) {
    __shared__ double s_d[4];
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double dl = 0.0;
    if (v < V) {
        const float xv = x[v];
        const int od = outdeg[v];
        contrib[slot[v]] = od > 0 ? xv / (float)od : 0.0f;
        if (od == 0 && (!master || bit_of(master, v))) dl = (double)xv;
    }
    const double t = block_sum<double>(dl, s_d);
    if (threadIdx.x == 0) dpart[blockIdx.x] = t;
}

// MSGApply of PageRank: x' = (1-d)/V + d * (merged + D/V), in place.
__global__ __launch_bounds__(256) void k_ph_pr_apply(const double *__restrict__ acc, float *__restrict__ x, int64_t V,
                                                     double base, double d, const double *__restrict__ Dp,
                                                     double inv_V, DevStep *step, DevStep *next,
                                                     const uint32_t *__restrict__ master) {
    __shared__ unsigned long long s_c[4];
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double dD = d * (*Dp) * inv_V;
    unsigned c = 0;
    if (v < V && (!master || bit_of(master, v))) {  // a part of a vertex-cut applies at its masters
        const float xn = (float)(base + d * acc[v] + dD);
        c = __float_as_uint(xn) != __float_as_uint(x[v]);
        x[v] = xn;
    }
    const unsigned long long t = block_sum<unsigned long long>((unsigned long long)c, s_c);
    if (threadIdx.x == 0) {
        if (t) atomicAdd(&step->changed, t);
        if (blockIdx.x == 0) *next = DevStep{};
    }
}

template <class T>
inline unsigned grid_for(T n, unsigned block) {
    return (unsigned)std::max<T>(1, (n + block - 1) / block);
}

}  // namespace

// ------------------------------------------------------------------ host

template <class K>
static int persistent_grid(gx_graph *g, K kernel, int block) {
    return g->num_cus * occupancy_per_cu(reinterpret_cast<const void *>(kernel), block);
}

// Persistent grid of the relaxation: whole multiples of the slice count (a
// pulling XCD's workgroups share its slice's units evenly).
static int relax_grid_for(gx_graph *g, const gx_params *p) {
    const int pg = p->algo == GX_CC ? persistent_grid(g, k_relax<false>, 256) : persistent_grid(g, k_relax<true>, 256);
    return std::max(PULL_SLICES, pg / PULL_SLICES * PULL_SLICES);
}

// Fix-up entries per relaxation workgroup: the records of the pull units a
// workgroup sweeps (the j-th workgroup on the XCD of slice x takes units j,
// j + nper, ... of slice x), maximised over x and j, so a region never
// overflows.
static uint32_t fix_cap_for(const gx_graph *g, const gx_params *p, int grid) {
    const DevGraph &d = g->d;
    const bool cc = p->algo == GX_CC;
    const bool has_pull = cc ? d.pull_sym != nullptr : d.pull_w != nullptr;
    if (!has_pull) return 0;
    const PullSlices &sl = cc ? d.pull_sym_off : d.pull_w_off;
    const std::vector<uint32_t> &recs = cc ? g->pull_sym_recs : g->pull_w_recs;
    const int64_t nper = grid / PULL_SLICES;
    uint64_t bound = 0;
    for (int x = 0; x < PULL_SLICES; x++)
        for (int64_t j = 0; j < nper; j++) {
            uint64_t sum = 0;
            for (int64_t u = sl.uoff[x] + j; u < sl.uoff[x + 1]; u += nper) sum += recs[(size_t)u];
            bound = std::max(bound, sum);
        }
    return (uint32_t)std::min<uint64_t>(bound, (1u << FIX_ROT_SHIFT) - 1u);
}

static size_t state_layout(gx_graph *g, const gx_params *p, Carver &c, gx_state *s) {
    const DevGraph &d = g->d;
    int64_t V = d.V;
    int32_t W = d.W;
    if (p->algo == GX_LP) {
        lp_layout(g, c, s);
    } else if (p->algo == GX_PAGERANK) {
        int32_t nt = d.pr_ntiles;
        s->x[0] = c.take<float>(V);
        s->x[1] = c.take<float>(V);
        s->contrib[0] = c.take<float>(V);
        s->contrib[1] = c.take<float>(V);
        s->synced = c.take<uint32_t>(V);
        s->head = c.take<double>(nt);
        s->tailp = c.take<double>(nt);
        s->spill_row = c.take<int32_t>(nt);
        s->dpart = c.take<double>(std::max<int64_t>(nt, grid_for<int64_t>(V, 256)));
        s->cpart = c.take<uint32_t>(std::max<int64_t>(nt, 1));
        s->Dval = c.take<double>(1);
        s->pr_fix_grid = (int)std::min<int64_t>(PR_FIX_MAX_GRID, std::max<int64_t>(1, (nt + PR_FIX_BLOCK - 1) / PR_FIX_BLOCK));
        s->fix_d = c.take<double>(s->pr_fix_grid);
        s->fix_c = c.take<unsigned long long>(s->pr_fix_grid);
        s->fix_done = c.take<uint32_t>(1);
    } else {
        int64_t Eimg = p->algo == GX_SSSP ? d.E : d.E_sym;
        s->val = c.take<uint32_t>(V);
        // byte maps padded to whole 32-vertex words (the sync set reads 32 at a time)
        s->front8[0] = c.take<uint8_t>((size_t)W * 32);
        s->front8[1] = c.take<uint8_t>((size_t)W * 32);
        s->dirty8 = c.take<uint8_t>((size_t)W * 32);
        s->list = c.take<uint4>(V);
        s->tile_start = c.take<uint32_t>(Eimg / PUSH_TILE + 2);
        s->snap = c.take<uint32_t>(V);
        s->relax_grid = relax_grid_for(g, p);
        s->fix_cap = fix_cap_for(g, p, s->relax_grid);
        s->fix = c.take<uint2>((size_t)s->relax_grid * s->fix_cap);
        s->fixn = c.take<uint32_t>(s->relax_grid);
    }
    if (p->phases) {
        if (p->algo == GX_PAGERANK) {
            s->acc_d = c.take<double>(V);
            s->Dscratch = c.take<double>(1);
            s->ph_steps = c.take<DevStep>(2);
        } else {
            s->acc = c.take<uint32_t>(V);
            s->junk8 = c.take<uint8_t>((size_t)W * 32);
        }
    }
    s->steps = c.take<DevStep>(STEP_RING);
    s->delta_blocks = (int)grid_for<int64_t>(W, 256);
    s->blk_cnt = c.take<uint32_t>(s->delta_blocks);
    s->delta_total = c.take<uint32_t>(1);
    return c.used;
}

static gx_status check_params(const gx_graph *g, const gx_params *p) {
    GX_REQUIRE(g, GX_EINVAL, "graph is NULL");
    GX_REQUIRE(p, GX_EINVAL, "params is NULL");
    GX_REQUIRE(!g->dev_error, GX_EDEVICE, "graph handle has a sticky device error");
    GX_REQUIRE(p->algo == GX_PAGERANK || p->algo == GX_SSSP || p->algo == GX_CC || p->algo == GX_LP, GX_EINVAL,
               "algo %d not supported by the plain engine", p->algo);
    GX_REQUIRE(p->delta_mode <= GX_DELTA_MASTERS, GX_EINVAL, "delta_mode %u invalid", p->delta_mode);
    GX_REQUIRE(p->delta_mode != GX_DELTA_MASTERS || g->d.master_rep, GX_EINVAL,
               "GX_DELTA_MASTERS needs a partitioned graph (flags)");
    GX_REQUIRE(p->phases <= GX_PHASES_MASTERS, GX_EINVAL, "phases %u invalid", p->phases);
    GX_REQUIRE(!p->phases || p->algo != GX_LP, GX_EINVAL, "the separate template calls serve PageRank, SSSP and CC");
    GX_REQUIRE(p->phases != GX_PHASES_MASTERS || (p->algo == GX_PAGERANK && g->d.outdeg_g && g->d.master), GX_EINVAL,
               "GX_PHASES_MASTERS is PageRank on a part loaded with flags, V_global and outdeg_global");
    if (p->algo == GX_PAGERANK) {
        GX_REQUIRE(g->needs & GX_NEED_IN, GX_EINVAL, "PageRank needs GX_NEED_IN");
        GX_REQUIRE(p->damping >= 0.f && p->damping < 1.f, GX_EINVAL, "damping %f out of [0,1)", p->damping);
    }
    if (p->algo == GX_SSSP) {
        GX_REQUIRE(g->needs & GX_NEED_OUT, GX_EINVAL, "SSSP needs GX_NEED_OUT");
        GX_REQUIRE(p->source >= -1 && p->source < g->d.V, GX_EINVAL, "source %d out of [-1,V)", p->source);
    }
    if (p->algo == GX_CC) GX_REQUIRE(g->needs & GX_NEED_SYM, GX_EINVAL, "CC needs GX_NEED_SYM");
    if (p->algo == GX_LP) {
        GX_REQUIRE(g->needs & GX_NEED_SYM, GX_EINVAL, "LP needs GX_NEED_SYM");
        int64_t slots = 0;
        for (int32_t d : g->host_symdeg)
            if (d > LP_MID_MAX) slots += 3 * (int64_t)d + 256;
        GX_REQUIRE(slots < (int64_t(1) << 32), GX_EINVAL, "LP hub tables would exceed 2^32 slots");
    }
    return GX_OK;
}

extern "C" gx_status gx_state_bytes(const gx_graph *g, const gx_params *p, size_t *bytes) {
    clear_error();
    GX_REQUIRE(bytes, GX_EINVAL, "bytes is NULL");
    gx_status st = check_params(g, p);
    if (st != GX_OK) return st;
    Carver c(nullptr, 0);
    gx_state tmp;
    *bytes = state_layout(const_cast<gx_graph *>(g), p, c, &tmp);
    return GX_OK;
}

extern "C" gx_status gx_state_init(gx_graph *g, const gx_params *p, void *dev_state, size_t bytes, void *stream,
                                   gx_state **out) {
    clear_error();
    GX_REQUIRE(out, GX_EINVAL, "out is NULL");
    *out = nullptr;
    gx_status st = check_params(g, p);
    if (st != GX_OK) return st;
    GX_REQUIRE(dev_state, GX_EINVAL, "dev_state is NULL");
    GX_REQUIRE(reinterpret_cast<uintptr_t>(dev_state) % ALIGN == 0, GX_EINVAL, "dev_state not 256-byte aligned");
    {
        Carver m(nullptr, 0);
        gx_state tmp;
        size_t need = state_layout(g, p, m, &tmp);
        GX_REQUIRE(need <= bytes, GX_ENOMEM, "state buffer too small: need %zu bytes, have %zu", need, bytes);
    }
    gx_state *s = new (std::nothrow) gx_state();
    GX_REQUIRE(s, GX_ENOMEM, "host allocation failed");
    s->g = g;
    s->p = *p;
    s->mem = dev_state;
    // GX_XCD_CHECK_SHIFT (tests only) offsets the XCD the odd pull workgroups
    // see, so that the rotation check fires without a real fault
    if (const char *e = std::getenv("GX_XCD_CHECK_SHIFT")) s->xcd_shift = (uint32_t)std::strtoul(e, nullptr, 10);
    Carver c(dev_state, bytes);
    state_layout(g, p, c, s);
    if (p->algo == GX_SSSP || p->algo == GX_CC) {
        const DevGraph &dg = g->d;
        // (the pull addresses values through a 32-bit buffer range)
        bool can_pull = dg.V < (int64_t(1) << 30) &&
                        (p->algo == GX_SSSP ? (dg.pull_w != nullptr) : (dg.pull_sym != nullptr));
        double frac = p->pull_fraction > 0.f ? (double)p->pull_fraction : 0.3;
        double Eimg = (double)(p->algo == GX_SSSP ? dg.E : dg.E_sym);
        s->pull_edges = (!can_pull || frac >= 1.0) ? 0xFFFFFFFFu : (uint32_t)std::max(1.0, std::ceil(frac * Eimg));
    }
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const DevGraph &d = g->d;
    int64_t V = d.V;
    if (p->algo == GX_LP) {
        gx_status ls = lp_init(s, hs);
        if (ls != GX_OK) {
            delete s;
            return ls;
        }
    } else if (p->algo == GX_PAGERANK) {
        const int64_t Vn = p->phases == GX_PHASES_MASTERS ? d.V_global : V;
        float x0 = V > 0 ? (float)(1.0 / (double)Vn) : 0.f;
        unsigned nb = grid_for<int64_t>(V, 256);
        hipLaunchKernelGGL(k_pr_init, dim3(nb), dim3(256), 0, hs, s->x[0], s->contrib[0], s->synced, d.outdeg,
                           d.pr_slot, V, x0, s->dpart, s->steps);
        hipLaunchKernelGGL(k_reduce_D, dim3(1), dim3(1024), 0, hs, s->dpart, (int)nb, s->Dval);
        (void)hipMemsetAsync(s->fix_done, 0, sizeof(uint32_t), hs);
    } else {
        int64_t n = std::max<int64_t>(V, d.W);
        const int32_t *rp = p->algo == GX_CC ? d.sym_rp : d.out_rp;
        // (padding bytes of the maps beyond V are cleared too)
        hipLaunchKernelGGL(k_min_init, dim3(grid_for<int64_t>(n, 256)), dim3(256), 0, hs, s->val, s->front8[0],
                           s->front8[1], s->dirty8, d.l2g, rp, V, p->algo, p->source, s->steps);
        if ((int64_t)d.W * 32 > V) {
            size_t pad = (size_t)d.W * 32 - (size_t)V;
            (void)hipMemsetAsync(s->front8[0] + V, 0, pad, hs);
            (void)hipMemsetAsync(s->front8[1] + V, 0, pad, hs);
            (void)hipMemsetAsync(s->dirty8 + V, 0, pad, hs);
        }
        if (p->phases && V > 0)
            hipLaunchKernelGGL(k_fill_u32, dim3(grid_for<int64_t>(V, 256)), dim3(256), 0, hs, s->acc, V, INF);
        // compaction of superstep 0 (each superstep then relaxes and compacts the
        // next); with separate template calls the first MSGGen does it
        if (V > 0 && !p->phases)
            hipLaunchKernelGGL(k_compact, dim3(grid_for<int64_t>(V, CBLOCK * CVT)), dim3(CBLOCK), 0, hs, s->front8[0],
                               s->front8[1], rp, s->val, s->snap, V, s->list, s->tile_start, s->steps,
                               s->steps + 1, (int)(s->pull_edges != 0xFFFFFFFFu), nullptr, nullptr, s->pull_edges);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("state init launch failed: %s", hipGetErrorString(e));
        delete s;
        return GX_EDEVICE;
    }
    *out = s;
    return GX_OK;
}

extern "C" gx_status gx_state_free(gx_state *s) {
    clear_error();
    delete s;
    return GX_OK;
}

// The current vertex values (PageRank ranks move between two buffers per
// superstep, except under separate template calls, which update in place).
static uint32_t *cur_values(const gx_state *s) {
    if (s->p.algo == GX_PAGERANK)
        return reinterpret_cast<uint32_t *>(s->x[s->p.phases ? 0 : (s->k & 1)]);
    if (s->p.algo == GX_LP) return s->lab[s->k & 1];
    return s->val;
}

extern "C" gx_status gx_state_values(gx_state *s, void **dev_values) {
    clear_error();
    GX_REQUIRE(s && dev_values, GX_EINVAL, "NULL argument");
    *dev_values = cur_values(s);
    return GX_OK;
}

extern "C" gx_status gx_state_frontier(gx_state *s, void **dev_bitmap) {
    clear_error();
    GX_REQUIRE(s && dev_bitmap, GX_EINVAL, "NULL argument");
    GX_REQUIRE(s->p.algo == GX_SSSP || s->p.algo == GX_CC, GX_EINVAL, "only SSSP and CC keep a frontier");
    // (separate template calls: the vertices the next MSGGen sends from)
    *dev_bitmap = s->front8[s->p.phases ? s->ph_p : (s->k & 1)];
    return GX_OK;
}

extern "C" gx_status gx_state_superstep(gx_state *s, int64_t *k) {
    clear_error();
    GX_REQUIRE(s && k, GX_EINVAL, "NULL argument");
    *k = s->k;
    return GX_OK;
}

// Process-wide pool of timing events (creating events per superstep costs
// more than the short supersteps themselves).  They only time kernels and are
// read after a stream synchronisation, so they skip the system-scope fence: a
// fenced record writes back and invalidates the caches between the kernels
// it separates, a gap of several microseconds per superstep.
static std::mutex g_ev_mu;
static std::vector<hipEvent_t> g_ev_free;

static hipEvent_t pool_event(gx_state *s) {
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    {
        std::lock_guard<std::mutex> lk(g_ev_mu);
        if (!g_ev_free.empty()) {
            hipEvent_t e = g_ev_free.back();
            g_ev_free.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

static void pool_return(hipEvent_t e) {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    g_ev_free.push_back(e);
}

// Process-wide pool of pinned buffers for reading superstep counters back.
constexpr int HOST_STEPS = 256;
static std::vector<DevStep *> g_hs_free;

static DevStep *host_steps_take() {
    {
        std::lock_guard<std::mutex> lk(g_ev_mu);
        if (!g_hs_free.empty()) {
            DevStep *p = g_hs_free.back();
            g_hs_free.pop_back();
            return p;
        }
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, HOST_STEPS * sizeof(DevStep), hipHostMallocDefault) != hipSuccess) return nullptr;
    return static_cast<DevStep *>(p);
}

static void host_steps_return(DevStep *p) {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    g_hs_free.push_back(p);
}

extern "C" gx_status gx_release_cached(void) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_ev_mu);
    hipError_t first = hipSuccess;
    for (hipEvent_t e : g_ev_free) {
        hipError_t r = hipEventDestroy(e);
        if (first == hipSuccess) first = r;
    }
    g_ev_free.clear();
    for (DevStep *p : g_hs_free) {
        hipError_t r = hipHostFree(p);
        if (first == hipSuccess) first = r;
    }
    g_hs_free.clear();
    GX_REQUIRE(first == hipSuccess, GX_EDEVICE, "releasing cached resources failed: %s", hipGetErrorString(first));
    return GX_OK;
}

// Enqueues superstep s->k on `hs` and advances s->k.
static gx_status enqueue_superstep(gx_state *s, hipStream_t hs) {
    const DevGraph &d = s->g->d;
    const gx_params &p = s->p;
    DevStep *step = s->steps + (s->k % STEP_RING);
    DevStep *next = s->steps + ((s->k + 1) % STEP_RING);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (p.timing) {
        e0 = pool_event(s);
        e1 = pool_event(s);
    }
    if (p.algo == GX_LP) {
        if (e0) (void)hipEventRecord(e0, hs);
        lp_enqueue(s, hs, step, next);
        if (e1) (void)hipEventRecord(e1, hs);
    } else if (p.algo == GX_PAGERANK) {
        int cur = (int)(s->k & 1);
        double dd = p.damping;
        PrApply ap{(1.0 - dd) / (double)d.V, dd, 0.0, d.outdeg, s->x[cur], s->x[cur ^ 1], s->contrib[cur ^ 1],
                   d.pr_slot};
        double inv_V = d.V > 0 ? 1.0 / (double)d.V : 0.0;
        if (d.V > 0) {
            if (e0) (void)hipEventRecord(e0, hs);
            auto pull = d.pr_tile == 256 ? k_pr_pull<1, PrApply> : d.pr_tile == 512 ? k_pr_pull<2, PrApply>
                      : d.pr_tile == 1024 ? k_pr_pull<4, PrApply> : k_pr_pull<8, PrApply>;
            hipLaunchKernelGGL(pull, dim3(d.pr_ntiles), dim3(PR_BLOCK), 0, hs, d.in_rp, d.pr_src, d.pr_tile_row,
                               d.E, s->contrib[cur], ap, s->Dval, inv_V, s->head, s->tailp, s->spill_row, s->dpart,
                               s->cpart);
            if (e1) (void)hipEventRecord(e1, hs);
            hipLaunchKernelGGL(k_pr_fix<PrApply>, dim3(s->pr_fix_grid), dim3(PR_FIX_BLOCK), 0, hs, d.in_rp, d.pr_ntiles,
                               d.pr_tile, s->head, s->tailp, s->spill_row, s->dpart, s->cpart, ap, s->Dval, inv_V,
                               step, next, s->fix_d, s->fix_c, s->fix_done);
        }
    } else {
        // superstep k: relax A_k (list built by the previous compaction), then
        // compact A_{k+1} for superstep k+1
        const int cur = (int)(s->k & 1);
        const bool cc = p.algo == GX_CC;
        const int32_t *rp = cc ? d.sym_rp : d.out_rp;
        DevStep *next2 = s->steps + ((s->k + 2) % STEP_RING);
        if (d.V > 0) {
            if (e0) (void)hipEventRecord(e0, hs);
            if (!cc) {
                const PullArgs pa{d.pull_w, d.pull_w_units, d.pull_w_off};
                hipLaunchKernelGGL(k_relax<true>, dim3(s->relax_grid), dim3(256), 0, hs, s->list, s->tile_start,
                                   (const void *)d.out_adj, pa, d.V, s->snap, s->val, s->front8[cur], s->front8[cur ^ 1],
                                   step, s->pull_edges, s->fix, s->fixn, s->fix_cap, s->xcd_shift);
            } else {
                const PullArgs pa{d.pull_sym, d.pull_sym_units, d.pull_sym_off};
                hipLaunchKernelGGL(k_relax<false>, dim3(s->relax_grid), dim3(256), 0, hs, s->list, s->tile_start,
                                   (const void *)d.sym_col, pa, d.V, s->snap, s->val, s->front8[cur], s->front8[cur ^ 1],
                                   step, s->pull_edges, s->fix, s->fixn, s->fix_cap, s->xcd_shift);
            }
            hipLaunchKernelGGL(k_fixup, dim3(s->relax_grid), dim3(256), 0, hs, s->fix, s->fixn, s->fix_cap, s->val,
                               step);
            if (e1) (void)hipEventRecord(e1, hs);
            hipLaunchKernelGGL(k_compact, dim3(grid_for<int64_t>(d.V, CBLOCK * CVT)), dim3(CBLOCK), 0, hs,
                               s->front8[cur ^ 1], s->front8[cur], rp, s->val, s->snap, d.V, s->list, s->tile_start,
                               next, next2, (int)(s->pull_edges != 0xFFFFFFFFu), step, s->dirty8, s->pull_edges);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("superstep launch failed: %s", hipGetErrorString(e));
        s->dev_error = true;
        return GX_EDEVICE;
    }
    if (e0 && e1) s->ev_pending.push_back({s->k, e0, e1});
    s->k++;
    return GX_OK;
}

// After a stream synchronisation: fold the pending kernel timings of
// supersteps before k_end (later ones were enqueued speculatively after
// convergence and do no work of the solve); with `per_step`, superstep k's
// time goes to per_step[k - k0] when in range.
static void collect_timings(gx_state *s, gx_step_stats *per_step = nullptr, int64_t k0 = 0, int64_t n = 0,
                            int64_t k_end = INT64_MAX) {
    for (auto &pr : s->ev_pending) {
        float ms = 0.f;
        if (pr.k < k_end && hipEventElapsedTime(&ms, pr.a, pr.b) == hipSuccess) {
            s->kernel_ms += ms;
            s->kernel_launches++;
            if (per_step && pr.k >= k0 && pr.k < k0 + n) per_step[pr.k - k0].kernel_ms = ms;
        }
        s->ev_pool.push_back(pr.a);
        s->ev_pool.push_back(pr.b);
    }
    s->ev_pending.clear();
}

// `next` is the slot of the following superstep: for SSSP/CC the number of
// vertices a superstep changed is the size of the next frontier.
static void to_stats(const gx_state *s, const DevStep &ds, const DevStep &next, gx_step_stats *o) {
    if (s->p.algo == GX_PAGERANK) {
        o->frontier = s->g->d.V;
        o->edges = s->g->d.E;
        o->pulled = 1;
        o->changed = (int64_t)ds.changed;
    } else if (s->p.algo == GX_LP) {
        o->frontier = lp_active(s);
        o->edges = s->g->d.E_sym;
        o->pulled = 1;
        o->changed = (int64_t)ds.changed;
    } else {
        o->frontier = (int64_t)ds.frontier;
        o->edges = (int64_t)(uint32_t)ds.list;
        o->pulled = ds.pad ? 1 : 0;
        o->changed = (int64_t)next.frontier;
    }
    o->kernel_ms = 0.0;
}

static gx_status read_steps(gx_state *s, int64_t kfirst, uint32_t n, hipStream_t hs, std::vector<DevStep> &out);

extern "C" gx_status gx_superstep(gx_state *s, void *stream, gx_step_stats *stats) {
    clear_error();
    GX_REQUIRE(s, GX_EINVAL, "state is NULL");
    GX_REQUIRE(!s->p.phases, GX_EINVAL, "this state is driven by gx_msg_gen / gx_msg_merge / gx_msg_apply");
    GX_REQUIRE(!s->dev_error && !s->g->dev_error, GX_EDEVICE, "sticky device error");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    int64_t k = s->k;
    gx_status st = enqueue_superstep(s, hs);
    if (st != GX_OK) return st;
    if (stats) {
        std::vector<DevStep> ds;
        st = read_steps(s, k, 2, hs, ds);
        if (st != GX_OK) return st;
        to_stats(s, ds[0], ds[1], stats);
        collect_timings(s, stats, k, 1);
    }
    return GX_OK;
}

// Copies the counters of supersteps [kfirst, kfirst + n) to out[] through the
// state's pinned buffer (ring-contiguous pieces, one synchronisation).
static gx_status read_steps(gx_state *s, int64_t kfirst, uint32_t n, hipStream_t hs, std::vector<DevStep> &out) {
    out.resize(n);
    if (!s->host_steps) s->host_steps = host_steps_take();
    GX_REQUIRE(s->host_steps, GX_ENOMEM, "pinned host allocation failed");
    for (uint32_t done = 0; done < n;) {
        uint32_t chunk = std::min<uint32_t>(n - done, HOST_STEPS);
        uint32_t copied = 0;
        while (copied < chunk) {
            int64_t k = kfirst + done + copied;
            uint32_t slot = (uint32_t)(k % STEP_RING);
            uint32_t run = std::min<uint32_t>(chunk - copied, STEP_RING - slot);
            GX_CHECK_HIP(hipMemcpyAsync(s->host_steps + copied, s->steps + slot, run * sizeof(DevStep),
                                        hipMemcpyDeviceToHost, hs),
                         s);
            copied += run;
        }
        GX_CHECK_HIP(hipStreamSynchronize(hs), s);
        std::memcpy(out.data() + done, s->host_steps, chunk * sizeof(DevStep));
        done += chunk;
    }
    for (uint32_t i = 0; i < n; i++)
        if (out[i].rot_mixed) {
            s->dev_error = true;
            set_error("superstep %lld pulled with workgroups dealt to the XCDs in more than one rotation; some "
                      "work units may have run on an XCD other than the one owning their destinations, so the "
                      "values may be wrong; run with pull_fraction >= 1 (push only) on this device",
                      (long long)(kfirst + i));
            return GX_EDEVICE;
        }
    return GX_OK;
}

// PageRank supersteps k .. k+n-1 as one HIP graph launch on `hs`.  The
// kernels' arguments depend only on the state's memory, the damping and the
// ring slot of k (which also fixes the buffer parity), so the graph is
// captured once, on the graph handle's private stream, and replayed by every
// run that starts from the same slot with the same count, also by a state
// created again in the same memory (what a reset does).  A superstep
// enqueues two kernels and no memory set.  Returns false, having enqueued
// nothing, when timing events are on, for a single superstep, or when capture
// is not available; the caller then enqueues the supersteps one by one.
static bool pr_replay(gx_state *s, uint32_t n, hipStream_t hs) {
    gx_graph *g = s->g;
    if (s->p.timing || n < 2 || g->d.V == 0) return false;
    const int64_t slot = s->k % STEP_RING, k0 = s->k;
    const double damping = s->p.damping;
    std::lock_guard<std::mutex> lk(g->pr_mu);
    hipGraphExec_t exec = nullptr;
    for (auto &e : g->pr_graphs)
        if (e.mem == s->mem && e.damping == damping && e.slot == slot && e.n == n) exec = e.exec;
    if (!exec) {
        if (!g->cap_stream && hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking) != hipSuccess) {
            g->cap_stream = nullptr;
            return false;
        }
        if (hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
        bool ok = true;
        for (uint32_t i = 0; i < n && ok; i++) ok = enqueue_superstep(s, g->cap_stream) == GX_OK;
        hipGraph_t graph = nullptr;
        ok = hipStreamEndCapture(g->cap_stream, &graph) == hipSuccess && ok && graph;
        ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        s->k = k0;
        (void)hipGetLastError();
        if (!ok) {
            s->dev_error = false;  // a capture that failed launched nothing
            clear_error();
            return false;
        }
        if (g->pr_graphs.size() >= gx_graph::PR_GRAPHS) {
            (void)hipGraphExecDestroy(g->pr_graphs.front().exec);
            g->pr_graphs.erase(g->pr_graphs.begin());
        }
        g->pr_graphs.push_back({s->mem, damping, slot, n, exec});
    }
    if (hipGraphLaunch(exec, hs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    s->k = k0 + n;
    return true;
}

extern "C" gx_status gx_run_until_converged(gx_state *s, uint32_t max_supersteps, void *stream, gx_run_stats *out,
                                            gx_step_stats *per_step) {
    clear_error();
    GX_REQUIRE(s, GX_EINVAL, "state is NULL");
    GX_REQUIRE(!s->p.phases, GX_EINVAL, "this state is driven by gx_msg_gen / gx_msg_merge / gx_msg_apply");
    GX_REQUIRE(!s->dev_error && !s->g->dev_error, GX_EDEVICE, "sticky device error");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    auto t0 = std::chrono::steady_clock::now();
    double ms0 = s->kernel_ms;
    int64_t l0 = s->kernel_launches;
    gx_run_stats rs{};
    std::vector<DevStep> host;
    gx_status result = GX_OK;
    const int64_t k_begin = s->k;
    if (s->p.algo == GX_PAGERANK) {
        // In chunks that leave the counter ring room for the chunk's slots
        // plus the following one, so no slot is reused before it is read.
        for (uint32_t done = 0; done < max_supersteps;) {
            const uint32_t g = std::min<uint32_t>(max_supersteps - done, STEP_RING - 2);
            const int64_t kfirst = s->k;
            if (!pr_replay(s, g, hs)) {
                for (uint32_t i = 0; i < g; i++) {
                    gx_status st = enqueue_superstep(s, hs);
                    if (st != GX_OK) return st;
                }
            }
            gx_status st = read_steps(s, kfirst, g + 1, hs, host);
            if (st != GX_OK) return st;
            for (uint32_t i = 0; i < g; i++) {
                gx_step_stats o;
                to_stats(s, host[i], host[i + 1], &o);
                if (per_step) per_step[done + i] = o;
                rs.edges += o.edges;
            }
            done += g;
        }
        rs.supersteps = max_supersteps;
        rs.converged = 0;
    } else {
        // Supersteps are enqueued in speculative groups and the host
        // synchronises once per group; supersteps enqueued after convergence
        // find an empty frontier, change nothing and cost a few microseconds
        // each, less than a host round trip.  The first group covers the
        // superstep count of the last converged run on this graph (which
        // includes the superstep that changed nothing, so a repeat of that
        // run converges inside the group; at least 6, at most 16), the later
        // ones 8 at a time.
        // (label propagation keeps no history: its first group covers 16, the
        // evaluation's cap of 15 plus one)
        const int hist = s->p.algo == GX_CC ? 1 : 0;
        const bool lp = s->p.algo == GX_LP;
        const uint32_t last = lp ? 16u : s->g->last_supersteps[hist].load(std::memory_order_relaxed);
        uint32_t done = 0, spec = std::min<uint32_t>(16, std::max<uint32_t>(6, last));
        bool conv = false;
        while (done < max_supersteps && !conv) {
            uint32_t g = std::min(spec, max_supersteps - done);
            int64_t kfirst = s->k;
            for (uint32_t i = 0; i < g; i++) {
                gx_status st = enqueue_superstep(s, hs);
                if (st != GX_OK) return st;
            }
            gx_status st = read_steps(s, kfirst, g + 1, hs, host);
            if (st != GX_OK) return st;
            for (uint32_t i = 0; i < g; i++) {
                gx_step_stats o;
                to_stats(s, host[i], host[i + 1], &o);
                if (per_step) per_step[done] = o;
                rs.edges += o.edges;
                done++;
                if (o.changed == 0) {
                    conv = true;
                    s->k = kfirst + i + 1;
                    break;
                }
            }
            spec = 8;
        }
        rs.supersteps = done;
        rs.converged = conv ? 1 : 0;
        if (conv && k_begin == 0 && !lp) s->g->last_supersteps[hist].store(done, std::memory_order_relaxed);
        if (!conv) {
            set_error("not converged after %u supersteps", max_supersteps);
            result = GX_ENOTCONVERGED;
        }
    }
    collect_timings(s, per_step, k_begin, rs.supersteps, k_begin + rs.supersteps);
    rs.edge_kernel_ms = s->kernel_ms - ms0;
    rs.edge_kernel_launches = s->kernel_launches - l0;
    rs.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (out) *out = rs;
    return result;
}

extern "C" gx_status gx_sync_delta(gx_state *s, int32_t *dev_gid, uint32_t *dev_val, uint32_t cap, uint32_t *count,
                                   int32_t *skippable, void *stream) {
    clear_error();
    GX_REQUIRE(s && count, GX_EINVAL, "NULL argument");
    GX_REQUIRE(cap == 0 || (dev_gid && dev_val), GX_EINVAL, "output buffers are NULL");
    GX_REQUIRE(!s->dev_error && !s->g->dev_error, GX_EDEVICE, "sticky device error");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const DevGraph &d = s->g->d;
    *count = 0;
    if (skippable) *skippable = 1;
    if (d.W == 0) return GX_OK;
    bool all = s->p.delta_mode == GX_DELTA_ALL;
    const uint32_t *remote = s->p.delta_mode == GX_DELTA_MASTERS              ? d.master_rep
                           : (s->p.algo == GX_CC || s->p.algo == GX_LP) ? d.remote_any
                                                                        : d.remote_out;
    // PageRank and LP compare with the synced copy (LP labels can return to an
    // earlier value); SSSP / CC values only fall, so the dirty map decides
    const bool by_copy = s->p.algo == GX_PAGERANK || s->p.algo == GX_LP;
    const uint32_t *vals = cur_values(s);
    uint8_t *dirty = by_copy ? nullptr : s->dirty8;
    uint32_t *synced = by_copy ? s->synced : nullptr;
    hipLaunchKernelGGL(k_delta_count, dim3(s->delta_blocks), dim3(256), 0, hs, d.W, d.V, remote, (int)all, dirty,
                       vals, synced, s->blk_cnt);
    hipLaunchKernelGGL(k_delta_emit, dim3(s->delta_blocks), dim3(256), 0, hs, d.W, d.V, remote, (int)all, dirty,
                       vals, synced, d.l2g, s->blk_cnt, s->delta_blocks, cap, dev_gid, dev_val, s->delta_total);
    GX_CHECK_HIP(hipGetLastError(), s);
    uint32_t total = 0;
    GX_CHECK_HIP(hipMemcpyAsync(&total, s->delta_total, 4, hipMemcpyDeviceToHost, hs), s);
    GX_CHECK_HIP(hipStreamSynchronize(hs), s);
    *count = total;
    if (skippable) *skippable = total == 0;
    if (total > cap) {
        set_error("sync set has %u entries, capacity %u", total, cap);
        return GX_ENOMEM;
    }
    return GX_OK;
}

// ------------------------------------------------------------ sync set, no allocation
// The per-workgroup counts of gx_sync_delta_noalloc live in this array: one
// copy per GPU, held until the process ends, shared by every call on that
// GPU.  Host code never passes its name to a kernel (on the host it is only a
// stand-in symbol): the device address of each GPU's copy is looked up once
// with hipGetSymbolAddress, with that GPU current, and kept in g_scratch_ptr.
// Every count a launch reads is written earlier in the same call, so nothing
// in the array has to start at zero.
constexpr int NOALLOC_SCRATCH_WORDS = 65536;  // 256 KiB: sync sets of up to 2^29 vertices
static __device__ __align__(256) uint32_t scratch[NOALLOC_SCRATCH_WORDS];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static uint32_t *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

static gx_status scratch_for_device(int device, uint32_t **out) {
    GX_REQUIRE(device >= 0 && device < NOALLOC_MAX_DEVICES, GX_EINVAL, "device ordinal %d out of range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void *ptr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) {
            set_error("hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                      hipGetErrorString(e == hipSuccess ? hipErrorInvalidSymbol : e));
            return GX_EDEVICE;
        }
        g_scratch_ptr[device] = static_cast<uint32_t *>(ptr);
    }
    *out = g_scratch_ptr[device];
    return GX_OK;
}

extern "C" gx_status gx_sync_delta_noalloc(gx_state *s, int32_t *dev_gid, uint32_t *dev_val, uint32_t cap,
                                           uint32_t *dev_count, void *stream) {
    clear_error();
    GX_REQUIRE(s && dev_count, GX_EINVAL, "NULL argument");
    GX_REQUIRE(cap == 0 || (dev_gid && dev_val), GX_EINVAL, "output buffers are NULL");
    GX_REQUIRE(!s->dev_error && !s->g->dev_error, GX_EDEVICE, "sticky device error");
    GX_REQUIRE(s->delta_blocks <= NOALLOC_SCRATCH_WORDS, GX_EINVAL,
               "gx_sync_delta_noalloc handles at most %lld vertices (graph has %lld)",
               (long long)NOALLOC_SCRATCH_WORDS * 256 * 32, (long long)s->g->d.V);
    uint32_t *cnt = nullptr;
    gx_status st = scratch_for_device(s->g->device, &cnt);
    if (st != GX_OK) return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const DevGraph &d = s->g->d;
    if (d.W == 0) {  // no vertices: the count is zero (a one-thread kernel, not a memset node)
        hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, hs, dev_count, 0u);
        GX_CHECK_HIP(hipGetLastError(), s);
        return GX_OK;
    }
    bool all = s->p.delta_mode == GX_DELTA_ALL;
    const uint32_t *remote = s->p.delta_mode == GX_DELTA_MASTERS              ? d.master_rep
                           : (s->p.algo == GX_CC || s->p.algo == GX_LP) ? d.remote_any
                                                                        : d.remote_out;
    // PageRank and LP compare with the synced copy (LP labels can return to an
    // earlier value); SSSP / CC values only fall, so the dirty map decides
    const bool by_copy = s->p.algo == GX_PAGERANK || s->p.algo == GX_LP;
    const uint32_t *vals = cur_values(s);
    uint8_t *dirty = by_copy ? nullptr : s->dirty8;
    uint32_t *synced = by_copy ? s->synced : nullptr;
    hipLaunchKernelGGL(k_delta_count, dim3(s->delta_blocks), dim3(256), 0, hs, d.W, d.V, remote, (int)all, dirty,
                       vals, synced, cnt);
    hipLaunchKernelGGL(k_delta_emit, dim3(s->delta_blocks), dim3(256), 0, hs, d.W, d.V, remote, (int)all, dirty,
                       vals, synced, d.l2g, cnt, s->delta_blocks, cap, dev_gid, dev_val, dev_count);
    GX_CHECK_HIP(hipGetLastError(), s);
    return GX_OK;
}

extern "C" gx_status gx_apply_delta(gx_state *s, const int32_t *dev_gid, const uint32_t *dev_val, uint32_t n,
                                    int64_t *active_next, void *stream) {
    clear_error();
    GX_REQUIRE(s, GX_EINVAL, "state is NULL");
    GX_REQUIRE(n == 0 || (dev_gid && dev_val), GX_EINVAL, "input buffers are NULL");
    GX_REQUIRE(!s->dev_error && !s->g->dev_error, GX_EDEVICE, "sticky device error");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const DevGraph &d = s->g->d;
    if (s->p.phases == GX_PHASES_MASTERS) {  // PageRank replicas take their masters' new ranks
        if (n > 0 && d.V > 0)
            hipLaunchKernelGGL(k_replica_set, dim3(grid_for<uint32_t>(n, 256)), dim3(256), 0, hs, dev_gid, dev_val, n,
                               d.l2g, d.V, d.master, reinterpret_cast<uint32_t *>(s->x[0]));
        GX_CHECK_HIP(hipGetLastError(), s);
        if (active_next) *active_next = 0;
        return GX_OK;
    }
    GX_REQUIRE(s->p.algo == GX_SSSP || s->p.algo == GX_CC, GX_EINVAL,
               "gx_apply_delta merges SSSP / CC values (and PageRank ranks under GX_PHASES_MASTERS)");
    GX_REQUIRE(!s->p.phases, GX_EINVAL, "gx_apply_delta serves SSSP / CC states driven by gx_superstep");
    if (d.V > 0) {
        // A_{k+1} (the frontier of the superstep about to run) and its counter slot
        uint8_t *front = s->front8[s->k & 1];
        DevStep *slot = s->steps + (s->k % STEP_RING), *slot2 = s->steps + ((s->k + 1) % STEP_RING);
        if (n > 0)
            hipLaunchKernelGGL(k_apply_delta, dim3(grid_for<uint32_t>(n, 256)), dim3(256), 0, hs, dev_gid, dev_val, n,
                               d.l2g, d.V, s->val, front);
        // rebuild the active list of A_{k+1} from the merged values
        hipLaunchKernelGGL(k_zero_step, dim3(1), dim3(1), 0, hs, slot);
        const int32_t *rp = s->p.algo == GX_CC ? d.sym_rp : d.out_rp;
        hipLaunchKernelGGL(k_compact, dim3(grid_for<int64_t>(d.V, CBLOCK * CVT)), dim3(CBLOCK), 0, hs, front,
                           s->front8[(s->k & 1) ^ 1], rp, s->val, s->snap, d.V, s->list, s->tile_start, slot, slot2,
                           (int)(s->pull_edges != 0xFFFFFFFFu), nullptr, nullptr, s->pull_edges);
        GX_CHECK_HIP(hipGetLastError(), s);
    }
    if (active_next) {
        *active_next = 0;
        if (d.V > 0) {
            DevStep ds{};
            GX_CHECK_HIP(hipMemcpyAsync(&ds, s->steps + (s->k % STEP_RING), sizeof ds, hipMemcpyDeviceToHost, hs), s);
            GX_CHECK_HIP(hipStreamSynchronize(hs), s);
            *active_next = (int64_t)ds.frontier;
        }
    }
    return GX_OK;
}

// ------------------------------------------------------------ separate template calls

static gx_status ph_check(gx_state *s) {
    GX_REQUIRE(s, GX_EINVAL, "state is NULL");
    GX_REQUIRE(s->p.phases, GX_EINVAL, "state was not initialised with gx_params.phases");
    GX_REQUIRE(!s->dev_error && !s->g->dev_error, GX_EDEVICE, "sticky device error");
    return GX_OK;
}

extern "C" gx_status gx_msg_gen(gx_state *s, void *stream) {
    clear_error();
    gx_status st = ph_check(s);
    if (st != GX_OK) return st;
    GX_REQUIRE(!s->ph_msgs, GX_EINVAL, "MSGGen: the previous messages have not been merged");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const DevGraph &d = s->g->d;
    if (d.V > 0) {
        if (s->p.algo == GX_PAGERANK) {
            const unsigned nb = grid_for<int64_t>(d.V, 256);
            const bool parts = s->p.phases == GX_PHASES_MASTERS;
            hipLaunchKernelGGL(k_ph_pr_gen, dim3(nb), dim3(256), 0, hs, s->x[0], parts ? d.outdeg_g : d.outdeg,
                               d.pr_slot, s->contrib[0], d.V, s->dpart, parts ? d.master : nullptr);
            hipLaunchKernelGGL(k_reduce_D, dim3(1), dim3(1024), 0, hs, s->dpart, (int)nb, s->Dval);
        } else {
            // the pending map's vertices become the active list (with the values
            // they send); the other map is cleared to collect the next changes
            const int32_t *rp = s->p.algo == GX_CC ? d.sym_rp : d.out_rp;
            DevStep *step = s->steps + (s->k % STEP_RING), *next = s->steps + ((s->k + 1) % STEP_RING);
            hipLaunchKernelGGL(k_compact, dim3(grid_for<int64_t>(d.V, CBLOCK * CVT)), dim3(CBLOCK), 0, hs,
                               s->front8[s->ph_p], s->front8[s->ph_p ^ 1], rp, s->val, s->snap, d.V, s->list,
                               s->tile_start, step, next, (int)(s->pull_edges != 0xFFFFFFFFu), nullptr, nullptr,
                               s->pull_edges);
        }
        GX_CHECK_HIP(hipGetLastError(), s);
    }
    s->ph_p ^= 1;
    s->ph_msgs = true;
    return GX_OK;
}

extern "C" gx_status gx_msg_merge(gx_state *s, void *stream) {
    clear_error();
    gx_status st = ph_check(s);
    if (st != GX_OK) return st;
    if (!s->ph_msgs) return GX_OK;  // nothing generated since the last merge
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const DevGraph &d = s->g->d;
    if (d.V > 0) {
        if (s->p.algo == GX_PAGERANK) {
            const PrStore ap{(double)s->p.damping, 0.0, s->acc_d};
            const double inv_V = 1.0 / (double)d.V;
            auto pull = d.pr_tile == 256 ? k_pr_pull<1, PrStore> : d.pr_tile == 512 ? k_pr_pull<2, PrStore>
                      : d.pr_tile == 1024 ? k_pr_pull<4, PrStore> : k_pr_pull<8, PrStore>;
            hipLaunchKernelGGL(pull, dim3(d.pr_ntiles), dim3(PR_BLOCK), 0, hs, d.in_rp, d.pr_src, d.pr_tile_row, d.E,
                               s->contrib[0], ap, s->Dscratch, inv_V, s->head, s->tailp, s->spill_row, s->dpart,
                               s->cpart);
            hipLaunchKernelGGL(k_pr_fix<PrStore>, dim3(s->pr_fix_grid), dim3(PR_FIX_BLOCK), 0, hs, d.in_rp,
                               d.pr_ntiles, d.pr_tile, s->head, s->tailp, s->spill_row, s->dpart, s->cpart, ap,
                               s->Dscratch, inv_V, s->ph_steps, s->ph_steps + 1, s->fix_d, s->fix_c, s->fix_done);
        } else {
            // the relaxation of the fused superstep, against the accumulator:
            // it combines the messages by minimum and changes no vertex value
            DevStep *step = s->steps + (s->k % STEP_RING);
            const uint8_t *cur = s->front8[s->ph_p ^ 1];
            if (s->p.algo == GX_SSSP) {
                const PullArgs pa{d.pull_w, d.pull_w_units, d.pull_w_off};
                hipLaunchKernelGGL(k_relax<true>, dim3(s->relax_grid), dim3(256), 0, hs, s->list, s->tile_start,
                                   (const void *)d.out_adj, pa, d.V, s->snap, s->acc, cur, s->junk8, step,
                                   s->pull_edges, s->fix, s->fixn, s->fix_cap, s->xcd_shift);
            } else {
                const PullArgs pa{d.pull_sym, d.pull_sym_units, d.pull_sym_off};
                hipLaunchKernelGGL(k_relax<false>, dim3(s->relax_grid), dim3(256), 0, hs, s->list, s->tile_start,
                                   (const void *)d.sym_col, pa, d.V, s->snap, s->acc, cur, s->junk8, step,
                                   s->pull_edges, s->fix, s->fixn, s->fix_cap, s->xcd_shift);
            }
            hipLaunchKernelGGL(k_fixup, dim3(s->relax_grid), dim3(256), 0, hs, s->fix, s->fixn, s->fix_cap, s->acc,
                               step);
        }
        GX_CHECK_HIP(hipGetLastError(), s);
    }
    s->ph_msgs = false;
    s->ph_merged = true;
    return GX_OK;
}

extern "C" gx_status gx_msg_apply(gx_state *s, void *stream, gx_step_stats *stats) {
    clear_error();
    gx_status st = ph_check(s);
    if (st != GX_OK) return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (stats) *stats = gx_step_stats{};
    if (!s->ph_merged) return GX_OK;  // nothing merged since the last apply
    const DevGraph &d = s->g->d;
    const int64_t k = s->k;
    DevStep *step = s->steps + (k % STEP_RING), *next = s->steps + ((k + 1) % STEP_RING);
    if (d.V > 0) {
        if (s->p.algo == GX_PAGERANK) {
            const bool parts = s->p.phases == GX_PHASES_MASTERS;
            const double Vn = (double)(parts ? d.V_global : d.V);
            hipLaunchKernelGGL(k_ph_pr_apply, dim3(grid_for<int64_t>(d.V, 256)), dim3(256), 0, hs, s->acc_d, s->x[0],
                               d.V, (1.0 - (double)s->p.damping) / Vn, (double)s->p.damping, s->Dval, 1.0 / Vn, step,
                               next, parts ? d.master : nullptr);
        } else {
            hipLaunchKernelGGL(k_ph_apply, dim3(grid_for<int64_t>(d.V, 256)), dim3(256), 0, hs, s->acc, s->val,
                               s->front8[s->ph_p], s->dirty8, d.V, step);
        }
        GX_CHECK_HIP(hipGetLastError(), s);
    }
    s->ph_merged = false;
    s->k++;
    if (stats && d.V > 0) {
        std::vector<DevStep> ds;
        st = read_steps(s, k, 1, hs, ds);
        if (st != GX_OK) return st;
        const bool pr = s->p.algo == GX_PAGERANK;
        stats->frontier = pr ? d.V : (int64_t)ds[0].frontier;
        stats->edges = pr ? d.E : (int64_t)(uint32_t)ds[0].list;
        stats->changed = (int64_t)ds[0].changed;
        stats->pulled = pr ? 1 : (ds[0].pad ? 1 : 0);
    }
    return GX_OK;
}

// ------------------------------------------------------------ PageRank across the parts of a vertex-cut

static gx_status parts_check(gx_state *s) {
    GX_REQUIRE(s, GX_EINVAL, "state is NULL");
    GX_REQUIRE(s->p.phases == GX_PHASES_MASTERS, GX_EINVAL, "state was not initialised with GX_PHASES_MASTERS");
    GX_REQUIRE(!s->dev_error && !s->g->dev_error, GX_EDEVICE, "sticky device error");
    return GX_OK;
}

extern "C" gx_status gx_dangling_get(gx_state *s, double *mass, void *stream) {
    clear_error();
    gx_status st = parts_check(s);
    if (st != GX_OK) return st;
    GX_REQUIRE(mass, GX_EINVAL, "mass is NULL");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    GX_CHECK_HIP(hipMemcpyAsync(mass, s->Dval, sizeof(double), hipMemcpyDeviceToHost, hs), s);
    GX_CHECK_HIP(hipStreamSynchronize(hs), s);
    return GX_OK;
}

extern "C" gx_status gx_dangling_set(gx_state *s, double mass, void *stream) {
    clear_error();
    gx_status st = parts_check(s);
    if (st != GX_OK) return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    s->D_host = mass;
    GX_CHECK_HIP(hipMemcpyAsync(s->Dval, &s->D_host, sizeof(double), hipMemcpyHostToDevice, hs), s);
    return GX_OK;
}

extern "C" gx_status gx_partial_emit(gx_state *s, int32_t *dev_gid, double *dev_val, uint32_t cap, uint32_t *count,
                                     void *stream) {
    clear_error();
    gx_status st = parts_check(s);
    if (st != GX_OK) return st;
    GX_REQUIRE(count, GX_EINVAL, "count is NULL");
    GX_REQUIRE(cap == 0 || (dev_gid && dev_val), GX_EINVAL, "output buffers are NULL");
    GX_REQUIRE(s->ph_merged, GX_EINVAL, "no merged messages to send");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const DevGraph &d = s->g->d;
    *count = 0;
    if (d.W == 0) return GX_OK;
    hipLaunchKernelGGL(k_part_count, dim3(s->delta_blocks), dim3(256), 0, hs, d.W, d.V, d.remote_any, d.master,
                       d.in_rp, s->blk_cnt);
    hipLaunchKernelGGL(k_part_emit, dim3(s->delta_blocks), dim3(256), 0, hs, d.W, d.V, d.remote_any, d.master,
                       d.in_rp, d.l2g, s->acc_d, s->blk_cnt, s->delta_blocks, cap, dev_gid, dev_val, s->delta_total);
    GX_CHECK_HIP(hipGetLastError(), s);
    uint32_t total = 0;
    GX_CHECK_HIP(hipMemcpyAsync(&total, s->delta_total, 4, hipMemcpyDeviceToHost, hs), s);
    GX_CHECK_HIP(hipStreamSynchronize(hs), s);
    *count = total;
    if (total > cap) {
        set_error("%u merged sums to send, capacity %u", total, cap);
        return GX_ENOMEM;
    }
    return GX_OK;
}

extern "C" gx_status gx_partial_add(gx_state *s, const int32_t *dev_gid, const double *dev_val, uint32_t n,
                                    void *stream) {
    clear_error();
    gx_status st = parts_check(s);
    if (st != GX_OK) return st;
    GX_REQUIRE(n == 0 || (dev_gid && dev_val), GX_EINVAL, "input buffers are NULL");
    GX_REQUIRE(s->ph_merged, GX_EINVAL, "merge this part's messages before adding other parts' sums");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const DevGraph &d = s->g->d;
    if (n > 0 && d.V > 0)
        hipLaunchKernelGGL(k_part_add, dim3(grid_for<uint32_t>(n, 256)), dim3(256), 0, hs, dev_gid, dev_val, n, d.l2g,
                           d.V, d.master, s->acc_d);
    GX_CHECK_HIP(hipGetLastError(), s);
    return GX_OK;
}
