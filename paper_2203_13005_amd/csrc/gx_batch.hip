// Batched lanes: B independent single-source problems over one resident
// graph, carried in a [V x B] state tile (B contiguous per vertex) by one
// persistent cooperative kernel per pass.  The evaluation of the paper runs
// several SSSP sources simultaneously to raise the arithmetic intensity
// (Section "Setup", first footnote); here the lanes are independent
// problems, each equal to its plain solve.
//
// SSSP (k_bsssp): per superstep
//   compaction: every (vertex, 32-lane group) whose lane mask is non-zero
//     and that has out-edges becomes one active entry; its 32 start-of-
//     superstep distances are copied to a snapshot row (Jacobi semantics per
//     lane); one 64-bit atomic per workgroup chunk reserves entries and edge
//     offsets; tiles of equal (entry, edge) work units record where they
//     start.
//   relaxation: 8 threads per work unit handle the unit's 32 lanes (4 each,
//     one 16-byte load of the destination's group); improvements are
//     folded by atomicMin per lane (no result awaited: a candidate below a
//     value read during the superstep already proves the lane changes), and
//     the group's improved-lane bits by one atomicOr into the next mask.
//   A grid barrier separates the phases; the loop ends when a superstep
//   activates no (vertex, lane) pair.
// PPR: per superstep four ordinary launches: a pull over equal in-edge
//   tiles (one wave per tile, lanes across the wave), rows crossing tiles
//   completed in tile order, and the per-lane dangling mass reduced in a
//   fixed two-level order, so every lane's arithmetic is independent of the
//   other lanes and of the launch shape.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "gx_device.h"
#include "gx_internal.h"
#include "gx_batch.h"

namespace gx {

// ------------------------------------------------------------------ SSSP

template <int BLOCK, int VT>
struct BsShared {
    static constexpr int T = BLOCK * VT;
    static constexpr int NW = BLOCK / 64;
    int32_t own[T];
    uint32_t base[T + 1];
    uint32_t mask[T + 1];
    uint32_t g[T + 1];
    unsigned long long scan[NW];
    unsigned long long base64;
    int32_t red[NW];
    unsigned long long cnt[NW];
    uint32_t lane[256];
    unsigned int flag;
};

// Phase 1 of batched superstep k: active (vertex, group) pairs -> entries,
// snapshots, tile starts.  Grid-strided over the V*G mask words.
template <int BLOCK, int VT>
__device__ __forceinline__ void bs_compact(const BsArgs &a, uint32_t k, BsShared<BLOCK, VT> &sh) {
    constexpr int T = BLOCK * VT;
    const int tid = threadIdx.x;
    const int64_t VG = a.V * (int64_t)a.G;
    const int slot = k & 3;
    const uint32_t *Mc = a.M[k & 1];
    uint32_t *Mn = a.M[(k + 1) & 1];
    if (blockIdx.x == 0 && tid == 0) {
        a.ctl->list[(k + 1) & 3] = 0;
        a.ctl->changed[(k + 1) & 3] = 0;
    }
    for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < VG; base += (int64_t)gridDim.x * BLOCK) {
        const int64_t i = base + tid;
        uint32_t word = 0, u = 0, g = 0;
        int32_t r0 = 0, deg = 0;
        if (i < VG) {
            word = Mc[i];
            Mn[i] = 0u;
            if (word) {
                u = (uint32_t)(i / a.G);
                g = (uint32_t)(i % a.G);
                r0 = a.rp[u];
                deg = a.rp[u + 1] - r0;
            }
        }
        const bool has = word && deg > 0;
        unsigned long long mine = has ? ((1ull << 32) | (uint32_t)deg) : 0ull, total;
        unsigned long long pre = block_excl_scan_u64(mine, &total, sh.scan);
        if (tid == 0) sh.base64 = total ? atomicAdd(&a.ctl->list[slot], total) : 0ull;
        __syncthreads();
        if (has) {
            unsigned long long pos = sh.base64 + pre;
            uint32_t idx = (uint32_t)(pos >> 32), off = (uint32_t)pos;
            a.list[idx] = make_uint4(off, (uint32_t)(r0 - (int32_t)off), word, g);
            const uint4 *src = reinterpret_cast<const uint4 *>(a.D + (size_t)u * a.B + a.l0 + g * 32);
            uint4 *dst = a.S + (size_t)idx * 8;
#pragma unroll
            for (int q = 0; q < 8; q++) dst[q] = src[q];
            uint32_t t0 = (off + T - 1) / T, t1 = (off + (uint32_t)deg - 1) / T;
            for (uint32_t t = t0; t <= t1; t++) a.tile_start[t] = idx;
        }
        __syncthreads();
    }
}

// Phase 2 of batched superstep k: relax the equal tiles of (entry, edge)
// work units; `it` indexes the per-lane activation counters.
template <int BLOCK, int VT>
__device__ __forceinline__ void bs_relax(const BsArgs &a, uint32_t k, uint32_t it, BsShared<BLOCK, VT> &sh) {
    constexpr int T = BLOCK * VT;
    constexpr int UNITS = BLOCK / 8;
    const int tid = threadIdx.x;
    const int slot = k & 3;
    uint32_t *Mn = a.M[(k + 1) & 1];
    const unsigned long long le = a.ctl->list[slot];
    const uint32_t L = (uint32_t)(le >> 32), EF = (uint32_t)le;
    const uint32_t ntiles = (EF + T - 1) / T;
    unsigned long long changed = 0;
    if (a.lane_cnt)
        for (int q = tid; q < 256; q += BLOCK) sh.lane[q] = 0;
    __syncthreads();
    const int sub = tid & 7;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t e0 = t * T;
        const int n = (int)min((uint32_t)T, EF - e0);
        const uint32_t s0 = a.tile_start[t];
        const uint32_t s1 = (t + 1 < ntiles) ? a.tile_start[t + 1] : L - 1;
        const int m = (int)(s1 - s0) + 1;
        for (int p = tid; p < n; p += BLOCK) sh.own[p] = 0;
        __syncthreads();
        for (int q = tid; q < m; q += BLOCK) {
            uint4 en = a.list[s0 + q];
            sh.base[q] = en.y + e0;
            sh.mask[q] = en.z;
            sh.g[q] = en.w;
            uint32_t rel = en.x - e0;
            if (q > 0 && rel < (uint32_t)n) sh.own[rel] = q;
        }
        __syncthreads();
        block_max_scan<VT>(sh.own, n, sh.red);
        // UB work units per 8-thread group at a time: their edge loads, then
        // their snapshot and destination loads, then the relaxations, all
        // loads unconditional (units past the tile's end repeat its last
        // unit with no lanes).  The lane minima go out as atomics whose
        // results are not awaited; only the mask atomics return, once.
        constexpr int UB = 4;
        for (int p0 = tid >> 3; p0 < n; p0 += UNITS * UB) {
            uint2 ed[UB];
            uint32_t my4[UB], gq[UB], jq[UB];
#pragma unroll
            for (int q = 0; q < UB; q++) {
                const int p = min(p0 + q * UNITS, n - 1);
                const int j = sh.own[p];
                jq[q] = (uint32_t)j;
                gq[q] = sh.g[j];
                my4[q] = (p0 + q * UNITS < n) ? (sh.mask[j] >> (sub * 4)) & 15u : 0u;
                ed[q] = a.adj[sh.base[j] + (uint32_t)p];
            }
            uint4 sn[UB], cur[UB];
#pragma unroll
            for (int q = 0; q < UB; q++) {
                sn[q] = a.S[(size_t)(s0 + jq[q]) * 8 + sub];
                cur[q] = *reinterpret_cast<const uint4 *>(a.D + (size_t)ed[q].x * a.B + a.l0 + gq[q] * 32 + sub * 4);
            }
            uint32_t cand[UB][4], word[UB];
#pragma unroll
            for (int q = 0; q < UB; q++) {
                const uint32_t snv[4] = {sn[q].x, sn[q].y, sn[q].z, sn[q].w};
                const uint32_t cv[4] = {cur[q].x, cur[q].y, cur[q].z, cur[q].w};
                uint32_t imp = 0;
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    cand[q][r] = sat_add(snv[r], ed[q].y);
                    // below a value read this superstep: the lane changes
                    if (((my4[q] >> r) & 1u) && cand[q][r] < cv[r]) imp |= 1u << r;
                }
                uint32_t w = imp << (sub * 4);
                w |= __shfl_xor(w, 1, 8);
                w |= __shfl_xor(w, 2, 8);
                w |= __shfl_xor(w, 4, 8);
                word[q] = w;
            }
#pragma unroll
            for (int q = 0; q < UB; q++) {
                const uint32_t imp = (word[q] >> (sub * 4)) & 15u;
                uint32_t *dp = a.D + (size_t)ed[q].x * a.B + a.l0 + gq[q] * 32 + sub * 4;
#pragma unroll
                for (int r = 0; r < 4; r++)
                    if ((imp >> r) & 1u) atomicMin(dp + r, cand[q][r]);
            }
            // The group leader ORs all UB words (a zero word changes nothing)
            // under one branch, so the returns are awaited once.
            if (sub == 0 && (word[0] | word[1] | word[2] | word[3])) {
                static_assert(UB == 4, "the branch above names the UB words");
                uint32_t prev[UB];
#pragma unroll
                for (int q = 0; q < UB; q++) prev[q] = atomicOr(&Mn[(size_t)ed[q].x * a.G + gq[q]], word[q]);
#pragma unroll
                for (int q = 0; q < UB; q++) {
                    const uint32_t nb = word[q] & ~prev[q];
                    changed += __popc(nb);
                    if (a.lane_cnt)
                        for (uint32_t mm = nb; mm; mm &= mm - 1) atomicAdd(&sh.lane[gq[q] * 32 + __ffs(mm) - 1], 1u);
                }
            }
        }
        __syncthreads();
    }
    unsigned long long tot = block_sum<unsigned long long>(changed, sh.cnt);
    if (tid == 0 && tot) atomicAdd(&a.ctl->changed[slot], tot);
    if (a.lane_cnt) {
        __syncthreads();
        for (int q = tid; q < (int)(a.G * 32); q += BLOCK)
            if (sh.lane[q]) atomicAdd(&a.lane_cnt[(size_t)it * a.B + a.l0 + q], sh.lane[q]);
    }
}

// One persistent cooperative launch runs supersteps until one activates no
// (vertex, lane) pair or max_steps have run; grid barriers separate phases.
template <int BLOCK, int VT>
__global__ __launch_bounds__(BLOCK) void k_bsssp(BsArgs a) {
    __shared__ BsShared<BLOCK, VT> sh;
    uint32_t k = a.k0;
    for (uint32_t it = 0; it < a.max_steps; it++, k++) {
        bs_compact<BLOCK, VT>(a, k, sh);
        if (!grid_sync(&a.ctl->bar, gridDim.x, &sh.flag, a.bar_ticks)) return;
        bs_relax<BLOCK, VT>(a, k, it, sh);
        if (!grid_sync(&a.ctl->bar, gridDim.x, &sh.flag, a.bar_ticks)) return;
        const unsigned long long ch =
            __hip_atomic_load(&a.ctl->changed[k & 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->steps = it + 1;
        if (ch == 0 && a.stop_when_idle) break;
    }
}

// The same phases as ordinary launches (serving: several pools overlap on
// their own streams, so no launch may rely on grid-wide co-residency).
template <int BLOCK, int VT>
__global__ __launch_bounds__(BLOCK) void k_bs_compact(BsArgs a, uint32_t k) {
    __shared__ BsShared<BLOCK, VT> sh;
    bs_compact<BLOCK, VT>(a, k, sh);
}
template <int BLOCK, int VT>
__global__ __launch_bounds__(BLOCK) void k_bs_relax(BsArgs a, uint32_t k, uint32_t it) {
    __shared__ BsShared<BLOCK, VT> sh;
    bs_relax<BLOCK, VT>(a, k, it, sh);
}

__global__ __launch_bounds__(256) void k_bs_fill(uint32_t *D, size_t n, uint32_t x) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) D[i] = x;
}

// Lane b of the pass starting at lane l0: D[src][b] = 0 and its mask bit.
__global__ __launch_bounds__(256) void k_bs_sources(uint32_t *D, uint32_t *M0, const int32_t *src, uint32_t B,
                                                    uint32_t l0, uint32_t width, uint32_t G) {
    uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= width) return;
    int32_t s = src[l0 + q];
    if (s < 0) return;
    D[(size_t)s * B + l0 + q] = 0u;
    atomicOr(&M0[(size_t)s * G + q / 32], 1u << (q & 31));
}

// Serving: re-initialise lane b (column of D over all V, its masks) and seed it.
__global__ __launch_bounds__(256) void k_bs_lane_reset(uint32_t *D, uint32_t *Mc, uint32_t *Mn, int64_t V, uint32_t B,
                                                       uint32_t G, uint32_t lane, int32_t src) {
    const uint32_t bit = 1u << (lane & 31), g = lane / 32;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (int64_t)gridDim.x * blockDim.x) {
        D[(size_t)v * B + lane] = (v == src) ? 0u : INF;
        uint32_t w = Mc[(size_t)v * G + g];
        uint32_t want = (v == src) ? (w | bit) : (w & ~bit);
        if (want != w) Mc[(size_t)v * G + g] = want;
        uint32_t w2 = Mn[(size_t)v * G + g];
        if (w2 & bit) Mn[(size_t)v * G + g] = w2 & ~bit;
    }
}

// ------------------------------------------------------------------ PPR

// Per-lane constants of one PPR superstep, held in registers: lane b =
// lane + 64 i is live when it is inside the processed width, holds a query
// and has not reached its end superstep (a finished lane is frozen: its
// values stay as they were after its last superstep, in x[end & 1]).
template <int LPT>
struct PprLanes {
    uint32_t bl[LPT];  // load column (clamped into the processed width)
    bool live[LPT];
    int32_t seed[LPT];
    double dc[LPT];    // dangling mass of the lane at the start of the superstep
    __device__ PprLanes(const BpArgs &a, uint32_t k, const double *Dcur, int lane) {
#pragma unroll
        for (int i = 0; i < LPT; i++) {
            const uint32_t b = lane + 64 * i;
            bl[i] = min(b, a.Bw - 1);
            const int32_t sd = b < a.Bw ? a.seed[b] : -1;
            live[i] = sd >= 0 && (!a.end || (int32_t)((uint32_t)a.end[b] - k) > 0);
            seed[i] = sd;
            dc[i] = b < a.Bw ? Dcur[b] : 0.0;
        }
    }
};

template <int LPT>
__device__ __forceinline__ void ppr_apply(const BpArgs &a, int32_t r, int od, const double (&acc)[LPT],
                                          const PprLanes<LPT> &L, float *x_out, float *c_out, double (&dang)[LPT],
                                          int lane) {
#pragma unroll
    for (int i = 0; i < LPT; i++) {
        if (!L.live[i]) continue;
        const uint32_t b = lane + 64 * i;
        double v = (double)a.d * acc[i];
        if (L.seed[i] == r) v += (1.0 - (double)a.d) + (double)a.d * L.dc[i];
        const float xn = (float)v;
        x_out[(size_t)r * a.B + b] = xn;
        c_out[(size_t)r * a.B + b] = od > 0 ? xn / (float)od : 0.0f;
        if (od == 0) dang[i] += (double)xn;
    }
}

// PPR phase P of superstep k: pull tiles, one wave per tile, lanes across
// the wave.  The tile's edges are streamed in order: the wave loads the
// tile's source ids at once (edge position p sits in lane p mod 64 of
// register p / 64), then loads the contribution rows of EB edges at a time
// before adding any, so the row loads of consecutive edges overlap whatever
// rows they belong to.  A running segment (the head of a row begun in an earlier
// tile, then the rows that start in this tile) closes when the position
// passes its end; row ends and out-degrees come from a window of 64 rows
// loaded one per lane.  Each lane adds its row's contributions in edge
// order, so results do not depend on the batching.
template <int LPT>
__device__ __forceinline__ void bp_pull(const BpArgs &a, uint32_t k, const double *Dcur) {
    constexpr int EB = 16 / (LPT == 3 ? 4 : LPT);  // edges whose rows are loaded before any is added
    constexpr int CR = BP_TILE / 64;               // source-id registers per lane
    __shared__ int2 s_win[4][64];        // per wave (blocks of 256 threads)
    const int lane = threadIdx.x & 63, wv = (threadIdx.x >> 6) & 3;
    const int64_t gwave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    float *x_out = a.x[(k + 1) & 1];
    const float *c_in = a.c[k & 1];
    float *c_out = a.c[(k + 1) & 1];
    const PprLanes<LPT> L(a, k, Dcur, lane);
    for (int64_t t = gwave; t < a.ntiles; t += nwaves) {
        const int32_t e0 = (int32_t)(t * BP_TILE);
        const int32_t e1 = (int32_t)std::min<int64_t>((int64_t)e0 + BP_TILE, a.E);
        const int n = e1 - e0;  // 0 only when E == 0
        const int32_t r_lo = a.trow[t], r_hi = a.trow[t + 1];
        const int nrows = r_hi - r_lo;
        if (lane == 0) a.spill[t] = -1;
        int32_t col[CR];
#pragma unroll
        for (int q = 0; q < CR; q++) col[q] = n > 0 ? a.in_col[e0 + min(lane + 64 * q, n - 1)] : 0;
        const int32_t first_start = r_lo < a.V ? a.in_rp[r_lo] : (int32_t)a.E;
        // Row window in LDS: entry j holds the end and out-degree of row
        // r_lo + wb + j.  (Values in LDS are waited for on their own counter;
        // a register loaded from global memory would make every later use wait
        // for all row loads in flight.)
        int wb = 0;
        auto load_window = [&]() {
            const int32_t rq = r_lo + wb + min(lane, nrows - wb - 1);
            const int32_t re = a.in_rp[rq + 1], od = a.outdeg[rq];
            s_win[wv][lane] = make_int2(re, od);
            __builtin_amdgcn_wave_barrier();
        };
        if (nrows > 0) load_window();
        double acc[LPT], dang[LPT];
#pragma unroll
        for (int i = 0; i < LPT; i++) {
            acc[i] = 0.0;
            dang[i] = 0.0;
        }
        // seg = -1: the head (positions before first_start); seg >= 0: row r_lo + seg
        int seg = -1;
        const int head_end = std::min(first_start, e1) - e0;
        int seg_end = head_end;
        auto close = [&]() {  // closes segment `seg` with the sum in acc, then moves to the next one
            if (seg < 0) {
                if (head_end > 0)
#pragma unroll
                    for (int i = 0; i < LPT; i++)
                        if (lane + 64 * i < (int)a.Bw) a.head[t * a.B + lane + 64 * i] = acc[i];
            } else {
                const int32_t r = r_lo + seg;
                const int2 w = s_win[wv][seg - wb];
                const int32_t re = w.x;
                if (re > e1) {  // continues into later tiles: a partial for the fix phase
#pragma unroll
                    for (int i = 0; i < LPT; i++)
                        if (lane + 64 * i < (int)a.Bw) a.tailp[t * a.B + lane + 64 * i] = acc[i];
                    if (lane == 0) a.spill[t] = r;
                } else {
                    ppr_apply<LPT>(a, r, w.y, acc, L, x_out, c_out, dang, lane);
                }
            }
#pragma unroll
            for (int i = 0; i < LPT; i++) acc[i] = 0.0;
            seg++;
            if (seg < nrows) {
                if (seg - wb == 64) {  // next window of rows
                    wb = seg;
                    __builtin_amdgcn_wave_barrier();
                    load_window();
                }
                seg_end = std::min(s_win[wv][seg - wb].x, e1) - e0;
            } else {
                seg_end = 0x7FFFFFFF;
            }
        };
        // Chunks of EB edges: the chunk's contribution rows are loaded at
        // once, then added segment by segment (one predicated pass over the
        // chunk's registers per segment, closes in between), so the loads of
        // a chunk overlap whatever rows they belong to and the adds keep
        // edge order.
        for (int p0 = 0; p0 < n; p0 += EB) {
            const int cnt = min(EB, n - p0);
            float v[EB][LPT];
#pragma unroll
            for (int jj = 0; jj < EB; jj++) {
                const int p = p0 + min(jj, cnt - 1);
                int32_t c = col[0];
#pragma unroll
                for (int q = 1; q < CR; q++)
                    if ((p >> 6) == q) c = col[q];
                const int32_t u = __shfl(c, p & 63, 64);
                const float *row = c_in + (size_t)u * a.B;
#pragma unroll
                for (int i = 0; i < LPT; i++) v[jj][i] = row[L.bl[i]];
            }
            int j = 0;
            while (j < cnt) {
                while (p0 + j >= seg_end) close();
                const int jend = min(seg_end - p0, cnt);
#pragma unroll
                for (int jj = 0; jj < EB; jj++)
                    if (jj >= j && jj < jend)
#pragma unroll
                        for (int i = 0; i < LPT; i++) acc[i] += (double)v[jj][i];
                j = jend;
            }
        }
        while (seg < nrows) close();  // the open segment, then rows with no edges left in this tile
#pragma unroll
        for (int i = 0; i < LPT; i++)
            if (lane + 64 * i < (int)a.Bw) a.dsum[t * a.B + lane + 64 * i] = dang[i];
    }
}

// Phase F: rows crossing tiles, summed in tile order.
template <int LPT>
__device__ __forceinline__ void bp_fix(const BpArgs &a, uint32_t k, const double *Dcur) {
    const int lane = threadIdx.x & 63;
    const int64_t gwave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    float *x_out = a.x[(k + 1) & 1];
    float *c_out = a.c[(k + 1) & 1];
    const PprLanes<LPT> L(a, k, Dcur, lane);
    for (int64_t t = gwave; t < a.ntiles; t += nwaves) {
        const int32_t r = a.spill[t];
        if (r < 0) continue;
        double acc[LPT], dang[LPT];
        const int32_t t_end = (a.in_rp[r + 1] - 1) / BP_TILE;
#pragma unroll
        for (int i = 0; i < LPT; i++) {
            dang[i] = 0.0;
            acc[i] = 0.0;
            const uint32_t b = lane + 64 * i;
            if (b >= a.Bw) continue;
            double s = a.tailp[t * a.B + b];
            for (int32_t t2 = (int32_t)t + 1; t2 <= t_end; t2++) s += a.head[(int64_t)t2 * a.B + b];
            acc[i] = s;
        }
        ppr_apply<LPT>(a, r, a.outdeg[r], acc, L, x_out, c_out, dang, lane);
#pragma unroll
        for (int i = 0; i < LPT; i++)
            if (lane + 64 * i < (int)a.Bw) a.dsum[t * a.B + lane + 64 * i] += dang[i];
    }
}

// Sum of p[i * stride] over i = 0 .. n-1 (n >= 1) in index order; the
// loads go out 16 at a time, the adds stay in order.
__device__ __forceinline__ double ordered_sum(const double *p, int64_t stride, int64_t n) {
    double s = 0.0;
    for (int64_t i0 = 0; i0 < n; i0 += 16) {
        double v[16];
#pragma unroll
        for (int j = 0; j < 16; j++) v[j] = p[std::min<int64_t>(i0 + j, n - 1) * stride];
#pragma unroll
        for (int j = 0; j < 16; j++)
            if (i0 + j < n) s += v[j];
    }
    return s;
}

// Phase D1: dangling partial per fixed chunk of BP_DCHUNK tiles.
__device__ __forceinline__ void bp_dang1(const BpArgs &a) {
    const int lane = threadIdx.x & 63;
    const int64_t gwave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t nchunks = (a.ntiles + BP_DCHUNK - 1) / BP_DCHUNK;
    const int64_t lgroups = (a.Bw + 63) / 64;
    for (int64_t w = gwave; w < nchunks * lgroups; w += nwaves) {
        const int64_t ch = w / lgroups;
        const uint32_t b = (uint32_t)((w % lgroups) * 64 + lane);
        if (b >= a.Bw) continue;
        const int64_t t0 = ch * BP_DCHUNK, t1 = std::min<int64_t>(t0 + BP_DCHUNK, a.ntiles);
        a.dpart[ch * a.B + b] = ordered_sum(a.dsum + t0 * a.B + b, a.B, t1 - t0);
    }
}

// Phase D2: per-lane total over the chunks, in chunk order.
__device__ __forceinline__ void bp_dang2(const BpArgs &a, double *Dnext) {
    const int lane = threadIdx.x & 63;
    const int64_t gwave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t nchunks = (a.ntiles + BP_DCHUNK - 1) / BP_DCHUNK;
    for (int64_t lg = gwave; lg * 64 < (int64_t)a.Bw; lg += nwaves) {
        const uint32_t b = (uint32_t)(lg * 64 + lane);
        if (b >= a.Bw) continue;
        Dnext[b] = ordered_sum(a.dpart + b, a.B, nchunks);
    }
}

// The four phases as ordinary launches (batched runs and serving).
template <int LPT>
__global__ __launch_bounds__(256) void k_bp_pull(BpArgs a, uint32_t k) { bp_pull<LPT>(a, k, a.D[k & 1]); }
template <int LPT>
__global__ __launch_bounds__(256) void k_bp_fix(BpArgs a, uint32_t k) { bp_fix<LPT>(a, k, a.D[k & 1]); }
__global__ __launch_bounds__(256) void k_bp_dang1(BpArgs a) { bp_dang1(a); }
__global__ __launch_bounds__(256) void k_bp_dang2(BpArgs a, uint32_t k) { bp_dang2(a, a.D[(k + 1) & 1]); }

__global__ __launch_bounds__(256) void k_bp_init(float *x, float *c, double *D, const int32_t *seed,
                                                 const int32_t *outdeg, int64_t V, uint32_t B) {
    const size_t n = (size_t)V * B;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int64_t v = (int64_t)(i / B);
        const uint32_t b = (uint32_t)(i % B);
        const float xv = seed[b] == v ? 1.0f : 0.0f;
        x[i] = xv;
        const int od = outdeg[v];
        c[i] = od > 0 ? xv / (float)od : 0.0f;
    }
    if (blockIdx.x == 0)
        for (uint32_t b = threadIdx.x; b < B; b += blockDim.x)
            D[b] = (seed[b] >= 0 && outdeg[seed[b]] == 0) ? 1.0 : 0.0;
}

// Serving: lane b restarts from its new seed (x = e_seed, D = dangling of seed).
__global__ __launch_bounds__(256) void k_bp_lane_reset(float *x, float *c, double *D, const int32_t *outdeg,
                                                       int64_t V, uint32_t B, uint32_t lane, int32_t seed) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (int64_t)gridDim.x * blockDim.x) {
        const float xv = v == seed ? 1.0f : 0.0f;
        x[(size_t)v * B + lane] = xv;
        const int od = outdeg[v];
        c[(size_t)v * B + lane] = od > 0 ? xv / (float)od : 0.0f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) D[lane] = outdeg[seed] == 0 ? 1.0 : 0.0;
}

// PPR tiles: first row whose first in-edge position is >= t * BP_TILE.
__global__ __launch_bounds__(256) void k_bp_tiles(const int32_t *in_rp, int64_t V, int64_t ntiles, int32_t *trow) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    if (t == ntiles) {
        trow[t] = (int32_t)V;
        return;
    }
    const int32_t key = (int32_t)(t * BP_TILE);
    int64_t lo = 0, hi = V;  // lower_bound over in_rp[0..V)
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (in_rp[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    trow[t] = t == 0 ? 0 : (int32_t)lo;
}

// Gathers lane b of a [V x B] tile into a contiguous vector.
__global__ __launch_bounds__(256) void k_lane_extract(const uint32_t *tile, int64_t V, uint32_t B, uint32_t lane,
                                                      uint32_t *out) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (int64_t)gridDim.x * blockDim.x)
        out[v] = tile[(size_t)v * B + lane];
}

// ------------------------------------------------------------------ host

const BsVariant *bs_variants(int *n) {
    static const BsVariant v[] = {
        {256, 4, (const void *)k_bsssp<256, 4>},  {256, 8, (const void *)k_bsssp<256, 8>},
        {512, 4, (const void *)k_bsssp<512, 4>},  {512, 8, (const void *)k_bsssp<512, 8>},
        {1024, 2, (const void *)k_bsssp<1024, 2>}, {1024, 4, (const void *)k_bsssp<1024, 4>},
    };
    *n = (int)(sizeof v / sizeof v[0]);
    return v;
}


// Workgroups of a cooperative (grid-barrier) launch.  By default at most
// max_per_cu per CU and at most half of the occupancy bound; a kernel whose
// phases run for milliseconds (batched PPR) passes max_per_cu = 0 to use
// the whole bound (the cooperative launch itself refuses a grid that cannot
// be resident at once).
int coop_grid(const void *kernel, int block, int num_cus, int want, int max_per_cu) {
    const int occ = occupancy_per_cu(kernel, block);
    int per_cu = max_per_cu > 0 ? std::max(1, std::min(max_per_cu, occ / 2)) : std::max(1, occ);
    int cap = per_cu * num_cus;
    if (want > 0) return std::min(want, cap);
    return cap;
}

void bs_layout(const DevGraph &d, uint32_t B, Carver &c, BsWork *w) {
    const uint32_t G = B / 32;
    const int64_t VG = d.V * (int64_t)G;
    w->M[0] = c.take<uint32_t>(VG);
    w->M[1] = c.take<uint32_t>(VG);
    w->list = c.take<uint4>(VG);
    w->S = c.take<uint4>(VG * 8);
    w->tile_start = c.take<uint32_t>((d.E * (int64_t)G) / BS_MIN_TILE + 2);
    w->ctl = c.take<BsCtl>(1);
    w->src = c.take<int32_t>(B);
}

void bp_layout(const DevGraph &d, uint32_t B, Carver &c, BpWork *w) {
    const int64_t nt = std::max<int64_t>(1, (d.E + BP_TILE - 1) / BP_TILE);
    const int64_t nchunks = (nt + BP_DCHUNK - 1) / BP_DCHUNK;
    w->ntiles = nt;
    w->x[0] = c.take<float>((size_t)d.V * B);
    w->x[1] = c.take<float>((size_t)d.V * B);
    w->c[0] = c.take<float>((size_t)d.V * B);
    w->c[1] = c.take<float>((size_t)d.V * B);
    w->head = c.take<double>(nt * B);
    w->tailp = c.take<double>(nt * B);
    w->dsum = c.take<double>(nt * B);
    w->dpart = c.take<double>(nchunks * B);
    w->D[0] = c.take<double>(B);
    w->D[1] = c.take<double>(B);
    w->spill = c.take<int32_t>(nt);
    w->trow = c.take<int32_t>(nt + 1);
    w->seed = c.take<int32_t>(2 * (size_t)B);  // seeds, then per-lane end supersteps
    w->end = w->seed + B;
}

// Wall-clock ticks a grid barrier may wait: BARRIER_LIMIT_S seconds at the
// device's constant wall-clock rate (a superstep phase of the batched
// kernel takes milliseconds; only a grid that is not co-resident waits that
// long).
unsigned long long barrier_limit_ticks(int device) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0)
        khz = 100000;  // 100 MHz, the gfx9 constant clock
    return (unsigned long long)(BARRIER_LIMIT_S * 1e3 * (double)khz);
}

hipError_t launch_coop(const void *kernel, int grid, int block, void *args, hipStream_t s) {
    void *params[] = {args};
    return hipLaunchCooperativeKernel(kernel, dim3(grid), dim3(block), params, 0, s);
}

}  // namespace gx

using namespace gx;

static gx_status check_batch(const gx_graph *g, int32_t algo, uint32_t B) {
    GX_REQUIRE(g, GX_EINVAL, "graph is NULL");
    GX_REQUIRE(!g->dev_error, GX_EDEVICE, "sticky device error on the graph");
    GX_REQUIRE(algo == GX_SSSP || algo == GX_PPR, GX_EINVAL, "batched algo must be GX_SSSP or GX_PPR");
    GX_REQUIRE(B >= 1 && B <= 256, GX_EINVAL, "B=%u out of [1,256]", B);
    if (algo == GX_SSSP) {
        GX_REQUIRE(B % 32 == 0, GX_EINVAL, "SSSP lanes must be a multiple of 32 (B=%u)", B);
        GX_REQUIRE(g->needs & GX_NEED_OUT, GX_EINVAL, "batched SSSP needs GX_NEED_OUT");
    } else {
        GX_REQUIRE(g->needs & GX_NEED_IN, GX_EINVAL, "batched PPR needs GX_NEED_IN");
    }
    return GX_OK;
}

extern "C" gx_status gx_batch_bytes(const gx_graph *g, int32_t algo, uint32_t B, size_t *bytes) {
    clear_error();
    GX_REQUIRE(bytes, GX_EINVAL, "bytes is NULL");
    gx_status st = check_batch(g, algo, B);
    if (st != GX_OK) return st;
    Carver c(nullptr, 0);
    if (algo == GX_SSSP) {
        BsWork w;
        bs_layout(g->d, B, c, &w);
    } else {
        BpWork w;
        bp_layout(g->d, B, c, &w);
    }
    *bytes = c.used;
    return GX_OK;
}

namespace gx {

// Runs SSSP lanes with one tuning; returns GX_OK / error.  out: [V x B] u32.
gx_status run_bsssp(gx_graph *g, const int32_t *dev_src, uint32_t B, BsWork &w, uint32_t *D, const gx_tune &tn,
                    hipStream_t s, int64_t *supersteps) {
    const DevGraph &d = g->d;
    int nv = 0;
    const BsVariant *vars = bs_variants(&nv);
    const BsVariant *var = nullptr;
    for (int i = 0; i < nv; i++)
        if (vars[i].block == tn.block && vars[i].block * vars[i].vt == tn.tile) var = &vars[i];
    GX_REQUIRE(var, GX_EINVAL, "unsupported tuning block=%u tile=%u", tn.block, tn.tile);
    GX_REQUIRE(tn.width % 32 == 0 && tn.width >= 32 && B % tn.width == 0, GX_EINVAL, "width %u invalid for B=%u",
               tn.width, B);
    const size_t n = (size_t)d.V * B;
    hipLaunchKernelGGL(k_bs_fill, dim3(std::min<size_t>(4096, (n + 255) / 256 + 1)), dim3(256), 0, s, D, n, INF);
    int64_t steps_max = 0;
    const int grid = coop_grid(var->fn, var->block, g->num_cus, (int)tn.grid, 2);
    for (uint32_t l0 = 0; l0 < B; l0 += tn.width) {
        const uint32_t G = tn.width / 32;
        GX_CHECK_HIP(hipMemsetAsync(w.M[0], 0, (size_t)d.V * G * 4, s), g);
        GX_CHECK_HIP(hipMemsetAsync(w.M[1], 0, (size_t)d.V * G * 4, s), g);
        GX_CHECK_HIP(hipMemsetAsync(w.ctl, 0, sizeof(BsCtl), s), g);
        hipLaunchKernelGGL(k_bs_sources, dim3((tn.width + 255) / 256), dim3(256), 0, s, D, w.M[0], dev_src, B, l0,
                           tn.width, G);
        BsArgs a{};
        a.rp = d.out_rp;
        a.adj = d.out_adj;
        a.V = d.V;
        a.B = B;
        a.l0 = l0;
        a.G = G;
        a.D = D;
        a.M[0] = w.M[0];
        a.M[1] = w.M[1];
        a.list = w.list;
        a.S = w.S;
        a.tile_start = w.tile_start;
        a.ctl = w.ctl;
        a.max_steps = (uint32_t)std::min<int64_t>(d.V + 2, 0x7FFFFFFF);
        a.k0 = 0;
        a.lane_cnt = nullptr;
        a.stop_when_idle = 1;
        a.bar_ticks = barrier_limit_ticks(g->device);
        GX_CHECK_HIP(launch_coop(var->fn, grid, var->block, &a, s), g);
        BsCtl ctl;
        GX_CHECK_HIP(hipMemcpyAsync(&ctl, w.ctl, sizeof ctl, hipMemcpyDeviceToHost, s), g);
        GX_CHECK_HIP(hipStreamSynchronize(s), g);
        if (ctl.bar.error) {
            set_error("grid barrier waited over %.0f s in batched SSSP (pass at lane %u, grid %d x %u)",
                      BARRIER_LIMIT_S, l0, grid, var->block);
            g->dev_error = true;
            return GX_EDEVICE;
        }
        steps_max = std::max<int64_t>(steps_max, ctl.steps);
    }
    if (supersteps) *supersteps = steps_max;
    return GX_OK;
}

gx_status run_bppr(gx_graph *g, const int32_t *dev_seed, uint32_t B, BpWork &w, float d_, uint32_t iters,
                   float *out, hipStream_t s, int grid_want) {
    const DevGraph &d = g->d;
    const int64_t nt = w.ntiles;
    hipLaunchKernelGGL(k_bp_tiles, dim3((unsigned)((nt + 1 + 255) / 256)), dim3(256), 0, s, d.in_rp, d.V, nt, w.trow);
    if (dev_seed != w.seed)
        GX_CHECK_HIP(hipMemcpyAsync(w.seed, dev_seed, B * 4, hipMemcpyDeviceToDevice, s), g);
    const size_t n = (size_t)d.V * B;
    hipLaunchKernelGGL(k_bp_init, dim3((unsigned)std::min<size_t>(8192, (n + 255) / 256 + 1)), dim3(256), 0, s,
                       w.x[0], w.c[0], w.D[0], w.seed, d.outdeg, d.V, B);
    BpArgs a{};
    a.in_rp = d.in_rp;
    a.in_col = d.in_col;
    a.outdeg = d.outdeg;
    a.trow = w.trow;
    a.ntiles = nt;
    a.V = d.V;
    a.E = d.E;
    a.B = B;
    a.Bw = B;
    a.d = d_;
    a.seed = w.seed;
    a.x[0] = w.x[0];
    a.x[1] = w.x[1];
    a.c[0] = w.c[0];
    a.c[1] = w.c[1];
    a.head = w.head;
    a.tailp = w.tailp;
    a.dsum = w.dsum;
    a.dpart = w.dpart;
    a.D[0] = w.D[0];
    a.D[1] = w.D[1];
    a.spill = w.spill;
    // four ordinary launches per superstep (measured faster than one
    // persistent kernel with grid barriers: each phase then runs at its own
    // full occupancy)
    const int grid = grid_want > 0 ? grid_want : 2 * g->num_cus;
    for (uint32_t k = 0; k < iters; k++) GX_CHECK_HIP(bp_launch_superstep(a, k, grid, s), g);
    GX_CHECK_HIP(hipMemcpyAsync(out, w.x[iters & 1], n * 4, hipMemcpyDeviceToDevice, s), g);
    GX_CHECK_HIP(hipStreamSynchronize(s), g);
    return GX_OK;
}

// ---- launchers of the ordinary-launch phases (serving)

hipError_t bs_launch_superstep(const BsArgs &a, uint32_t k, uint32_t it, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_bs_compact<256, 8>), dim3(grid), dim3(256), 0, s, a, k);
    hipLaunchKernelGGL((k_bs_relax<256, 8>), dim3(grid), dim3(256), 0, s, a, k, it);
    return hipGetLastError();
}

hipError_t bp_launch_superstep(const BpArgs &a, uint32_t k, int grid, hipStream_t s) {
    const uint32_t lpt = (a.Bw + 63) / 64;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const int cus = device_cus(dev);
    // the pull keeps its row gathers in flight from every wave the CUs hold
#define GX_BP_PHASES(L)                                                                                  \
    hipLaunchKernelGGL(k_bp_pull<L>,                                                                     \
                       dim3(std::max(grid, cus * occupancy_per_cu((const void *)k_bp_pull<L>, 256))),  \
                       dim3(256), 0, s, a, k);                                                          \
    hipLaunchKernelGGL(k_bp_fix<L>, dim3(grid), dim3(256), 0, s, a, k);
    switch (lpt) {
        case 1: GX_BP_PHASES(1) break;
        case 2: GX_BP_PHASES(2) break;
        case 3: GX_BP_PHASES(3) break;
        default: GX_BP_PHASES(4) break;
    }
#undef GX_BP_PHASES
    hipLaunchKernelGGL(k_bp_dang1, dim3(grid), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_bp_dang2, dim3(grid), dim3(256), 0, s, a, k);
    return hipGetLastError();
}

hipError_t bs_lane_reset(uint32_t *D, uint32_t *Mc, uint32_t *Mn, int64_t V, uint32_t B, uint32_t G, uint32_t lane,
                         int32_t src, hipStream_t s) {
    unsigned nb = (unsigned)std::min<int64_t>(2048, (V + 255) / 256 + 1);
    hipLaunchKernelGGL(k_bs_lane_reset, dim3(nb), dim3(256), 0, s, D, Mc, Mn, V, B, G, lane, src);
    return hipGetLastError();
}

hipError_t bp_lane_reset(float *x, float *c, double *D, const int32_t *outdeg, int64_t V, uint32_t B, uint32_t lane,
                         int32_t seed, hipStream_t s) {
    unsigned nb = (unsigned)std::min<int64_t>(2048, (V + 255) / 256 + 1);
    hipLaunchKernelGGL(k_bp_lane_reset, dim3(nb), dim3(256), 0, s, x, c, D, outdeg, V, B, lane, seed);
    return hipGetLastError();
}

hipError_t bp_make_tiles(const int32_t *in_rp, int64_t V, int64_t ntiles, int32_t *trow, hipStream_t s) {
    hipLaunchKernelGGL(k_bp_tiles, dim3((unsigned)((ntiles + 1 + 255) / 256)), dim3(256), 0, s, in_rp, V, ntiles,
                       trow);
    return hipGetLastError();
}

hipError_t lane_extract(const uint32_t *tile, int64_t V, uint32_t B, uint32_t lane, uint32_t *out, hipStream_t s) {
    unsigned nb = (unsigned)std::min<int64_t>(2048, (V + 255) / 256 + 1);
    hipLaunchKernelGGL(k_lane_extract, dim3(nb), dim3(256), 0, s, tile, V, B, lane, out);
    return hipGetLastError();
}

gx_tune default_tune(uint32_t B) {
    gx_tune t{};
    t.block = 256;
    t.tile = 2048;
    t.width = B;
    t.grid = 0;
    return t;
}

}  // namespace gx

static gx_status batch_common(gx_graph *g, int32_t algo, const int32_t *sources, uint32_t B, void *dev_work,
                              size_t work_bytes, void *dev_out, BsWork *bsw, BpWork *bpw) {
    gx_status st = check_batch(g, algo, B);
    if (st != GX_OK) return st;
    GX_REQUIRE(sources && dev_work && dev_out, GX_EINVAL, "NULL argument");
    GX_REQUIRE(reinterpret_cast<uintptr_t>(dev_work) % ALIGN == 0, GX_EINVAL, "dev_work not 256-byte aligned");
    GX_REQUIRE(reinterpret_cast<uintptr_t>(dev_out) % 16 == 0, GX_EINVAL, "dev_out not 16-byte aligned");
    for (uint32_t b = 0; b < B; b++)
        GX_REQUIRE(sources[b] >= 0 && sources[b] < g->d.V, GX_EINVAL, "sources[%u]=%d out of [0,V)", b, sources[b]);
    Carver c(dev_work, work_bytes);
    if (algo == GX_SSSP) bs_layout(g->d, B, c, bsw);
    else bp_layout(g->d, B, c, bpw);
    GX_REQUIRE(c.fits(), GX_ENOMEM, "workspace too small: need %zu bytes, have %zu", c.used, work_bytes);
    return GX_OK;
}

extern "C" gx_status gx_batch_run(gx_graph *g, int32_t algo, const int32_t *sources, uint32_t B, float damping,
                                  uint32_t iters, void *dev_work, size_t work_bytes, void *dev_out,
                                  const gx_tune *tune, void *stream, gx_run_stats *out) {
    clear_error();
    BsWork bsw;
    BpWork bpw;
    gx_status st = batch_common(g, algo, sources, B, dev_work, work_bytes, dev_out, &bsw, &bpw);
    if (st != GX_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto t0 = std::chrono::steady_clock::now();
    gx_run_stats rs{};
    if (algo == GX_SSSP) {
        gx_tune tn = tune ? *tune : default_tune(B);
        if (tn.block == 0) tn.block = 256;
        if (tn.tile == 0) tn.tile = tn.block * 8;
        if (tn.width == 0) tn.width = B;
        GX_CHECK_HIP(hipMemcpyAsync(bsw.src, sources, B * 4, hipMemcpyHostToDevice, s), g);
        int64_t steps = 0;
        st = run_bsssp(g, bsw.src, B, bsw, static_cast<uint32_t *>(dev_out), tn, s, &steps);
        if (st != GX_OK) return st;
        rs.supersteps = steps;
        rs.converged = 1;
    } else {
        GX_REQUIRE(damping >= 0.f && damping < 1.f, GX_EINVAL, "damping %f out of [0,1)", damping);
        GX_CHECK_HIP(hipMemcpyAsync(bpw.seed, sources, B * 4, hipMemcpyHostToDevice, s), g);
        st = run_bppr(g, bpw.seed, B, bpw, damping, iters, static_cast<float *>(dev_out), s,
                      tune ? (int)tune->grid : 0);
        if (st != GX_OK) return st;
        rs.supersteps = iters;
        rs.edges = (int64_t)iters * g->d.E;
    }
    rs.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (out) *out = rs;
    return GX_OK;
}

// Autotune results kept on disk when GX_TUNE_CACHE names a file: one line
// per (graph signature, algorithm, lanes, iterations) with the chosen shape
// and its time.  The signature hashes the graph's size, its out-degrees and
// the device's CU count (FNV-1a), so a cached shape is reused only for the
// same graph on the same kind of device.
namespace {
struct TuneKey {
    uint64_t sig;
    int32_t algo;
    uint32_t B, iters;
    bool operator<(const TuneKey &o) const {
        return std::tie(sig, algo, B, iters) < std::tie(o.sig, o.algo, o.B, o.iters);
    }
};
struct TuneCache {
    std::mutex mu;
    std::string path;  // the file the map was read from
    std::map<TuneKey, std::pair<gx_tune, double>> map;
};
TuneCache &tune_cache() {
    static TuneCache c;
    return c;
}

uint64_t graph_signature(const gx_graph *g) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; i++) {
            h ^= (v >> (8 * i)) & 0xFFu;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)g->d.V);
    mix((uint64_t)g->d.E);
    mix((uint64_t)g->num_cus);
    for (int32_t d : g->host_outdeg) mix((uint64_t)(uint32_t)d);
    return h;
}

// Reads the file named by GX_TUNE_CACHE into the map (again when the name
// changes); returns false when the variable is not set.
bool tune_cache_open(TuneCache &c) {
    const char *p = std::getenv("GX_TUNE_CACHE");
    if (!p || !*p) return false;
    if (c.path == p) return true;
    c.path = p;
    c.map.clear();
    if (FILE *f = std::fopen(p, "r")) {
        unsigned long long sig;
        int algo;
        unsigned B, iters, block, tile, width, grid;
        double ms;
        while (std::fscanf(f, "%llx %d %u %u %u %u %u %u %lf", &sig, &algo, &B, &iters, &block, &tile, &width,
                           &grid, &ms) == 9)
            c.map[TuneKey{sig, algo, B, iters}] = {gx_tune{block, tile, width, grid}, ms};
        std::fclose(f);
    }
    return true;
}
}  // namespace

extern "C" gx_status gx_batch_autotune(gx_graph *g, int32_t algo, const int32_t *sources, uint32_t B, float damping,
                                       uint32_t iters, void *dev_work, size_t work_bytes, void *dev_out,
                                       void *stream, gx_tune *best, double *best_ms) {
    clear_error();
    GX_REQUIRE(best, GX_EINVAL, "best is NULL");
    BsWork bsw;
    BpWork bpw;
    gx_status st = batch_common(g, algo, sources, B, dev_work, work_bytes, dev_out, &bsw, &bpw);
    if (st != GX_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const TuneKey key{graph_signature(g), algo, B, algo == GX_PPR ? iters : 0u};
    {
        TuneCache &tc = tune_cache();
        std::lock_guard<std::mutex> lk(tc.mu);
        auto it = tune_cache_open(tc) ? tc.map.find(key) : tc.map.end();
        if (it != tc.map.end()) {  // a stored shape: run it once so dev_out holds its result
            *best = it->second.first;
            if (best_ms) *best_ms = it->second.second;
            if (algo == GX_SSSP) {
                GX_CHECK_HIP(hipMemcpyAsync(bsw.src, sources, B * 4, hipMemcpyHostToDevice, s), g);
                return run_bsssp(g, bsw.src, B, bsw, static_cast<uint32_t *>(dev_out), *best, s, nullptr);
            }
            GX_CHECK_HIP(hipMemcpyAsync(bpw.seed, sources, B * 4, hipMemcpyHostToDevice, s), g);
            return run_bppr(g, bpw.seed, B, bpw, damping, iters, static_cast<float *>(dev_out), s, (int)best->grid);
        }
    }
    std::vector<gx_tune> cands;
    if (algo == GX_SSSP) {
        int nv = 0;
        const BsVariant *vars = bs_variants(&nv);
        for (uint32_t width = 32; width <= B; width *= 2) {
            if (B % width) continue;
            for (int i = 0; i < nv; i++) cands.push_back(gx_tune{vars[i].block, vars[i].block * vars[i].vt, width, 0});
        }
        GX_CHECK_HIP(hipMemcpyAsync(bsw.src, sources, B * 4, hipMemcpyHostToDevice, s), g);
    } else {
        for (int frac : {1, 2, 4}) cands.push_back(gx_tune{256, BP_TILE, B, (uint32_t)(g->num_cus * frac)});
        GX_CHECK_HIP(hipMemcpyAsync(bpw.seed, sources, B * 4, hipMemcpyHostToDevice, s), g);
    }
    const size_t n = (size_t)g->d.V * B;
    std::vector<uint32_t> ref, cur;
    double bms = 1e300;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GX_CHECK_HIP(hipEventCreate(&e0), g);
    GX_CHECK_HIP(hipEventCreate(&e1), g);
    gx_status result = GX_OK;
    for (size_t ci = 0; ci < cands.size() && result == GX_OK; ci++) {
        const gx_tune &tn = cands[ci];
        (void)hipEventRecord(e0, s);
        if (algo == GX_SSSP)
            result = run_bsssp(g, bsw.src, B, bsw, static_cast<uint32_t *>(dev_out), tn, s, nullptr);
        else
            result = run_bppr(g, bpw.seed, B, bpw, damping, iters, static_cast<float *>(dev_out), s, (int)tn.grid);
        (void)hipEventRecord(e1, s);
        if (result != GX_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
            result = GX_EDEVICE;
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        // every candidate must reproduce the first candidate's tile exactly
        cur.resize(n);
        if (hipMemcpy(cur.data(), dev_out, n * 4, hipMemcpyDeviceToHost) != hipSuccess) {
            result = GX_EDEVICE;
            break;
        }
        if (ci == 0) ref.swap(cur);
        else if (std::memcmp(ref.data(), cur.data(), n * 4) != 0) {
            set_error("autotune candidate block=%u tile=%u width=%u grid=%u changed the result", tn.block, tn.tile,
                      tn.width, tn.grid);
            result = GX_EDEVICE;
            break;
        }
        if (ms < bms) {
            bms = ms;
            *best = tn;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != GX_OK) return result;
    if (best_ms) *best_ms = bms;
    {
        TuneCache &tc = tune_cache();
        std::lock_guard<std::mutex> lk(tc.mu);
        if (tune_cache_open(tc)) {
            tc.map[key] = {*best, bms};
            if (FILE *f = std::fopen(tc.path.c_str(), "a")) {
                std::fprintf(f, "%llx %d %u %u %u %u %u %u %.6f\n", (unsigned long long)key.sig, key.algo, key.B,
                             key.iters, best->block, best->tile, best->width, best->grid, bms);
                std::fclose(f);
            }
        }
    }
    // leave the best candidate's result in dev_out
    if (algo == GX_SSSP)
        return run_bsssp(g, bsw.src, B, bsw, static_cast<uint32_t *>(dev_out), *best, s, nullptr);
    return run_bppr(g, bpw.seed, B, bpw, damping, iters, static_cast<float *>(dev_out), s, (int)best->grid);
}
