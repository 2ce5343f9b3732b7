// Label propagation (community-detection form) on the symmetric adjacency.
//
// The paper's evaluation runs "LP" capped at 15 iterations (Section "Setup",
// first footnote) through the algorithm template (Section "Algorithm
// Template"): MSGGen sends a vertex's label along each of its edges in both
// directions, MSGMerge gathers the labels bound for a vertex, MSGApply keeps
// the most frequent one (the smallest on a tie).  One superstep reads the
// labels of its start (lab[k & 1]) and writes lab[(k + 1) & 1].
//
// The merge is a mode over a multiset, so it is computed where the messages
// meet: every vertex reads its distinct neighbours' labels and counts them.
// Vertices are grouped by degree so each group's counting fits its size:
//   classes 0..4 (d <= 4 .. 64): one lane group of width G = 4 .. 64 per
//     vertex, each lane one neighbour, counts by G lane shuffles and the
//     winner by a butterfly maximum of (count, ~label);
//   class 5 (64 < d <= LP_MID_MAX): one workgroup per vertex, labels counted
//     in an LDS hash table at most half full;
//   class 6 (hubs): neighbours cut into chunks; each chunk counts in LDS and
//     adds its (label, count) pairs to the hub's table in device memory; a
//     second kernel takes each hub's maximum and clears its table.
// Counts are exact integers and the winner is the unique maximum of
// (count, ~label), so the result does not depend on the order of the atomics.
#include <algorithm>
#include <vector>

#include "gx_device.h"
#include "gx_internal.h"

using namespace gx;

namespace {

constexpr int LP_BLOCK = 256;

__device__ __forceinline__ unsigned long long lp_key(uint32_t count, uint32_t label) {
    return ((unsigned long long)count << 32) | (unsigned long long)(0xFFFFFFFFu - label);
}

__device__ __forceinline__ uint32_t lp_hash(uint32_t x) { return x * 0x9E3779B1u; }

// Changed-label counts of a workgroup go to the superstep's counter; block 0
// clears the following superstep's slot (nothing else touches it meanwhile).
__device__ __forceinline__ void lp_count_changed(unsigned c, DevStep *step, DevStep *next,
                                                 unsigned long long *s_c) {
    const unsigned long long t = block_sum<unsigned long long>((unsigned long long)c, s_c);
    if (threadIdx.x == 0) {
        if (t) atomicAdd(&step->changed, t);
        if (blockIdx.x == 0 && next) *next = DevStep{};
    }
}

__global__ __launch_bounds__(LP_BLOCK) void k_lp_init(uint32_t *lab0, uint32_t *lab1, uint32_t *synced,
                                                      const int32_t *__restrict__ l2g, int64_t V, DevStep *step0) {
    const int64_t v = (int64_t)blockIdx.x * LP_BLOCK + threadIdx.x;
    if (v == 0) *step0 = DevStep{};
    if (v >= V) return;
    const uint32_t l = l2g ? (uint32_t)l2g[v] : (uint32_t)v;
    lab0[v] = l;
    lab1[v] = l;
    synced[v] = l;
}

__global__ __launch_bounds__(LP_BLOCK) void k_lp_tab_clear(uint2 *tab, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * LP_BLOCK + threadIdx.x;
    if (i < n) tab[i] = make_uint2(LP_NONE, 0u);
}

template <int G>
__global__ __launch_bounds__(LP_BLOCK) void k_lp_group(const uint32_t *__restrict__ list, int64_t n,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       const uint32_t *__restrict__ lab, uint32_t *__restrict__ nxt,
                                                       DevStep *step, DevStep *next) {
    __shared__ unsigned long long s_c[LP_BLOCK / 64];
    const int64_t i = ((int64_t)blockIdx.x * LP_BLOCK + threadIdx.x) / G;
    const int j = threadIdx.x & (G - 1);
    const int base = (threadIdx.x & 63) - j;  // first lane of this vertex's group
    const bool ok = i < n;
    uint32_t v = 0;
    int32_t a = 0, d = 0;
    if (ok) {
        v = list[i];
        a = rp[v];
        d = rp[v + 1] - a;
    }
    const uint32_t L = (ok && j < d) ? lab[col[a + j]] : LP_NONE;
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < G; q++) c += (uint32_t)(__shfl(L, base + q, 64) == L);
    unsigned long long key = L != LP_NONE ? lp_key(c, L) : 0ull;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        const unsigned long long k2 = __shfl_xor(key, o, 64);
        key = k2 > key ? k2 : key;
    }
    unsigned chg = 0;
    if (ok && j == 0) {
        const uint32_t nl = 0xFFFFFFFFu - (uint32_t)key;
        nxt[v] = nl;
        chg = nl != lab[v];
    }
    lp_count_changed(chg, step, next, s_c);
}

// One workgroup per vertex of the mid class; the table holds the next power
// of two at or above 2d slots, so it is at most half full.
__global__ __launch_bounds__(LP_BLOCK) void k_lp_mid(const uint32_t *__restrict__ list, int64_t n,
                                                     const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                     const uint32_t *__restrict__ lab, uint32_t *__restrict__ nxt,
                                                     DevStep *step, DevStep *next) {
    __shared__ uint32_t s_key[LP_MID_SLOTS];
    __shared__ uint32_t s_cnt[LP_MID_SLOTS];
    __shared__ unsigned long long s_best[LP_BLOCK / 64];
    __shared__ unsigned long long s_c[LP_BLOCK / 64];
    const int tid = threadIdx.x;
    unsigned chg = 0;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint32_t v = list[i];
        const int32_t a = rp[v], d = rp[v + 1] - a;
        int lg = 7;
        while ((1 << lg) < 2 * d) lg++;
        const int slots = 1 << lg;
        for (int s = tid; s < slots; s += LP_BLOCK) {
            s_key[s] = LP_NONE;
            s_cnt[s] = 0;
        }
        __syncthreads();
        for (int e = tid; e < d; e += LP_BLOCK) {
            const uint32_t L = lab[col[a + e]];
            uint32_t h = lp_hash(L) >> (32 - lg);
            for (;;) {
                const uint32_t k = atomicCAS(&s_key[h], LP_NONE, L);
                if (k == LP_NONE || k == L) {
                    atomicAdd(&s_cnt[h], 1u);
                    break;
                }
                h = (h + 1) & (uint32_t)(slots - 1);
            }
        }
        __syncthreads();
        unsigned long long best = 0;
        for (int s = tid; s < slots; s += LP_BLOCK) {
            const uint32_t k = s_key[s];
            if (k != LP_NONE) {
                const unsigned long long key = lp_key(s_cnt[s], k);
                best = key > best ? key : best;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long b2 = __shfl_down(best, o, 64);
            best = b2 > best ? b2 : best;
        }
        if ((tid & 63) == 0) s_best[tid >> 6] = best;
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < LP_BLOCK / 64; w++) best = s_best[w] > best ? s_best[w] : best;
            const uint32_t nl = 0xFFFFFFFFu - (uint32_t)best;
            nxt[v] = nl;
            chg += nl != lab[v];
        }
        __syncthreads();
    }
    lp_count_changed(chg, step, next, s_c);
}

// Hub chunks: each workgroup counts its chunk's labels in an LDS table
// (labels that find no free slot within a few probes go straight to the
// hub's table) and adds the chunk's (label, count) pairs to the hub's table.
constexpr int LP_CHUNK_SLOTS = 4096;
constexpr int LP_CHUNK_PROBES = 16;

__device__ __forceinline__ void lp_tab_add(uint2 *tab, uint32_t slots, uint32_t L, uint32_t c) {
    uint32_t h = (lp_hash(L) >> 7) & (slots - 1);
    for (;;) {
        const uint32_t k = atomicCAS(&tab[h].x, LP_NONE, L);
        if (k == LP_NONE || k == L) {
            atomicAdd(&tab[h].y, c);
            return;
        }
        h = (h + 1) & (slots - 1);
    }
}

__global__ __launch_bounds__(LP_BLOCK) void k_lp_hub_count(const uint4 *__restrict__ chunks,
                                                           const uint2 *__restrict__ hub,
                                                           const int32_t *__restrict__ col,
                                                           const uint32_t *__restrict__ lab, uint2 *tab) {
    __shared__ uint32_t s_key[LP_CHUNK_SLOTS];
    __shared__ uint32_t s_cnt[LP_CHUNK_SLOTS];
    const uint4 ch = chunks[blockIdx.x];
    const uint2 hb = hub[ch.x];
    uint2 *t = tab + hb.x;
    for (int s = threadIdx.x; s < LP_CHUNK_SLOTS; s += LP_BLOCK) {
        s_key[s] = LP_NONE;
        s_cnt[s] = 0;
    }
    __syncthreads();
    for (uint32_t e = ch.y + threadIdx.x; e < ch.z; e += LP_BLOCK) {
        const uint32_t L = lab[col[e]];
        uint32_t h = lp_hash(L) >> 20;  // 12 bits: LP_CHUNK_SLOTS
        bool done = false;
        for (int p = 0; p < LP_CHUNK_PROBES; p++) {
            const uint32_t k = atomicCAS(&s_key[h], LP_NONE, L);
            if (k == LP_NONE || k == L) {
                atomicAdd(&s_cnt[h], 1u);
                done = true;
                break;
            }
            h = (h + 1) & (LP_CHUNK_SLOTS - 1);
        }
        if (!done) lp_tab_add(t, hb.y, L, 1u);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < LP_CHUNK_SLOTS; s += LP_BLOCK)
        if (s_key[s] != LP_NONE) lp_tab_add(t, hb.y, s_key[s], s_cnt[s]);
}

// One workgroup per hub: the maximum of (count, ~label) over its table,
// which is cleared for the next superstep on the way.
__global__ __launch_bounds__(LP_BLOCK) void k_lp_hub_pick(const uint32_t *__restrict__ hubs, int64_t n,
                                                          const uint2 *__restrict__ hub, uint2 *tab,
                                                          const uint32_t *__restrict__ lab, uint32_t *__restrict__ nxt,
                                                          DevStep *step, DevStep *next) {
    __shared__ unsigned long long s_best[LP_BLOCK / 64];
    __shared__ unsigned long long s_c[LP_BLOCK / 64];
    unsigned chg = 0;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint2 hb = hub[i];
        uint2 *t = tab + hb.x;
        unsigned long long best = 0;
        for (uint32_t s = threadIdx.x; s < hb.y; s += LP_BLOCK) {
            const uint2 q = t[s];
            if (q.x != LP_NONE) {
                const unsigned long long key = lp_key(q.y, q.x);
                best = key > best ? key : best;
                t[s] = make_uint2(LP_NONE, 0u);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long b2 = __shfl_down(best, o, 64);
            best = b2 > best ? b2 : best;
        }
        if ((threadIdx.x & 63) == 0) s_best[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < LP_BLOCK / 64; w++) best = s_best[w] > best ? s_best[w] : best;
            const uint32_t v = hubs[i];
            const uint32_t nl = 0xFFFFFFFFu - (uint32_t)best;
            nxt[v] = nl;
            chg += nl != lab[v];
        }
        __syncthreads();
    }
    lp_count_changed(chg, step, next, s_c);
}

int lp_class_of(int32_t d) {
    if (d <= 0) return -1;
    if (d <= 4) return 0;
    if (d <= 8) return 1;
    if (d <= 16) return 2;
    if (d <= 32) return 3;
    if (d <= 64) return 4;
    if (d <= LP_MID_MAX) return 5;
    return 6;
}

uint32_t lp_hub_slots(int32_t d) {
    uint32_t s = 256;
    while (s < (uint32_t)d + (uint32_t)d / 2) s *= 2;  // load at most 2/3
    return s;
}

// Class sizes, hub chunks and hub table slots from the host copy of the
// symmetric degrees.
void lp_shape(const gx_graph *g, int64_t off[LP_CLASSES + 1], int64_t *nchunks, int64_t *tab_slots) {
    int64_t cnt[LP_CLASSES] = {};
    *nchunks = 0;
    *tab_slots = 0;
    for (int32_t d : g->host_symdeg) {
        const int c = lp_class_of(d);
        if (c < 0) continue;
        cnt[c]++;
        if (c == LP_CLASSES - 1) {
            *nchunks += (d + LP_HUB_CHUNK - 1) / LP_HUB_CHUNK;
            *tab_slots += lp_hub_slots(d);
        }
    }
    off[0] = 0;
    for (int c = 0; c < LP_CLASSES; c++) off[c + 1] = off[c] + cnt[c];
}

template <class T>
unsigned blocks_for(T n, int b) {
    return (unsigned)std::max<T>(1, (n + b - 1) / b);
}

}  // namespace

namespace gx {

size_t lp_layout(gx_graph *g, Carver &c, gx_state *s) {
    const int64_t V = g->d.V;
    lp_shape(g, s->lp_off, &s->lp_nchunks, &s->lp_tab_slots);
    s->lab[0] = c.take<uint32_t>(V);
    s->lab[1] = c.take<uint32_t>(V);
    s->synced = c.take<uint32_t>(V);
    s->lp_list = c.take<uint32_t>(std::max<int64_t>(1, s->lp_off[LP_CLASSES]));
    const int64_t hubs = s->lp_off[LP_CLASSES] - s->lp_off[LP_CLASSES - 1];
    s->lp_chunks = c.take<uint4>(std::max<int64_t>(1, s->lp_nchunks));
    s->lp_hub = c.take<uint2>(std::max<int64_t>(1, hubs));
    s->lp_tab = c.take<uint2>(std::max<int64_t>(1, s->lp_tab_slots));
    return c.used;
}

// Builds the class lists (ascending vertex order inside a class), the hub
// chunks and table offsets on the host, uploads them, and initialises the
// labels to the global ids.  Synchronises `hs` (the host arrays are freed
// on return).
gx_status lp_init(gx_state *s, hipStream_t hs) {
    const gx_graph *g = s->g;
    const DevGraph &d = g->d;
    const int64_t V = d.V;
    std::vector<uint32_t> list((size_t)std::max<int64_t>(1, s->lp_off[LP_CLASSES]));
    std::vector<uint4> chunks((size_t)std::max<int64_t>(1, s->lp_nchunks));
    const int64_t hubs = s->lp_off[LP_CLASSES] - s->lp_off[LP_CLASSES - 1];
    std::vector<uint2> hub((size_t)std::max<int64_t>(1, hubs));
    {
        int64_t pos[LP_CLASSES];
        for (int c = 0; c < LP_CLASSES; c++) pos[c] = s->lp_off[c];
        int64_t nch = 0, slot = 0;
        for (int64_t v = 0; v < V; v++) {
            const int32_t deg = g->host_symdeg[(size_t)v];
            const int c = lp_class_of(deg);
            if (c < 0) continue;
            list[(size_t)pos[c]++] = (uint32_t)v;
        }
        // hub chunks need the hubs' first symmetric entries: prefix sums of the degrees
        int64_t acc = 0;
        int64_t h = 0;
        for (int64_t v = 0; v < V; v++) {
            const int32_t deg = g->host_symdeg[(size_t)v];
            if (lp_class_of(deg) == LP_CLASSES - 1) {
                const uint32_t slots = lp_hub_slots(deg);
                hub[(size_t)h] = make_uint2((uint32_t)slot, slots);
                for (int64_t e = 0; e < deg; e += LP_HUB_CHUNK)
                    chunks[(size_t)nch++] = make_uint4((uint32_t)h, (uint32_t)(acc + e),
                                                       (uint32_t)(acc + std::min<int64_t>(deg, e + LP_HUB_CHUNK)), 0u);
                slot += slots;
                h++;
            }
            acc += deg;
        }
    }
    if (V > 0) {
        hipLaunchKernelGGL(k_lp_init, dim3(blocks_for<int64_t>(V, LP_BLOCK)), dim3(LP_BLOCK), 0, hs, s->lab[0],
                           s->lab[1], s->synced, d.l2g, V, s->steps);
        if (s->lp_tab_slots > 0)
            hipLaunchKernelGGL(k_lp_tab_clear, dim3(blocks_for<int64_t>(s->lp_tab_slots, LP_BLOCK)), dim3(LP_BLOCK), 0,
                               hs, s->lp_tab, s->lp_tab_slots);
        if (s->lp_off[LP_CLASSES] > 0)
            GX_CHECK_HIP(hipMemcpyAsync(s->lp_list, list.data(), (size_t)s->lp_off[LP_CLASSES] * 4,
                                        hipMemcpyHostToDevice, hs), s);
        if (s->lp_nchunks > 0) {
            GX_CHECK_HIP(hipMemcpyAsync(s->lp_chunks, chunks.data(), (size_t)s->lp_nchunks * sizeof(uint4),
                                        hipMemcpyHostToDevice, hs), s);
            GX_CHECK_HIP(hipMemcpyAsync(s->lp_hub, hub.data(), (size_t)hubs * sizeof(uint2), hipMemcpyHostToDevice,
                                        hs), s);
        }
    } else {
        hipLaunchKernelGGL(k_lp_init, dim3(1), dim3(LP_BLOCK), 0, hs, s->lab[0], s->lab[1], s->synced, d.l2g,
                           (int64_t)0, s->steps);
    }
    GX_CHECK_HIP(hipGetLastError(), s);
    GX_CHECK_HIP(hipStreamSynchronize(hs), s);
    return GX_OK;
}

// One superstep: labels lab[k & 1] -> lab[(k + 1) & 1]; the changed count
// goes to `step`, `next` is cleared for the following superstep.
void lp_enqueue(gx_state *s, hipStream_t hs, DevStep *step, DevStep *next) {
    const DevGraph &d = s->g->d;
    const int cur = (int)(s->k & 1);
    const uint32_t *lab = s->lab[cur];
    uint32_t *nxt = s->lab[cur ^ 1];
    const int64_t *off = s->lp_off;
    // (every launch below may clear `next`; the first one always runs)
    auto group = [&](auto kern, int c, int G) {
        const int64_t n = off[c + 1] - off[c];
        hipLaunchKernelGGL(kern, dim3(blocks_for<int64_t>(std::max<int64_t>(1, n) * G, LP_BLOCK)), dim3(LP_BLOCK), 0,
                           hs, s->lp_list + off[c], n, d.sym_rp, d.sym_col, lab, nxt, step, next);
    };
    group(k_lp_group<4>, 0, 4);
    group(k_lp_group<8>, 1, 8);
    group(k_lp_group<16>, 2, 16);
    group(k_lp_group<32>, 3, 32);
    group(k_lp_group<64>, 4, 64);
    const int64_t nmid = off[6] - off[5];
    if (nmid > 0)
        hipLaunchKernelGGL(k_lp_mid, dim3((unsigned)std::min<int64_t>(nmid, (int64_t)s->g->num_cus * 8)),
                           dim3(LP_BLOCK), 0, hs, s->lp_list + off[5], nmid, d.sym_rp, d.sym_col, lab, nxt, step,
                           nullptr);
    const int64_t nhub = off[7] - off[6];
    if (nhub > 0) {
        hipLaunchKernelGGL(k_lp_hub_count, dim3((unsigned)s->lp_nchunks), dim3(LP_BLOCK), 0, hs, s->lp_chunks,
                           s->lp_hub, d.sym_col, lab, s->lp_tab);
        hipLaunchKernelGGL(k_lp_hub_pick, dim3((unsigned)std::min<int64_t>(nhub, (int64_t)s->g->num_cus * 4)),
                           dim3(LP_BLOCK), 0, hs, s->lp_list + off[6], nhub, s->lp_hub, s->lp_tab, lab, nxt, step,
                           nullptr);
    }
}

// Vertices an LP superstep computes (those with at least one neighbour).
int64_t lp_active(const gx_state *s) { return s->lp_off[LP_CLASSES]; }

}  // namespace gx
