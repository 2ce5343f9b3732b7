// Batched-lane engine: argument blocks, workspace layouts and launchers
// shared by gx_batch.hip and the serving scheduler.
#pragma once

#include "gx_device.h"
#include "gx_internal.h"

namespace gx {

constexpr int BS_MIN_TILE = 1024;  // smallest SSSP work tile among the variants
constexpr int BP_TILE = 256;       // in-edges per PPR pull tile (one wave)
constexpr int BP_DCHUNK = 256;     // tiles per first-level dangling partial
constexpr double BARRIER_LIMIT_S = 20.0;  // longest wait of a grid barrier before it reports an error

struct BsCtl {
    GridBar bar;
    unsigned long long list[4];     // per superstep slot: (entries << 32) | units
    unsigned long long changed[4];  // (vertex, lane) activations
    unsigned int steps;             // supersteps run by the last launch
    unsigned int pad[3];
};

struct BsArgs {
    const int32_t *rp;
    const uint2 *adj;
    int64_t V;
    uint32_t B, l0, G;  // lane stride, first lane of the pass, 32-lane groups in the pass
    uint32_t *D;
    uint32_t *M[2];
    uint4 *list;
    uint4 *S;
    uint32_t *tile_start;
    BsCtl *ctl;
    uint32_t max_steps;
    uint32_t k0;          // global superstep index of the first superstep (mask parity)
    uint32_t *lane_cnt;   // optional [max_steps x B] activations per lane and superstep
    uint32_t stop_when_idle;
    unsigned long long bar_ticks;  // wall-clock ticks a grid barrier waits before reporting an error
};

struct BsWork {
    uint32_t *M[2];
    uint4 *list;
    uint4 *S;
    uint32_t *tile_start;
    BsCtl *ctl;
    int32_t *src;
};

struct BsVariant {
    uint32_t block, vt;
    const void *fn;
};

struct BpArgs {
    const int32_t *in_rp, *in_col, *outdeg, *trow;
    int64_t ntiles, V, E;
    uint32_t B;   // lane stride of the tiles
    uint32_t Bw;  // lanes processed (0..Bw-1); the rest keep their values untouched
    float d;
    const int32_t *seed;  // per lane; -1 = free lane
    const int32_t *end;   // per lane: first superstep it no longer runs (NULL: every lane runs every superstep)
    float *x[2], *c[2];
    double *head, *tailp, *dsum, *dpart, *D[2];  // D[k & 1]: dangling mass of superstep k
    int32_t *spill;
};

struct BpWork {
    int64_t ntiles;
    float *x[2], *c[2];
    double *head, *tailp, *dsum, *dpart, *D[2];
    int32_t *spill, *trow, *seed, *end;
};

const BsVariant *bs_variants(int *n);
int coop_grid(const void *kernel, int block, int num_cus, int want, int max_per_cu);
void bs_layout(const DevGraph &d, uint32_t B, Carver &c, BsWork *w);
void bp_layout(const DevGraph &d, uint32_t B, Carver &c, BpWork *w);
hipError_t launch_coop(const void *kernel, int grid, int block, void *args, hipStream_t s);
unsigned long long barrier_limit_ticks(int device);
gx_tune default_tune(uint32_t B);

hipError_t bs_launch_superstep(const BsArgs &a, uint32_t k, uint32_t it, int grid, hipStream_t s);
hipError_t bp_launch_superstep(const BpArgs &a, uint32_t k, int grid, hipStream_t s);
hipError_t bs_lane_reset(uint32_t *D, uint32_t *Mc, uint32_t *Mn, int64_t V, uint32_t B, uint32_t G, uint32_t lane,
                         int32_t src, hipStream_t s);
hipError_t bp_lane_reset(float *x, float *c, double *D, const int32_t *outdeg, int64_t V, uint32_t B, uint32_t lane,
                         int32_t seed, hipStream_t s);
hipError_t bp_make_tiles(const int32_t *in_rp, int64_t V, int64_t ntiles, int32_t *trow, hipStream_t s);
hipError_t lane_extract(const uint32_t *tile, int64_t V, uint32_t B, uint32_t lane, uint32_t *out, hipStream_t s);

}  // namespace gx
