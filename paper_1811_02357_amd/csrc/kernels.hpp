// kernels.hpp -- launch interface of the IRT-PS kernels (internal to libirtps).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "traverse.hpp"

namespace irtps {
namespace kern {

constexpr int kMaxLights = 64;
constexpr int kNumCounters = 5;  // IRTPS_NUM_COUNTERS
// Tracer tiles: one 256-thread block covers tile_w x (256 / tile_w) pixels.
constexpr int kTileThreads = 256;
__host__ __device__ inline int tile_rows(int tile_w) { return kTileThreads / tile_w; }
// Tile width of the direct-shading kernels (tiles of 8 x 32 samples).
constexpr int kDirectTileW = 8;
__host__ __device__ inline int tiles_for(int W, int H, int tile_w) {
    const int th = tile_rows(tile_w);
    return ((W + tile_w - 1) / tile_w) * ((H + th - 1) / th);
}
// Most tracer tiles over the schedule's tile widths (8..64).
__host__ __device__ inline int max_trace_tiles(int W, int H) {
    int m = 0;
    for (int tw = 8; tw <= 64; tw *= 2) m = tiles_for(W, H, tw) > m ? tiles_for(W, H, tw) : m;
    return m;
}
// Chunks: the single-job tracer hands out pixels by chunks of one wave's 64,
// tile_w x (64 / tile_w) of them, in row-major chunk order.
constexpr int kChunkPixels = 64;
__host__ __device__ inline int chunk_rows(int tile_w) { return kChunkPixels / tile_w; }
__host__ __device__ inline int chunks_for(int W, int H, int tile_w) {
    const int th = chunk_rows(tile_w);
    return ((W + tile_w - 1) / tile_w) * ((H + th - 1) / th);
}
__host__ __device__ inline int max_trace_chunks(int W, int H) {
    int m = 0;
    for (int tw = 8; tw <= 64; tw *= 2) m = chunks_for(W, H, tw) > m ? chunks_for(W, H, tw) : m;
    return m;
}
constexpr int kMaxMgLevels = 16;
constexpr int kFlagQuadrature = 1;
constexpr int kFlagFlat = 4;
constexpr int kFlagShadowPs = 8;  // IRTPS_FLAG_SHADOW_AWARE_PS
constexpr int kFlagRobust = 32;   // IRTPS_FLAG_ROBUST_INTEGRATION

// Eq.4 solve matrix, rows x, y, z over the K lights (passed by value).
struct PsMatrix {
    float m[3][kMaxLights];
};

// Calibrated lights: unit directions and intensities (passed by value).
struct LightSet {
    int K;
    float l[kMaxLights][3];
    float s[kMaxLights];
};

// A heightfield with its apron-max pyramid (level offsets in floats).
struct SurfaceArgs {
    const float* H;
    const float* pyr;  // apron-max levels, then the four quadrant maxima
    int W, Hh;
    int levels;
    int quad_off;      // floats from pyr to the block tables (escape windows, quadrant maxima)
    int off[trv::kMaxLevels];
    int wc[trv::kMaxLevels];  // cells per row of every level
};

struct TraceArgs {
    SurfaceArgs sa;
    const float* n;    // [H][W][3]
    const float* rho;  // [C][H][W]
    const float* S;    // [H][W][K]
    const float* env;  // [He][We][C]
    float* G;          // [H][W][K][C]: per-pixel sums during the trace, then the means
    unsigned long long* counters;  // 4 x u64 or null
    int env_h, env_w;
    int C, K;
    int spp, B, t, tag, flags;
    int ready_batch;   // lanes that must have a result before the wave shades
    int tile_shift;    // tile (batched tracer) or chunk (single-job tracer) width 2^tile_shift
    uint32_t key0, key1;
    // Single-job tracer only (the batched one leaves both null): the chunks in
    // the order they are handed out (a permutation), or null: row-major; and
    // per chunk the sum of its pixels' times in wall-clock ticks, then one slot
    // for the launch's chunk queue (both cleared by the launcher), or null:
    // each wave takes a fixed stride of the chunks.
    const int* order;
    unsigned* tile_cost;
    float* records;       // per-path mode: segment records (split_record_bytes), or null
    // Single-job tracer: per pixel the C sums of its escapes' terms, [H][W][C];
    // G then keeps the per-light hit sums and correct() forms the means.  Null:
    // G holds the means.
    float* esc_sums;
    // Walls (the known environment as geometry), or box_z <= 0: none.  A ray
    // that leaves the surface and meets a wall below box_z adds the wall
    // texel's term like a surface hit (row box_S, weight beta times its albedo).
    float box_z;
    int box_th, box_tw;
    const float* box_albedo;  // [4][th][tw][C]
    const float* box_S;       // [4][th][tw][K]
};

// The walls of the box: height and texture size (the walls' own direct light,
// box_shade, goes to S [4][th][tw][K]).
struct BoxArgs {
    float z;
    int th, tw;
};

// Small problems can trace one path per (pixel, sample) lane: each lane records
// its segments' outcomes (code: the hit sample q, or -(texel + 1) for an escape;
// then C weights), and a second pass adds them into G pixel by pixel in (sample,
// segment) order -- the same sums as the per-pixel tracer, with spp times the
// lanes.  Measured on MI355X it pays up to 128 x 128 pixels (64 x 64: 30% off
// the solve; 128 x 128: even; 256 x 256: the per-pixel tracer is 1.8x faster).
// Bytes of the records, or 0 where the mode does not apply.
constexpr long long kSplitMaxPixels = 16384;
constexpr long long kSplitMaxBytes = 64LL << 20;
__host__ __device__ inline long long split_record_bytes(long long npx, int C, int spp, int B) {
    if (npx > kSplitMaxPixels || B < 1 || spp < 1) return 0;
    const long long b = npx * spp * B * (1 + C) * 4;
    return b <= kSplitMaxBytes ? b : 0;
}

// Multigrid levels of a W x H grid, offsets (in floats) into the workspace.
// Levels of at most kMgTailNodes nodes (from `tail` to the coarsest) run in one
// single-block launch per V-cycle.
constexpr int kMgTailNodes = 4096;
constexpr long long kMgTailLdsBytes = 65536;
// Blocks of 256 threads for n elements, and near-horizon tiles (16 x 16) of a
// W x H surface: the units of the flattened multi-job grids.
constexpr int kNearTile = 16;
__host__ __device__ inline int flat_blocks(long long n) { return (int)((n + 255) / 256); }
__host__ __device__ inline int near_tiles(int W, int H) {
    return ((W + kNearTile - 1) / kNearTile) * ((H + kNearTile - 1) / kNearTile);
}
struct MgPlan {
    int levels;
    int tail;  // first level with at most kMgTailNodes nodes
    int W[kMaxMgLevels], H[kMaxMgLevels];
    long long xoff[kMaxMgLevels], boff[kMaxMgLevels];
    long long keyoff;  // uint32s: [0] the anchor's minimum, [1] the largest surface change (D_H)
    long long total;   // floats
};

// One reconstruction as the multi-job kernels see it (device memory).
struct JobDesc {
    int W, Hh, C, K;
    int spp, B, t, T;
    int rho_mode, flags, cycles_cold, cycles_warm;
    float stop_tol;     // > 0: the iteration whose D_H is below it is the last (T lowered to t + 1)
    uint32_t key0, key1;
    int active;         // 0: skipped by every multi-job kernel
    int tile_shift, ready_batch;  // the tracer's schedule for this job
    int pyr_levels, quad_off;
    int pyr_wc[trv::kMaxLevels], pyr_hc[trv::kMaxLevels], pyr_off[trv::kMaxLevels];
    MgPlan mg;
    // First block of this job in the flattened grids of the batch (jobs in
    // table order, each with only the blocks it needs): multigrid level l
    // (smoothing, prolongation; 0 blocks from the tail level on), restriction
    // l -> l+1, and the near-horizon tiles.
    int mg_bstart[kMaxMgLevels], rs_bstart[kMaxMgLevels], near_bstart;
    const float* I0;     // [K][C][H][W]
    const float* env;    // [He][We][C]
    int env_h, env_w;
    float* A;            // [K][C][H][W]
    float* S;            // [H][W][K]
    float* G;            // [H][W][K][C]
    float* pyr;          // pyramid + quadrant maxima
    float* mg_ws;        // multigrid workspace
    float* n;            // [H][W][3]
    float* rho;          // [C][H][W]
    float* depth;        // [H][W]
    float* E;            // [K][C][H][W] or null
    unsigned long long* counters;  // 4 x u64 or null
    float M[3][kMaxLights];
    float L[kMaxLights][3];
    float s[kMaxLights];
};

// Largest extents over the jobs of a batch, used to size the grids.
struct BatchShape {
    int njobs;
    int max_npx;             // largest W * H
    int max_direct_tiles;    // largest tiles_for(W, H, kDirectTileW)
    int max_pyr_cells[trv::kMaxLevels];
    int max_pyr_levels;
    int max_rows, max_cols;  // largest H, W
    int max_mg_tail;         // largest first tail level
    long long max_mg_tail_floats;  // largest LDS need of the tail levels
    int mg_blocks[kMaxMgLevels], rs_blocks[kMaxMgLevels], near_blocks;  // flattened grid sizes
    int max_cycles_cold, max_cycles_warm;
    int max_KCnpx;           // largest K * C * W * H
    int max_K1, max_K3;      // largest light count of the grey and of the colour jobs (0: none)
};

hipError_t ps_solve(int npx, int C, int K, const PsMatrix& M, const float* A, float* n, float* rho,
                    hipStream_t st);
// Eq.4 per pixel over the lights with S[p][k] > 0 (at least three), else all.
hipError_t ps_solve_masked(int npx, int C, int K, const PsMatrix& M, const LightSet& L, const float* A,
                           const float* S, float* n, float* rho, hipStream_t st);
// box_z > 0: the walls of that height block shadow rays too.
hipError_t direct(const SurfaceArgs& sa, const float* n, const LightSet& L, int flat, float* S,
                  hipStream_t st, float box_z = 0.0f);
// The walls' direct irradiance at texel centres, S [4][th][tw][K].
hipError_t box_shade(int W, int H, const BoxArgs& b, const LightSet& L, float* S, hipStream_t st);
// The single-job tracer (per-pixel, or per-path for small problems).  With
// tile_cost set it first clears the chunk costs and the queue slot.
hipError_t trace(TraceArgs a, hipStream_t st);
// order[0..tiles) = the tiles (or chunks) by descending cost (ties in any order).
hipError_t order_tiles(const unsigned* cost, int tiles, int* order, hipStream_t st);
// Stage 5.  With esc_sums (the tracer's escape sums, esc_sums in TraceArgs) G
// holds hit sums and each mean is formed here as (G + esc) / spp, the
// tracer's own finishing arithmetic.
hipError_t correct(int npx, int C, int K, int rho_mode, int cumulative, const float* I0,
                   const float* Aprev, const float* G, const float* S, const float* rho, float* E,
                   float* Anext, hipStream_t st, const float* esc_sums = nullptr, int spp = 1);
hipError_t compose(int npx, int C, int K, const float* rho, const float* S, const float* G, float* I,
                   hipStream_t st);
// Apron-max levels of P at pyr, then the block tables at pyr + quad_off.
hipError_t build_pyramid(int W, int Hh, const float* H, const trv::Pyramid& P, float* pyr,
                         long long quad_off, hipStream_t st);
// Robust integration: after the least-squares V-cycles, `rounds` rounds of the
// Huber M-estimator (threshold delta), each a right-hand side from the shrunk
// edge residuals and `cycles` more V-cycles.  rounds = 0: least squares.
struct Robust {
    float delta = 0.0f;
    int rounds = 0;
    int cycles = 0;
};
// The loop's robust integration (IRTPS_FLAG_ROBUST_INTEGRATION).
constexpr float kRobustDelta = 0.1f;
constexpr int kRobustRounds = 6;
constexpr int kRobustCycles = 2;
// With measure_change (Hinit == Hout), the largest |H_new - H_old| over the
// nodes is left, as float bits, in uint32 [1] of the key area of ws
// (change_key_of(plan, ws)).
hipError_t integrate(const MgPlan& plan, const float* n, const float* Hinit, int cycles, float* Hout,
                     float* ws, hipStream_t st, bool measure_change = false, const Robust& robust = Robust{});
inline unsigned* change_key_of(const MgPlan& plan, float* ws) {
    return reinterpret_cast<unsigned*>(ws + plan.keyoff) + 1;
}
// ---- the r-ray variant (Sec. IV, the tracing paragraph; Fig. 5) ----
// One path per pixel, on sample 0's counters of the gather, that leaves for the
// environment on its r-th ray: E[p][c] = (albedo product of its r - 1 hits)
// pi L_env,c, valid; any other path leaves E[p] = 0, not valid.  w0 (float
// 1 / 0) and valid (uint8 1 / 0) may each be null.
constexpr int kExactRShift = 8;  // IRTPS_FLAG_EXACT_R(r) = r << 8, r in 1..7
inline int exact_r_of(int flags) { return (flags >> kExactRShift) & 7; }
hipError_t trace_exact_r(const SurfaceArgs& sa, int C, const float* n, const float* rho, const float* env,
                         int He, int We, int r, int t, int tag, uint32_t key0, uint32_t key1, int flat, float* E,
                         float* w0, unsigned char* valid, hipStream_t st);

// Pull-push fill of the pixels without a value: levels of 2 x 2 aggregates
// (ragged edges keep the children that exist) down to 1 x 1, each a weight
// plane [h][w] at woff and (levels >= 1) a value plane [h][w][C] at voff, in
// floats from the region's start; `total` floats in all.  Level 0's values are
// the image being filled; the solve keeps them in the region too, at v0off
// (total_v0 floats then).
constexpr int kMaxFillLevels = 32;
struct FillPlan {
    int levels;
    int w[kMaxFillLevels], h[kMaxFillLevels];
    long long woff[kMaxFillLevels], voff[kMaxFillLevels];
    long long total, v0off, total_v0;
};
inline FillPlan fill_plan(int W, int H, int C) {
    FillPlan f{};
    auto up64 = [](long long x) { return (x + 63) & ~63LL; };
    f.w[0] = W;
    f.h[0] = H;
    f.levels = 1;
    while ((f.w[f.levels - 1] > 1 || f.h[f.levels - 1] > 1) && f.levels < kMaxFillLevels) {
        f.w[f.levels] = (f.w[f.levels - 1] + 1) / 2;
        f.h[f.levels] = (f.h[f.levels - 1] + 1) / 2;
        ++f.levels;
    }
    long long off = 0;
    for (int l = 0; l < f.levels; ++l) {
        const long long cells = (long long)f.w[l] * f.h[l];
        f.woff[l] = off;
        off = up64(off + cells);
        f.voff[l] = l ? off : -1;
        if (l) off = up64(off + cells * C);
    }
    f.total = off;
    f.v0off = off;
    f.total_v0 = up64(off + (long long)W * H * C);
    return f;
}
// w0[p] = valid[p] ? 1 : 0 (the region's level-0 weights).
hipError_t fill_weights(long long npx, const unsigned char* valid, float* ws, hipStream_t st);
// Pull from level 0 (weights in ws, values v0 [npx][C]) up to 1 x 1, then push
// back down to level 1: a coarse cell holds the weighted mean of its children
// with a value and their summed weight; going down, a cell of weight 0 takes
// its parent's value.
hipError_t fill_pull_push(const FillPlan& fp, int C, const float* v0, float* ws, hipStream_t st);
// Level 0's push, in place: pixels of weight 0 take their parent's value (0 for
// a 1 x 1 image).
hipError_t fill_push0(const FillPlan& fp, int C, float* v0, const float* ws, hipStream_t st);
// Level 0's push written into G [p][k][c] for every light k (the r-ray image is
// the same for all lights).
hipError_t fill_push0_broadcast(const FillPlan& fp, int C, int K, const float* v0, const float* ws, float* G,
                                hipStream_t st);

hipError_t fill_f32(float* p, float v, long long n, hipStream_t st);
hipError_t fill_u64_zero(unsigned long long* p, int n, hipStream_t st);
hipError_t add_u64(unsigned long long* p, unsigned long long v, hipStream_t st);
// ---- multi-job launches: grid.y walks the job table, the tracer a tile queue ----
// Persistent tracer over (job, tile) pairs; `queue` (one uint32) is cleared here.
hipError_t trace_multi(const JobDesc* jobs, int C, const int2* tiles, int ntiles, unsigned* queue,
                       int tag, int resident_blocks, hipStream_t st);
// t = 0, counters and E cleared.
hipError_t batch_begin(const JobDesc* jobs, const BatchShape& bs, hipStream_t st);
hipError_t batch_pyramid(const JobDesc* jobs, const BatchShape& bs, hipStream_t st);
hipError_t batch_direct(const JobDesc* jobs, const BatchShape& bs, hipStream_t st);
hipError_t batch_correct(const JobDesc* jobs, const BatchShape& bs, int unused, hipStream_t st);
// from_A = 0: PS of I0 (t = 0); 1: PS of A.
hipError_t batch_ps(const JobDesc* jobs, const BatchShape& bs, int from_A, hipStream_t st);
// cold != 0: from zero with each job's cold cycle count, else warm from depth.
hipError_t batch_integrate(const JobDesc* jobs, const BatchShape& bs, int cold, hipStream_t st);
hipError_t batch_advance(JobDesc* jobs, int njobs, hipStream_t st);

// ---- probes ----
// out: blocks x 256 uint32.
hipError_t probe_valu(int blocks, int iters, int active, int kind, uint32_t* out, hipStream_t st);
hipError_t probe_philox(long long count, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                        hipStream_t st);
hipError_t probe_sample(long long count, const float* n, const float* u, float* d, hipStream_t st);
hipError_t probe_env(long long count, const float* d, int He, int We, int* rc, hipStream_t st);
hipError_t probe_traverse(const SurfaceArgs& sa, int flat, long long count, const int* ij,
                          const float* d, int* q, hipStream_t st);

}  // namespace kern
}  // namespace irtps
