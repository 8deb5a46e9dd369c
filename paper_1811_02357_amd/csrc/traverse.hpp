// traverse.hpp -- ray against the grid-line heightfield on gfx950.
//
// The surface is linear between neighbouring samples along every grid line.
// A ray leaves a sample; it is tested where it crosses each vertical line
// x = X and each horizontal line y = Y, in order of its parameter t (an x-line
// first on a tie).  A crossing hits when the ray is strictly below the surface
// there; the shading sample is the nearer end of that grid segment.  The ray
// escapes at the first crossing outside the domain, or when it is at or above
// the highest sample and not descending.
//
// Two walks give the same answer bit for bit.  The flat walk visits every
// crossing.  The pyramid walk skips, in one step, every crossing inside a
// pyramid cell when the ray's height over the cell's t-range (exact: fmaf is
// monotone in t) is at or above the cell's maximum; that maximum is taken over
// the cell grown by one sample, which covers the samples any crossing in the
// cell can read after binary32 rounding of its minor coordinate (off by far
// less than a sample).  Cells touching the domain border are never skipped, so
// the escape test is always taken at the same crossing as in the flat walk.
// Escape windows and horizon bounds end a pyramid walk early only when no
// crossing ahead can hit, which is the flat walk's result too; the near horizon
// bound alone lets a walk start past the crossings it proves to miss.
#pragma once

#include "device_math.hpp"

namespace irtps {
namespace trv {

constexpr int kMaxLevels = 16;
// Quadrant maxima are kept per 2^kQuadShift x 2^kQuadShift block of samples.
constexpr int kQuadShift = 3;
__host__ __device__ inline int quad_cells(int n) { return (n + (1 << kQuadShift) - 1) >> kQuadShift; }

// Escape windows: per block and quadrant of travel, the maxima over the
// samples a ray starting in the block can read within 16, 64 and 256 samples of
// horizontal travel (escape_scale(k)), and the quadrant maximum; each is raised
// by 2e-3 + 2e-6 |max| so that a test against it survives the rounding of the
// ray's heights.
constexpr int kEscapeScales = 3;
__host__ __device__ inline int escape_scale(int k) { return 16 << (2 * k); }
__host__ __device__ inline float escape_margin(float m) { return fmaf(2e-6f, fabsf(m), m + 2e-3f); }

// Horizon bounds, which let most rising rays leave at their first step.  From
// sample p, a crossing can read a sample r (offsets a, b >= 0 along the travel
// quadrant) only after at least tmin(a, b) of horizontal travel: an x-line
// crossing at column a reads rows within one of the ray's, so after
// sqrt(a^2 + (b-1)^2) at least, and a y-line crossing after sqrt((a-1)^2 + b^2).
// A ray of slope s (rise per unit of horizontal travel) stays at or above
// escape_margin(h_r) at every such crossing when s >= (escape_margin(h_r) - h_p)
// / tmin(a, b).  Three bounds on that slope, each conservative:
//   near: per sample and quadrant, the exact maximum over the samples read
//     within kHorizonReach of travel;
//   mid: per block and quadrant, over the blocks up to kMidBlocks blocks ahead,
//     with the block-to-block distance less 1.5 (>= kHorizonReach) and the
//     block's lowest sample for h_p;
//   far: the same over 64 x 64 super-blocks up to kFarSupers ahead (distance >=
//     kMidBlocks blocks) and the quadrant maximum at 2048 samples.
// The mid and far maxima are convex in h_p; each is stored as its chord over the
// block's height range, a + k h_p, raised to cover rounding.
constexpr int kHorizonReach = 24;
constexpr int kMidBlocks = 32;
constexpr int kSuperShift = 6;
constexpr int kFarSupers = 32;
constexpr float kFarQuadrantTravel = 2048.0f;
__host__ __device__ inline int super_cells(int n) { return (n + (1 << kSuperShift) - 1) >> kSuperShift; }

// The block tables that follow the pyramid levels, in floats from their start
// (which is 64-float aligned), for a QW x QH block grid with plane p4 =
// QW QH rounded up to a multiple of 4, and s4 = the super-block count rounded
// up to a multiple of 4:
//   escape windows  float4 [4 quadrants][QH][QW]      at 0
//   block maxima    [QH][QW]                          at 16 p4
//   row-window maxima [2 x-directions][3 scales][QH][QW] at 17 p4
//   quadrant maxima [4 quadrants][QH][QW]             at 25 p4
//   block minima    [QH][QW]                          at 29 p4
//   horizon bounds  float4 [4 quadrants][QH][QW]      at 30 p4: (a_mid, k_mid, a_far, k_far)
//   super-block maxima [SH][SW]                       at 46 p4
//   near horizons   float4 [Hh][W]                    at 46 p4 + s4: the four quadrants of a sample
__host__ __device__ inline long long block_plane4(int QW, int QH) { return ((long long)QW * QH + 3) / 4 * 4; }
__host__ __device__ inline long long super_plane4(int W, int Hh) {
    return ((long long)super_cells(W) * super_cells(Hh) + 3) / 4 * 4;
}
__host__ __device__ inline long long near_horizon_offset(int W, int Hh) {
    return 46 * block_plane4(quad_cells(W), quad_cells(Hh)) + super_plane4(W, Hh);
}
__host__ __device__ inline long long block_tables_floats(int W, int Hh) {
    return near_horizon_offset(W, Hh) + 4LL * W * Hh;
}

// Apron-max pyramid.  Level l has cells (cx, cy), cx < wc[l], cy < hc[l];
// cell (cx, cy) spans samples [cx 2^l, (cx+1) 2^l] x [cy 2^l, (cy+1) 2^l].
struct Pyramid {
    int levels;
    int wc[kMaxLevels];
    int hc[kMaxLevels];
    long long off[kMaxLevels];
};

// A surface as one lane sees it.  Level l of the pyramid has
// ceil((W-1)/2^l) x ceil((H-1)/2^l) cells stored from offset lvl[l].x with
// lvl[l].y cells per row; the table lives in LDS so that a per-lane level
// index does not spill.  Cells that come within two samples of the domain
// border hold +inf (never skipped).
struct Surface {
    const float* H;      // [Hh][W]
    const float* pyr;    // apron maxima, levels concatenated
    const float* quad;   // 4 quadrant maxima [q][QH][QW] over blocks, q = (dx < 0) + 2 (dy < 0)
    const float4* esc;   // escape windows [q][QH][QW]: maxima within escape_scale(0..2), quadrant max
    const float4* hzb;   // horizon bounds [q][QH][QW]: (a_mid, k_mid, a_far, k_far)
    const float* nearh;  // near horizons [Hh][W][q]
    const int2* lvl;     // LDS copy of (offset, cells per row) of every level
    int W, Hh;
    int QW, QH;          // blocks of the quadrant tables
    int top;             // index of the 1x1 level
    int Wm1, Hm1;        // W - 1, Hh - 1
    float fWm1, fHm1;    // the same as floats
    float hmax;          // highest sample
};

// Loads through a 32-bit byte offset from a wave-uniform base, so that the
// address is one scalar base plus one vector offset.  Every table a walk reads
// (samples, pyramid, escape windows, horizons) is below 2^32 bytes: W H <= 2^28
// (the largest, four near horizons per sample, ends 16 bytes short of it).
template <class T>
__device__ __forceinline__ T ld32(const T* base, unsigned idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(T));
}

// Per-ray state shared by both walks.  The cell search uses the origin nudged
// by kNudge along the travel direction (nx0, ny0); crossings use the exact
// origin (i0, j0).
struct Ray {
    float nx0, ny0, oz, dx, dy, dz;
    float slope;           // rise per unit of horizontal travel, rounded down (0 if not rising)
    float ainv_x, ainv_y;  // |1/dx|, |1/dy| (+inf for a zero component)
    int i0, j0, sx, sy;
    int qrow;              // first block row of the ray's quadrant in the escape windows
};

// Cells are chosen at the ray's position nudged this far along the travel
// direction, so that a ray sitting on a cell edge picks the cell ahead.  The
// one-sample apron of every cell covers the nudge.
constexpr float kNudge = 0.03125f;

// The ray's start, direction, quadrant and slope: all that the horizon test
// and the shading of an escape read.
__device__ __forceinline__ void ray_begin(Ray& r, const Surface& S, int i0, int j0, float dx, float dy, float dz) {
    r.i0 = i0;
    r.j0 = j0;
    r.oz = ld32(S.H, (unsigned)(j0 * S.W + i0));
    r.dx = dx;
    r.dy = dy;
    r.dz = dz;
    r.sx = signbit(dx) ? -1 : 1;
    r.sy = signbit(dy) ? -1 : 1;
    r.qrow = ((r.sx < 0 ? 1 : 0) + (r.sy < 0 ? 2 : 0)) * S.QH;
    // dz / |(dx, dy)| from the hardware reciprocal square root (within a few ulp),
    // shrunk by 1e-5 so that it never exceeds the exact slope
    const float hd2 = fmaf(dx, dx, dy * dy);
    r.slope = (dz > 0.0f && hd2 > 0.0f) ? dz * __builtin_amdgcn_rsqf(hd2) * 0.99999f : 0.0f;
}

// The rest, which only a walk reads: the nudged origin and the reciprocals.
__device__ __forceinline__ void ray_finish(Ray& r) {
    r.nx0 = (float)r.i0 + (float)r.sx * kNudge;
    r.ny0 = (float)r.j0 + (float)r.sy * kNudge;
    r.ainv_x = fabsf(1.0f / r.dx);
    r.ainv_y = fabsf(1.0f / r.dy);
}

__device__ __forceinline__ Ray make_ray(const Surface& S, int i0, int j0, float dx, float dy,
                                        float dz) {
    Ray r;
    ray_begin(r, S, i0, j0, dx, dy, dz);
    ray_finish(r);
    return r;
}

// t of the m-th crossing: (X - ox) / dx with X - ox = sx m exact, written as
// m |1/dx| (the sign flip is exact, so this is (sx m)(1/dx) bit for bit).
__device__ __forceinline__ float t_x(const Ray& r, int m) { return (float)m * r.ainv_x; }
__device__ __forceinline__ float t_y(const Ray& r, int m) { return (float)m * r.ainv_y; }

enum : int { kMiss = 0, kHit = 1, kGoOn = 2 };

// A rising ray at height z in a block escapes when, over each stretch of
// horizontal travel, its lowest height clears the highest sample it can read
// there: z clears the first window; after escape_scale(k) of travel it has
// risen at least slope escape_scale(k) and clears the next window; after the
// last scale, the quadrant maximum (win.w).  z grows with t exactly as the
// crossings compute it (fma, monotone); the windows carry the rounding margin.
__device__ __forceinline__ bool escapes(float z, float slope, const float4& win) {
    // all four tests, without short-circuit branches
    return ((int)(z >= win.x) & (int)(fmaf(slope, (float)escape_scale(0), z) >= win.y) &
            (int)(fmaf(slope, (float)escape_scale(1), z) >= win.z) &
            (int)(fmaf(slope, (float)escape_scale(2), z) >= win.w)) != 0;
}

// Smallest crossing index m >= 1 whose t = m ainv (the walk's own product) is
// >= t_lim, with that t.  The answer is within one of ceil(t_lim |d|): ainv and
// each product round to within 2^-24 relative, so with t_lim |d| (the travel
// along the axis, at most the domain's side, < 2^15) the exact threshold moves
// by less than 2^-8 of an index, and the rounded estimate by less than 2^-9;
// both ceilings therefore differ by at most one.  For ainv = inf (no travel
// along the axis) the result is m = 1, t = inf.
__device__ __forceinline__ int first_index_at_or_after(float ainv, float d_abs, float t_lim, float& t_m) {
    const float est = fmaxf(ceilf(t_lim * d_abs), 1.0f);
    const float lo = est - 1.0f, hi = est + 1.0f;
    const float t_lo = lo * ainv, t_est = est * ainv, t_hi = hi * ainv;
    const bool take_lo = lo >= 1.0f && t_lo >= t_lim;
    const bool take_est = t_est >= t_lim;
    t_m = take_lo ? t_lo : (take_est ? t_est : t_hi);
    return (int)(take_lo ? lo : (take_est ? est : hi));
}

// Finest pyramid level the walker tries to skip (cells of 4 x 4 sample gaps).
constexpr int kMinSkipLevel = 2;
// Resumable walk.  (mx, tX) and (my, tY) name the next crossing of each family;
// every crossing before min(tX, tY) has been evaluated or lies in a skipped
// cell.  level < 0 walks every crossing.
struct Walker {
    Ray r;
    float tX, tY;
    int mx, my, level;
};

// The crossing state of a walker whose ray has begun (ray_begin): the ray's
// remaining fields and the first crossing of each family.
__device__ __forceinline__ void walker_finish(Walker& w, bool flat) {
    ray_finish(w.r);
    w.mx = 1;
    w.my = 1;
    w.level = flat ? -1 : kMinSkipLevel;
    // a ray along z has no crossings: t = inf on both families ends the walk
    const bool vertical = w.r.dx == 0.0f && w.r.dy == 0.0f;
    w.tX = vertical ? __builtin_inff() : t_x(w.r, 1);
    w.tY = vertical ? __builtin_inff() : t_y(w.r, 1);
}

__device__ __forceinline__ void walker_init(Walker& w, const Surface& S, int i0, int j0, float dx,
                                            float dy, float dz, bool flat) {
    ray_begin(w.r, S, i0, j0, dx, dy, dz);
    walker_finish(w, flat);
}

// Quadrant index of a ray: 0..3 = (dx < 0) + 2 (dy < 0).
__device__ __forceinline__ unsigned quadrant(const Ray& r) { return (r.sx < 0 ? 1u : 0u) + (r.sy < 0 ? 2u : 0u); }

// True when the start sample's horizon bounds for the ray's quadrant (near
// bound hn, block bounds hb) prove that no crossing can hit: the walk's result
// is then kMiss and no step is needed.  A ray that descends is never let go.
__device__ __forceinline__ bool leaves_at_once(const Ray& r, float hn, const float4& hb) {
    // not descending: its height at travel T is at least oz + slope T
    const float s = r.slope;
    return ((int)(r.dz >= 0.0f) & (int)(s >= hn) & (int)(s >= fmaf(hb.y, r.oz, hb.x)) &
            (int)(s >= fmaf(hb.w, r.oz, hb.z))) != 0;
}

// The start sample's horizon bounds for a walker: 2 when all three prove that
// no crossing can hit (as leaves_at_once); 1 when only the near bound holds,
// which proves it for every crossing within kHorizonReach of horizontal travel
// (such a crossing reads only samples within that travel, and a rising ray of
// at least the bound's slope is at or above their escape margins there); 0
// otherwise.  Reads only what ray_begin sets; a flat walk never asks.
__device__ __forceinline__ int horizon_class(const Ray& r, const Surface& S) {
    const unsigned q = quadrant(r);
    const float hn = ld32(S.nearh, (unsigned)(r.j0 * S.W + r.i0) * 4u + q);
    const float4 hb = ld32(S.hzb, __umul24((unsigned)r.qrow + ((unsigned)r.j0 >> kQuadShift), (unsigned)S.QW) +
                                      ((unsigned)r.i0 >> kQuadShift));
    const float s = r.slope;
    const bool near = ((int)(r.dz >= 0.0f) & (int)(s >= hn)) != 0;
    const bool far = ((int)(s >= fmaf(hb.y, r.oz, hb.x)) & (int)(s >= fmaf(hb.w, r.oz, hb.z))) != 0;
    return near ? (far ? 2 : 1) : 0;
}

// A walker whose near bound holds (horizon_class 1) resumes both crossing
// families at their first crossing at or after the parameter of kHorizonReach
// of horizontal travel, rounded down (the hardware reciprocal square root is
// within a few ulp; the 0.999 keeps the limit below the exact one), so that no
// crossing beyond that travel is passed over.  The crossings passed over all
// miss, and one outside the domain is followed only by others outside it (the
// domain is convex and the walk's coordinates are monotone in t), so the
// result is the flat walk's.  Called straight after walker_finish (or
// walker_init), before the walker's first step.
__device__ __forceinline__ void walker_skip_near(Walker& w) {
    const Ray& r = w.r;
    const float hd2 = fmaf(r.dx, r.dx, r.dy * r.dy);
    if (!(hd2 > 0.0f)) return;  // a ray along z has no crossings
    const float t_lim = (float)kHorizonReach * __builtin_amdgcn_rsqf(hd2) * 0.999f;
    // the search returns the walk's own products m |1/d|, so a family that
    // moves no further keeps its first crossing bit for bit
    w.mx = first_index_at_or_after(r.ainv_x, fabsf(r.dx), t_lim, w.tX);
    w.my = first_index_at_or_after(r.ainv_y, fabsf(r.dy), t_lim, w.tY);
}

// The same, reading the bounds of the ray's start sample (never in a flat walk).
__device__ __forceinline__ bool leaves_at_once(const Walker& w, const Surface& S) {
    const Ray& r = w.r;
    if (w.level < 0) return false;
    const unsigned q = quadrant(r);
    const float hn = ld32(S.nearh, (unsigned)(r.j0 * S.W + r.i0) * 4u + q);
    const float4 hb = ld32(S.hzb, __umul24((unsigned)r.qrow + ((unsigned)r.j0 >> kQuadShift), (unsigned)S.QW) +
                                      ((unsigned)r.i0 >> kQuadShift));
    return leaves_at_once(r, hn, hb);
}

// One step: a pyramid cell test (skip it, climb, descend or give up to crossing
// evaluation), or the evaluation of the next crossing.  Returns kGoOn, kHit
// (qi, qj set) or kMiss.  kEscapeWindows adds the escape-window test to every
// cell test; walks whose rays were already offered the horizon test at their
// start (the tracer's) do better without it.
template <bool kEscapeWindows>
__device__ __forceinline__ int walker_step(Walker& w, const Surface& S, int& qi, int& qj) {
    const Ray& r = w.r;
    const bool xline = w.tX <= w.tY;  // the next crossing is on an x-line (first on a tie)
    // t_now = inf (no crossing left: a ray along z) ends the walk in this step:
    // z_now is +inf (caught just below), or -inf or NaN, and then the position
    // is not interior and the crossing's minor coordinate is not in the domain
    const float t_now = xline ? w.tX : w.tY;
    const float z_now = fmaf(t_now, r.dz, r.oz);
    const bool rising = r.dz >= 0.0f;
    // at or above every sample and not descending: no crossing ahead can hit
    if (z_now >= S.hmax && rising) return kMiss;
    // The walker's next state is computed as values and stored once at the
    // end: with one store per field, divergent lanes need no register copies
    // where the branches join (the step is the tracer's inner loop).
    int mx = w.mx, my = w.my, level = w.level;
    float tX = w.tX, tY = w.tY;
    bool cross = true;  // evaluate the crossing at t_now in this step
    if (level >= kMinSkipLevel) {
        const float px = fmaf(t_now, r.dx, r.nx0);
        const float py = fmaf(t_now, r.dy, r.ny0);
        if (px >= 2.0f && px <= (float)(S.W - 3) && py >= 2.0f && py <= (float)(S.Hh - 3)) {
            const int l = level;
            const unsigned ix = (unsigned)px, iy = (unsigned)py;  // px, py > 0: truncation is floor
            // Escape windows of the block holding the (nudged) position: every
            // sample a later crossing can read within escape_scale(k) of travel
            // lies in window k (one sample behind the block going +, the lerp's
            // second sample and the nudge included), and everything ahead in the
            // block-aligned quadrant.
            float4 win = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (kEscapeWindows)
                win = ld32(S.esc, __umul24((unsigned)r.qrow + (iy >> kQuadShift), (unsigned)S.QW) + (ix >> kQuadShift));
            const unsigned cx = ix >> l, cy = iy >> l;
            const int2 lv = S.lvl[l];
            const float cmax = ld32(S.pyr, (unsigned)lv.x + __umul24(cy, (unsigned)lv.y) + cx);  // +inf near the border
            // both loads are issued before either result is tested (one wait)
            if (kEscapeWindows) __asm__ volatile("" : : "v"(cmax), "v"(win.x), "v"(win.y), "v"(win.z), "v"(win.w));
            // exit of the cell along the ray (computed while the loads are in
            // flight): the crossing index of its far edge in x and in y, >= 1
            // because the nudged position lies beyond the origin's lines
            const int size = 1 << l;
            const int ex = (int)(cx << l) - r.i0, ey = (int)(cy << l) - r.j0;
            const int mxa = r.sx > 0 ? ex + size : -ex;
            const int mya = r.sy > 0 ? ey + size : -ey;
            const float txe = t_x(r, mxa), tye = t_y(r, mya);
            const bool x_exit = txe <= tye;
            const float t_exit = x_exit ? txe : tye;
            const float z_exit = fmaf(t_exit, r.dz, r.oz);
            if (kEscapeWindows && rising && escapes(z_now, r.slope, win)) return kMiss;
            // every crossing with t in [t_now, t_exit) lies in the grown cell and
            // the ray is at or above its maximum over that range (t_exit is finite:
            // a ray with no travel along either axis never gets here)
            const bool skip = ((int)(z_now >= cmax) & (int)(z_exit >= cmax) & (int)(t_exit > t_now)) != 0;
            if (skip) {
                // Resume at the first crossing of each family at or after t_exit:
                // the exit line itself for the family the ray leaves through (t is
                // strictly increasing in the index), a search for the other.
                float t_o;
                const int m_o = first_index_at_or_after(x_exit ? r.ainv_y : r.ainv_x,
                                                        fabsf(x_exit ? r.dy : r.dx), t_exit, t_o);
                mx = x_exit ? mxa : m_o;
                tX = x_exit ? t_exit : t_o;
                my = x_exit ? m_o : mya;
                tY = x_exit ? t_o : t_exit;
            }
            // a skip climbs a level; a failed test descends one, or, at the
            // finest skip level, falls through to the crossing.  A skipped cell
            // is finite, so it keeps two samples from every border: 2^(l+1) <=
            // W - 3 < 2^top, and the level climbed to is still below the 1x1
            // top level (whose cell is +inf), so no clamp is needed.
            level = skip ? l + 1 : (l > kMinSkipLevel ? l - 1 : l);
            cross = !skip && l <= kMinSkipLevel;
        }
    }
    int res = kGoOn;
    if (cross) {
        // Evaluate the nearer crossing at t = t_now and height z_now.  It hits
        // when the ray is strictly below the surface there; the shading sample
        // is the nearer end of that grid segment.
        const int m = xline ? mx : my;
        const int o_major = xline ? r.i0 : r.j0;
        const int major = __mul24(xline ? r.sx : r.sy, m) + o_major;  // sx, sy are +-1
        const int last_major = xline ? S.Wm1 : S.Hm1;
        const float last_minor = xline ? S.fHm1 : S.fWm1;
        const float minor = fmaf(t_now, xline ? r.dy : r.dx, (float)(xline ? r.j0 : r.i0));
        if ((unsigned)major > (unsigned)last_major || !(minor >= 0.0f && minor <= last_minor)) {
            res = kMiss;  // the ray has left the domain
        } else {
            const float fm = floorf(minor);
            const int m0 = (int)fm;
            const float f = minor - fm;
            const unsigned idx0 = xline ? __umul24((unsigned)m0, (unsigned)S.W) + (unsigned)major
                                        : __umul24((unsigned)major, (unsigned)S.W) + (unsigned)m0;
            // the segment's second sample (the first again when the crossing is on a
            // sample: then the lerp below returns h0 without reading past the border)
            const unsigned step1 = f != 0.0f ? (xline ? (unsigned)S.W : 1u) : 0u;
            const float h0 = ld32(S.H, idx0);
            const float h1 = ld32(S.H, idx0 + step1);
            // h0 + f (h1 - h0), clamped to the segment's range (the median of the three)
            const float h = __builtin_amdgcn_fmed3f(fmaf(f, h1 - h0, h0), h0, h1);
            if (z_now < h) {
                const int qm = f < 0.5f ? m0 : m0 + 1;
                qi = xline ? major : qm;
                qj = xline ? qm : major;
                res = kHit;
            } else {
                const int m1 = m + 1;
                const float t1 = (float)m1 * (xline ? r.ainv_x : r.ainv_y);
                mx = xline ? m1 : mx;
                tX = xline ? t1 : tX;
                my = xline ? my : m1;
                tY = xline ? tY : t1;
            }
        }
    }
    w.mx = mx;
    w.my = my;
    w.tX = tX;
    w.tY = tY;
    w.level = level;
    return res;
}

// Whole walk in one call (shadow rays, probes).
__device__ __forceinline__ bool walk(const Surface& S, bool flat, int i0, int j0, float dx, float dy,
                                     float dz, int& qi, int& qj) {
    Walker w;
    walker_init(w, S, i0, j0, dx, dy, dz, flat);
    if (leaves_at_once(w, S)) return false;
    for (;;) {
        const int res = walker_step<true>(w, S, qi, qj);
        if (res != kGoOn) return res == kHit;
    }
}

}  // namespace trv
}  // namespace irtps
