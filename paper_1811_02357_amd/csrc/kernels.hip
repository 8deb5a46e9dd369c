// kernels.hip -- HIP kernels of the IRT-PS hot path for gfx950 (MI355X).
//
// Every kernel is a plain per-sample or per-pixel map over HBM-resident planes;
// the only dense arithmetic is the 3xK photometric-stereo product, far too
// small for MFMA.  The tracer is the hot loop.  Each step exists as a
// per-element device function used by two kinds of kernel: single-job kernels
// (arguments by value) and multi-job kernels that walk a job table in device
// memory (grid.y = job, or a persistent tile queue for the tracer), so that a
// batch of reconstructions of different sizes runs as one launch per step.
#include "kernels.hpp"

#include <atomic>

#include "device_math.hpp"
#include "traverse.hpp"

namespace irtps {
namespace kern {

using trv::Surface;

// Blocks are dealt round-robin over the 8 XCDs; remap so that each XCD gets a
// contiguous run of tiles (neighbouring tiles share that XCD's L2).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int per = (nb + 7) / 8;
    const int xcd = b % 8, k = b / 8;
    return xcd * per + k;
}

// Every kernel that walks rays first copies the pyramid's level table (offset
// and cells per row) to LDS (constant indices only) and then builds its
// Surface view on that table.
__device__ __forceinline__ void load_level_table(const int* off, const int* wc, int2* s_lvl) {
#pragma unroll
    for (int l = 0; l < trv::kMaxLevels; ++l)
        if ((int)threadIdx.x == l) s_lvl[l] = make_int2(off[l], wc[l]);
    __syncthreads();
}

__device__ __forceinline__ Surface make_surface(const float* H, const float* pyr, int W, int Hh,
                                                int levels, int quad_off, const int2* s_lvl) {
    Surface S;
    S.H = H;
    S.pyr = pyr;
    S.lvl = s_lvl;
    S.W = W;
    S.Hh = Hh;
    S.QW = trv::quad_cells(W);
    S.QH = trv::quad_cells(Hh);
    const float* tab = pyr + quad_off;
    const long long p4 = trv::block_plane4(S.QW, S.QH);
    S.esc = reinterpret_cast<const float4*>(tab);
    S.quad = tab + 25 * p4;
    S.hzb = reinterpret_cast<const float4*>(tab + 30 * p4);
    S.nearh = tab + trv::near_horizon_offset(W, Hh);
    S.top = levels - 1;
    S.Wm1 = W - 1;
    S.Hm1 = Hh - 1;
    S.fWm1 = (float)(W - 1);
    S.fHm1 = (float)(Hh - 1);
    S.hmax = S.quad[0];  // quadrant (+x, +y) of block (0, 0): every sample
    return S;
}

__device__ __forceinline__ Surface make_surface(const SurfaceArgs& a, const int2* s_lvl) {
    return make_surface(a.H, a.pyr, a.W, a.Hh, a.levels, a.quad_off, s_lvl);
}

// ===========================================================================
// Per-element bodies.

// Eq.4: g_c = M A_c (sum over lights in order, fused), albedo = |g_c|,
// normal = sum_c g_c normalised.  M rows have stride kMaxLights.
template <int C>
__device__ __forceinline__ void ps_px(int p, int npx, int K, const float* __restrict__ M,
                                      const float* __restrict__ A, float* __restrict__ n,
                                      float* __restrict__ rho) {
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
        // unrolled so that several image loads are in flight (sums in k order)
#pragma unroll 16
        for (int k = 0; k < K; ++k) {
            const float a = A[((size_t)k * C + c) * npx + p];
            g0 = fmaf(M[k], a, g0);
            g1 = fmaf(M[kMaxLights + k], a, g1);
            g2 = fmaf(M[2 * kMaxLights + k], a, g2);
        }
        rho[(size_t)c * npx + p] = sqrtf(fmaf(g0, g0, fmaf(g1, g1, g2 * g2)));
        sx = sx + g0;
        sy = sy + g1;
        sz = sz + g2;
    }
    const float len = sqrtf(fmaf(sx, sx, fmaf(sy, sy, sz * sz)));
    float nx = 0.0f, ny = 0.0f, nz = 1.0f;
    if (len > 0.0f) {
        nx = sx / len;
        ny = sy / len;
        nz = sz / len;
    }
    n[3 * (size_t)p + 0] = nx;
    n[3 * (size_t)p + 1] = ny;
    n[3 * (size_t)p + 2] = nz;
}

// Eq.4 over the lights that reach pixel p: light k is kept when its direct
// irradiance S[p][k] = s_k max(0, n_t . l_k) V_k(H_t) is positive.  With at
// least three kept lights whose 3x3 normal matrix passes the conditioning test
// of the all-light matrix (det > 1e-7 (trace/3)^3), the pixel's own solve
// matrix (L_p^T L_p)^-1 L_p^T is built in binary64 from the kept rows in light
// order (adjugate over determinant) and rounded to binary32, one column per
// kept light as the sums reach it; dropped lights add nothing.  Otherwise the
// all-light M.  The sums per channel and component still run in light order.
template <int C>
__device__ __forceinline__ void ps_px_masked(int p, int npx, int K, const float* __restrict__ M,
                                             const float* __restrict__ l, const float* __restrict__ s,
                                             const float* __restrict__ A, const float* __restrict__ Srow,
                                             float* __restrict__ n, float* __restrict__ rho) {
    unsigned long long kept = 0ull;
    int nkept = 0;
    // normal matrix of the kept rows (symmetric: six sums; a product is the
    // same in either operand order)
    double a00 = 0.0, a01 = 0.0, a02 = 0.0, a11 = 0.0, a12 = 0.0, a22 = 0.0;
    for (int k = 0; k < K; ++k) {
        if (!(Srow[k] > 0.0f)) continue;
        kept |= 1ull << k;
        ++nkept;
        const double sk = (double)s[k];
        const double x = sk * (double)l[3 * k], y = sk * (double)l[3 * k + 1], z = sk * (double)l[3 * k + 2];
        a00 = a00 + x * x;
        a01 = a01 + x * y;
        a02 = a02 + x * z;
        a11 = a11 + y * y;
        a12 = a12 + y * z;
        a22 = a22 + z * z;
    }
    // adjugate (cofactor c_ab of entry (a, b)), determinant, inverse = c_ba / det
    const double c00 = a11 * a22 - a12 * a12;
    const double c01 = -(a01 * a22 - a12 * a02);
    const double c02 = a01 * a12 - a11 * a02;
    const double c10 = -(a01 * a22 - a02 * a12);
    const double c11 = a00 * a22 - a02 * a02;
    const double c12 = -(a00 * a12 - a01 * a02);
    const double c20 = a01 * a12 - a02 * a11;
    const double c21 = -(a00 * a12 - a02 * a01);
    const double c22 = a00 * a11 - a01 * a01;
    const double det = a00 * c00 + a01 * c01 + a02 * c02;
    const double tr3 = (a00 + a11 + a22) / 3.0;
    const bool own = nkept >= 3 && det > 1e-7 * tr3 * tr3 * tr3;
    double i00 = 0, i01 = 0, i02 = 0, i10 = 0, i11 = 0, i12 = 0, i20 = 0, i21 = 0, i22 = 0;
    if (own) {
        i00 = c00 / det; i01 = c10 / det; i02 = c20 / det;
        i10 = c01 / det; i11 = c11 / det; i12 = c21 / det;
        i20 = c02 / det; i21 = c12 / det; i22 = c22 / det;
    }
    float g[C][3];
#pragma unroll
    for (int c = 0; c < C; ++c) g[c][0] = g[c][1] = g[c][2] = 0.0f;
    for (int k = 0; k < K; ++k) {
        float m0, m1, m2;
        if (own) {
            if (!((kept >> k) & 1ull)) continue;
            const double sk = (double)s[k];
            const double x = sk * (double)l[3 * k], y = sk * (double)l[3 * k + 1], z = sk * (double)l[3 * k + 2];
            m0 = (float)(i00 * x + i01 * y + i02 * z);
            m1 = (float)(i10 * x + i11 * y + i12 * z);
            m2 = (float)(i20 * x + i21 * y + i22 * z);
        } else {
            m0 = M[k];
            m1 = M[kMaxLights + k];
            m2 = M[2 * kMaxLights + k];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float a = A[((size_t)k * C + c) * npx + p];
            g[c][0] = fmaf(m0, a, g[c][0]);
            g[c][1] = fmaf(m1, a, g[c][1]);
            g[c][2] = fmaf(m2, a, g[c][2]);
        }
    }
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        rho[(size_t)c * npx + p] = sqrtf(fmaf(g[c][0], g[c][0], fmaf(g[c][1], g[c][1], g[c][2] * g[c][2])));
        sx = sx + g[c][0];
        sy = sy + g[c][1];
        sz = sz + g[c][2];
    }
    const float len = sqrtf(fmaf(sx, sx, fmaf(sy, sy, sz * sz)));
    float nx = 0.0f, ny = 0.0f, nz = 1.0f;
    if (len > 0.0f) {
        nx = sx / len;
        ny = sy / len;
        nz = sz / len;
    }
    n[3 * (size_t)p + 0] = nx;
    n[3 * (size_t)p + 1] = ny;
    n[3 * (size_t)p + 2] = nz;
}

// ---------------------------------------------------------------------------
// The box: four walls on the borders of the sample grid (x = 0, x = W - 1,
// y = 0, y = H - 1) up to height z, open above.

// A ray from (x0, y0, z0) along l (l.z > 0) that reaches height z inside the
// walls' footprint leaves through the open top (one starting at or above z
// is out already).
__device__ __forceinline__ bool over_rim(float z, float xmax, float ymax, float x0, float y0, float z0, float lx,
                                         float ly, float lz) {
    if (z0 >= z) return true;
    const float t = (z - z0) / lz;
    const float x = fmaf(t, lx, x0), y = fmaf(t, ly, y0);
    return x >= 0.0f && x <= xmax && y >= 0.0f && y <= ymax;
}

// floor(f) clamped to [0, n - 1].
__device__ __forceinline__ int clamp_texel(float f, int n) {
    return !(f >= 0.0f) ? 0 : (f >= (float)(n - 1) ? n - 1 : (int)f);
}

// The texel ((wall th + row) tw + col) of the wall that a ray leaving the
// surface from sample (i0, j0) at height z0 meets below the rim: the first
// wall plane ahead (a corner counts as the x wall); -1 when the ray passes
// over the walls.
__device__ __forceinline__ int wall_texel(float z, int th, int tw, int W, int Hh, int i0, int j0, float z0,
                                          float dx, float dy, float dz) {
    const float xmax = (float)(W - 1), ymax = (float)(Hh - 1);
    const float x0 = (float)i0, y0 = (float)j0;
    const float inf = __builtin_inff();
    const float tx = dx > 0.0f ? (xmax - x0) / dx : (dx < 0.0f ? -x0 / dx : inf);
    const float ty = dy > 0.0f ? (ymax - y0) / dy : (dy < 0.0f ? -y0 / dy : inf);
    const bool xwall = tx <= ty;
    const float t = xwall ? tx : ty;
    if (t == inf) return -1;
    const float zw = fmaf(t, dz, z0);
    if (!(zw < z)) return -1;
    const int wall = xwall ? (dx > 0.0f ? 1 : 0) : (dy > 0.0f ? 3 : 2);
    const float u = xwall ? fmaf(t, dy, y0) : fmaf(t, dx, x0);
    const float len = xwall ? ymax : xmax;
    const int col = clamp_texel((u / len) * (float)tw, tw);
    const int row = clamp_texel((zw / z) * (float)th, th);
    return (wall * th + row) * tw + col;
}

// The walls' own direct light at texel centres: a wall faces into the box, so
// its cosine with light k is a coordinate of l_k; the light reaches the
// point when its ray leaves through the open top.  One lane per texel.
__global__ void __launch_bounds__(256) k_box_shade(int W, int Hh, BoxArgs b, LightSet L, float* __restrict__ Sw) {
    const int x = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (x >= 4 * b.th * b.tw) return;
    const int wall = x / (b.th * b.tw), row = (x / b.tw) % b.th, col = x % b.tw;
    const float xmax = (float)(W - 1), ymax = (float)(Hh - 1);
    const float len = wall < 2 ? ymax : xmax;
    const float u = (((float)col + 0.5f) / (float)b.tw) * len;
    const float zc = (((float)row + 0.5f) / (float)b.th) * b.z;
    const float px = wall == 0 ? 0.0f : (wall == 1 ? xmax : u);
    const float py = wall == 2 ? 0.0f : (wall == 3 ? ymax : u);
    for (int k = 0; k < L.K; ++k) {
        const float lx = L.l[k][0], ly = L.l[k][1], lz = L.l[k][2];
        const float c = wall == 0 ? lx : (wall == 1 ? -lx : (wall == 2 ? ly : -ly));
        Sw[(size_t)x * L.K + k] = (c > 0.0f && over_rim(b.z, xmax, ymax, px, py, zc, lx, ly, lz)) ? L.s[k] * c : 0.0f;
    }
}

// Walker steps per pass of the shadow-ray loop.
constexpr int kDirectSteps = 8;

// Eq.2 without albedo, with cast shadows: an any-hit walk from sample p towards
// each light k facing it.  The wave's (pixel, light) walks are dealt to lanes as
// they free up (item 64 k + j is light k of lane j's pixel, p_self of lane j, -1
// for none), so the wave waits for its mean lane's work plus one walk rather
// than for its slowest pixel's lights.  Each S value depends on its pixel and
// light only.
__device__ __forceinline__ void direct_wave(const Surface& S, int p_self, const float* __restrict__ n, int K,
                                            const float* __restrict__ L, const float* __restrict__ s, bool flat,
                                            float* __restrict__ S_out, float box_z = 0.0f) {
    const int lane = (int)(threadIdx.x & 63);
    const unsigned long long below = (1ull << lane) - 1ull;
    const int total = 64 * K;
    int cur = lane, next = 64, p = -1, k = 0;
    bool fresh = true, have = false, done = false;
    float c = 0.0f;
    trv::Walker w;
    for (;;) {
        for (;;) {
            const bool want = !have && !done && !fresh;
            const unsigned long long m = __ballot(want);
            if (want) {
                cur = next + __popcll(m & below);
                fresh = true;
            }
            next += __popcll(m);
            const int pj = __shfl(p_self, cur & 63);
            if (fresh) {
                fresh = false;
                if (cur >= total) {
                    done = true;
                } else if (pj >= 0) {
                    p = pj;
                    k = cur >> 6;
                    const int i = p % S.W, j = p / S.W;
                    const float nx = n[3 * (size_t)p], ny = n[3 * (size_t)p + 1], nz = n[3 * (size_t)p + 2];
                    const float lx = L[3 * k], ly = L[3 * k + 1], lz = L[3 * k + 2];
                    c = fmaf(nx, lx, fmaf(ny, ly, nz * lz));
                    // with walls, a light that the rim hides needs no walk
                    if (c > 0.0f && (box_z <= 0.0f || over_rim(box_z, (float)(S.W - 1), (float)(S.Hh - 1), (float)i,
                                                               (float)j, S.H[p], lx, ly, lz))) {
                        trv::walker_init(w, S, i, j, lx, ly, lz, flat);
                        have = true;
                    } else {
                        S_out[(size_t)p * K + k] = 0.0f;
                    }
                }
            }
            if (!__any(!have && !done)) break;
        }
        if (__all(done)) break;
        if (have) {
            int qi, qj;
            int res = trv::walker_step<true>(w, S, qi, qj);
#pragma unroll
            for (int u = 1; u < kDirectSteps; ++u)
                if (res == trv::kGoOn) res = trv::walker_step<true>(w, S, qi, qj);
            if (res != trv::kGoOn) {
                S_out[(size_t)p * K + k] = res == trv::kHit ? 0.0f : s[k] * c;
                have = false;
            }
        }
    }
}


// The pixel a direct-shading thread takes: block b of nb covers a tile of
// kDirectTileW x (256 / kDirectTileW) samples (XCD-aware order), or -1 past the
// image.  Shadow rays of nearby samples cross similar terrain, so compact tiles
// keep a wave's walks alike in length.
__device__ __forceinline__ int direct_pixel(int W, int Hh, int b, int nb) {
    const int th = tile_rows(kDirectTileW);
    const int tiles_x = (W + kDirectTileW - 1) / kDirectTileW;
    const int tile = xcd_tile(b, nb);
    if (tile >= tiles_x * ((Hh + th - 1) / th)) return -1;
    const int i = (tile % tiles_x) * kDirectTileW + ((int)threadIdx.x % kDirectTileW);
    const int j = (tile / tiles_x) * th + ((int)threadIdx.x / kDirectTileW);
    return (i < W && j < Hh) ? j * W + i : -1;
}

// Stage 5 for one pixel p: Grow[k C + c] and Srow[k] are that pixel's gathered
// and direct values (images and E are [k][c][p]).
template <int C>
__device__ __forceinline__ void correct_px(int p, int npx, int K, int rho_mode, int cumulative,
                                           const float* __restrict__ I0, const float* __restrict__ Aprev,
                                           const float* Grow, const float* Srow,
                                           const float* __restrict__ rho, float* __restrict__ E,
                                           float* __restrict__ Anext) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float rt;
        if (rho_mode == 0) {
            float num = 0.0f, den = 0.0f;
            // unrolled so that several image loads are in flight (the sums
            // still run over k in order)
#pragma unroll 16
            for (int k = 0; k < K; ++k) {
                const size_t x = ((size_t)k * C + c) * npx + p;
                const float v = Srow[k] + Grow[k * C + c];
                num = fmaf(I0[x], v, num);
                den = fmaf(v, v, den);
            }
            rt = den > 0.0f ? num / den : 0.0f;
        } else {
            rt = rho[(size_t)c * npx + p];
        }
#pragma unroll 16
        for (int k = 0; k < K; ++k) {
            const size_t x = ((size_t)k * C + c) * npx + p;
            const float e = rt * Grow[k * C + c];
            if (E) E[x] = e;
            Anext[x] = (cumulative ? Aprev[x] : I0[x]) - e;
        }
    }
}

// Rows of a pixel-major array (w floats per pixel, rows r0.. r0+n-1 contiguous
// from src) into LDS with a row stride of w + 1 (odd: lanes reading their own
// rows hit distinct banks).  Loads are coalesced across the block, and each
// lane issues kStageBatch of them before it stores any, so that a wave keeps
// that many in flight (LDS, not registers, limits these blocks per CU).
constexpr int kStageBatch = 32;
__device__ __forceinline__ void stage_rows(const float* __restrict__ src, int n, int w, float* dst) {
    const unsigned magic = 0xFFFFFFFFu / (unsigned)w + 1u;  // x / w = umulhi(x, magic) for x < 2^32 / w
    const int total = n * w, nt = (int)blockDim.x;
    for (int base = (int)threadIdx.x; base < total; base += kStageBatch * nt) {
        float v[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int x = base + u * nt;
            v[u] = x < total ? src[x] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int x = base + u * nt;
            if (x < total) {
                const int r = (int)__umulhi((unsigned)x, magic);
                dst[r * (w + 1) + (x - r * w)] = v[u];
            }
        }
    }
}

// Pixels per correction block: 64 when both staged rows fit 64 KB of LDS.
__host__ __device__ inline int correct_rows(int K, int C) { return 64 * (K * C + K + 2) <= 16384 ? 64 : 32; }

// Forward render: images = albedo (S + G).
template <int C>
__device__ __forceinline__ void compose_px(int p, int npx, int K, const float* __restrict__ rho,
                                           const float* __restrict__ S, const float* __restrict__ G,
                                           float* __restrict__ I) {
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const size_t x = ((size_t)k * C + c) * npx + p;
            I[x] = rho[(size_t)c * npx + p] * (S[(size_t)p * K + k] + G[((size_t)p * K + k) * C + c]);
        }
    }
}

// Apron-max pyramid, level 0: max over the 4 x 4 samples around cell (cx, cy);
// +inf for a cell that comes within two samples of the border (the walker never
// skips those, so the escape test is always taken where the flat walk takes it).
__device__ __forceinline__ void pyr0_cell(int c, int W, int Hh, int wc, const float* __restrict__ H,
                                          float* __restrict__ out) {
    const int cx = c % wc, cy = c / wc;
    if (cx < 2 || cx + 1 > W - 3 || cy < 2 || cy + 1 > Hh - 3) {
        out[c] = __builtin_inff();
        return;
    }
    float m = H[(size_t)(cy - 1) * W + cx - 1];
    for (int y = cy - 1; y <= cy + 2; ++y)
        for (int x = cx - 1; x <= cx + 2; ++x) {
            const float v = H[(size_t)y * W + x];
            m = v > m ? v : m;
        }
    out[c] = m;
}

// Level l+1 from level l: max of the four children; +inf where one is missing
// (the cell reaches past the border) or +inf (it touches the border margin).
__device__ __forceinline__ void pyr_reduce_cell(int c, const float* __restrict__ in, int wi, int hi,
                                                float* __restrict__ out, int wo) {
    const int cx = c % wo, cy = c / wo;
    float m = -__builtin_inff();
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            const int x = 2 * cx + dx, y = 2 * cy + dy;
            const float v = (x < wi && y < hi) ? in[(size_t)y * wi + x] : __builtin_inff();
            m = v > m ? v : m;
        }
    out[c] = m;
}

// The block tables (layout in traverse.hpp), from the block maxima of H.
struct BlockTables {
    float4* esc;
    float* bmax;
    float* rowmax;
    float* quad;
    float* bmin;
    float4* hzb;
    float* smax;
    float4* nearh;
    int QW, QH;
    int SW, SH;       // super-blocks
    long long plane;  // QW QH
};

__device__ __forceinline__ BlockTables block_tables(float* tab, int W, int Hh) {
    BlockTables t;
    t.QW = trv::quad_cells(W);
    t.QH = trv::quad_cells(Hh);
    t.plane = (long long)t.QW * t.QH;
    const long long p4 = trv::block_plane4(t.QW, t.QH);
    t.esc = reinterpret_cast<float4*>(tab);
    t.bmax = tab + 16 * p4;
    t.rowmax = tab + 17 * p4;
    t.quad = tab + 25 * p4;
    t.bmin = tab + 29 * p4;
    t.hzb = reinterpret_cast<float4*>(tab + 30 * p4);
    t.smax = tab + 46 * p4;
    t.nearh = reinterpret_cast<float4*>(tab + trv::near_horizon_offset(W, Hh));
    t.SW = trv::super_cells(W);
    t.SH = trv::super_cells(Hh);
    return t;
}

// Block maxima and minima of H over 8 x 8 sample blocks.
__device__ __forceinline__ void quad_block(int b, int W, int Hh, const float* __restrict__ H,
                                           const BlockTables& t) {
    const int bx = b % t.QW, by = b / t.QW;
    const int x0 = bx << trv::kQuadShift, y0 = by << trv::kQuadShift;
    const int x1 = min(x0 + (1 << trv::kQuadShift), W), y1 = min(y0 + (1 << trv::kQuadShift), Hh);
    float m = H[(size_t)y0 * W + x0], n = m;
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) {
            const float v = H[(size_t)y * W + x];
            m = v > m ? v : m;
            n = v < n ? v : n;
        }
    t.bmax[b] = m;
    t.bmin[b] = n;
}

// Super-block maxima: the largest block maximum of each 64 x 64 super-block.
__device__ __forceinline__ void super_block(int c, const BlockTables& t) {
    constexpr int kBlocks = 1 << (trv::kSuperShift - trv::kQuadShift);
    const int sx = c % t.SW, sy = c / t.SW;
    const int bx0 = sx * kBlocks, by0 = sy * kBlocks;
    const int bx1 = min(bx0 + kBlocks, t.QW), by1 = min(by0 + kBlocks, t.QH);
    float m = t.bmax[(size_t)by0 * t.QW + bx0];
    for (int y = by0; y < by1; ++y)
        for (int x = bx0; x < bx1; ++x) {
            const float v = t.bmax[(size_t)y * t.QW + x];
            m = v > m ? v : m;
        }
    t.smax[c] = m;
}

// A bound computed in binary32 raised above every rounding of its terms.
__device__ __forceinline__ float raise_bound(float m) { return isinf(m) ? m : m + fabsf(m) * 1e-5f + 1e-7f; }

// Square root at compile time (Newton's iteration in binary64; the tables
// built with it keep a relative slack far above its error).
constexpr double ce_sqrt(double x) {
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 64; ++i) r = 0.5 * (r + x / r);
    return r;
}

// 1 / d for the mid bound between a block and the block (ca, cb) blocks ahead:
// d = max(kHorizonReach, gap - 1.5), gap the least distance between their
// samples; rounded up to binary32.
struct MidInverse {
    float v[trv::kMidBlocks + 2][trv::kMidBlocks + 2];
};
constexpr MidInverse mid_inverse() {
    MidInverse t{};
    constexpr int kBS = 1 << trv::kQuadShift;
    for (int cb = 0; cb < trv::kMidBlocks + 2; ++cb)
        for (int ca = 0; ca < trv::kMidBlocks + 2; ++ca) {
            const double gx = ca * kBS - (kBS - 1) > 0 ? ca * kBS - (kBS - 1) : 0;
            const double gy = cb * kBS - (kBS - 1) > 0 ? cb * kBS - (kBS - 1) : 0;
            double d = ce_sqrt(gx * gx + gy * gy) * (1.0 - 1e-9) - 1.5;
            d = d > (double)trv::kHorizonReach ? d : (double)trv::kHorizonReach;
            t.v[cb][ca] = (float)(1.0 / d * (1.0 + 1e-7));
        }
    return t;
}
__constant__ MidInverse k_mid_inv = mid_inverse();

// Mid and far horizon bounds of block b for quadrant q (run after the block,
// super-block and quadrant maxima).  For each far region R with maximum M_R at
// least d_R of travel away, the slope needed from a sample of height h is
// (escape_margin(M_R) - h) / d_R; the maximum over the regions is convex in h,
// so its chord between the block's lowest and highest sample bounds it there.
__device__ __forceinline__ void horizon_block(int b, int q, const BlockTables& t) {
    const int bx = b % t.QW, by = b / t.QW;
    const int sx = (q & 1) ? -1 : 1, sy = (q & 2) ? -1 : 1;
    const float lo = t.bmin[b], hi = t.bmax[b];
    constexpr int kBS = 1 << trv::kQuadShift;
    float mid_lo = -__builtin_inff(), mid_hi = -__builtin_inff();
    for (int cb = 0; cb <= trv::kMidBlocks + 1; ++cb) {
        const int cy = by + sy * cb;
        if (cy < 0 || cy >= t.QH) break;
        for (int ca = 0; ca <= trv::kMidBlocks + 1; ++ca) {
            const int cx = bx + sx * ca;
            if (cx < 0 || cx >= t.QW) break;
            const float inv = k_mid_inv.v[cb][ca];
            const float M = trv::escape_margin(t.bmax[(size_t)cy * t.QW + cx]);
            mid_lo = fmaxf(mid_lo, (M - lo) * inv);
            mid_hi = fmaxf(mid_hi, (M - hi) * inv);
        }
    }
    // far: super-blocks ahead of the block (the one holding it included), then
    // everything else in the quadrant at kFarQuadrantTravel or more
    constexpr int kSS = 1 << trv::kSuperShift;
    const int X0 = bx * kBS, Y0 = by * kBS;
    const int hx = X0 >> trv::kSuperShift, hy = Y0 >> trv::kSuperShift;
    const float mid_floor = (float)(trv::kMidBlocks * kBS);
    const float Mq = trv::escape_margin(t.quad[q * t.plane + b]);
    float far_lo = (Mq - lo) / trv::kFarQuadrantTravel, far_hi = (Mq - hi) / trv::kFarQuadrantTravel;
    for (int cb = 0; cb <= trv::kFarSupers + 1; ++cb) {
        const int cy = hy + sy * cb;
        if (cy < 0 || cy >= t.SH) break;
        const int y0 = cy * kSS, y1 = y0 + kSS - 1;
        const float gy = (float)max(0, max(y0 - (Y0 + kBS - 1), Y0 - y1));
        for (int ca = 0; ca <= trv::kFarSupers + 1; ++ca) {
            const int cx = hx + sx * ca;
            if (cx < 0 || cx >= t.SW) break;
            const int x0 = cx * kSS, x1 = x0 + kSS - 1;
            const float gx = (float)max(0, max(x0 - (X0 + kBS - 1), X0 - x1));
            // hardware square root and reciprocal (within 1 ulp each), the
            // distance lowered and its inverse raised by far more than that
            float d = __builtin_amdgcn_sqrtf(fmaf(gx, gx, gy * gy)) * (1.0f - 1e-6f) - 1.5f;
            d = d > mid_floor ? d : mid_floor;
            const float inv = __builtin_amdgcn_rcpf(d) * (1.0f + 1e-6f);
            const float M = trv::escape_margin(t.smax[(size_t)cy * t.SW + cx]);
            far_lo = fmaxf(far_lo, (M - lo) * inv);
            far_hi = fmaxf(far_hi, (M - hi) * inv);
        }
    }
    // chords a + k h through (lo, f(lo)) and (hi, f(hi)), evaluated in binary64
    // and raised by more than the rounding of a, k and of fma(k, h, a)
    auto chord = [&](float f_lo, float f_hi, float& a_out, float& k_out) {
        const double flo = raise_bound(f_lo), fhi = raise_bound(f_hi);
        const double k = hi > lo ? (fhi - flo) / ((double)hi - (double)lo) : 0.0;
        const double a = flo - k * (double)lo;
        const double hm = fabs((double)lo) > fabs((double)hi) ? fabs((double)lo) : fabs((double)hi);
        const double slack = 0x1p-21 * (fabs(a) + fabs(k) * hm) + 1e-7;
        a_out = (float)(a + slack);
        k_out = (float)k;
    };
    float am, km, af, kf;
    chord(mid_lo, mid_hi, am, km);
    chord(far_lo, far_hi, af, kf);
    t.hzb[q * t.plane + b] = make_float4(am, km, af, kf);
}

// Near horizons of a 16 x 16 tile of samples, from an LDS copy of
// escape_margin(H) with an apron of kHorizonReach + 1 (-inf outside the domain).
constexpr int kNearApron = trv::kHorizonReach + 1;
constexpr int kNearSpan = kNearTile + 2 * kNearApron;
constexpr int kNearOff = kNearApron + 1;  // offsets 0 .. kNearApron along each axis

// 1 / tmin(a, b) with tmin lowered by 0.01 per minor offset and 1e-6 relative
// (the rounding of crossing positions), 0 where tmin exceeds kHorizonReach; and
// per row b the last a with a weight (tmin grows with a).  Computed at compile
// time in binary64 and rounded up to binary32.
struct NearWeights {
    float w[kNearOff][kNearOff];
    int last[kNearOff];
};
constexpr NearWeights near_weights() {
    NearWeights t{};
    for (int b = 0; b < kNearOff; ++b) {
        t.last[b] = -1;
        for (int a = 0; a < kNearOff; ++a) {
            const double am = a - 1.01 > 0.0 ? a - 1.01 : 0.0, bm = b - 1.01 > 0.0 ? b - 1.01 : 0.0;
            const double tx = a >= 1 ? ce_sqrt((double)a * a + bm * bm) : 1e300;
            const double ty = b >= 1 ? ce_sqrt(am * am + (double)b * b) : 1e300;
            const double tt = (tx < ty ? tx : ty) * (1.0 - 1e-6);
            t.w[b][a] = tt <= (double)trv::kHorizonReach ? (float)(1.0 / tt * (1.0 + 1e-7)) : 0.0f;
            if (t.w[b][a] > 0.0f) t.last[b] = a;
        }
    }
    return t;
}
__constant__ NearWeights k_near_w = near_weights();

__device__ __forceinline__ void near_tile(int W, int Hh, const float* __restrict__ H, int tile_x, int tile_y,
                                          float4* __restrict__ nearh, float* s_e) {
    const int X0 = tile_x * kNearTile - kNearApron, Y0 = tile_y * kNearTile - kNearApron;
    for (int k = threadIdx.x; k < kNearSpan * kNearSpan; k += blockDim.x) {
        const int x = X0 + k % kNearSpan, y = Y0 + k / kNearSpan;
        s_e[k] = (x >= 0 && x < W && y >= 0 && y < Hh) ? trv::escape_margin(H[(size_t)y * W + x]) : -__builtin_inff();
    }
    __syncthreads();
    const int tx = threadIdx.x % kNearTile, ty = threadIdx.x / kNearTile;
    const int x = tile_x * kNearTile + tx, y = tile_y * kNearTile + ty;
    if (x >= W || y >= Hh) return;
    const float hp = H[(size_t)y * W + x];
    // the four quadrants together (q = (dx < 0) + 2 (dy < 0)): one weight
    // serves four independent terms
    const float* c = s_e + (ty + kNearApron) * kNearSpan + (tx + kNearApron);
    float m0 = -__builtin_inff(), m1 = m0, m2 = m0, m3 = m0;
#pragma unroll 1
    for (int b = 0; b < kNearOff; ++b) {
        const float* up = c + b * kNearSpan;  // dy >= 0
        const float* dn = c - b * kNearSpan;  // dy < 0
        const int last = k_near_w.last[b];
#pragma unroll 2
        for (int a = b == 0 ? 1 : 0; a <= last; ++a) {  // (0, 0) is the sample itself
            const float w = k_near_w.w[b][a];
            m0 = fmaxf(m0, (up[a] - hp) * w);
            m1 = fmaxf(m1, (up[-a] - hp) * w);
            m2 = fmaxf(m2, (dn[a] - hp) * w);
            m3 = fmaxf(m3, (dn[-a] - hp) * w);
        }
    }
    const float m[4] = {raise_bound(m0), raise_bound(m1), raise_bound(m2), raise_bound(m3)};
    nearh[(size_t)y * W + x] = make_float4(m[0], m[1], m[2], m[3]);
}

// Quadrant maxima over blocks: quad[q][by][bx] = max of H over samples (x, y)
// with x >= 8 bx (sx > 0) or x <= 8 bx + 7 (sx < 0), and the same along y,
// q = (sx < 0) + 2 (sy < 0).  Rows fill planes 0 (suffix along x) and 1
// (prefix); columns fill planes 2 and 3 (prefix along y of planes 0 and 1) and
// finish 0 and 1 (suffix along y) in place.
__device__ __forceinline__ void quad_row(int j, const BlockTables& t) {
    const float* row = t.bmax + (size_t)j * t.QW;
    float* suf = t.quad + (size_t)j * t.QW;
    float* pre = t.quad + t.plane + (size_t)j * t.QW;
    float m = row[t.QW - 1];
    for (int x = t.QW - 1; x >= 0; --x) {
        const float v = row[x];
        m = v > m ? v : m;
        suf[x] = m;
    }
    m = row[0];
    for (int x = 0; x < t.QW; ++x) {
        const float v = row[x];
        m = v > m ? v : m;
        pre[x] = m;
    }
}

__device__ __forceinline__ void quad_col(int i, const BlockTables& t) {
    const int QW = t.QW, QH = t.QH;
    for (int h = 0; h < 2; ++h) {
        float* src = t.quad + h * t.plane;        // sx = +1 (h = 0) or -1 (h = 1), rows done
        float* pre = t.quad + (h + 2) * t.plane;  // sy = -1
        float m = src[i];
        for (int y = 0; y < QH; ++y) {
            const float v = src[(size_t)y * QW + i];
            m = v > m ? v : m;
            pre[(size_t)y * QW + i] = m;
        }
        m = src[(size_t)(QH - 1) * QW + i];
        for (int y = QH - 1; y >= 0; --y) {
            const float v = src[(size_t)y * QW + i];
            m = v > m ? v : m;
            src[(size_t)y * QW + i] = m;
        }
    }
}

// Block range of escape window k along one axis for travel direction s: a
// ray in block c can read samples from one before the block to scale + 9
// past its start going +, mirrored going -, i.e. blocks [c - 1, c + scale/8 + 1]
// or [c - scale/8 - 1, c + 1], clamped to the grid.
__device__ __forceinline__ void escape_range(int c, int k, bool forward, int n, int& lo, int& hi) {
    const int reach = (trv::escape_scale(k) >> trv::kQuadShift) + 1;
    lo = forward ? c - 1 : c - reach;
    hi = forward ? c + reach : c + 1;
    lo = lo < 0 ? 0 : lo;
    hi = hi > n - 1 ? n - 1 : hi;
}

// Row pass: rowmax[xdir][k][by][bx] = max of the block maxima of row by over
// the x-range of window k (xdir 0: +x, 1: -x).
__device__ __forceinline__ void escape_row(int b, const BlockTables& t) {
    const int bx = b % t.QW, by = b / t.QW;
    const float* row = t.bmax + (size_t)by * t.QW;
    for (int xd = 0; xd < 2; ++xd)
        for (int k = 0; k < trv::kEscapeScales; ++k) {
            int lo, hi;
            escape_range(bx, k, xd == 0, t.QW, lo, hi);
            float m = row[lo];
            for (int x = lo + 1; x <= hi; ++x) m = row[x] > m ? row[x] : m;
            t.rowmax[(xd * trv::kEscapeScales + k) * t.plane + b] = m;
        }
}

// Column pass: esc[q][by][bx] = (max of rowmax[xdir(q)][k] over the y-range of
// window k, k = 0..2; quadrant maximum), each with the escape margin.  Runs
// after the quadrant maxima.
__device__ __forceinline__ void escape_col(int b, const BlockTables& t) {
    const int bx = b % t.QW, by = b / t.QW;
    for (int q = 0; q < 4; ++q) {
        float m[trv::kEscapeScales + 1];
        for (int k = 0; k < trv::kEscapeScales; ++k) {
            int lo, hi;
            escape_range(by, k, (q & 2) == 0, t.QH, lo, hi);
            const float* col = t.rowmax + ((q & 1) * trv::kEscapeScales + k) * t.plane + bx;
            float v = col[(size_t)lo * t.QW];
            for (int y = lo + 1; y <= hi; ++y) {
                const float u = col[(size_t)y * t.QW];
                v = u > v ? u : v;
            }
            m[k] = trv::escape_margin(v);
        }
        m[3] = trv::escape_margin(t.quad[q * t.plane + b]);
        t.esc[q * t.plane + b] = make_float4(m[0], m[1], m[2], m[3]);
    }
}

// Integration: right-hand side of the normal equations at node v.
__device__ __forceinline__ void grad_at(const float* n, size_t v, float& p, float& q) {
    const float nz0 = n[3 * v + 2];
    const float nz = nz0 > 0.05f ? nz0 : 0.05f;
    p = -(n[3 * v + 0] / nz);
    q = -(n[3 * v + 1] / nz);
}

__device__ __forceinline__ void mg_rhs_node(int v, int W, int Hh, const float* __restrict__ n,
                                            float* __restrict__ b) {
    const int i = v % W, j = v / W;
    float p, q;
    grad_at(n, v, p, q);
    float acc = 0.0f;
    float pn, qn;
    if (i > 0) { grad_at(n, v - 1, pn, qn); acc = acc + (pn + p) * 0.5f; }
    if (i < W - 1) { grad_at(n, v + 1, pn, qn); acc = acc - (p + pn) * 0.5f; }
    if (j > 0) { grad_at(n, v - W, pn, qn); acc = acc + (qn + q) * 0.5f; }
    if (j < Hh - 1) { grad_at(n, v + W, pn, qn); acc = acc - (q + qn) * 0.5f; }
    b[v] = acc;
}

// Robust integration (Huber M-estimator by half-quadratic splitting): the
// right-hand side for edge targets g + shrink(residual) against the current
// level-0 surface X, shrink(r) being the part of r beyond +-delta.  An edge's
// target depends on its two ends only, so both of its nodes compute the same
// value.
__device__ __forceinline__ float huber_shrink(float r, float delta) {
    return r > delta ? r - delta : (r < -delta ? r + delta : 0.0f);
}
__device__ __forceinline__ float robust_target(const float* __restrict__ n, const float* __restrict__ X,
                                               size_t a, size_t b, bool xedge, float delta) {
    float pa, qa, pb, qb;
    grad_at(n, a, pa, qa);
    grad_at(n, b, pb, qb);
    const float g = xedge ? (pa + pb) * 0.5f : (qa + qb) * 0.5f;
    return g + huber_shrink((X[b] - X[a]) - g, delta);
}
__device__ __forceinline__ void mg_rhs_robust_node(int v, int W, int Hh, const float* __restrict__ n,
                                                   const float* __restrict__ X, float delta,
                                                   float* __restrict__ b) {
    const int i = v % W, j = v / W;
    float acc = 0.0f;
    if (i > 0) acc = acc + robust_target(n, X, v - 1, v, true, delta);
    if (i < W - 1) acc = acc - robust_target(n, X, v, v + 1, true, delta);
    if (j > 0) acc = acc + robust_target(n, X, v - W, v, false, delta);
    if (j < Hh - 1) acc = acc - robust_target(n, X, v, v + W, false, delta);
    b[v] = acc;
}

// Edge weights of level `shift`: horizontal edges of row J carry the number of
// finest rows in that aggregate, vertical edges of column I its column count.
__device__ __forceinline__ float w_row(int H0, int shift, int J) {
    const int s = 1 << shift, rows = H0 - J * s;
    return (float)(rows < s ? rows : s);
}
__device__ __forceinline__ float w_col(int W0, int shift, int I) {
    const int s = 1 << shift, cols = W0 - I * s;
    return (float)(cols < s ? cols : s);
}

// One red-black Gauss-Seidel update of node v (if it has the given colour).
__device__ __forceinline__ void mg_smooth_node(int v, int Wl, int Hl, int shift, int W0, int H0,
                                               float* __restrict__ X, const float* __restrict__ b,
                                               int colour) {
    const int I = v % Wl, J = v / Wl;
    if (((I + J) & 1) != colour) return;
    const float wx = w_row(H0, shift, J), wy = w_col(W0, shift, I);
    float num = b[v], den = 0.0f;
    if (I > 0) { num = fmaf(wx, X[v - 1], num); den = den + wx; }
    if (I < Wl - 1) { num = fmaf(wx, X[v + 1], num); den = den + wx; }
    if (J > 0) { num = fmaf(wy, X[v - Wl], num); den = den + wy; }
    if (J < Hl - 1) { num = fmaf(wy, X[v + Wl], num); den = den + wy; }
    if (den > 0.0f) X[v] = num / den;
}

__device__ __forceinline__ float mg_resid(int Wl, int Hl, int shift, int W0, int H0, const float* X,
                                          const float* b, int I, int J) {
    const size_t v = (size_t)J * Wl + I;
    const float wx = w_row(H0, shift, J), wy = w_col(W0, shift, I);
    const float xv = X[v];
    float lx = 0.0f;
    if (I > 0) lx = fmaf(wx, xv - X[v - 1], lx);
    if (I < Wl - 1) lx = fmaf(wx, xv - X[v + 1], lx);
    if (J > 0) lx = fmaf(wy, xv - X[v - Wl], lx);
    if (J < Hl - 1) lx = fmaf(wy, xv - X[v + Wl], lx);
    return b[v] - lx;
}

// Coarse right-hand side = sum of the four fine residuals; coarse guess = 0.
__device__ __forceinline__ void mg_restrict_node(int v, int Wf, int Hf, int shift, int W0, int H0,
                                                 const float* __restrict__ Xf, const float* __restrict__ bf,
                                                 int Wc, float* __restrict__ bc, float* __restrict__ Xc) {
    const int I = v % Wc, J = v / Wc;
    float acc = 0.0f;
    for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
            const int fi = 2 * I + di, fj = 2 * J + dj;
            if (fi < Wf && fj < Hf) acc = acc + mg_resid(Wf, Hf, shift, W0, H0, Xf, bf, fi, fj);
        }
    bc[v] = acc;
    Xc[v] = 0.0f;
}

__device__ __forceinline__ void mg_prolong_node(int v, int Wf, float* __restrict__ Xf, int Wc,
                                                const float* __restrict__ Xc) {
    const int I = v % Wf, J = v / Wf;
    Xf[v] = Xf[v] + 2.0f * Xc[(size_t)(J / 2) * Wc + I / 2];
}

// The V-cycle's small levels, from plan.tail to the coarsest, by one block:
// the same node updates in the same colour and level order as the per-level
// launches (nodes of one colour are independent), with a block barrier
// between passes.  The coarsest grid (at most 4 x 4) gets 16 red-black sweeps.
// The levels' X and b live in LDS for the duration (s_mg, mg_tail_floats(m)
// floats): X and b of level tail come in, X of level tail goes back.
__host__ __device__ inline long long mg_tail_floats(const MgPlan& m) { return m.keyoff - m.xoff[m.tail]; }
constexpr int kMgTailThreads = 1024;

// Passes over levels of at most 64 nodes run in the first wave alone: its lanes
// see each other's LDS writes in program order, so a compiler fence replaces the
// block barrier between passes.
constexpr int kMgWaveNodes = 64;
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void mg_tail(const MgPlan& m, int W0, int H0, float* ws, float* s_mg) {
    const int top = m.levels - 1;
    const long long base = m.xoff[m.tail];
    auto X = [&](int l) { return s_mg + (m.xoff[l] - base); };
    auto B = [&](int l) { return s_mg + (m.boff[l] - base); };
    const int n0 = m.W[m.tail] * m.H[m.tail];
    for (int v = threadIdx.x; v < n0; v += blockDim.x) {
        X(m.tail)[v] = ws[m.xoff[m.tail] + v];
        B(m.tail)[v] = ws[m.boff[m.tail] + v];
    }
    __syncthreads();
    // one pass of `body` over level l's nodes: the whole block, or wave 0 alone
    auto pass = [&](int n, bool wave, auto body) {
        if (wave) {
            for (int v = threadIdx.x; v < n; v += 64) body(v);
            wave_sync();
        } else {
            for (int v = threadIdx.x; v < n; v += blockDim.x) body(v);
            __syncthreads();
        }
    };
    auto smooth = [&](int l, int sweeps, bool wave) {
        const int n = m.W[l] * m.H[l];
        for (int sw = 0; sw < sweeps; ++sw)
            for (int colour = 0; colour < 2; ++colour)
                pass(n, wave, [&](int v) { mg_smooth_node(v, m.W[l], m.H[l], l, W0, H0, X(l), B(l), colour); });
    };
    auto restrict_to = [&](int l, bool wave) {  // level l -> l + 1
        pass(m.W[l + 1] * m.H[l + 1], wave, [&](int v) {
            mg_restrict_node(v, m.W[l], m.H[l], l, W0, H0, X(l), B(l), m.W[l + 1], B(l + 1), X(l + 1));
        });
    };
    auto prolong_from = [&](int l, bool wave) {  // level l + 1 -> l
        pass(m.W[l] * m.H[l], wave, [&](int v) { mg_prolong_node(v, m.W[l], X(l), m.W[l + 1], X(l + 1)); });
    };
    // levels from lw on have at most kMgWaveNodes nodes (the coarsest always does)
    int lw = top;
    while (lw > m.tail && m.W[lw - 1] * m.H[lw - 1] <= kMgWaveNodes) --lw;
    for (int l = m.tail; l < lw; ++l) {
        smooth(l, 2, false);
        restrict_to(l, false);
    }
    if (threadIdx.x < 64) {
        for (int l = lw; l < top; ++l) {
            smooth(l, 2, true);
            restrict_to(l, true);
        }
        smooth(top, 16, true);
        for (int l = top - 1; l >= lw; --l) {
            prolong_from(l, true);
            smooth(l, 2, true);
        }
    }
    __syncthreads();
    for (int l = lw - 1; l >= m.tail; --l) {
        prolong_from(l, false);
        smooth(l, 2, false);
    }
    for (int v = threadIdx.x; v < n0; v += blockDim.x) ws[m.xoff[m.tail] + v] = X(m.tail)[v];
}

// Order-preserving map of binary32 (no NaN) to uint32.
__device__ __forceinline__ unsigned order_key(float f) {
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float order_val(unsigned k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Minimum of X + 0 over the nodes v = start, start + stride, ... below n into
// *key: each thread strides, the block reduces (wave shuffles, then LDS) and
// issues one atomic.  The minimum does not depend on the order.
__device__ __forceinline__ void min_key_strided(const float* __restrict__ X, long long start, long long stride,
                                                int n, unsigned* key) {
    __shared__ unsigned s_min[4];  // one per wave of a 256-thread block
    unsigned k = 0xffffffffu;
    for (long long v = start; v < n; v += stride) {
        const unsigned o = order_key(X[v] + 0.0f);  // +0.0f: one zero
        k = o < k ? o : k;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned other = __shfl_xor(k, o);
        k = other < k ? other : k;
    }
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = k;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned m = s_min[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = s_min[w] < m ? s_min[w] : m;
        atomicMin(key, m);
    }
}

// ---------------------------------------------------------------------------
// Eq.5-7: per pixel, spp cosine-weighted paths of up to B segments, for one
// tile of 2^tile_shift x (256 >> tile_shift) pixels (one 256-thread block).
// One lane owns one pixel.  Its K x C hit sums live in that pixel's row of the
// pixel-major output G[p][k][c] (only this lane touches it); the C environment
// sums stay in registers.  Each lane runs its own sequence of segments: the
// wave alternates a traversal phase, in which every lane advances its own ray
// until at least ready_batch lanes (or all that still have work) have finished
// theirs, with a phase that shades the finished segments and starts the next
// ones.  A lane's segments are summed in (sample, bounce) order.
constexpr int kStepsPerVote = 4;
// Shading rounds in a row for segments the horizon bounds let go at once.
constexpr int kEscapeRounds = 3;

// One hit's share: g[k C + c] = fma(wgt[c], Sq[k], g[k C + c]) for every light
// and channel, in that order per element.  With vec4, four lights at a time
// through float4 loads and stores of S and G (same arithmetic).
template <int C>
__device__ __forceinline__ void accumulate_hit(float* __restrict__ g, const float* __restrict__ Sq,
                                               const float (&wgt)[C], int K, bool vec4) {
    if (vec4) {
        for (int m = 0; m < K; m += 4) {
            const float4 s4 = *reinterpret_cast<const float4*>(Sq + m);
            const float sv[4] = {s4.x, s4.y, s4.z, s4.w};
            float4* g4 = reinterpret_cast<float4*>(g + m * C);
            // the 4C elements of these four lights are C float4s of G: element
            // e = 4x + i is light e / C, channel e % C
#pragma unroll
            for (int x = 0; x < C; ++x) {
                const float4 t = g4[x];
                float tv[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) tv[i] = fmaf(wgt[(4 * x + i) % C], sv[(4 * x + i) / C], tv[i]);
                g4[x] = make_float4(tv[0], tv[1], tv[2], tv[3]);
            }
        }
    } else {
        for (int k = 0; k < K; ++k) {
            const float sq = Sq[k];
#pragma unroll
            for (int c = 0; c < C; ++c) g[k * C + c] = fmaf(wgt[c], sq, g[k * C + c]);
        }
    }
}

template <int C>
__device__ __forceinline__ void trace_tile(const TraceArgs& a, const Surface& S, int tile) {
    const int tw = 1 << a.tile_shift;
    const int tiles_x = (a.sa.W + tw - 1) >> a.tile_shift;
    const int i = (tile % tiles_x) * tw + ((int)threadIdx.x & (tw - 1));
    const int j = (tile / tiles_x) * (kTileThreads >> a.tile_shift) + ((int)threadIdx.x >> a.tile_shift);
    const bool live = i < a.sa.W && j < a.sa.Hh;
    const int npx = a.sa.W * a.sa.Hh;
    const int p = live ? j * a.sa.W + i : 0;
    const bool flat = (a.flags & kFlagFlat) != 0;
    const int K = a.K;
    const int KC = K * C;
    const int batch = a.ready_batch;
    float* __restrict__ gp = a.G + (size_t)p * KC;  // this pixel's sums
    // whole float4 rows of S (and of the walls' S) and G when K is a multiple of
    // 4 and the rows are 16-byte aligned
    const bool vec4 = (K & 3) == 0 && (reinterpret_cast<uintptr_t>(a.G) & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(a.S) & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(a.box_S) & 15) == 0;
    const bool box = a.box_z > 0.0f;

    if (live)
        for (int x = 0; x < KC; ++x) gp[x] = 0.0f;
    float eacc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) eacc[c] = 0.0f;
    // wave-wide event counts (uniform across the wave, so they live in SGPRs)
    unsigned long long n_seg = 0, n_hit = 0, n_esc = 0, n_cont = 0;

    int M = 0;
    if (a.flags & kFlagQuadrature) {
        M = 1;
        while (M * M < a.spp) ++M;
    }

    // lane state
    bool finished = !live || a.B < 1;
    bool ready = false;  // current segment has a result
    int s = 0, b = 1;    // current sample and segment
    int res = trv::kGoOn, qi = 0, qj = 0;
    float beta[C];
#pragma unroll
    for (int c = 0; c < C; ++c) beta[c] = 1.0f;
    int ci = i, cj = j;  // sample the current segment starts from
    trv::Walker w;
    w.mx = 1;  // no walk pending (a pending walk has crossing index 0)
    bool need_setup = !finished;
    int chain = 0;  // shading rounds since the last traversal phase

    for (;;) {
        n_seg += __popcll(__ballot(need_setup));
        if (need_setup) {
            float u1, u2;
            if (M > 0 && b == 1) {
                u1 = ((float)(s / M) + 0.5f) / (float)M;
                u2 = ((float)(s % M) + 0.5f) / (float)M;
            } else {
                const dm::U4 r = dm::philox((uint32_t)p, (uint32_t)s, (uint32_t)a.t * 256u + (uint32_t)b,
                                            (uint32_t)a.tag, a.key0, a.key1);
                u1 = dm::unit24(r.x);
                u2 = dm::unit24(r.y);
            }
            const float* nq = a.n + 3 * (cj * a.sa.W + ci);
            const dm::V3 d = dm::cosine_dir(nq[0], nq[1], nq[2], u1, u2);
            trv::ray_begin(w.r, S, ci, cj, d.x, d.y, d.z);
            // a segment the horizon bounds let go is ready at once (an escape);
            // the walker state of the others is completed when the next
            // traversal phase starts, so that the set-up passes of rounds that
            // only shade escapes leave it out
            const int hz = flat ? 0 : trv::horizon_class(w.r, S);
            ready = hz == 2;
            // a pending walk has crossing index 0 (a walker's are >= 1) and
            // keeps the horizon class in its level field until then
            w.mx = hz == 2 ? 1 : 0;
            w.level = hz;
            res = trv::kMiss;
            need_setup = false;
        }
        if (__all(finished)) break;
        // Segments let go at once are shaded (and replaced) straight away, for a
        // few rounds, so that their lanes do not sit out a traversal phase.
        if (chain < kEscapeRounds && __any(!finished && ready)) {
            ++chain;
        } else {
        chain = 0;
        if (w.mx == 0) {
            // walks that only the near horizon bound clears start past its reach
            const bool pass_near = w.level == 1;
            trv::walker_finish(w, flat);
            if (pass_near) trv::walker_skip_near(w);
        }
        // traversal phase
        for (;;) {
            // a few walker steps per pair of ballots: a lane that finishes early
            // waits out the remaining steps, but the wave votes less often
#pragma unroll
            for (int u = 0; u < kStepsPerVote; ++u) {
                if (!finished && !ready) {
                    res = trv::walker_step<false>(w, S, qi, qj);
                    ready = res != trv::kGoOn;
                }
            }
            const int n_act = __popcll(__ballot(!finished));
            const int n_rdy = __popcll(__ballot(!finished && ready));
            if (n_rdy >= (n_act < batch ? n_act : batch)) break;
        }
        }
        // shading phase
        {
            const bool shade = !finished && ready;
            n_esc += __popcll(__ballot(shade && res == trv::kMiss));
            n_hit += __popcll(__ballot(shade && res != trv::kMiss));
            n_cont += __popcll(__ballot(shade && res != trv::kMiss && b < a.B));
        }
        if (!finished && ready) {
            bool next_sample = true;
            // an escape that meets a wall is shaded like a surface hit, from
            // the wall texel's albedo and direct light, and ends the path
            const int wt = (box && res == trv::kMiss)
                               ? wall_texel(a.box_z, a.box_th, a.box_tw, a.sa.W, a.sa.Hh, ci, cj, w.r.oz, w.r.dx,
                                            w.r.dy, w.r.dz)
                               : -1;
            if (res == trv::kMiss && wt < 0) {
                int er, ec;
                dm::env_texel(w.r.dx, w.r.dy, w.r.dz, a.env_h, a.env_w, er, ec);
                const float* L = a.env + (er * a.env_w + ec) * C;
#pragma unroll
                for (int c = 0; c < C; ++c) eacc[c] = fmaf(beta[c], dm::kPi * L[c], eacc[c]);
            } else {
                const int q = qj * a.sa.W + qi;
                const bool on_wall = wt >= 0;
                float wgt[C];
#pragma unroll
                for (int c = 0; c < C; ++c)
                    wgt[c] = beta[c] * (on_wall ? a.box_albedo[(size_t)wt * C + c] : a.rho[c * npx + q]);
                accumulate_hit<C>(gp, on_wall ? a.box_S + (size_t)wt * K : a.S + (size_t)q * K, wgt, K, vec4);
                if (!on_wall && b < a.B) {
#pragma unroll
                    for (int c = 0; c < C; ++c) beta[c] = wgt[c];
                    ci = qi;
                    cj = qj;
                    ++b;
                    next_sample = false;
                }
            }
            if (next_sample) {
                ++s;
                b = 1;
#pragma unroll
                for (int c = 0; c < C; ++c) beta[c] = 1.0f;
                ci = i;
                cj = j;
                finished = s >= a.spp;
            }
            need_setup = !finished;
        }
    }
    if (live) {
        const float fspp = (float)a.spp;
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int c = 0; c < C; ++c) gp[k * C + c] = (gp[k * C + c] + eacc[c]) / fspp;
        }
    }
    if (a.counters && (threadIdx.x & 63) == 0) {
        // one atomic per wave and counter
        atomicAdd(&a.counters[0], n_seg);
        atomicAdd(&a.counters[1], n_hit);
        atomicAdd(&a.counters[2], n_esc);
        atomicAdd(&a.counters[3], n_cont);
    }
}

// A lane whose pixel is done idles until this many lanes of its wave are done
// (or no lane has work left); the wave then finishes them together and they
// take new pixels.
constexpr int kRefillBatch = 4;

// The single-job per-pixel tracer: the same per-pixel work as trace_tile (each
// pixel's samples and segments in order, the same sums), but lanes are not
// bound to one pixel.  A wave takes chunks of 64 pixels from the launch's queue
// (or a fixed stride of them) and hands their pixels to lanes as the lanes
// free up, so that a wave does not wait for its slowest pixel.
template <int C>
__device__ __forceinline__ void trace_pixels(const TraceArgs& a, const Surface& S) {
    const int W = a.sa.W, Hh = a.sa.Hh;
    const int npx = W * Hh;
    const int sh = a.tile_shift;  // chunk width 2^sh
    const int tw = 1 << sh;
    const int chunks_x = (W + tw - 1) >> sh;
    const int nchunks = chunks_for(W, Hh, tw);
    const bool flat = (a.flags & kFlagFlat) != 0;
    const int K = a.K;
    const int KC = K * C;
    const int batch = a.ready_batch;
    const bool vec4 = (K & 3) == 0 && (reinterpret_cast<uintptr_t>(a.G) & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(a.S) & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(a.box_S) & 15) == 0;
    const bool box = a.box_z > 0.0f;
    const int lane = (int)(threadIdx.x & 63);
    unsigned* queue = a.tile_cost ? a.tile_cost + nchunks : nullptr;
    const int nwaves = (int)(gridDim.x * (blockDim.x >> 6));
    // wave-uniform: the next chunk of the fixed stride, the current chunk and
    // its next pixel, and whether the chunks have run out
    int stride_next = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    int cur = 0, pos = kChunkPixels;
    bool drained = false;

    int M = 0;
    if (a.flags & kFlagQuadrature) {
        M = 1;
        while (M * M < a.spp) ++M;
    }
    // wave-wide event counts (uniform across the wave, so they live in SGPRs)
    unsigned long long n_seg = 0, n_hit = 0, n_esc = 0, n_cont = 0;

    // lane state: the pixel held (if any) and its progress
    bool has = false;      // a pixel is held
    bool finished = true;  // no segment left to trace (no pixel, or all samples done)
    int i = 0, j = 0;      // the pixel
    bool ready = false;
    int s = 0, b = 1;
    int res = trv::kGoOn, qi = 0, qj = 0;
    float beta[C], eacc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        beta[c] = 1.0f;
        eacc[c] = 0.0f;
    }
    int ci = 0, cj = 0;
    trv::Walker w;
    w.mx = 1;  // no walk pending (a pending walk has crossing index 0)
    bool need_setup = false;
    int chain = 0;

    for (;;) {
        // finish the lanes whose pixels are done, a few at a time
        {
            const int n_done = __popcll(__ballot(has && finished));
            const int n_busy = __popcll(__ballot(!finished));
            if (n_done > 0 && (n_done >= kRefillBatch || n_busy == 0)) {
                if (has && finished) {
                    if (a.esc_sums) {
                        // G keeps the hit sums; correct() forms the means
                        float* ep = a.esc_sums + (size_t)(j * W + i) * C;
#pragma unroll
                        for (int c = 0; c < C; ++c) ep[c] = eacc[c];
                    } else {
                        // G = (hit sums + escape sum) / spp
                        float* gp = a.G + (size_t)(j * W + i) * KC;
                        const float fspp = (float)a.spp;
                        for (int k = 0; k < K; ++k) {
#pragma unroll
                            for (int c = 0; c < C; ++c) gp[k * C + c] = (gp[k * C + c] + eacc[c]) / fspp;
                        }
                    }
                    // the pixel's time: its start was subtracted when it was taken
                    // (modulo 2^32, exact while a chunk's total stays below 2^32 ticks)
                    if (a.tile_cost)
                        atomicAdd(&a.tile_cost[(j >> (6 - sh)) * chunks_x + (i >> sh)], (unsigned)wall_clock64());
                    has = false;
                }
            }
        }
        // lanes without a pixel take the next ones of the wave's chunk, and the
        // wave takes a new chunk when that one runs out
        while (!drained) {
            const unsigned long long want = __ballot(!has);
            if (want == 0ull) break;
            const int n = __popcll(want);
            const int rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(want >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((unsigned)want, 0u));
            const int avail = kChunkPixels - pos;
            int next = -1;
            if (n > avail) {
                int k;
                if (queue) {
                    const int leader = __ffsll((long long)__ballot(true)) - 1;
                    unsigned v = 0u;
                    if (lane == leader) v = atomicAdd(queue, 1u);
                    k = (int)__shfl(v, leader);
                } else {
                    k = stride_next;
                    stride_next += nwaves;
                }
                if (k >= nchunks) drained = true;
                else next = a.order ? a.order[k] : k;
            }
            int c_take = -1, loc = 0;
            if (!has) {
                if (rank < avail) {
                    c_take = cur;
                    loc = pos + rank;
                } else if (next >= 0) {
                    c_take = next;
                    loc = rank - avail;
                }
            }
            const int ii = c_take >= 0 ? (c_take % chunks_x) * tw + (loc & (tw - 1)) : 0;
            const int jj = c_take >= 0 ? (c_take / chunks_x) * (kChunkPixels >> sh) + (loc >> sh) : 0;
            const bool take = c_take >= 0 && ii < W && jj < Hh;  // else the lane asks again (a ragged chunk)
            // each pixel taken starts its chunk's clock now: the wave subtracts
            // the start times at once, per chunk
            if (a.tile_cost) {
                const unsigned now = (unsigned)wall_clock64();
                const unsigned n_cur = (unsigned)__popcll(__ballot(take && c_take == cur));
                const unsigned n_next = (unsigned)__popcll(__ballot(take && c_take != cur));
                if (lane == __ffsll((long long)__ballot(true)) - 1) {
                    if (n_cur) atomicSub(&a.tile_cost[cur], now * n_cur);
                    if (n_next) atomicSub(&a.tile_cost[next], now * n_next);
                }
            }
            if (next >= 0) {
                cur = next;
                pos = n - avail;
            } else {
                pos += n < avail ? n : avail;
            }
            if (take) {
                has = true;
                i = ii;
                j = jj;
                float* gp = a.G + (size_t)(jj * W + ii) * KC;
                for (int x = 0; x < KC; ++x) gp[x] = 0.0f;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    beta[c] = 1.0f;
                    eacc[c] = 0.0f;
                }
                s = 0;
                b = 1;
                ci = i;
                cj = j;
                finished = a.B < 1;
                need_setup = !finished;
            }
        }
        if (!__any(has)) break;        // the chunks have run out and every pixel is finished
        if (__all(finished)) continue;  // every held pixel is done: finish them
        n_seg += __popcll(__ballot(need_setup));
        if (need_setup) {
            float u1, u2;
            if (M > 0 && b == 1) {
                u1 = ((float)(s / M) + 0.5f) / (float)M;
                u2 = ((float)(s % M) + 0.5f) / (float)M;
            } else {
                // The key enters each setup as an opaque scalar, so that the
                // round keys are derived here with scalar adds instead of being
                // held through the whole loop (spilled to vector lanes and read
                // back one by one).
                uint32_t k0 = a.key0, k1 = a.key1;
                __asm__ volatile("" : "+s"(k0), "+s"(k1));
                const dm::U4 r = dm::philox((uint32_t)(j * W + i), (uint32_t)s, (uint32_t)a.t * 256u + (uint32_t)b,
                                            (uint32_t)a.tag, k0, k1);
                u1 = dm::unit24(r.x);
                u2 = dm::unit24(r.y);
            }
            const float* nq = a.n + 3 * (cj * W + ci);
            const dm::V3 d = dm::cosine_dir(nq[0], nq[1], nq[2], u1, u2);
            trv::ray_begin(w.r, S, ci, cj, d.x, d.y, d.z);
            // a segment the horizon bounds let go is ready at once (an escape);
            // the walker state of the others is completed when the next
            // traversal phase starts, so that the set-up passes of rounds that
            // only shade escapes leave it out
            const int hz = flat ? 0 : trv::horizon_class(w.r, S);
            ready = hz == 2;
            // a pending walk has crossing index 0 (a walker's are >= 1) and
            // keeps the horizon class in its level field until then
            w.mx = hz == 2 ? 1 : 0;
            w.level = hz;
            res = trv::kMiss;
            need_setup = false;
        }
        // Segments let go at once are shaded (and replaced) straight away, for a
        // few rounds, so that their lanes do not sit out a traversal phase.
        if (chain < kEscapeRounds && __any(!finished && ready)) {
            ++chain;
        } else {
            chain = 0;
            if (w.mx == 0) {
                // walks that only the near horizon bound clears start past its reach
                const bool pass_near = w.level == 1;
                trv::walker_finish(w, flat);
                if (pass_near) trv::walker_skip_near(w);
            }
            // traversal phase: a few walker steps per pair of ballots
            for (;;) {
#pragma unroll
                for (int u = 0; u < kStepsPerVote; ++u) {
                    if (!finished && !ready) {
                        res = trv::walker_step<false>(w, S, qi, qj);
                        ready = res != trv::kGoOn;
                    }
                }
                const int n_act = __popcll(__ballot(!finished));
                const int n_rdy = __popcll(__ballot(!finished && ready));
                if (n_rdy >= (n_act < batch ? n_act : batch)) break;
            }
        }
        // shading phase
        {
            const bool shade = !finished && ready;
            n_esc += __popcll(__ballot(shade && res == trv::kMiss));
            n_hit += __popcll(__ballot(shade && res != trv::kMiss));
            n_cont += __popcll(__ballot(shade && res != trv::kMiss && b < a.B));
        }
        if (!finished && ready) {
            bool next_sample = true;
            // an escape that meets a wall is shaded like a surface hit, from
            // the wall texel's albedo and direct light, and ends the path
            const int wt = (box && res == trv::kMiss)
                               ? wall_texel(a.box_z, a.box_th, a.box_tw, W, Hh, ci, cj, w.r.oz, w.r.dx, w.r.dy,
                                            w.r.dz)
                               : -1;
            if (res == trv::kMiss && wt < 0) {
                int er, ec;
                dm::env_texel(w.r.dx, w.r.dy, w.r.dz, a.env_h, a.env_w, er, ec);
                const float* L = a.env + (er * a.env_w + ec) * C;
#pragma unroll
                for (int c = 0; c < C; ++c) eacc[c] = fmaf(beta[c], dm::kPi * L[c], eacc[c]);
            } else {
                const int q = qj * W + qi;
                const bool on_wall = wt >= 0;
                float wgt[C];
#pragma unroll
                for (int c = 0; c < C; ++c)
                    wgt[c] = beta[c] * (on_wall ? a.box_albedo[(size_t)wt * C + c] : a.rho[c * npx + q]);
                accumulate_hit<C>(a.G + (size_t)(j * W + i) * KC, on_wall ? a.box_S + (size_t)wt * K : a.S + (size_t)q * K,
                                  wgt, K, vec4);
                if (!on_wall && b < a.B) {
#pragma unroll
                    for (int c = 0; c < C; ++c) beta[c] = wgt[c];
                    ci = qi;
                    cj = qj;
                    ++b;
                    next_sample = false;
                }
            }
            if (next_sample) {
                ++s;
                b = 1;
#pragma unroll
                for (int c = 0; c < C; ++c) beta[c] = 1.0f;
                ci = i;
                cj = j;
                finished = s >= a.spp;
            }
            need_setup = !finished;
        }
    }
    if (a.counters && lane == 0) {
        // one atomic per wave and counter
        atomicAdd(&a.counters[0], n_seg);
        atomicAdd(&a.counters[1], n_hit);
        atomicAdd(&a.counters[2], n_esc);
        atomicAdd(&a.counters[3], n_cont);
    }
}

// ===========================================================================
// Single-job kernels.

template <int C>
__global__ void __launch_bounds__(256) k_ps_solve(int npx, int K, PsMatrix M, const float* __restrict__ A,
                                                  float* __restrict__ n, float* __restrict__ rho) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npx) return;
    ps_px<C>(p, npx, K, &M.m[0][0], A, n, rho);
}


template <int C>
__global__ void __launch_bounds__(256) k_ps_solve_masked(int npx, int K, PsMatrix M, LightSet L,
                                                         const float* __restrict__ A, const float* __restrict__ S,
                                                         float* __restrict__ n, float* __restrict__ rho) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npx) return;
    ps_px_masked<C>(p, npx, K, &M.m[0][0], &L.l[0][0], L.s, A, S + (size_t)p * K, n, rho);
}

__global__ void __launch_bounds__(256) k_direct(SurfaceArgs sa, const float* __restrict__ n, LightSet L,
                                                int flat, float* __restrict__ S_out, float box_z) {
    __shared__ int2 s_lvl[trv::kMaxLevels];
    load_level_table(sa.off, sa.wc, s_lvl);
    const int p = direct_pixel(sa.W, sa.Hh, blockIdx.x, gridDim.x);
    const Surface S = make_surface(sa, s_lvl);
    direct_wave(S, p, n, L.K, &L.l[0][0], L.s, flat != 0, S_out, box_z);
}

// The tracers are issue- and latency-bound: the lane-bound ones ask for seven
// waves per SIMD (at most 72 VGPRs; eight force spills to scratch, six measured
// slower).  The single-job tracer, whose lanes take new pixels, holds more
// state across its loop and does best with six (80 VGPRs and more scalar
// registers, so fewer values parked in vector lanes; five and seven measured
// slower).
#define IRTPS_TRACER_OCCUPANCY __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 7)))
#define IRTPS_REFILL_OCCUPANCY __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 6)))

// Per-path mode, first pass: lane (s, p) traces sample s of pixel p (Eq.5-7, the
// same segment arithmetic as trace_tile) and records every segment: code q for
// a hit at sample q with weights beta albedo(q), or -(texel + 1) for an escape
// with weights beta.  Records are planes [1 + C][B][spp][npx].
template <int C>
__global__ void IRTPS_TRACER_OCCUPANCY k_trace_paths(TraceArgs a) {
    __shared__ int2 s_lvl[trv::kMaxLevels];
    load_level_table(a.sa.off, a.sa.wc, s_lvl);
    const int W = a.sa.W, npx = W * a.sa.Hh;
    const int idx = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const bool live = idx < npx * a.spp;
    const int s = live ? idx / npx : 0;
    const int p = live ? idx - s * npx : 0;
    const Surface S = make_surface(a.sa, s_lvl);
    unsigned cnt[4] = {0u, 0u, 0u, 0u};  // segments, hits, escapes, continuations
    if (live) {
        const bool flat = (a.flags & kFlagFlat) != 0;
        int M = 0;
        if (a.flags & kFlagQuadrature) {
            M = 1;
            while (M * M < a.spp) ++M;
        }
        const size_t plane = (size_t)npx * a.spp * a.B;
        int ci = p % W, cj = p / W;
        float beta[C];
#pragma unroll
        for (int c = 0; c < C; ++c) beta[c] = 1.0f;
        for (int b = 1; b <= a.B; ++b) {
            ++cnt[0];
            float u1, u2;
            if (M > 0 && b == 1) {
                u1 = ((float)(s / M) + 0.5f) / (float)M;
                u2 = ((float)(s % M) + 0.5f) / (float)M;
            } else {
                const dm::U4 r = dm::philox((uint32_t)p, (uint32_t)s, (uint32_t)a.t * 256u + (uint32_t)b,
                                            (uint32_t)a.tag, a.key0, a.key1);
                u1 = dm::unit24(r.x);
                u2 = dm::unit24(r.y);
            }
            const float* nq = a.n + 3 * (cj * W + ci);
            const dm::V3 d = dm::cosine_dir(nq[0], nq[1], nq[2], u1, u2);
            trv::Walker w;
            trv::walker_init(w, S, ci, cj, d.x, d.y, d.z, flat);
            int res = trv::kMiss, qi = 0, qj = 0;
            if (!trv::leaves_at_once(w, S)) {
                do {
                    res = trv::walker_step<false>(w, S, qi, qj);
                } while (res == trv::kGoOn);
            }
            const size_t r = ((size_t)(b - 1) * a.spp + s) * npx + p;
            if (res == trv::kMiss) {
                ++cnt[2];
                const int wt = a.box_z > 0.0f ? wall_texel(a.box_z, a.box_th, a.box_tw, W, a.sa.Hh, ci, cj, w.r.oz,
                                                           w.r.dx, w.r.dy, w.r.dz)
                                              : -1;
                if (wt >= 0) {  // a wall: code npx + texel, weight beta times its albedo
                    a.records[r] = __int_as_float(npx + wt);
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        a.records[(1 + c) * plane + r] = beta[c] * a.box_albedo[(size_t)wt * C + c];
                    break;
                }
                int er, ec;
                dm::env_texel(w.r.dx, w.r.dy, w.r.dz, a.env_h, a.env_w, er, ec);
                a.records[r] = __int_as_float(-(er * a.env_w + ec) - 1);
#pragma unroll
                for (int c = 0; c < C; ++c) a.records[(1 + c) * plane + r] = beta[c];
                break;
            }
            ++cnt[1];
            const int q = qj * W + qi;
            float wgt[C];
#pragma unroll
            for (int c = 0; c < C; ++c) wgt[c] = beta[c] * a.rho[c * npx + q];
            a.records[r] = __int_as_float(q);
#pragma unroll
            for (int c = 0; c < C; ++c) a.records[(1 + c) * plane + r] = wgt[c];
            if (b >= a.B) break;
            ++cnt[3];
#pragma unroll
            for (int c = 0; c < C; ++c) beta[c] = wgt[c];
            ci = qi;
            cj = qj;
        }
    }
    if (a.counters) {
        // one atomic per wave and counter
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            unsigned x = cnt[i];
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
            if ((threadIdx.x & 63) == 0 && x) atomicAdd(&a.counters[i], (unsigned long long)x);
        }
    }
}

// Per-path mode, second pass: pixel p's records in (sample, segment) order,
// summed exactly as trace_tile sums them, then the means.
template <int C>
__global__ void __launch_bounds__(256) k_gather_paths(TraceArgs a) {
    const int npx = a.sa.W * a.sa.Hh;
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= npx) return;
    const int K = a.K, KC = K * C;
    float* __restrict__ gp = a.G + (size_t)p * KC;
    const bool vec4 = (K & 3) == 0 && (reinterpret_cast<uintptr_t>(a.G) & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(a.S) & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(a.box_S) & 15) == 0;
    for (int x = 0; x < KC; ++x) gp[x] = 0.0f;
    float eacc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) eacc[c] = 0.0f;
    const size_t plane = (size_t)npx * a.spp * a.B;
    for (int s = 0; s < a.spp; ++s)
        for (int b = 1; b <= a.B; ++b) {
            const size_t r = ((size_t)(b - 1) * a.spp + s) * npx + p;
            const int code = __float_as_int(a.records[r]);
            float w[C];
#pragma unroll
            for (int c = 0; c < C; ++c) w[c] = a.records[(1 + c) * plane + r];
            if (code < 0) {
                const float* L = a.env + (size_t)(-code - 1) * C;
#pragma unroll
                for (int c = 0; c < C; ++c) eacc[c] = fmaf(w[c], dm::kPi * L[c], eacc[c]);
                break;
            }
            if (code >= npx) {  // a wall texel ends the path
                accumulate_hit<C>(gp, a.box_S + (size_t)(code - npx) * K, w, K, vec4);
                break;
            }
            accumulate_hit<C>(gp, a.S + (size_t)code * K, w, K, vec4);
        }
    const float fspp = (float)a.spp;
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int c = 0; c < C; ++c) gp[k * C + c] = (gp[k * C + c] + eacc[c]) / fspp;
    }
}

// ---------------------------------------------------------------------------
// The r-ray variant: one lane per pixel follows sample 0's path (the gather's
// counters for s = 0) through at most r segments.  Only a path whose r-th ray
// escapes gives its pixel a value: the albedo products of its r - 1 hits times
// pi times the environment texel that ray reaches.
template <int C>
__global__ void __launch_bounds__(256) k_trace_exact_r(SurfaceArgs sa, const float* __restrict__ n,
                                                       const float* __restrict__ rho,
                                                       const float* __restrict__ env, int He, int We, int r,
                                                       int t, int tag, uint32_t key0, uint32_t key1, int flat,
                                                       float* __restrict__ E, float* __restrict__ w0,
                                                       unsigned char* __restrict__ valid) {
    __shared__ int2 s_lvl[trv::kMaxLevels];
    load_level_table(sa.off, sa.wc, s_lvl);
    const int W = sa.W, npx = W * sa.Hh;
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= npx) return;
    const Surface S = make_surface(sa, s_lvl);
    float beta[C], out[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        beta[c] = 1.0f;
        out[c] = 0.0f;
    }
    bool ok = false;
    int ci = p % W, cj = p / W;
    for (int b = 1; b <= r; ++b) {
        const dm::U4 u = dm::philox((uint32_t)p, 0u, (uint32_t)t * 256u + (uint32_t)b, (uint32_t)tag, key0, key1);
        const float* nq = n + 3 * (cj * W + ci);
        const dm::V3 d = dm::cosine_dir(nq[0], nq[1], nq[2], dm::unit24(u.x), dm::unit24(u.y));
        trv::Walker w;
        trv::walker_init(w, S, ci, cj, d.x, d.y, d.z, flat != 0);
        int res = trv::kMiss, qi = 0, qj = 0;
        if (!trv::leaves_at_once(w, S)) {
            do {
                res = trv::walker_step<false>(w, S, qi, qj);
            } while (res == trv::kGoOn);
        }
        if (res == trv::kMiss) {
            if (b == r) {
                int er, ec;
                dm::env_texel(w.r.dx, w.r.dy, w.r.dz, He, We, er, ec);
                const float* L = env + ((size_t)er * We + ec) * C;
#pragma unroll
                for (int c = 0; c < C; ++c) out[c] = beta[c] * (dm::kPi * L[c]);
                ok = true;
            }
            break;
        }
        if (b == r) break;  // the r-th ray met the surface
        const int q = qj * W + qi;
#pragma unroll
        for (int c = 0; c < C; ++c) beta[c] = beta[c] * rho[(size_t)c * npx + q];
        ci = qi;
        cj = qj;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) E[(size_t)p * C + c] = out[c];
    if (w0) w0[p] = ok ? 1.0f : 0.0f;
    if (valid) valid[p] = ok ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_fill_weights(long long npx, const unsigned char* __restrict__ valid,
                                                      float* __restrict__ w0) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npx) w0[p] = valid[p] ? 1.0f : 0.0f;
}

// Pull one level: coarse cell u averages its children (fine cells 2I + di,
// 2J + dj, taken in the order dj, then di) that carry weight, weighted by it.
template <int C>
__global__ void __launch_bounds__(256) k_fill_pull(const float* __restrict__ wf, const float* __restrict__ vf,
                                                   int fw, int fh, float* __restrict__ wc,
                                                   float* __restrict__ vc, int cw, int ch) {
    const int u = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (u >= cw * ch) return;
    const int I = u % cw, J = u / cw;
    float den = 0.0f, num[C];
#pragma unroll
    for (int c = 0; c < C; ++c) num[c] = 0.0f;
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
        for (int di = 0; di < 2; ++di) {
            const int fi = 2 * I + di, fj = 2 * J + dj;
            if (fi >= fw || fj >= fh) continue;
            const size_t f = (size_t)fj * fw + fi;
            const float wgt = wf[f];
            if (!(wgt > 0.0f)) continue;
#pragma unroll
            for (int c = 0; c < C; ++c) num[c] = fmaf(wgt, vf[f * C + c], num[c]);
            den = den + wgt;
        }
    wc[u] = den;
#pragma unroll
    for (int c = 0; c < C; ++c) vc[(size_t)u * C + c] = den > 0.0f ? num[c] / den : 0.0f;
}

// Push one level, in place: a fine cell of weight 0 takes its parent's value
// (vc null: no parent, the value is 0).
template <int C>
__global__ void __launch_bounds__(256) k_fill_push(const float* __restrict__ wf, float* __restrict__ vf, int fw,
                                                   int fh, const float* __restrict__ vc, int cw) {
    const int f = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (f >= fw * fh || wf[f] > 0.0f) return;
    const int i = f % fw, j = f / fw;
    const size_t u = (size_t)(j / 2) * cw + i / 2;
#pragma unroll
    for (int c = 0; c < C; ++c) vf[(size_t)f * C + c] = vc ? vc[u * C + c] : 0.0f;
}

// Level 0's push into G [p][k][c]: one lane per element of G, so the stores
// are contiguous across the wave.
template <int C>
__global__ void __launch_bounds__(256) k_fill_push0_broadcast(const float* __restrict__ w0,
                                                              const float* __restrict__ v0, int W, int Hh,
                                                              const float* __restrict__ v1, int cw, int K,
                                                              float* __restrict__ G) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long KC = (long long)K * C;
    if (x >= KC * W * Hh) return;
    const int p = (int)(x / KC);
    const int c = (int)(x % KC) % C;
    float v;
    if (w0[p] > 0.0f) {
        v = v0[(size_t)p * C + c];
    } else {
        const int i = p % W, j = p / W;
        v = v1 ? v1[((size_t)(j / 2) * cw + i / 2) * C + c] : 0.0f;
    }
    G[x] = v;
}

// Persistent: the grid is at most what the GPU holds at once, and each wave
// works until the chunks run out (see trace_pixels).
template <int C>
__global__ void IRTPS_REFILL_OCCUPANCY k_trace(TraceArgs a) {
    __shared__ int2 s_lvl[trv::kMaxLevels];
    load_level_table(a.sa.off, a.sa.wc, s_lvl);
    const Surface S = make_surface(a.sa, s_lvl);
    trace_pixels<C>(a, S);
}

// Tiles (the single-job tracer's chunks) by descending cost: a counting sort
// over kOrderBuckets cost classes in
// one block (classes of 2^s ticks, s the least shift that fits the largest
// cost).  Slots within a class go by LDS atomics, so ties fall in any order;
// the trace does not depend on the order.
constexpr int kOrderBuckets = 4096;
constexpr int kOrderThreads = 1024;
__global__ void __launch_bounds__(kOrderThreads) k_order_tiles(const unsigned* __restrict__ cost, int tiles,
                                                                int* __restrict__ order) {
    __shared__ unsigned s_cnt[kOrderBuckets];
    __shared__ unsigned s_part[kOrderThreads];
    const int tid = (int)threadIdx.x;
    unsigned mx = 0;
    for (int t = tid; t < tiles; t += kOrderThreads) mx = cost[t] > mx ? cost[t] : mx;
    s_part[tid] = mx;
    for (int b = tid; b < kOrderBuckets; b += kOrderThreads) s_cnt[b] = 0u;
    __syncthreads();
    for (int h = kOrderThreads / 2; h > 0; h >>= 1) {
        if (tid < h && s_part[tid + h] > s_part[tid]) s_part[tid] = s_part[tid + h];
        __syncthreads();
    }
    mx = s_part[0];
    int sh = 0;
    while ((mx >> sh) >= (unsigned)kOrderBuckets) ++sh;
    __syncthreads();  // every thread has read s_part[0]
    // class k = kOrderBuckets - 1 - (cost >> sh): the heaviest tiles come first
    for (int t = tid; t < tiles; t += kOrderThreads) atomicAdd(&s_cnt[kOrderBuckets - 1 - (cost[t] >> sh)], 1u);
    __syncthreads();
    // exclusive scan of the counts: each thread sums its 4 classes, the block
    // scans the partial sums, then each thread writes its classes' starts
    constexpr int per = kOrderBuckets / kOrderThreads;
    unsigned loc = 0;
#pragma unroll
    for (int i = 0; i < per; ++i) loc += s_cnt[tid * per + i];
    s_part[tid] = loc;
    __syncthreads();
    for (int h = 1; h < kOrderThreads; h <<= 1) {
        const unsigned v = tid >= h ? s_part[tid - h] : 0u;
        __syncthreads();
        s_part[tid] += v;
        __syncthreads();
    }
    unsigned start = s_part[tid] - loc;
#pragma unroll
    for (int i = 0; i < per; ++i) {
        const unsigned c = s_cnt[tid * per + i];
        s_cnt[tid * per + i] = start;
        start += c;
    }
    __syncthreads();
    for (int t = tid; t < tiles; t += kOrderThreads) {
        const unsigned slot = atomicAdd(&s_cnt[kOrderBuckets - 1 - (cost[t] >> sh)], 1u);
        order[slot] = t;
    }
}

template <int C>
__global__ void __launch_bounds__(64) k_correct(int npx, int K, int rho_mode, int cumulative,
                                                const float* __restrict__ I0, const float* __restrict__ Aprev,
                                                const float* __restrict__ G, const float* __restrict__ S,
                                                const float* __restrict__ rho, float* __restrict__ E,
                                                float* __restrict__ Anext, const float* __restrict__ esc,
                                                int spp) {
    extern __shared__ float sm[];
    const int KC = K * C, rows = correct_rows(K, C);
    const int p0 = blockIdx.x * rows;
    const int n = npx - p0 < rows ? npx - p0 : rows;
    float* sG = sm;
    float* sS = sm + rows * (KC + 1);
    stage_rows(G + (size_t)p0 * KC, n, KC, sG);
    stage_rows(S + (size_t)p0 * K, n, K, sS);
    __syncthreads();
    const int t = threadIdx.x;
    if (esc && t < n) {
        // the means from the tracer's hit and escape sums, as its finish forms them
        float* row = sG + t * (KC + 1);
        const float fspp = (float)spp;
        float e[C];
#pragma unroll
        for (int c = 0; c < C; ++c) e[c] = esc[(size_t)(p0 + t) * C + c];
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int c = 0; c < C; ++c) row[k * C + c] = (row[k * C + c] + e[c]) / fspp;
        }
    }
    if (t < n)
        correct_px<C>(p0 + t, npx, K, rho_mode, cumulative, I0, Aprev, sG + t * (KC + 1), sS + t * (K + 1), rho, E,
                      Anext);
}

template <int C>
__global__ void __launch_bounds__(256) k_compose(int npx, int K, const float* __restrict__ rho,
                                                 const float* __restrict__ S, const float* __restrict__ G,
                                                 float* __restrict__ I) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npx) return;
    compose_px<C>(p, npx, K, rho, S, G, I);
}

__global__ void __launch_bounds__(256) k_pyr_level0(int W, int Hh, const float* __restrict__ H,
                                                    float* __restrict__ out, int wc, int hc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= wc * hc) return;
    pyr0_cell(c, W, Hh, wc, H, out);
}

__global__ void __launch_bounds__(256) k_pyr_reduce(const float* __restrict__ in, int wi, int hi,
                                                    float* __restrict__ out, int wo, int ho) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= wo * ho) return;
    pyr_reduce_cell(c, in, wi, hi, out, wo);
}

__global__ void __launch_bounds__(256) k_quad_blocks(int W, int Hh, const float* __restrict__ H,
                                                    float* __restrict__ tab) {
    const BlockTables t = block_tables(tab, W, Hh);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < t.plane) quad_block(b, W, Hh, H, t);
}

__global__ void __launch_bounds__(256) k_super_blocks(int W, int Hh, float* __restrict__ tab) {
    const BlockTables t = block_tables(tab, W, Hh);
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < t.SW * t.SH) super_block(c, t);
}

__global__ void __launch_bounds__(256) k_horizon_blocks(int W, int Hh, float* __restrict__ tab) {
    const BlockTables t = block_tables(tab, W, Hh);
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < 4 * t.plane) horizon_block((int)(v >> 2), (int)(v & 3), t);
}

__global__ void __launch_bounds__(256) k_horizon_near(int W, int Hh, const float* __restrict__ H,
                                                      float* __restrict__ tab) {
    __shared__ float s_e[kNearSpan * kNearSpan];
    const BlockTables t = block_tables(tab, W, Hh);
    near_tile(W, Hh, H, blockIdx.x, blockIdx.y, t.nearh, s_e);
}

__global__ void __launch_bounds__(64) k_quad_rows(int W, int Hh, float* __restrict__ tab) {
    const BlockTables t = block_tables(tab, W, Hh);
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < t.QH) quad_row(j, t);
}

__global__ void __launch_bounds__(64) k_quad_cols(int W, int Hh, float* __restrict__ tab) {
    const BlockTables t = block_tables(tab, W, Hh);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < t.QW) quad_col(i, t);
}

__global__ void __launch_bounds__(256) k_escape_rows(int W, int Hh, float* __restrict__ tab) {
    const BlockTables t = block_tables(tab, W, Hh);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < t.plane) escape_row(b, t);
}

__global__ void __launch_bounds__(256) k_escape_cols(int W, int Hh, float* __restrict__ tab) {
    const BlockTables t = block_tables(tab, W, Hh);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < t.plane) escape_col(b, t);
}

__global__ void __launch_bounds__(256) k_mg_rhs(int W, int Hh, const float* __restrict__ n,
                                                float* __restrict__ b) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < W * Hh) mg_rhs_node(v, W, Hh, n, b);
}
__global__ void __launch_bounds__(256) k_mg_rhs_robust(int W, int Hh, const float* __restrict__ n,
                                                       const float* __restrict__ X, float delta,
                                                       float* __restrict__ b) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < W * Hh) mg_rhs_robust_node(v, W, Hh, n, X, delta, b);
}

__global__ void __launch_bounds__(256) k_mg_smooth(int Wl, int Hl, int shift, int W0, int H0,
                                                   float* __restrict__ X, const float* __restrict__ b,
                                                   int colour) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < Wl * Hl) mg_smooth_node(v, Wl, Hl, shift, W0, H0, X, b, colour);
}

__global__ void __launch_bounds__(256) k_mg_restrict(int Wf, int Hf, int shift, int W0, int H0,
                                                     const float* __restrict__ Xf,
                                                     const float* __restrict__ bf, int Wc, int Hc,
                                                     float* __restrict__ bc, float* __restrict__ Xc) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < Wc * Hc) mg_restrict_node(v, Wf, Hf, shift, W0, H0, Xf, bf, Wc, bc, Xc);
}

__global__ void __launch_bounds__(256) k_mg_prolong(int Wf, int Hf, float* __restrict__ Xf, int Wc,
                                                    const float* __restrict__ Xc) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < Wf * Hf) mg_prolong_node(v, Wf, Xf, Wc, Xc);
}

__global__ void __launch_bounds__(kMgTailThreads) k_mg_tail(MgPlan m, int W0, int H0, float* ws) {
    extern __shared__ float s_mg[];
    mg_tail(m, W0, H0, ws, s_mg);
}

__global__ void k_fill_u32(unsigned* p, unsigned v, int n) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) p[x] = v;
}

__global__ void k_fill_f32(float* p, float v, long long n) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) p[x] = v;
}

__global__ void k_copy_f32(float* __restrict__ dst, const float* __restrict__ src, long long n) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) dst[x] = src[x];
}

__global__ void __launch_bounds__(256) k_min_key(const float* __restrict__ X, int n, unsigned* key) {
    min_key_strided(X, (long long)blockIdx.x * blockDim.x + threadIdx.x, (long long)gridDim.x * blockDim.x, n, key);
}

// Largest of d >= 0 over a 256-thread block, one atomic per block into *key
// (float bits of non-negative values order as unsigned integers).
__device__ __forceinline__ void block_max_into(float d, unsigned* key) {
    __shared__ unsigned s_max[4];
    unsigned k = __float_as_uint(d);
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned other = __shfl_xor(k, o);
        k = other > k ? other : k;
    }
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = k;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned m = s_max[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = s_max[w] > m ? s_max[w] : m;
        atomicMax(key, m);
    }
}

// H = X - min(X); with change_key, also the largest |H_new - H_old| where out
// holds H_old on entry (D_H of the paper's stop rule).
__global__ void __launch_bounds__(256) k_anchor(const float* __restrict__ X, int n, const unsigned* key,
                                                float* __restrict__ out, unsigned* change_key) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    float d = 0.0f;
    if (v < n) {
        const float h = X[v] - order_val(*key);
        if (change_key) d = fabsf(h - out[v]);
        out[v] = h;
    }
    if (change_key) block_max_into(d, change_key);
}

// ===========================================================================
// Multi-job kernels: blockIdx.y selects the job; blocks past a job's extent
// return at once.

// A job takes part in the iteration steps while t < T; the t = 0 steps (PS of
// I0, cold integration) run for every active job.
__device__ __forceinline__ bool iterating(const JobDesc& J) { return J.active && J.t < J.T; }

// The job that owns block b of a flattened grid: the last job whose first
// block (start(J)) is <= b (starts are non-decreasing in table order).
template <class Start>
__device__ __forceinline__ int job_of_block(const JobDesc* __restrict__ jobs, int njobs, int b, Start start) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start(jobs[mid]) <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ bool participates(const JobDesc& J, int init) {
    return init ? J.active != 0 : iterating(J);
}

__device__ __forceinline__ TraceArgs job_trace_args(const JobDesc& J, int tag) {
    TraceArgs a{};  // every field not set below is zero or null (no walls)
    a.sa.H = J.depth;
    a.sa.pyr = J.pyr;
    a.sa.W = J.W;
    a.sa.Hh = J.Hh;
    a.sa.levels = J.pyr_levels;
    a.sa.quad_off = J.quad_off;
#pragma unroll
    for (int l = 0; l < trv::kMaxLevels; ++l) {
        a.sa.off[l] = J.pyr_off[l];
        a.sa.wc[l] = J.pyr_wc[l];
    }
    a.n = J.n;
    a.rho = J.rho;
    a.S = J.S;
    a.env = J.env;
    a.G = J.G;
    a.counters = J.counters;
    a.order = nullptr;
    a.tile_cost = nullptr;
    a.records = nullptr;
    a.env_h = J.env_h;
    a.env_w = J.env_w;
    a.C = J.C;
    a.K = J.K;
    a.spp = J.spp;
    a.B = J.B;
    a.t = J.t;
    a.tag = tag;
    a.flags = J.flags & (kFlagQuadrature | kFlagFlat);
    a.ready_batch = J.ready_batch;
    a.tile_shift = J.tile_shift;
    a.key0 = J.key0;
    a.key1 = J.key1;
    return a;
}

// Persistent tracer: each block takes (job, tile) pairs from a queue.
template <int C>
__global__ void IRTPS_TRACER_OCCUPANCY k_trace_multi(const JobDesc* __restrict__ jobs,
                                                     const int2* __restrict__ tiles, int ntiles,
                                                     unsigned* queue, int tag) {
    __shared__ int2 s_lvl[trv::kMaxLevels];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();  // every thread has read s_item before it is replaced
        if (item >= ntiles) return;
        const int2 jt = tiles[item];
        const JobDesc& J = jobs[jt.x];
        if (!iterating(J)) continue;  // uniform per block; s_item was read above
        const TraceArgs a = job_trace_args(J, tag);
        load_level_table(a.sa.off, a.sa.wc, s_lvl);
        const Surface S = make_surface(a.sa, s_lvl);
        trace_tile<C>(a, S, jt.y);
        __syncthreads();  // s_lvl is reloaded for the next item
    }
}

__global__ void __launch_bounds__(256) k_begin_multi(JobDesc* jobs) {
    JobDesc& J = jobs[blockIdx.y];
    if (blockIdx.x == 0 && threadIdx.x == 0) J.t = 0;
    if (!J.active) return;
    if (J.counters && blockIdx.x == 0 && threadIdx.x < kNumCounters) J.counters[threadIdx.x] = 0ull;
    if (J.E) {
        const long long n = (long long)J.K * J.C * J.W * J.Hh;
        for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
             x += (long long)gridDim.x * blockDim.x)
            J.E[x] = 0.0f;
    }
}

__global__ void k_advance_multi(JobDesc* jobs, int njobs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < njobs && iterating(jobs[j])) {
        jobs[j].t += 1;
        if (jobs[j].counters) jobs[j].counters[4] += 1ull;  // IRT iterations run
    }
}

template <int C>
__global__ void __launch_bounds__(256) k_ps_multi(const JobDesc* __restrict__ jobs, int from_A) {
    const JobDesc& J = jobs[blockIdx.y];
    const int npx = J.W * J.Hh;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (!participates(J, !from_A) || J.C != C || p >= npx) return;
    // after a correction, the shadow-aware solve uses this iteration's S
    if (from_A && (J.flags & kFlagShadowPs))
        ps_px_masked<C>(p, npx, J.K, &J.M[0][0], &J.L[0][0], J.s, J.A, J.S + (size_t)p * J.K, J.n, J.rho);
    else
        ps_px<C>(p, npx, J.K, &J.M[0][0], from_A ? J.A : J.I0, J.n, J.rho);
}

__global__ void __launch_bounds__(256) k_direct_multi(const JobDesc* __restrict__ jobs) {
    __shared__ int2 s_lvl[trv::kMaxLevels];
    const JobDesc& J = jobs[blockIdx.y];
    load_level_table(J.pyr_off, J.pyr_wc, s_lvl);
    const int p = direct_pixel(J.W, J.Hh, blockIdx.x, gridDim.x);
    if (!iterating(J)) return;  // uniform per block
    const Surface S = make_surface(J.depth, J.pyr, J.W, J.Hh, J.pyr_levels, J.quad_off, s_lvl);
    direct_wave(S, p, J.n, J.K, &J.L[0][0], J.s, (J.flags & kFlagFlat) != 0, J.S);
}

template <int C>
__global__ void __launch_bounds__(64) k_correct_multi(const JobDesc* __restrict__ jobs) {
    extern __shared__ float sm[];
    const JobDesc& J = jobs[blockIdx.y];
    const int npx = J.W * J.Hh;
    const int K = J.K, KC = J.K * C, rows = correct_rows(K, C);
    const int p0 = blockIdx.x * rows;
    if (!iterating(J) || J.C != C || p0 >= npx) return;  // uniform per block
    const int n = npx - p0 < rows ? npx - p0 : rows;
    float* sG = sm;
    float* sS = sm + rows * (KC + 1);
    stage_rows(J.G + (size_t)p0 * KC, n, KC, sG);
    stage_rows(J.S + (size_t)p0 * K, n, K, sS);
    __syncthreads();
    const int t = threadIdx.x;
    if (t >= n) return;
    const bool cumulative = (J.flags & 2) != 0;
    // the last iteration writes E; with a stop rule any iteration may be the last
    float* E = (J.t == J.T - 1 || J.stop_tol > 0.0f) ? J.E : nullptr;
    correct_px<C>(p0 + t, npx, K, J.rho_mode, cumulative ? 1 : 0, J.I0, (cumulative && J.t > 0) ? J.A : J.I0,
                  sG + t * (KC + 1), sS + t * (K + 1), J.rho, E, J.A);
}

__global__ void __launch_bounds__(256) k_pyr0_multi(const JobDesc* __restrict__ jobs) {
    const JobDesc& J = jobs[blockIdx.y];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (!iterating(J) || c >= J.pyr_wc[0] * J.pyr_hc[0]) return;
    pyr0_cell(c, J.W, J.Hh, J.pyr_wc[0], J.depth, J.pyr);
}

__global__ void __launch_bounds__(256) k_pyr_reduce_multi(const JobDesc* __restrict__ jobs, int l) {
    const JobDesc& J = jobs[blockIdx.y];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (!iterating(J) || l >= J.pyr_levels || c >= J.pyr_wc[l] * J.pyr_hc[l]) return;
    pyr_reduce_cell(c, J.pyr + J.pyr_off[l - 1], J.pyr_wc[l - 1], J.pyr_hc[l - 1], J.pyr + J.pyr_off[l],
                    J.pyr_wc[l]);
}

__global__ void __launch_bounds__(256) k_quad_blocks_multi(const JobDesc* __restrict__ jobs) {
    const JobDesc& J = jobs[blockIdx.y];
    const BlockTables t = block_tables(J.pyr + J.quad_off, J.W, J.Hh);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (iterating(J) && b < t.plane) quad_block(b, J.W, J.Hh, J.depth, t);
}

__global__ void __launch_bounds__(256) k_super_blocks_multi(const JobDesc* __restrict__ jobs) {
    const JobDesc& J = jobs[blockIdx.y];
    const BlockTables t = block_tables(J.pyr + J.quad_off, J.W, J.Hh);
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (iterating(J) && c < t.SW * t.SH) super_block(c, t);
}

__global__ void __launch_bounds__(256) k_horizon_blocks_multi(const JobDesc* __restrict__ jobs) {
    const JobDesc& J = jobs[blockIdx.y];
    const BlockTables t = block_tables(J.pyr + J.quad_off, J.W, J.Hh);
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (iterating(J) && v < 4 * t.plane) horizon_block((int)(v >> 2), (int)(v & 3), t);
}

// the flattened grid holds each job's near-horizon tiles
__global__ void __launch_bounds__(256) k_horizon_near_multi(const JobDesc* __restrict__ jobs, int njobs) {
    __shared__ float s_e[kNearSpan * kNearSpan];
    const int jb = job_of_block(jobs, njobs, blockIdx.x, [](const JobDesc& J) { return J.near_bstart; });
    const JobDesc& J = jobs[jb];
    const int tiles_x = (J.W + kNearTile - 1) / kNearTile;
    const int tile = (int)blockIdx.x - J.near_bstart;
    if (!iterating(J) || tile >= near_tiles(J.W, J.Hh)) return;  // uniform per block
    const BlockTables t = block_tables(J.pyr + J.quad_off, J.W, J.Hh);
    near_tile(J.W, J.Hh, J.depth, tile % tiles_x, tile / tiles_x, t.nearh, s_e);
}

__global__ void __launch_bounds__(64) k_quad_rows_multi(const JobDesc* __restrict__ jobs) {
    const JobDesc& J = jobs[blockIdx.y];
    const BlockTables t = block_tables(J.pyr + J.quad_off, J.W, J.Hh);
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (iterating(J) && j < t.QH) quad_row(j, t);
}

__global__ void __launch_bounds__(64) k_quad_cols_multi(const JobDesc* __restrict__ jobs) {
    const JobDesc& J = jobs[blockIdx.y];
    const BlockTables t = block_tables(J.pyr + J.quad_off, J.W, J.Hh);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (iterating(J) && i < t.QW) quad_col(i, t);
}

__global__ void __launch_bounds__(256) k_escape_rows_multi(const JobDesc* __restrict__ jobs) {
    const JobDesc& J = jobs[blockIdx.y];
    const BlockTables t = block_tables(J.pyr + J.quad_off, J.W, J.Hh);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (iterating(J) && b < t.plane) escape_row(b, t);
}

__global__ void __launch_bounds__(256) k_escape_cols_multi(const JobDesc* __restrict__ jobs) {
    const JobDesc& J = jobs[blockIdx.y];
    const BlockTables t = block_tables(J.pyr + J.quad_off, J.W, J.Hh);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (iterating(J) && b < t.plane) escape_col(b, t);
}

__global__ void __launch_bounds__(256) k_mg_rhs_multi(const JobDesc* __restrict__ jobs, int cold) {
    const JobDesc& J = jobs[blockIdx.y];
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (participates(J, cold) && v < J.W * J.Hh) mg_rhs_node(v, J.W, J.Hh, J.n, J.mg_ws + J.mg.boff[0]);
}

// X0 <- depth (warm) or 0 (cold).
__global__ void __launch_bounds__(256) k_mg_init_multi(const JobDesc* __restrict__ jobs, int cold) {
    const JobDesc& J = jobs[blockIdx.y];
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (!participates(J, cold) || v >= J.W * J.Hh) return;
    J.mg_ws[J.mg.xoff[0] + v] = cold ? 0.0f : J.depth[v];
}

// A job takes part in V-cycle c only while c is below its own cycle count.
__device__ __forceinline__ bool in_cycle(const JobDesc& J, int c, int cold) {
    return participates(J, cold) && c < (cold ? J.cycles_cold : J.cycles_warm);
}

__global__ void __launch_bounds__(256) k_mg_smooth_multi(const JobDesc* __restrict__ jobs, int njobs, int l,
                                                         int colour, int c, int cold) {
    const int jb = job_of_block(jobs, njobs, blockIdx.x, [l](const JobDesc& J) { return J.mg_bstart[l]; });
    const JobDesc& J = jobs[jb];
    const int v = (blockIdx.x - J.mg_bstart[l]) * blockDim.x + threadIdx.x;
    if (!in_cycle(J, c, cold) || l >= J.mg.tail || v >= J.mg.W[l] * J.mg.H[l]) return;
    mg_smooth_node(v, J.mg.W[l], J.mg.H[l], l, J.W, J.Hh, J.mg_ws + J.mg.xoff[l], J.mg_ws + J.mg.boff[l],
                   colour);
}

__global__ void __launch_bounds__(256) k_mg_restrict_multi(const JobDesc* __restrict__ jobs, int njobs, int l,
                                                           int c, int cold) {
    const int jb = job_of_block(jobs, njobs, blockIdx.x, [l](const JobDesc& J) { return J.rs_bstart[l]; });
    const JobDesc& J = jobs[jb];
    const int v = (blockIdx.x - J.rs_bstart[l]) * blockDim.x + threadIdx.x;
    if (!in_cycle(J, c, cold) || l >= J.mg.tail || v >= J.mg.W[l + 1] * J.mg.H[l + 1]) return;
    mg_restrict_node(v, J.mg.W[l], J.mg.H[l], l, J.W, J.Hh, J.mg_ws + J.mg.xoff[l], J.mg_ws + J.mg.boff[l],
                     J.mg.W[l + 1], J.mg_ws + J.mg.boff[l + 1], J.mg_ws + J.mg.xoff[l + 1]);
}

__global__ void __launch_bounds__(kMgTailThreads) k_mg_tail_multi(const JobDesc* __restrict__ jobs, int c, int cold) {
    extern __shared__ float s_mg[];
    const JobDesc& J = jobs[blockIdx.y];
    if (!in_cycle(J, c, cold)) return;  // uniform per block
    mg_tail(J.mg, J.W, J.Hh, J.mg_ws, s_mg);
}

__global__ void __launch_bounds__(256) k_mg_prolong_multi(const JobDesc* __restrict__ jobs, int njobs, int l,
                                                          int c, int cold) {
    const int jb = job_of_block(jobs, njobs, blockIdx.x, [l](const JobDesc& J) { return J.mg_bstart[l]; });
    const JobDesc& J = jobs[jb];
    const int v = (blockIdx.x - J.mg_bstart[l]) * blockDim.x + threadIdx.x;
    if (!in_cycle(J, c, cold) || l >= J.mg.tail || v >= J.mg.W[l] * J.mg.H[l]) return;
    mg_prolong_node(v, J.mg.W[l], J.mg_ws + J.mg.xoff[l], J.mg.W[l + 1], J.mg_ws + J.mg.xoff[l + 1]);
}

__global__ void __launch_bounds__(256) k_min_key_multi(const JobDesc* __restrict__ jobs, int init, int cold) {
    const JobDesc& J = jobs[blockIdx.y];
    if (!participates(J, cold)) return;
    unsigned* key = reinterpret_cast<unsigned*>(J.mg_ws + J.mg.keyoff);
    if (init) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            key[0] = 0xffffffffu;
            key[1] = 0u;  // D_H
        }
        return;
    }
    const int n = J.W * J.Hh;
    min_key_strided(J.mg_ws + J.mg.xoff[0], (long long)blockIdx.x * blockDim.x + threadIdx.x,
                    (long long)gridDim.x * blockDim.x, n, key);
}

__global__ void __launch_bounds__(256) k_anchor_multi(const JobDesc* __restrict__ jobs, int cold) {
    const JobDesc& J = jobs[blockIdx.y];
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (!participates(J, cold)) return;  // uniform per block
    unsigned* key = reinterpret_cast<unsigned*>(J.mg_ws + J.mg.keyoff);
    const bool measure = !cold && J.stop_tol > 0.0f;  // uniform per block
    float d = 0.0f;
    if (v < J.W * J.Hh) {
        const float h = J.mg_ws[J.mg.xoff[0] + v] - order_val(key[0]);
        if (measure) d = fabsf(h - J.depth[v]);
        J.depth[v] = h;
    }
    if (measure) block_max_into(d, key + 1);
}

// The paper's stop rule: a job whose surface changed by less than stop_tol in
// this iteration ends with it (T lowered to t + 1; t advances afterwards).
__global__ void k_stop_multi(JobDesc* jobs, int njobs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= njobs) return;
    JobDesc& J = jobs[j];
    if (!iterating(J) || !(J.stop_tol > 0.0f)) return;
    const unsigned* key = reinterpret_cast<const unsigned*>(J.mg_ws + J.mg.keyoff);
    if (__uint_as_float(key[1]) < J.stop_tol) J.T = J.t + 1;
}

// ===========================================================================
// Probes.
// Issue-rate probe: each lane runs `iters` rounds of eight independent 32-bit
// integer chains (a shift and a xor-add each: 16 VALU instructions per round, no
// memory access in the loop).  Lanes at or above `active` of their wave skip the
// work (the wave still issues it with those lanes masked off).  A counted, timed
// launch gives the wave64 VALU instructions the chip retires per second, and how
// that rate depends on the active lanes.
// VALU issue-rate probe: each round 16 independent wave64 instructions of one
// kind -- 0: integer shift and xor-add pairs (compiler-chosen encodings), 1:
// register moves, 2: fp32 fma -- on the lanes below `active`; no memory access
// in the loop.  One kernel per kind, so that a round holds nothing else; kinds
// 1 and 2 are written out so that each round is exactly those 16 instructions.
template <int KIND>
__global__ void __launch_bounds__(256) k_probe_valu(int iters, int active, uint32_t* out) {
    uint32_t x[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = threadIdx.x * 0x9E3779B9u + blockIdx.x * 0x85EBCA6Bu + (uint32_t)r;
    float f[4] = {(float)x[0], (float)x[1], (float)x[2], (float)x[3]};
    const bool on = (int)(threadIdx.x & 63) < active;
    for (int i = 0; i < iters; ++i) {
        if (on) {
            if (KIND == 0) {
#pragma unroll
                for (int r = 0; r < 8; ++r) x[r] = (x[r] ^ (x[r] >> 7)) + 0x7F4A7C15u;
            } else if (KIND == 1) {
                __asm__ volatile(
                    "v_mov_b32 %0, %4\n v_mov_b32 %1, %4\n v_mov_b32 %2, %4\n v_mov_b32 %3, %4\n"
                    "v_mov_b32 %0, %5\n v_mov_b32 %1, %5\n v_mov_b32 %2, %5\n v_mov_b32 %3, %5\n"
                    "v_mov_b32 %0, %4\n v_mov_b32 %1, %4\n v_mov_b32 %2, %4\n v_mov_b32 %3, %4\n"
                    "v_mov_b32 %0, %5\n v_mov_b32 %1, %5\n v_mov_b32 %2, %5\n v_mov_b32 %3, %5\n"
                    : "=v"(x[0]), "=v"(x[1]), "=v"(x[2]), "=v"(x[3])
                    : "v"(x[4]), "v"(x[5]));
            } else {
                __asm__ volatile(
                    "v_fma_f32 %0, %4, %6, %5\n v_fma_f32 %1, %5, %6, %4\n v_fma_f32 %2, %4, %6, %4\n v_fma_f32 %3, %5, %6, %5\n"
                    "v_fma_f32 %0, %5, %6, %4\n v_fma_f32 %1, %4, %6, %5\n v_fma_f32 %2, %5, %6, %5\n v_fma_f32 %3, %4, %6, %4\n"
                    "v_fma_f32 %0, %4, %6, %5\n v_fma_f32 %1, %5, %6, %4\n v_fma_f32 %2, %4, %6, %4\n v_fma_f32 %3, %5, %6, %5\n"
                    "v_fma_f32 %0, %5, %6, %4\n v_fma_f32 %1, %4, %6, %5\n v_fma_f32 %2, %5, %6, %5\n v_fma_f32 %3, %4, %6, %4\n"
                    : "=v"(f[0]), "=v"(f[1]), "=v"(f[2]), "=v"(f[3])
                    : "v"(__uint_as_float(x[4])), "v"(__uint_as_float(x[5])), "v"(0.5f));
            }
        }
        __asm__ volatile("" ::: "memory");  // keeps the masked body inside the loop
    }
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) acc ^= x[r];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc ^= __float_as_uint(f[r]);
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ void k_probe_philox(long long count, const uint32_t* ctr, uint32_t k0, uint32_t k1,
                               uint32_t* out) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    const dm::U4 o = dm::philox(ctr[4 * r], ctr[4 * r + 1], ctr[4 * r + 2], ctr[4 * r + 3], k0, k1);
    out[4 * r] = o.x;
    out[4 * r + 1] = o.y;
    out[4 * r + 2] = o.z;
    out[4 * r + 3] = o.w;
}

__global__ void k_probe_sample(long long count, const float* n, const float* u, float* d) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    const dm::V3 v = dm::cosine_dir(n[3 * r], n[3 * r + 1], n[3 * r + 2], u[2 * r], u[2 * r + 1]);
    d[3 * r] = v.x;
    d[3 * r + 1] = v.y;
    d[3 * r + 2] = v.z;
}

__global__ void k_probe_env(long long count, const float* d, int He, int We, int* rc) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    int row, col;
    dm::env_texel(d[3 * r], d[3 * r + 1], d[3 * r + 2], He, We, row, col);
    rc[2 * r] = row;
    rc[2 * r + 1] = col;
}

__global__ void k_probe_traverse(SurfaceArgs sa, int flat, long long count, const int* ij,
                                 const float* d, int* q) {
    __shared__ int2 s_lvl[trv::kMaxLevels];
    load_level_table(sa.off, sa.wc, s_lvl);
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    const int i0 = ij[2 * r], j0 = ij[2 * r + 1];
    if (i0 < 0 || i0 >= sa.W || j0 < 0 || j0 >= sa.Hh) {  // not a sample: reported, not traced
        q[2 * r] = -2;
        q[2 * r + 1] = -2;
        return;
    }
    const Surface S = make_surface(sa, s_lvl);
    int qi = -1, qj = -1;
    const bool hit = trv::walk(S, flat != 0, i0, j0, d[3 * r], d[3 * r + 1], d[3 * r + 2], qi, qj);
    q[2 * r] = hit ? qi : -1;
    q[2 * r + 1] = hit ? qj : -1;
}

// ===========================================================================
// Host launchers.
static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t ps_solve(int npx, int C, int K, const PsMatrix& M, const float* A, float* n, float* rho,
                    hipStream_t st) {
    const unsigned g = blocks_for(npx, 256);
    if (C == 1) hipLaunchKernelGGL(k_ps_solve<1>, dim3(g), dim3(256), 0, st, npx, K, M, A, n, rho);
    else hipLaunchKernelGGL(k_ps_solve<3>, dim3(g), dim3(256), 0, st, npx, K, M, A, n, rho);
    return hipGetLastError();
}

hipError_t ps_solve_masked(int npx, int C, int K, const PsMatrix& M, const LightSet& L, const float* A,
                           const float* S, float* n, float* rho, hipStream_t st) {
    const unsigned g = blocks_for(npx, 256);
    if (C == 1) hipLaunchKernelGGL(k_ps_solve_masked<1>, dim3(g), dim3(256), 0, st, npx, K, M, L, A, S, n, rho);
    else hipLaunchKernelGGL(k_ps_solve_masked<3>, dim3(g), dim3(256), 0, st, npx, K, M, L, A, S, n, rho);
    return hipGetLastError();
}

hipError_t direct(const SurfaceArgs& sa, const float* n, const LightSet& L, int flat, float* S,
                  hipStream_t st, float box_z) {
    const int tiles = tiles_for(sa.W, sa.Hh, kDirectTileW);
    hipLaunchKernelGGL(k_direct, dim3((tiles + 7) / 8 * 8), dim3(256), 0, st, sa, n, L, flat, S, box_z);
    return hipGetLastError();
}

hipError_t box_shade(int W, int H, const BoxArgs& b, const LightSet& L, float* S, hipStream_t st) {
    const long long n = 4LL * b.th * b.tw;
    hipLaunchKernelGGL(k_box_shade, dim3(blocks_for(n, 256)), dim3(256), 0, st, W, H, b, L, S);
    return hipGetLastError();
}

hipError_t order_tiles(const unsigned* cost, int tiles, int* order, hipStream_t st) {
    hipLaunchKernelGGL(k_order_tiles, dim3(1), dim3(kOrderThreads), 0, st, cost, tiles, order);
    return hipGetLastError();
}

// Blocks of the single-job tracer that the current device holds at once (its
// compute units times the blocks per unit at the tracer's occupancy), cached
// per device.
constexpr int kMaxDevices = 64;
static int trace_resident_blocks(int C) {
    static std::atomic<int> cache[2][kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = -1;
    if (dev >= 0) {
        const int v = cache[C == 1 ? 0 : 1][dev].load(std::memory_order_relaxed);
        if (v > 0) return v;
    }
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev < 0 ? 0 : dev) != hipSuccess || cus < 1)
        cus = 256;
    const void* f = C == 1 ? reinterpret_cast<const void*>(&k_trace<1>) : reinterpret_cast<const void*>(&k_trace<3>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, 256, 0) != hipSuccess || per < 1) per = 1;
    const int v = cus * per;
    if (dev >= 0) cache[C == 1 ? 0 : 1][dev].store(v, std::memory_order_relaxed);
    return v;
}

hipError_t trace(TraceArgs a, hipStream_t st) {
    if (a.records) {
        const int npx = a.sa.W * a.sa.Hh;
        if (split_record_bytes(npx, a.C, a.spp, a.B) == 0) return hipErrorInvalidValue;
        const unsigned g1 = blocks_for((long long)npx * a.spp, 256), g2 = blocks_for(npx, 256);
        if (a.C == 1) {
            hipLaunchKernelGGL(k_trace_paths<1>, dim3(g1), dim3(256), 0, st, a);
            hipLaunchKernelGGL(k_gather_paths<1>, dim3(g2), dim3(256), 0, st, a);
        } else {
            hipLaunchKernelGGL(k_trace_paths<3>, dim3(g1), dim3(256), 0, st, a);
            hipLaunchKernelGGL(k_gather_paths<3>, dim3(g2), dim3(256), 0, st, a);
        }
        return hipGetLastError();
    }
    const int chunks = chunks_for(a.sa.W, a.sa.Hh, 1 << a.tile_shift);
    if (a.tile_cost)  // chunk costs and the queue slot start at zero
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for((long long)chunks + 1, 256)), dim3(256), 0, st, a.tile_cost,
                           0u, chunks + 1);
    // at most the blocks the GPU holds at once (4 waves, so 4 chunks, per block)
    const int want = (chunks + 3) / 4;
    const int held = trace_resident_blocks(a.C);
    const int grid = want < held ? want : held;
    if (a.C == 1) hipLaunchKernelGGL(k_trace<1>, dim3(grid), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_trace<3>, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t correct(int npx, int C, int K, int rho_mode, int cumulative, const float* I0,
                   const float* Aprev, const float* G, const float* S, const float* rho, float* E,
                   float* Anext, hipStream_t st, const float* esc_sums, int spp) {
    const int rows = correct_rows(K, C);
    const unsigned g = blocks_for(npx, rows);
    const size_t lds = sizeof(float) * rows * (K * C + 1 + K + 1);
    if (C == 1)
        hipLaunchKernelGGL(k_correct<1>, dim3(g), dim3(64), lds, st, npx, K, rho_mode, cumulative, I0, Aprev, G, S,
                           rho, E, Anext, esc_sums, spp);
    else
        hipLaunchKernelGGL(k_correct<3>, dim3(g), dim3(64), lds, st, npx, K, rho_mode, cumulative, I0, Aprev, G, S,
                           rho, E, Anext, esc_sums, spp);
    return hipGetLastError();
}

hipError_t compose(int npx, int C, int K, const float* rho, const float* S, const float* G, float* I,
                   hipStream_t st) {
    const unsigned g = blocks_for(npx, 256);
    if (C == 1) hipLaunchKernelGGL(k_compose<1>, dim3(g), dim3(256), 0, st, npx, K, rho, S, G, I);
    else hipLaunchKernelGGL(k_compose<3>, dim3(g), dim3(256), 0, st, npx, K, rho, S, G, I);
    return hipGetLastError();
}

hipError_t build_pyramid(int W, int Hh, const float* H, const trv::Pyramid& P, float* pyr,
                         long long quad_off, hipStream_t st) {
    float* tab = pyr + quad_off;
    const int QW = trv::quad_cells(W), QH = trv::quad_cells(Hh);
    const unsigned gb = blocks_for((long long)QW * QH, 256);
    hipLaunchKernelGGL(k_quad_blocks, dim3(gb), dim3(256), 0, st, W, Hh, H, tab);
    hipLaunchKernelGGL(k_quad_rows, dim3(blocks_for(QH, 64)), dim3(64), 0, st, W, Hh, tab);
    hipLaunchKernelGGL(k_quad_cols, dim3(blocks_for(QW, 64)), dim3(64), 0, st, W, Hh, tab);
    hipLaunchKernelGGL(k_escape_rows, dim3(gb), dim3(256), 0, st, W, Hh, tab);
    hipLaunchKernelGGL(k_escape_cols, dim3(gb), dim3(256), 0, st, W, Hh, tab);
    const long long supers = (long long)trv::super_cells(W) * trv::super_cells(Hh);
    hipLaunchKernelGGL(k_super_blocks, dim3(blocks_for(supers, 256)), dim3(256), 0, st, W, Hh, tab);
    hipLaunchKernelGGL(k_horizon_blocks, dim3(blocks_for(4LL * QW * QH, 256)), dim3(256), 0, st, W, Hh, tab);
    hipLaunchKernelGGL(k_horizon_near, dim3(blocks_for(W, kNearTile), blocks_for(Hh, kNearTile)), dim3(256), 0, st,
                       W, Hh, H, tab);
    hipLaunchKernelGGL(k_pyr_level0, dim3(blocks_for((long long)P.wc[0] * P.hc[0], 256)), dim3(256), 0,
                       st, W, Hh, H, pyr + P.off[0], P.wc[0], P.hc[0]);
    for (int l = 1; l < P.levels; ++l)
        hipLaunchKernelGGL(k_pyr_reduce, dim3(blocks_for((long long)P.wc[l] * P.hc[l], 256)), dim3(256),
                           0, st, pyr + P.off[l - 1], P.wc[l - 1], P.hc[l - 1], pyr + P.off[l], P.wc[l],
                           P.hc[l]);
    return hipGetLastError();
}

// Blocks of the anchor's minimum reduction (each strides over the grid).
constexpr unsigned kMinKeyBlocks = 512;

hipError_t integrate(const MgPlan& plan, const float* n, const float* Hinit, int cycles, float* Hout,
                     float* ws, hipStream_t st, bool measure_change, const Robust& robust) {
    if (measure_change && Hinit != Hout) return hipErrorInvalidValue;
    const int W0 = plan.W[0], H0 = plan.H[0];
    const int npx = W0 * H0;
    float* X[kMaxMgLevels];
    float* b[kMaxMgLevels];
    for (int l = 0; l < plan.levels; ++l) {
        X[l] = ws + plan.xoff[l];
        b[l] = ws + plan.boff[l];
    }
    unsigned* key = reinterpret_cast<unsigned*>(ws + plan.keyoff);
    hipLaunchKernelGGL(k_mg_rhs, dim3(blocks_for(npx, 256)), dim3(256), 0, st, W0, H0, n, b[0]);
    if (Hinit)
        hipLaunchKernelGGL(k_copy_f32, dim3(blocks_for(npx, 256)), dim3(256), 0, st, X[0], Hinit,
                           (long long)npx);
    else
        hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(npx, 256)), dim3(256), 0, st, X[0], 0.0f,
                           (long long)npx);
    auto smooth = [&](int l, int sweeps) {
        const int nl = plan.W[l] * plan.H[l];
        for (int s = 0; s < sweeps; ++s)
            for (int colour = 0; colour < 2; ++colour)
                hipLaunchKernelGGL(k_mg_smooth, dim3(blocks_for(nl, 256)), dim3(256), 0, st, plan.W[l],
                                   plan.H[l], l, W0, H0, X[l], b[l], colour);
    };
    // the plan chose the tail so that its levels fit the default 64 KiB of LDS
    if ((long long)sizeof(float) * mg_tail_floats(plan) > kMgTailLdsBytes) return hipErrorInvalidValue;
    auto vcycle = [&]() {
        for (int l = 0; l < plan.tail; ++l) {
            smooth(l, 2);
            const int nc = plan.W[l + 1] * plan.H[l + 1];
            hipLaunchKernelGGL(k_mg_restrict, dim3(blocks_for(nc, 256)), dim3(256), 0, st, plan.W[l],
                               plan.H[l], l, W0, H0, X[l], b[l], plan.W[l + 1], plan.H[l + 1], b[l + 1],
                               X[l + 1]);
        }
        hipLaunchKernelGGL(k_mg_tail, dim3(1), dim3(kMgTailThreads), sizeof(float) * mg_tail_floats(plan), st,
                           plan, W0, H0, ws);
        for (int l = plan.tail - 1; l >= 0; --l) {
            hipLaunchKernelGGL(k_mg_prolong, dim3(blocks_for(plan.W[l] * plan.H[l], 256)), dim3(256), 0,
                               st, plan.W[l], plan.H[l], X[l], plan.W[l + 1], X[l + 1]);
            smooth(l, 2);
        }
    };
    for (int c = 0; c < cycles; ++c) vcycle();
    for (int r = 0; r < robust.rounds; ++r) {
        hipLaunchKernelGGL(k_mg_rhs_robust, dim3(blocks_for(npx, 256)), dim3(256), 0, st, W0, H0, n, X[0],
                           robust.delta, b[0]);
        for (int c = 0; c < robust.cycles; ++c) vcycle();
    }
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, key, 0xffffffffu, 1);
    unsigned* change = measure_change ? change_key_of(plan, ws) : nullptr;
    if (change) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, change, 0u, 1);
    const unsigned gm = blocks_for(npx, 256) < kMinKeyBlocks ? blocks_for(npx, 256) : kMinKeyBlocks;
    hipLaunchKernelGGL(k_min_key, dim3(gm), dim3(256), 0, st, X[0], npx, key);
    hipLaunchKernelGGL(k_anchor, dim3(blocks_for(npx, 256)), dim3(256), 0, st, X[0], npx, key, Hout, change);
    return hipGetLastError();
}

hipError_t trace_exact_r(const SurfaceArgs& sa, int C, const float* n, const float* rho, const float* env,
                         int He, int We, int r, int t, int tag, uint32_t key0, uint32_t key1, int flat, float* E,
                         float* w0, unsigned char* valid, hipStream_t st) {
    const long long npx = (long long)sa.W * sa.Hh;
    const dim3 g(blocks_for(npx, 256)), b(256);
    if (C == 1)
        hipLaunchKernelGGL(k_trace_exact_r<1>, g, b, 0, st, sa, n, rho, env, He, We, r, t, tag, key0, key1, flat, E,
                           w0, valid);
    else
        hipLaunchKernelGGL(k_trace_exact_r<3>, g, b, 0, st, sa, n, rho, env, He, We, r, t, tag, key0, key1, flat, E,
                           w0, valid);
    return hipGetLastError();
}

hipError_t fill_weights(long long npx, const unsigned char* valid, float* ws, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_weights, dim3(blocks_for(npx, 256)), dim3(256), 0, st, npx, valid, ws);
    return hipGetLastError();
}

hipError_t fill_pull_push(const FillPlan& fp, int C, const float* v0, float* ws, hipStream_t st) {
    for (int l = 0; l + 1 < fp.levels; ++l) {
        const float* vf = l ? ws + fp.voff[l] : v0;
        const long long cells = (long long)fp.w[l + 1] * fp.h[l + 1];
        const dim3 g(blocks_for(cells, 256)), b(256);
        if (C == 1)
            hipLaunchKernelGGL(k_fill_pull<1>, g, b, 0, st, ws + fp.woff[l], vf, fp.w[l], fp.h[l], ws + fp.woff[l + 1],
                               ws + fp.voff[l + 1], fp.w[l + 1], fp.h[l + 1]);
        else
            hipLaunchKernelGGL(k_fill_pull<3>, g, b, 0, st, ws + fp.woff[l], vf, fp.w[l], fp.h[l], ws + fp.woff[l + 1],
                               ws + fp.voff[l + 1], fp.w[l + 1], fp.h[l + 1]);
    }
    for (int l = fp.levels - 2; l >= 1; --l) {
        const long long cells = (long long)fp.w[l] * fp.h[l];
        const dim3 g(blocks_for(cells, 256)), b(256);
        if (C == 1)
            hipLaunchKernelGGL(k_fill_push<1>, g, b, 0, st, ws + fp.woff[l], ws + fp.voff[l], fp.w[l], fp.h[l],
                               ws + fp.voff[l + 1], fp.w[l + 1]);
        else
            hipLaunchKernelGGL(k_fill_push<3>, g, b, 0, st, ws + fp.woff[l], ws + fp.voff[l], fp.w[l], fp.h[l],
                               ws + fp.voff[l + 1], fp.w[l + 1]);
    }
    return hipGetLastError();
}

hipError_t fill_push0(const FillPlan& fp, int C, float* v0, const float* ws, hipStream_t st) {
    const long long cells = (long long)fp.w[0] * fp.h[0];
    const float* v1 = fp.levels > 1 ? ws + fp.voff[1] : nullptr;
    const int cw = fp.levels > 1 ? fp.w[1] : 1;
    const dim3 g(blocks_for(cells, 256)), b(256);
    if (C == 1)
        hipLaunchKernelGGL(k_fill_push<1>, g, b, 0, st, ws + fp.woff[0], v0, fp.w[0], fp.h[0], v1, cw);
    else
        hipLaunchKernelGGL(k_fill_push<3>, g, b, 0, st, ws + fp.woff[0], v0, fp.w[0], fp.h[0], v1, cw);
    return hipGetLastError();
}

hipError_t fill_push0_broadcast(const FillPlan& fp, int C, int K, const float* v0, const float* ws, float* G,
                                hipStream_t st) {
    const long long n = (long long)fp.w[0] * fp.h[0] * K * C;
    const float* v1 = fp.levels > 1 ? ws + fp.voff[1] : nullptr;
    const int cw = fp.levels > 1 ? fp.w[1] : 1;
    const dim3 g(blocks_for(n, 256)), b(256);
    if (C == 1)
        hipLaunchKernelGGL(k_fill_push0_broadcast<1>, g, b, 0, st, ws + fp.woff[0], v0, fp.w[0], fp.h[0], v1, cw, K,
                           G);
    else
        hipLaunchKernelGGL(k_fill_push0_broadcast<3>, g, b, 0, st, ws + fp.woff[0], v0, fp.w[0], fp.h[0], v1, cw, K,
                           G);
    return hipGetLastError();
}

hipError_t fill_f32(float* p, float v, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t fill_u64_zero(unsigned long long* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned*>(p), 0u, 2 * n);
    return hipGetLastError();
}

__global__ void k_add_u64(unsigned long long* p, unsigned long long v) {
    if (threadIdx.x == 0) *p += v;
}

hipError_t add_u64(unsigned long long* p, unsigned long long v, hipStream_t st) {
    hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(64), 0, st, p, v);
    return hipGetLastError();
}

// ---- multi-job ----
hipError_t trace_multi(const JobDesc* jobs, int C, const int2* tiles, int ntiles, unsigned* queue,
                       int tag, int resident_blocks, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, queue, 0u, 1);
    // enough resident blocks to fill every CU several times over; the queue balances them
    int grid = resident_blocks;
    if (grid > ntiles) grid = ntiles;
    if (C == 1)
        hipLaunchKernelGGL(k_trace_multi<1>, dim3(grid), dim3(256), 0, st, jobs, tiles, ntiles, queue, tag);
    else
        hipLaunchKernelGGL(k_trace_multi<3>, dim3(grid), dim3(256), 0, st, jobs, tiles, ntiles, queue, tag);
    return hipGetLastError();
}

hipError_t batch_begin(const JobDesc* jobs, const BatchShape& bs, hipStream_t st) {
    hipLaunchKernelGGL(k_begin_multi, dim3(256, bs.njobs), dim3(256), 0, st, const_cast<JobDesc*>(jobs));
    return hipGetLastError();
}

hipError_t batch_advance(JobDesc* jobs, int njobs, hipStream_t st) {
    hipLaunchKernelGGL(k_advance_multi, dim3(blocks_for(njobs, 64)), dim3(64), 0, st, jobs, njobs);
    return hipGetLastError();
}

hipError_t batch_ps(const JobDesc* jobs, const BatchShape& bs, int from_A, hipStream_t st) {
    const dim3 g(blocks_for(bs.max_npx, 256), bs.njobs);
    hipLaunchKernelGGL(k_ps_multi<1>, g, dim3(256), 0, st, jobs, from_A);
    hipLaunchKernelGGL(k_ps_multi<3>, g, dim3(256), 0, st, jobs, from_A);
    return hipGetLastError();
}

hipError_t batch_pyramid(const JobDesc* jobs, const BatchShape& bs, hipStream_t st) {
    const long long qcells = (long long)trv::quad_cells(bs.max_cols) * trv::quad_cells(bs.max_rows);
    hipLaunchKernelGGL(k_quad_blocks_multi, dim3(blocks_for(qcells, 256), bs.njobs), dim3(256), 0, st, jobs);
    hipLaunchKernelGGL(k_quad_rows_multi, dim3(blocks_for(trv::quad_cells(bs.max_rows), 64), bs.njobs), dim3(64), 0,
                       st, jobs);
    hipLaunchKernelGGL(k_quad_cols_multi, dim3(blocks_for(trv::quad_cells(bs.max_cols), 64), bs.njobs), dim3(64), 0,
                       st, jobs);
    hipLaunchKernelGGL(k_escape_rows_multi, dim3(blocks_for(qcells, 256), bs.njobs), dim3(256), 0, st, jobs);
    hipLaunchKernelGGL(k_escape_cols_multi, dim3(blocks_for(qcells, 256), bs.njobs), dim3(256), 0, st, jobs);
    const long long supers = (long long)trv::super_cells(bs.max_cols) * trv::super_cells(bs.max_rows);
    hipLaunchKernelGGL(k_super_blocks_multi, dim3(blocks_for(supers, 256), bs.njobs), dim3(256), 0, st, jobs);
    hipLaunchKernelGGL(k_horizon_blocks_multi, dim3(blocks_for(4 * qcells, 256), bs.njobs), dim3(256), 0, st, jobs);
    if (bs.near_blocks > 0)
        hipLaunchKernelGGL(k_horizon_near_multi, dim3(bs.near_blocks), dim3(256), 0, st, jobs, bs.njobs);
    hipLaunchKernelGGL(k_pyr0_multi, dim3(blocks_for(bs.max_pyr_cells[0], 256), bs.njobs), dim3(256), 0, st,
                       jobs);
    for (int l = 1; l < bs.max_pyr_levels; ++l)
        hipLaunchKernelGGL(k_pyr_reduce_multi, dim3(blocks_for(bs.max_pyr_cells[l], 256), bs.njobs), dim3(256),
                           0, st, jobs, l);
    return hipGetLastError();
}

hipError_t batch_direct(const JobDesc* jobs, const BatchShape& bs, hipStream_t st) {
    hipLaunchKernelGGL(k_direct_multi, dim3((bs.max_direct_tiles + 7) / 8 * 8, bs.njobs), dim3(256), 0, st,
                       jobs);
    return hipGetLastError();
}

hipError_t batch_correct(const JobDesc* jobs, const BatchShape& bs, int /*last_only*/, hipStream_t st) {
    // LDS for the largest light count of each channel count; rows per block
    // never exceed what that allows (correct_rows shrinks with K C)
    for (int C = 1; C <= 3; C += 2) {
        const int K = C == 1 ? bs.max_K1 : bs.max_K3;
        if (K == 0) continue;
        int need = 0;  // the largest staging area any job of this channel count uses
        for (int k = 1; k <= K; ++k) {
            const int r = correct_rows(k, C) * (k * C + 1 + k + 1);
            need = r > need ? r : need;
        }
        const dim3 g(blocks_for(bs.max_npx, 32), bs.njobs);  // enough blocks for 32-row jobs too
        const size_t lds = sizeof(float) * need;
        if (C == 1) hipLaunchKernelGGL(k_correct_multi<1>, g, dim3(64), lds, st, jobs);
        else hipLaunchKernelGGL(k_correct_multi<3>, g, dim3(64), lds, st, jobs);
    }
    return hipGetLastError();
}

hipError_t batch_integrate(const JobDesc* jobs, const BatchShape& bs, int cold, hipStream_t st) {
    const int nj = bs.njobs;
    const dim3 gpx(blocks_for(bs.max_npx, 256), nj);
    hipLaunchKernelGGL(k_mg_rhs_multi, gpx, dim3(256), 0, st, jobs, cold);
    hipLaunchKernelGGL(k_mg_init_multi, gpx, dim3(256), 0, st, jobs, cold);
    const int cycles = cold ? bs.max_cycles_cold : bs.max_cycles_warm;
    if ((long long)sizeof(float) * bs.max_mg_tail_floats > kMgTailLdsBytes) return hipErrorInvalidValue;
    const int L = bs.max_mg_tail;  // every job's per-level part
    for (int c = 0; c < cycles; ++c) {
        for (int l = 0; l < L; ++l) {
            for (int s = 0; s < 2; ++s)
                for (int colour = 0; colour < 2; ++colour)
                    hipLaunchKernelGGL(k_mg_smooth_multi, dim3(bs.mg_blocks[l]), dim3(256), 0, st, jobs, nj, l,
                                       colour, c, cold);
            hipLaunchKernelGGL(k_mg_restrict_multi, dim3(bs.rs_blocks[l]), dim3(256), 0, st, jobs, nj, l, c, cold);
        }
        hipLaunchKernelGGL(k_mg_tail_multi, dim3(1, nj), dim3(kMgTailThreads), sizeof(float) * bs.max_mg_tail_floats,
                           st, jobs, c, cold);
        for (int l = L - 1; l >= 0; --l) {
            hipLaunchKernelGGL(k_mg_prolong_multi, dim3(bs.mg_blocks[l]), dim3(256), 0, st, jobs, nj, l, c, cold);
            for (int s = 0; s < 2; ++s)
                for (int colour = 0; colour < 2; ++colour)
                    hipLaunchKernelGGL(k_mg_smooth_multi, dim3(bs.mg_blocks[l]), dim3(256), 0, st, jobs, nj, l,
                                       colour, c, cold);
        }
    }
    hipLaunchKernelGGL(k_min_key_multi, dim3(1, nj), dim3(64), 0, st, jobs, 1, cold);
    const unsigned gm = gpx.x < kMinKeyBlocks ? gpx.x : kMinKeyBlocks;
    hipLaunchKernelGGL(k_min_key_multi, dim3(gm, nj), dim3(256), 0, st, jobs, 0, cold);
    hipLaunchKernelGGL(k_anchor_multi, gpx, dim3(256), 0, st, jobs, cold);
    if (!cold)
        hipLaunchKernelGGL(k_stop_multi, dim3(blocks_for(nj, 64)), dim3(64), 0, st, const_cast<JobDesc*>(jobs), nj);
    return hipGetLastError();
}

hipError_t probe_valu(int blocks, int iters, int active, int kind, uint32_t* out, hipStream_t st) {
    if (kind == 0) hipLaunchKernelGGL(k_probe_valu<0>, dim3(blocks), dim3(256), 0, st, iters, active, out);
    else if (kind == 1) hipLaunchKernelGGL(k_probe_valu<1>, dim3(blocks), dim3(256), 0, st, iters, active, out);
    else hipLaunchKernelGGL(k_probe_valu<2>, dim3(blocks), dim3(256), 0, st, iters, active, out);
    return hipGetLastError();
}

hipError_t probe_philox(long long count, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                        hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_philox, dim3(blocks_for(count, 256)), dim3(256), 0, st, count, ctr, k0, k1,
                       out);
    return hipGetLastError();
}

hipError_t probe_sample(long long count, const float* n, const float* u, float* d, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_sample, dim3(blocks_for(count, 256)), dim3(256), 0, st, count, n, u, d);
    return hipGetLastError();
}

hipError_t probe_env(long long count, const float* d, int He, int We, int* rc, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_env, dim3(blocks_for(count, 256)), dim3(256), 0, st, count, d, He, We, rc);
    return hipGetLastError();
}

hipError_t probe_traverse(const SurfaceArgs& sa, int flat, long long count, const int* ij,
                          const float* d, int* q, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_traverse, dim3(blocks_for(count, 256)), dim3(256), 0, st, sa, flat, count,
                       ij, d, q);
    return hipGetLastError();
}

}  // namespace kern
}  // namespace irtps
