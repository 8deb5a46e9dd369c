// host.hpp -- host-side helpers shared by the C ABI translation units:
// status and HIP error plumbing, workspace plans, the Eq.4 matrix, validation.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "irtps.h"
#include "kernels.hpp"

namespace irtps {
namespace host {


inline thread_local int g_last_hip = 0;

inline int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return IRTPS_ERR_DEVICE;
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        const hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hip_fail(e_);     \
    } while (0)

#define STATUS_TRY(expr)                               \
    do {                                               \
        const int s_ = (expr);                         \
        if (s_ != IRTPS_OK) return s_;                 \
    } while (0)

constexpr size_t kAlign = 256;

// The tracer's schedule: tile width 2^tile_shift and the lanes that must hold a
// finished segment before a wave shades them.  Any schedule gives the same
// bits.  Forced values (irtps_set_schedule) win over the tuning table, which
// wins over the default 16 x 16 tiles, 32 lanes (tune.cpp).
struct Schedule {
    int tile_shift;
    int ready_batch;
};
Schedule schedule_for(int W, int H, int C, int K, int B);

// Event pairs around tracer launches while profiling is on (per thread).
struct Profiler {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};
inline thread_local Profiler g_prof;

inline hipError_t traced(const kern::TraceArgs& ta, hipStream_t st) {
    if (!g_prof.on) return kern::trace(ta, st);
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, st);
    if (e == hipSuccess) e = kern::trace(ta, st);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        return e;
    }
    g_prof.ev.emplace_back(a, b);
    return hipSuccess;
}

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Sides up to 16384 keep the pyramid within trv::kMaxLevels levels and every
// pixel index within int32.
inline bool dims_ok(int W, int H) { return W >= 2 && H >= 2 && W <= 16384 && H <= 16384 && (long long)W * H <= (1LL << 28); }
inline bool channels_ok(int C) { return C == 1 || C == 3; }
inline bool lights_ok(int K) { return K >= 3 && K <= kern::kMaxLights; }
// A box: a positive finite height, textures of 1..4096 texels a side, albedo given.
inline bool box_ok(const irtps_box* b) {
    return b && b->height > 0.0f && b->height <= 3.0e38f && b->tex_h >= 1 && b->tex_w >= 1 && b->tex_h <= 4096 &&
           b->tex_w <= 4096 && b->albedo_dev;
}
inline kern::BoxArgs box_args(const irtps_box* b) {
    kern::BoxArgs a{};
    a.z = b->height;
    a.th = b->tex_h;
    a.tw = b->tex_w;
    return a;
}
// Bytes of the walls' direct irradiance [4][tex_h][tex_w][K] (0 without a box).
inline size_t box_shade_bytes(const irtps_box* b, int K) {
    return b ? align_up(sizeof(float) * 4 * (size_t)b->tex_h * (size_t)b->tex_w * (size_t)K) : 0;
}

inline trv::Pyramid pyramid_plan(int W, int H) {
    trv::Pyramid P{};
    int wc = W - 1, hc = H - 1;
    long long off = 0;
    int l = 0;
    for (;;) {
        P.wc[l] = wc;
        P.hc[l] = hc;
        P.off[l] = off;
        off += (long long)wc * hc;
        ++l;
        if (wc == 1 && hc == 1) break;
        wc = (wc + 1) / 2;
        hc = (hc + 1) / 2;
    }
    P.levels = l;
    return P;
}

inline long long pyramid_level_floats(const trv::Pyramid& P) {
    const int t = P.levels - 1;
    return (P.off[t] + (long long)P.wc[t] * P.hc[t] + 63) / 64 * 64;
}

// Apron-max levels followed by the four quadrant-maximum planes.
inline long long pyramid_floats(int W, int H) {
    return pyramid_level_floats(pyramid_plan(W, H)) + trv::block_tables_floats(W, H);
}

inline kern::MgPlan mg_plan(int W, int H) {
    kern::MgPlan m{};
    m.W[0] = W;
    m.H[0] = H;
    m.levels = 1;
    while ((m.W[m.levels - 1] > 4 || m.H[m.levels - 1] > 4) && m.levels < kern::kMaxMgLevels) {
        m.W[m.levels] = (m.W[m.levels - 1] + 1) / 2;
        m.H[m.levels] = (m.H[m.levels - 1] + 1) / 2;
        ++m.levels;
    }
    long long off = 0;
    for (int l = 0; l < m.levels; ++l) {
        const long long n = (long long)m.W[l] * m.H[l];
        m.xoff[l] = off;
        off += (n + 63) / 64 * 64;
        m.boff[l] = off;
        off += (n + 63) / 64 * 64;
    }
    m.keyoff = off;
    off += 64;
    m.total = off;
    // the tail: the first level of at most kMgTailNodes nodes whose X and b,
    // with those of every coarser level, fit the tail kernel's LDS
    m.tail = 0;
    while ((long long)m.W[m.tail] * m.H[m.tail] > kern::kMgTailNodes ||
           (long long)sizeof(float) * (m.keyoff - m.xoff[m.tail]) > kern::kMgTailLdsBytes)
        ++m.tail;
    return m;
}

// Eq.3-4 in binary64: A = L^T L, inverse by the adjugate, M = A^-1 L^T.
inline int ps_matrix_host(int K, const float* l, const float* s, float* M) {
    if (K < 3 || !l || !M) return K < 3 ? IRTPS_ERR_SINGULAR_LIGHTS : IRTPS_ERR_INVALID_ARG;
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int k = 0; k < K; ++k) {
        const double sk = s ? (double)s[k] : 1.0;
        const double v[3] = {sk * (double)l[3 * k], sk * (double)l[3 * k + 1], sk * (double)l[3 * k + 2]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A[a][b] = A[a][b] + v[a] * v[b];
    }
    double adj_t[3][3];  // cofactor matrix C[a][b]; inverse = C^T / det
    adj_t[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    adj_t[0][1] = -(A[1][0] * A[2][2] - A[1][2] * A[2][0]);
    adj_t[0][2] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    adj_t[1][0] = -(A[0][1] * A[2][2] - A[0][2] * A[2][1]);
    adj_t[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
    adj_t[1][2] = -(A[0][0] * A[2][1] - A[0][1] * A[2][0]);
    adj_t[2][0] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
    adj_t[2][1] = -(A[0][0] * A[1][2] - A[0][2] * A[1][0]);
    adj_t[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
    const double det = A[0][0] * adj_t[0][0] + A[0][1] * adj_t[0][1] + A[0][2] * adj_t[0][2];
    const double mean_eig = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
    if (!(det > 1e-7 * mean_eig * mean_eig * mean_eig)) return IRTPS_ERR_SINGULAR_LIGHTS;
    for (int k = 0; k < K; ++k) {
        const double sk = s ? (double)s[k] : 1.0;
        const double v[3] = {sk * (double)l[3 * k], sk * (double)l[3 * k + 1], sk * (double)l[3 * k + 2]};
        for (int a = 0; a < 3; ++a) {
            const double i0 = adj_t[0][a] / det, i1 = adj_t[1][a] / det, i2 = adj_t[2][a] / det;
            M[(size_t)a * K + k] = (float)(i0 * v[0] + i1 * v[1] + i2 * v[2]);
        }
    }
    return IRTPS_OK;
}

inline int make_lights(int K, const float* l, const float* s, kern::LightSet& L) {
    if (!lights_ok(K) || !l) return IRTPS_ERR_INVALID_ARG;
    std::memset(&L, 0, sizeof(L));
    L.K = K;
    for (int k = 0; k < K; ++k) {
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(l[3 * k + a])) return IRTPS_ERR_INVALID_ARG;
            L.l[k][a] = l[3 * k + a];
        }
        L.s[k] = s ? s[k] : 1.0f;
        if (!std::isfinite(L.s[k])) return IRTPS_ERR_INVALID_ARG;
    }
    return IRTPS_OK;
}

inline int make_psmatrix(int K, const float* l, const float* s, kern::PsMatrix& M) {
    if (!lights_ok(K)) return K < 3 ? IRTPS_ERR_SINGULAR_LIGHTS : IRTPS_ERR_INVALID_ARG;
    float tmp[3 * kern::kMaxLights];
    STATUS_TRY(ps_matrix_host(K, l, s, tmp));
    std::memset(&M, 0, sizeof(M));
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < K; ++k) M.m[a][k] = tmp[(size_t)a * K + k];
    return IRTPS_OK;
}

inline kern::SurfaceArgs surface(int W, int H, const float* depth, const float* pyr) {
    kern::SurfaceArgs sa;
    sa.H = depth;
    sa.pyr = pyr;
    sa.W = W;
    sa.Hh = H;
    const trv::Pyramid P = pyramid_plan(W, H);
    sa.levels = P.levels;
    sa.quad_off = (int)pyramid_level_floats(P);
    for (int l = 0; l < trv::kMaxLevels; ++l) {
        sa.off[l] = l < P.levels ? (int)P.off[l] : 0;
        sa.wc[l] = l < P.levels ? P.wc[l] : 0;
    }
    return sa;
}

// Workspace layout of one solve (byte offsets, each 256-aligned).
struct SolveLayout {
    size_t A, S, G, pyr, mg, tile_cost, tile_order, total;
    kern::MgPlan plan;
};

inline SolveLayout solve_layout(int W, int H, int C, int K) {
    SolveLayout L{};
    const size_t npx = (size_t)W * H;
    size_t off = 0;
    L.A = off;
    off = align_up(off + sizeof(float) * npx * K * C);
    L.S = off;
    off = align_up(off + sizeof(float) * npx * K);
    L.G = off;
    off = align_up(off + sizeof(float) * npx * K * C);
    L.pyr = off;
    off = align_up(off + sizeof(float) * (size_t)pyramid_floats(W, H));
    L.plan = mg_plan(W, H);
    L.mg = off;
    off = align_up(off + sizeof(float) * (size_t)L.plan.total);
    L.tile_cost = off;  // the tracer's chunk costs, then its queue slot
    off = align_up(off + sizeof(unsigned) * ((size_t)kern::max_trace_chunks(W, H) + 1));
    L.tile_order = off;
    off = align_up(off + sizeof(int) * (size_t)kern::max_trace_chunks(W, H));
    L.total = off;
    return L;
}

// The solve's workspace: the layout above, then a tail: with the r-ray variant
// its pull-push levels, else for small problems the per-path tracer's segment
// records, and for the others the per-pixel tracer's escape sums.
inline size_t split_bytes(int W, int H, int C, int spp, int B) {
    return align_up((size_t)kern::split_record_bytes((long long)W * H, C, spp, B));
}
inline size_t fill_bytes(int W, int H, int C) {
    return align_up(sizeof(float) * (size_t)kern::fill_plan(W, H, C).total_v0);
}
inline size_t esc_sum_bytes(int W, int H, int C) { return align_up(sizeof(float) * (size_t)W * H * C); }
inline size_t tail_bytes(int W, int H, int C, const irtps_params* pa) {
    if (kern::exact_r_of(pa->flags)) return fill_bytes(W, H, C);
    const size_t rec = split_bytes(W, H, C, pa->spp, pa->bounces);
    return rec ? rec : esc_sum_bytes(W, H, C);
}
// ... and, with a box, the walls' direct irradiance after the tail.
inline size_t solve_workspace_bytes(const irtps_problem* pr, const irtps_params* pa) {
    const int W = pr->width, H = pr->height, C = pr->channels, K = pr->num_lights;
    return solve_layout(W, H, C, K).total + tail_bytes(W, H, C, pa) + box_shade_bytes(pr->box, K);
}

inline int check_problem(const irtps_problem* pr, const irtps_params* pa) {
    if (!pr || !pa) return IRTPS_ERR_INVALID_ARG;
    if (!dims_ok(pr->width, pr->height) || !channels_ok(pr->channels) || !lights_ok(pr->num_lights))
        return IRTPS_ERR_INVALID_ARG;
    if (!pr->images_dev || !pr->light_dirs_host || !pr->env_dev || pr->env_h < 1 || pr->env_w < 1)
        return IRTPS_ERR_INVALID_ARG;
    if (pa->spp < 1 || pa->bounces < 0 || pa->bounces > 8 || pa->iterations < 0 ||
        pa->iterations > 1000 || (pa->rho_mode != IRTPS_RHO_FIT && pa->rho_mode != IRTPS_RHO_PREV) ||
        pa->mg_cycles_cold < 0 || pa->mg_cycles_warm < 0 || !(pa->stop_tol >= 0.0f) ||
        !(pa->stop_tol <= 3.0e38f) ||
        (pa->flags & ~(IRTPS_FLAG_QUADRATURE | IRTPS_FLAG_LITERAL_CUMULATIVE | IRTPS_FLAG_FLAT_TRAVERSAL |
                       IRTPS_FLAG_SHADOW_AWARE_PS | IRTPS_FLAG_GRAPH | IRTPS_FLAG_ROBUST_INTEGRATION |
                       IRTPS_FLAG_EXACT_R_MASK)))
        return IRTPS_ERR_INVALID_ARG;
    // the r-ray image is one per solve, the walls' light one per light
    if (pr->box && (!box_ok(pr->box) || kern::exact_r_of(pa->flags))) return IRTPS_ERR_INVALID_ARG;
    return IRTPS_OK;
}


// Pinned host staging for uploads of job tables (per thread).  A buffer is
// reused only after the copy that read it has completed.
struct Staging {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};
inline thread_local Staging g_stage;

inline hipError_t upload(void* dst_dev, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    Staging& S = g_stage;
    hipError_t e = hipSuccess;
    if (S.done) {
        e = hipEventSynchronize(S.done);
        if (e != hipSuccess) return e;
    } else {
        e = hipEventCreateWithFlags(&S.done, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    if (S.cap < bytes) {
        if (S.host) (void)hipHostFree(S.host);
        S.host = nullptr;
        S.cap = 0;
        e = hipHostMalloc(&S.host, bytes, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        S.cap = bytes;
    }
    std::memcpy(S.host, src, bytes);
    e = hipMemcpyAsync(dst_dev, S.host, bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(S.done, st);
    return e;
}

}  // namespace host
}  // namespace irtps
