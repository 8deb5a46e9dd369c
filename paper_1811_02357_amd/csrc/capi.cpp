// capi.cpp -- the C ABI of libirtps (include/irtps.h): validation, workspace
// layout and the host side of the IRT-PS loop (Sec. IV of the paper).
#include "irtps.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <list>
#include <mutex>
#include <vector>

#include "host.hpp"
#include "kernels.hpp"

using namespace irtps;

using namespace irtps::host;

extern "C" {

static_assert(kern::kNumCounters == IRTPS_NUM_COUNTERS, "counter count");

int irtps_abi_version(void) { return IRTPS_ABI_VERSION; }

const char* irtps_status_string(int status) {
    switch (status) {
        case IRTPS_OK: return "ok";
        case IRTPS_ERR_INVALID_ARG: return "invalid argument";
        case IRTPS_ERR_SINGULAR_LIGHTS: return "singular light configuration";
        case IRTPS_ERR_WORKSPACE: return "workspace missing or too small";
        case IRTPS_ERR_OOM: return "job larger than the memory budget";
        case IRTPS_ERR_DEVICE: return "HIP error";
        case IRTPS_ERR_CANCELLED: return "cancelled";
        case IRTPS_ERR_NOT_FOUND: return "unknown job";
        case IRTPS_ERR_BUSY: return "job not finished";
        default: return "unknown status";
    }
}

int irtps_last_hip_error(void) { return g_last_hip; }

int irtps_ps_matrix(int32_t K, const float* light_dirs_host, const float* light_intensity_host,
                    float* M_host) {
    if (K > kern::kMaxLights) return IRTPS_ERR_INVALID_ARG;
    return ps_matrix_host(K, light_dirs_host, light_intensity_host, M_host);
}

int irtps_workspace_bytes(const irtps_problem* problem, const irtps_params* params, size_t* bytes) {
    STATUS_TRY(check_problem(problem, params));
    if (!bytes) return IRTPS_ERR_INVALID_ARG;
    *bytes = solve_workspace_bytes(problem, params);
    return IRTPS_OK;
}

}  // extern "C"

namespace {

// The solve's launches for one (problem, params, outputs, workspace), on st.
int solve_launches(const irtps_problem* pr, const irtps_params* pa, const irtps_outputs* out, void* ws,
                   const kern::PsMatrix& M, const kern::LightSet& Ls, hipStream_t st) {
    const int W = pr->width, H = pr->height, C = pr->channels, K = pr->num_lights;
    const SolveLayout lay = solve_layout(W, H, C, K);
    const int r_exact = kern::exact_r_of(pa->flags);
    const size_t rec_bytes = r_exact ? 0 : split_bytes(W, H, C, pa->spp, pa->bounces);
    char* base = static_cast<char*>(ws);
    float* A = reinterpret_cast<float*>(base + lay.A);
    float* S = reinterpret_cast<float*>(base + lay.S);
    float* G = reinterpret_cast<float*>(base + lay.G);
    float* pyr = reinterpret_cast<float*>(base + lay.pyr);
    float* mg = reinterpret_cast<float*>(base + lay.mg);
    unsigned* tile_cost = reinterpret_cast<unsigned*>(base + lay.tile_cost);
    int* tile_order = reinterpret_cast<int*>(base + lay.tile_order);
    const int npx = W * H;
    const int cold = pa->mg_cycles_cold ? pa->mg_cycles_cold : 8;
    const int warm = pa->mg_cycles_warm ? pa->mg_cycles_warm : 4;
    const bool cumulative = (pa->flags & IRTPS_FLAG_LITERAL_CUMULATIVE) != 0;
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(out->counters_dev);

    kern::Robust robust;  // the M-estimator of stage 1: least squares, or Huber
    if (pa->flags & IRTPS_FLAG_ROBUST_INTEGRATION) {
        robust.delta = kern::kRobustDelta;
        robust.rounds = kern::kRobustRounds;
        robust.cycles = kern::kRobustCycles;
    }

    // the walls' direct light: the lights do not move, so once per solve
    const irtps_box* box = pr->box;
    float* wall_S = box ? reinterpret_cast<float*>(base + lay.total + tail_bytes(W, H, C, pa)) : nullptr;
    if (box) HIP_TRY(kern::box_shade(W, H, box_args(box), Ls, wall_S, st));
    const float box_z = box ? box->height : 0.0f;

    if (cnt) HIP_TRY(kern::fill_u64_zero(cnt, IRTPS_NUM_COUNTERS, st));
    // t = 0: plain photometric stereo and integration (stage 1)
    HIP_TRY(kern::ps_solve(npx, C, K, M, pr->images_dev, out->normals_dev, out->albedo_dev, st));
    HIP_TRY(kern::integrate(lay.plan, out->normals_dev, nullptr, cold, out->depth_dev, mg, st, false, robust));
    if (out->indirect_dev) HIP_TRY(kern::fill_f32(out->indirect_dev, 0.0f, (long long)npx * K * C, st));

    const kern::SurfaceArgs sa = surface(W, H, out->depth_dev, pyr);
    const bool stop = pa->stop_tol > 0.0f;
    int run = 0;  // IRT iterations run
    for (int t = 0; t < pa->iterations; ++t) {
        HIP_TRY(kern::build_pyramid(W, H, out->depth_dev, pyramid_plan(W, H), pyr, sa.quad_off, st));
        HIP_TRY(kern::direct(sa, out->normals_dev, Ls, (pa->flags & IRTPS_FLAG_FLAT_TRAVERSAL) ? 1 : 0, S, st,
                             box_z));
        // stage 5: subtract; the cumulative reading starts from A_0 = I0
        const float* Aprev = (cumulative && t > 0) ? A : pr->images_dev;
        // the last iteration writes E; with a stop rule any iteration may be the last
        float* E = (t == pa->iterations - 1 || stop) ? out->indirect_dev : nullptr;
        if (r_exact) {
            // the r-ray variant: one environment image, its holes filled, as G of every light
            const kern::FillPlan fp = kern::fill_plan(W, H, C);
            float* fill = reinterpret_cast<float*>(base + lay.total);
            float* v0 = fill + fp.v0off;
            HIP_TRY(kern::trace_exact_r(sa, C, out->normals_dev, out->albedo_dev, pr->env_dev, pr->env_h, pr->env_w,
                                        r_exact, t, IRTPS_TAG_SOLVE, (uint32_t)pa->seed, (uint32_t)(pa->seed >> 32),
                                        (pa->flags & IRTPS_FLAG_FLAT_TRAVERSAL) ? 1 : 0, v0, fill + fp.woff[0],
                                        nullptr, st));
            HIP_TRY(kern::fill_pull_push(fp, C, v0, fill, st));
            HIP_TRY(kern::fill_push0_broadcast(fp, C, K, v0, fill, G, st));
            HIP_TRY(kern::correct(npx, C, K, pa->rho_mode, cumulative ? 1 : 0, pr->images_dev, Aprev, G, S,
                                  out->albedo_dev, E, A, st));
        } else {
            kern::TraceArgs ta{};
            ta.sa = sa;
            ta.n = out->normals_dev;
            ta.rho = out->albedo_dev;
            ta.S = S;
            ta.env = pr->env_dev;
            ta.G = G;
            ta.counters = cnt;
            ta.env_h = pr->env_h;
            ta.env_w = pr->env_w;
            ta.C = C;
            ta.K = K;
            ta.spp = pa->spp;
            ta.B = pa->bounces;
            ta.t = t;
            ta.tag = IRTPS_TAG_SOLVE;
            ta.flags = pa->flags & (IRTPS_FLAG_QUADRATURE | IRTPS_FLAG_FLAT_TRAVERSAL);
            ta.key0 = (uint32_t)pa->seed;
            ta.key1 = (uint32_t)(pa->seed >> 32);
            if (box) {
                ta.box_z = box->height;
                ta.box_th = box->tex_h;
                ta.box_tw = box->tex_w;
                ta.box_albedo = box->albedo_dev;
                ta.box_S = wall_S;
            }
            const Schedule sched = schedule_for(W, H, C, K, pa->bounces);
            ta.ready_batch = sched.ready_batch;
            ta.tile_shift = sched.tile_shift;
            // Each launch records its pixels' times per chunk; from the second
            // iteration on, the chunks go out heaviest first by the previous
            // iteration's times, so that the launch ends on short ones (the
            // surface changes little between iterations).
            ta.tile_cost = tile_cost;
            // a small problem traces one path per (pixel, sample) lane instead;
            // a larger one hands its escape sums to the correction, which forms
            // the means
            ta.records = rec_bytes ? reinterpret_cast<float*>(base + lay.total) : nullptr;
            ta.esc_sums = rec_bytes ? nullptr : reinterpret_cast<float*>(base + lay.total);
            if (t > 0 && !ta.records) {
                HIP_TRY(kern::order_tiles(tile_cost, kern::chunks_for(W, H, 1 << sched.tile_shift), tile_order, st));
                ta.order = tile_order;
            }
            HIP_TRY(traced(ta, st));
            HIP_TRY(kern::correct(npx, C, K, pa->rho_mode, cumulative ? 1 : 0, pr->images_dev, Aprev, G, S,
                                  out->albedo_dev, E, A, st, ta.esc_sums, pa->spp));
        }
        if (pa->flags & IRTPS_FLAG_SHADOW_AWARE_PS)  // per pixel, the lights that reach it (S of H_t, n_t)
            HIP_TRY(kern::ps_solve_masked(npx, C, K, M, Ls, A, S, out->normals_dev, out->albedo_dev, st));
        else
            HIP_TRY(kern::ps_solve(npx, C, K, M, A, out->normals_dev, out->albedo_dev, st));
        HIP_TRY(kern::integrate(lay.plan, out->normals_dev, out->depth_dev, warm, out->depth_dev, mg, st, stop,
                                robust));
        ++run;
        if (stop) {
            // the paper's stop rule: D_H = max |H_{t+1} - H_t| below the tolerance
            unsigned bits = 0;
            HIP_TRY(hipMemcpyAsync(&bits, kern::change_key_of(lay.plan, mg), sizeof(bits), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            float dh;
            std::memcpy(&dh, &bits, sizeof(dh));
            if (dh < pa->stop_tol) break;
        }
    }
    if (cnt) HIP_TRY(kern::add_u64(cnt + 4, (unsigned long long)run, st));
    return IRTPS_OK;
}

// ---- hipGraph cache of whole solves ----------------------------------------
// A solve with IRTPS_FLAG_GRAPH is captured once into a graph keyed by every
// value its launches depend on (the problem, params, output and workspace
// pointers, the lights and the tracer schedule); a later call with the same key
// replays it.  Most recent first, at most kMaxSolveGraphs.
struct SolveGraph {
    std::vector<char> key;
    hipGraphExec_t exec = nullptr;
};
std::mutex g_solve_graph_mu;
std::list<SolveGraph> g_solve_graphs;
constexpr size_t kMaxSolveGraphs = 8;

template <class T>
void put(std::vector<char>& k, const T& v) {
    const char* p = reinterpret_cast<const char*>(&v);
    k.insert(k.end(), p, p + sizeof(T));
}

std::vector<char> solve_key(const irtps_problem* pr, const irtps_params* pa, const irtps_outputs* out, void* ws,
                            const kern::PsMatrix& M, const kern::LightSet& Ls) {
    std::vector<char> k;
    put(k, *pr);
    put(k, *pa);
    put(k, *out);
    put(k, ws);
    put(k, M);
    put(k, Ls);
    if (pr->box) put(k, *pr->box);  // the problem holds only its host address
    const Schedule sc = schedule_for(pr->width, pr->height, pr->channels, pr->num_lights, pa->bounces);
    put(k, sc.tile_shift);
    put(k, sc.ready_batch);
    return k;
}

int solve_graphed(const irtps_problem* pr, const irtps_params* pa, const irtps_outputs* out, void* ws,
                  const kern::PsMatrix& M, const kern::LightSet& Ls, hipStream_t st) {
    std::vector<char> key = solve_key(pr, pa, out, ws, M, Ls);
    std::lock_guard<std::mutex> lock(g_solve_graph_mu);
    for (auto it = g_solve_graphs.begin(); it != g_solve_graphs.end(); ++it) {
        if (it->key == key) {
            g_solve_graphs.splice(g_solve_graphs.begin(), g_solve_graphs, it);
            HIP_TRY(hipGraphLaunch(g_solve_graphs.front().exec, st));
            return IRTPS_OK;
        }
    }
    // the tracer's timing events are not captured
    const bool prof = g_prof.on;
    g_prof.on = false;
    hipGraph_t graph = nullptr;
    hipError_t eb = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) {
        g_prof.on = prof;
        return hip_fail(eb);
    }
    const int rc = solve_launches(pr, pa, out, ws, M, Ls, st);
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    g_prof.on = prof;
    if (rc != IRTPS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess) return hip_fail(ec);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return hip_fail(ei);
    g_solve_graphs.push_front(SolveGraph{std::move(key), exec});
    while (g_solve_graphs.size() > kMaxSolveGraphs) {
        (void)hipGraphExecDestroy(g_solve_graphs.back().exec);
        g_solve_graphs.pop_back();
    }
    HIP_TRY(hipGraphLaunch(exec, st));
    return IRTPS_OK;
}

}  // namespace

extern "C" {

int irtps_solve(const irtps_problem* pr, const irtps_params* pa, const irtps_outputs* out, void* ws,
                size_t ws_bytes, void* stream) {
    STATUS_TRY(check_problem(pr, pa));
    if (!out || !out->normals_dev || !out->albedo_dev || !out->depth_dev) return IRTPS_ERR_INVALID_ARG;
    const int K = pr->num_lights;
    if (!ws || ws_bytes < solve_workspace_bytes(pr, pa) || (reinterpret_cast<uintptr_t>(ws) % kAlign))
        return IRTPS_ERR_WORKSPACE;
    const bool graph = (pa->flags & IRTPS_FLAG_GRAPH) != 0;
    // a graph cannot hold the stop rule's read-back, nor run on the legacy stream
    if (graph && (pa->stop_tol > 0.0f || stream == nullptr)) return IRTPS_ERR_INVALID_ARG;
    kern::PsMatrix M;
    kern::LightSet Ls;
    STATUS_TRY(make_psmatrix(K, pr->light_dirs_host, pr->light_intensity_host, M));
    STATUS_TRY(make_lights(K, pr->light_dirs_host, pr->light_intensity_host, Ls));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return graph ? solve_graphed(pr, pa, out, ws, M, Ls, st) : solve_launches(pr, pa, out, ws, M, Ls, st);
}

int irtps_ps_solve(int32_t W, int32_t H, int32_t C, int32_t K, const float* light_dirs_host,
                   const float* light_intensity_host, const float* A_dev, float* normals_dev,
                   float* albedo_dev, void* stream) {
    if (!dims_ok(W, H) || !channels_ok(C) || !A_dev || !normals_dev || !albedo_dev) return IRTPS_ERR_INVALID_ARG;
    kern::PsMatrix M;
    STATUS_TRY(make_psmatrix(K, light_dirs_host, light_intensity_host, M));
    HIP_TRY(kern::ps_solve(W * H, C, K, M, A_dev, normals_dev, albedo_dev, reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_ps_solve_masked(int32_t W, int32_t H, int32_t C, int32_t K, const float* light_dirs_host,
                          const float* light_intensity_host, const float* A_dev, const float* S_dev,
                          float* normals_dev, float* albedo_dev, void* stream) {
    if (!dims_ok(W, H) || !channels_ok(C) || !A_dev || !S_dev || !normals_dev || !albedo_dev)
        return IRTPS_ERR_INVALID_ARG;
    kern::PsMatrix M;
    kern::LightSet Ls;
    STATUS_TRY(make_psmatrix(K, light_dirs_host, light_intensity_host, M));
    STATUS_TRY(make_lights(K, light_dirs_host, light_intensity_host, Ls));
    HIP_TRY(kern::ps_solve_masked(W * H, C, K, M, Ls, A_dev, S_dev, normals_dev, albedo_dev,
                                  reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_integrate_workspace_bytes(int32_t W, int32_t H, size_t* bytes) {
    if (!dims_ok(W, H) || !bytes) return IRTPS_ERR_INVALID_ARG;
    *bytes = align_up(sizeof(float) * (size_t)mg_plan(W, H).total);
    return IRTPS_OK;
}

int irtps_integrate(int32_t W, int32_t H, const float* normals_dev, const float* depth_init_dev,
                    int32_t cycles, float* depth_dev, void* ws_dev, size_t ws_bytes, void* stream) {
    if (!dims_ok(W, H) || !normals_dev || !depth_dev || cycles < 0) return IRTPS_ERR_INVALID_ARG;
    const kern::MgPlan plan = mg_plan(W, H);
    if (!ws_dev || ws_bytes < sizeof(float) * (size_t)plan.total || (reinterpret_cast<uintptr_t>(ws_dev) % kAlign))
        return IRTPS_ERR_WORKSPACE;
    HIP_TRY(kern::integrate(plan, normals_dev, depth_init_dev, cycles, depth_dev, static_cast<float*>(ws_dev),
                            reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_integrate_robust(int32_t W, int32_t H, const float* normals_dev, const float* depth_init_dev,
                           int32_t cycles, float delta, int32_t rounds, int32_t rcycles, float* depth_dev,
                           void* ws_dev, size_t ws_bytes, void* stream) {
    if (!dims_ok(W, H) || !normals_dev || !depth_dev || cycles < 0 || rounds < 0 || rcycles < 0 ||
        !(delta >= 0.0f) || !(delta <= 3.0e38f))
        return IRTPS_ERR_INVALID_ARG;
    const kern::MgPlan plan = mg_plan(W, H);
    if (!ws_dev || ws_bytes < sizeof(float) * (size_t)plan.total || (reinterpret_cast<uintptr_t>(ws_dev) % kAlign))
        return IRTPS_ERR_WORKSPACE;
    kern::Robust robust;
    robust.delta = delta;
    robust.rounds = rounds;
    robust.cycles = rcycles;
    HIP_TRY(kern::integrate(plan, normals_dev, depth_init_dev, cycles, depth_dev, static_cast<float*>(ws_dev),
                            reinterpret_cast<hipStream_t>(stream), false, robust));
    return IRTPS_OK;
}

int irtps_pyramid_bytes(int32_t W, int32_t H, size_t* bytes) {
    if (!dims_ok(W, H) || !bytes) return IRTPS_ERR_INVALID_ARG;
    *bytes = sizeof(float) * (size_t)pyramid_floats(W, H);
    return IRTPS_OK;
}

int irtps_build_pyramid(int32_t W, int32_t H, const float* depth_dev, float* pyramid_dev, void* stream) {
    if (!dims_ok(W, H) || !depth_dev || !pyramid_dev) return IRTPS_ERR_INVALID_ARG;
    const trv::Pyramid P = pyramid_plan(W, H);
    HIP_TRY(kern::build_pyramid(W, H, depth_dev, P, pyramid_dev, pyramid_level_floats(P),
                                reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_direct(int32_t W, int32_t H, int32_t K, const float* depth_dev, const float* normals_dev,
                 const float* light_dirs_host, const float* light_intensity_host, const float* pyramid_dev,
                 float* S_dev, const irtps_box* box, void* stream) {
    if (!dims_ok(W, H) || !depth_dev || !normals_dev || !pyramid_dev || !S_dev) return IRTPS_ERR_INVALID_ARG;
    if (box && !(box->height > 0.0f && box->height <= 3.0e38f)) return IRTPS_ERR_INVALID_ARG;
    kern::LightSet Ls;
    STATUS_TRY(make_lights(K, light_dirs_host, light_intensity_host, Ls));
    HIP_TRY(kern::direct(surface(W, H, depth_dev, pyramid_dev), normals_dev, Ls, 0, S_dev,
                         reinterpret_cast<hipStream_t>(stream), box ? box->height : 0.0f));
    return IRTPS_OK;
}

int irtps_box_shade(int32_t W, int32_t H, int32_t K, const irtps_box* box, const float* light_dirs_host,
                    const float* light_intensity_host, float* wall_S_dev, void* stream) {
    if (!dims_ok(W, H) || !box_ok(box) || !wall_S_dev) return IRTPS_ERR_INVALID_ARG;
    kern::LightSet Ls;
    STATUS_TRY(make_lights(K, light_dirs_host, light_intensity_host, Ls));
    HIP_TRY(kern::box_shade(W, H, box_args(box), Ls, wall_S_dev, reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_trace(int32_t W, int32_t H, int32_t C, int32_t K, const float* depth_dev, const float* normals_dev,
                const float* albedo_dev, const float* S_dev, const float* env_dev, int32_t env_h,
                int32_t env_w, const float* pyramid_dev, int32_t spp, int32_t B, uint64_t seed, int32_t t,
                int32_t tag, int32_t flags, float* G_dev, uint64_t* counters_dev, const irtps_box* box,
                const float* wall_S_dev, void* stream) {
    if (!dims_ok(W, H) || !channels_ok(C) || !lights_ok(K) || !depth_dev || !normals_dev || !albedo_dev ||
        !S_dev || !env_dev || env_h < 1 || env_w < 1 || !pyramid_dev || spp < 1 || B < 0 || B > 8 || t < 0 ||
        t >= (1 << 23) || tag < 0 || !G_dev ||
        (flags & ~(IRTPS_FLAG_QUADRATURE | IRTPS_FLAG_FLAT_TRAVERSAL)) || (box && (!box_ok(box) || !wall_S_dev)))
        return IRTPS_ERR_INVALID_ARG;
    kern::TraceArgs ta{};
    ta.sa = surface(W, H, depth_dev, pyramid_dev);
    ta.n = normals_dev;
    ta.rho = albedo_dev;
    ta.S = S_dev;
    ta.env = env_dev;
    ta.G = G_dev;
    ta.counters = reinterpret_cast<unsigned long long*>(counters_dev);
    ta.env_h = env_h;
    ta.env_w = env_w;
    ta.C = C;
    ta.K = K;
    ta.spp = spp;
    ta.B = B;
    ta.t = t;
    ta.tag = tag;
    ta.flags = flags;
    ta.key0 = (uint32_t)seed;
    ta.key1 = (uint32_t)(seed >> 32);
    if (box) {
        ta.box_z = box->height;
        ta.box_th = box->tex_h;
        ta.box_tw = box->tex_w;
        ta.box_albedo = box->albedo_dev;
        ta.box_S = wall_S_dev;
    }
    const Schedule sched = schedule_for(W, H, C, K, B);
    ta.ready_batch = sched.ready_batch;
    ta.tile_shift = sched.tile_shift;
    HIP_TRY(traced(ta, reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_trace_exact_r(int32_t W, int32_t H, int32_t C, const float* depth_dev, const float* normals_dev,
                        const float* albedo_dev, const float* env_dev, int32_t env_h, int32_t env_w,
                        const float* pyramid_dev, int32_t r, uint64_t seed, int32_t t, int32_t tag, int32_t flags,
                        float* E_dev, unsigned char* valid_dev, void* stream) {
    if (!dims_ok(W, H) || !channels_ok(C) || !depth_dev || !normals_dev || !albedo_dev || !env_dev || env_h < 1 ||
        env_w < 1 || !pyramid_dev || r < 1 || r > 7 || t < 0 || t >= (1 << 23) || tag < 0 || !E_dev ||
        (flags & ~IRTPS_FLAG_FLAT_TRAVERSAL))
        return IRTPS_ERR_INVALID_ARG;
    HIP_TRY(kern::trace_exact_r(surface(W, H, depth_dev, pyramid_dev), C, normals_dev, albedo_dev, env_dev, env_h,
                                env_w, r, t, tag, (uint32_t)seed, (uint32_t)(seed >> 32),
                                (flags & IRTPS_FLAG_FLAT_TRAVERSAL) ? 1 : 0, E_dev, nullptr, valid_dev,
                                reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_fill_workspace_bytes(int32_t W, int32_t H, int32_t C, size_t* bytes) {
    if (!dims_ok(W, H) || !channels_ok(C) || !bytes) return IRTPS_ERR_INVALID_ARG;
    *bytes = align_up(sizeof(float) * (size_t)kern::fill_plan(W, H, C).total);
    return IRTPS_OK;
}

int irtps_fill_missing(int32_t W, int32_t H, int32_t C, float* E_dev, const unsigned char* valid_dev, void* ws_dev,
                       size_t ws_bytes, void* stream) {
    if (!dims_ok(W, H) || !channels_ok(C) || !E_dev || !valid_dev) return IRTPS_ERR_INVALID_ARG;
    const kern::FillPlan fp = kern::fill_plan(W, H, C);
    if (!ws_dev || ws_bytes < sizeof(float) * (size_t)fp.total || (reinterpret_cast<uintptr_t>(ws_dev) % kAlign))
        return IRTPS_ERR_WORKSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    float* ws = static_cast<float*>(ws_dev);
    HIP_TRY(kern::fill_weights((long long)W * H, valid_dev, ws + fp.woff[0], st));
    HIP_TRY(kern::fill_pull_push(fp, C, E_dev, ws, st));
    HIP_TRY(kern::fill_push0(fp, C, E_dev, ws, st));
    return IRTPS_OK;
}

int irtps_correct(int32_t W, int32_t H, int32_t C, int32_t K, int32_t rho_mode, int32_t flags,
                  const float* I0_dev, const float* A_prev_dev, const float* G_dev, const float* S_dev,
                  const float* albedo_dev, float* E_dev, float* A_next_dev, void* stream) {
    const bool cumulative = (flags & IRTPS_FLAG_LITERAL_CUMULATIVE) != 0;
    if (!dims_ok(W, H) || !channels_ok(C) || !lights_ok(K) || !I0_dev || !G_dev || !S_dev || !albedo_dev ||
        !A_next_dev || (cumulative && !A_prev_dev) || (rho_mode != IRTPS_RHO_FIT && rho_mode != IRTPS_RHO_PREV))
        return IRTPS_ERR_INVALID_ARG;
    HIP_TRY(kern::correct(W * H, C, K, rho_mode, cumulative ? 1 : 0, I0_dev, cumulative ? A_prev_dev : I0_dev,
                          G_dev, S_dev, albedo_dev, E_dev, A_next_dev, reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_render_workspace_bytes(int32_t W, int32_t H, int32_t C, int32_t K, const irtps_box* box,
                                 size_t* bytes) {
    if (!dims_ok(W, H) || !channels_ok(C) || !lights_ok(K) || !bytes || (box && !box_ok(box)))
        return IRTPS_ERR_INVALID_ARG;
    const size_t npx = (size_t)W * H;
    *bytes = align_up(sizeof(float) * npx * K) + align_up(sizeof(float) * npx * K * C) +
             align_up(sizeof(float) * (size_t)pyramid_floats(W, H)) + box_shade_bytes(box, K);
    return IRTPS_OK;
}

int irtps_render(int32_t W, int32_t H, int32_t C, int32_t K, const float* depth_dev, const float* normals_dev,
                 const float* albedo_dev, const float* light_dirs_host, const float* light_intensity_host,
                 const float* env_dev, int32_t env_h, int32_t env_w, int32_t spp, int32_t B, uint64_t seed,
                 float* images_dev, void* ws_dev, size_t ws_bytes, const irtps_box* box, void* stream) {
    size_t need = 0;
    STATUS_TRY(irtps_render_workspace_bytes(W, H, C, K, box, &need));
    if (!depth_dev || !normals_dev || !albedo_dev || !env_dev || env_h < 1 || env_w < 1 || !images_dev ||
        spp < 1 || B < 0 || B > 8)
        return IRTPS_ERR_INVALID_ARG;
    if (!ws_dev || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws_dev) % kAlign)) return IRTPS_ERR_WORKSPACE;
    kern::LightSet Ls;
    STATUS_TRY(make_lights(K, light_dirs_host, light_intensity_host, Ls));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t npx = (size_t)W * H;
    char* base = static_cast<char*>(ws_dev);
    float* S = reinterpret_cast<float*>(base);
    float* G = reinterpret_cast<float*>(base + align_up(sizeof(float) * npx * K));
    float* pyr = reinterpret_cast<float*>(base + align_up(sizeof(float) * npx * K) + align_up(sizeof(float) * npx * K * C));
    float* wall_S = reinterpret_cast<float*>(reinterpret_cast<char*>(pyr) +
                                             align_up(sizeof(float) * (size_t)pyramid_floats(W, H)));
    const kern::SurfaceArgs sa = surface(W, H, depth_dev, pyr);
    HIP_TRY(kern::build_pyramid(W, H, depth_dev, pyramid_plan(W, H), pyr, sa.quad_off, st));
    HIP_TRY(kern::direct(sa, normals_dev, Ls, 0, S, st, box ? box->height : 0.0f));
    kern::TraceArgs ta{};
    if (box) {
        HIP_TRY(kern::box_shade(W, H, box_args(box), Ls, wall_S, st));
        ta.box_z = box->height;
        ta.box_th = box->tex_h;
        ta.box_tw = box->tex_w;
        ta.box_albedo = box->albedo_dev;
        ta.box_S = wall_S;
    }
    ta.sa = sa;
    ta.n = normals_dev;
    ta.rho = albedo_dev;
    ta.S = S;
    ta.env = env_dev;
    ta.G = G;
    ta.counters = nullptr;
    ta.env_h = env_h;
    ta.env_w = env_w;
    ta.C = C;
    ta.K = K;
    ta.spp = spp;
    ta.B = B;
    ta.t = 0;
    ta.tag = IRTPS_TAG_RENDER;
    ta.flags = 0;
    ta.key0 = (uint32_t)seed;
    ta.key1 = (uint32_t)(seed >> 32);
    const Schedule sched = schedule_for(W, H, C, K, B);
    ta.ready_batch = sched.ready_batch;
    ta.tile_shift = sched.tile_shift;
    HIP_TRY(traced(ta, st));
    HIP_TRY(kern::compose((int)npx, C, K, albedo_dev, S, G, images_dev, st));
    return IRTPS_OK;
}



int irtps_profile_begin(void) {
    for (auto& pr : g_prof.ev) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    g_prof.ev.clear();
    g_prof.on = true;
    return IRTPS_OK;
}

int irtps_profile_end(double* trace_ms, int64_t* launches) {
    double total = 0.0;
    hipError_t err = hipSuccess;
    for (auto& pr : g_prof.ev) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(pr.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (e != hipSuccess && err == hipSuccess) err = e;
        total += ms;
    }
    const int64_t n = (int64_t)g_prof.ev.size();
    for (auto& pr : g_prof.ev) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    g_prof.ev.clear();
    g_prof.on = false;
    if (trace_ms) *trace_ms = total;
    if (launches) *launches = n;
    if (err != hipSuccess) return hip_fail(err);
    return IRTPS_OK;
}

int irtps_probe_valu(int32_t blocks, int32_t iters, int32_t active_lanes, int32_t kind, uint32_t* out_dev,
                     void* stream) {
    if (blocks < 1 || blocks > (1 << 24) || iters < 0 || active_lanes < 1 || active_lanes > 64 || kind < 0 ||
        kind > 2 || !out_dev)
        return IRTPS_ERR_INVALID_ARG;
    HIP_TRY(kern::probe_valu(blocks, iters, active_lanes, kind, out_dev, reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_probe_philox(int64_t count, const uint32_t* ctr_dev, uint64_t seed, uint32_t* out_dev, void* stream) {
    if (count < 0 || (count > 0 && (!ctr_dev || !out_dev))) return IRTPS_ERR_INVALID_ARG;
    HIP_TRY(kern::probe_philox(count, ctr_dev, (uint32_t)seed, (uint32_t)(seed >> 32), out_dev,
                               reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_probe_sample(int64_t count, const float* normals_dev, const float* u_dev, float* dirs_dev, void* stream) {
    if (count < 0 || (count > 0 && (!normals_dev || !u_dev || !dirs_dev))) return IRTPS_ERR_INVALID_ARG;
    HIP_TRY(kern::probe_sample(count, normals_dev, u_dev, dirs_dev, reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_probe_env_texel(int64_t count, const float* dirs_dev, int32_t env_h, int32_t env_w, int32_t* rc_dev,
                          void* stream) {
    if (count < 0 || env_h < 1 || env_w < 1 || (count > 0 && (!dirs_dev || !rc_dev))) return IRTPS_ERR_INVALID_ARG;
    HIP_TRY(kern::probe_env(count, dirs_dev, env_h, env_w, rc_dev, reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

int irtps_probe_traverse(int32_t W, int32_t H, const float* depth_dev, const float* pyramid_dev, int32_t flat,
                         int64_t count, const int32_t* ij_dev, const float* dirs_dev, int32_t* q_dev,
                         void* stream) {
    if (!dims_ok(W, H) || !depth_dev || !pyramid_dev || count < 0 || (count > 0 && (!ij_dev || !dirs_dev || !q_dev)))
        return IRTPS_ERR_INVALID_ARG;
    HIP_TRY(kern::probe_traverse(surface(W, H, depth_dev, pyramid_dev), flat, count, ij_dev, dirs_dev, q_dev,
                                 reinterpret_cast<hipStream_t>(stream)));
    return IRTPS_OK;
}

}  // extern "C"
