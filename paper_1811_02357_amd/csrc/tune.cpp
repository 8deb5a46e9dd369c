// tune.cpp -- the tracer's schedule: lookup, forcing, autotuning, persistence.
//
// A schedule is the tracer's tile shape (2^s x 256/2^s pixels per 256-thread
// block) and the number of lanes of a wave that must hold a finished segment
// before the wave shades (the rays-per-wave batch).  Neither changes a result
// bit: each lane's pixel, its random numbers and the order of its sums are the
// same under every schedule.  The autotuner times the candidates on the caller's
// own problem and keeps the fastest per class (device architecture, image side
// class, light-count class, channels, bounces); the table persists as JSON.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "host.hpp"
#include "irtps.h"

namespace irtps {
namespace host {

namespace {

constexpr int kDefaultShift = 4;   // 16 x 16 tiles
constexpr int kDefaultBatch = 32;  // half a wave
constexpr int kShifts[] = {3, 4, 5, 6};
constexpr int kBatches[] = {24, 32, 40, 48, 56};
constexpr int kRepeats = 2;

struct Key {
    int side, kcls, C, B;
    bool operator<(const Key& o) const {
        return std::tie(side, kcls, C, B) < std::tie(o.side, o.kcls, o.C, o.B);
    }
};

struct Entry {
    Schedule s;
    float ms;
};

std::mutex g_mu;
std::map<Key, Entry> g_table;  // entries for this process's device architecture
int g_forced_shift = 0;        // 0: automatic
int g_forced_batch = 0;

int ceil_log2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

Key key_for(int W, int H, int C, int K, int B) {
    // side class: log2 of the geometric-mean side, rounded
    const int side = (int)std::lround(0.5 * std::log2((double)W * (double)H));
    return Key{side, ceil_log2(K), C, std::min(std::max(B, 1), 8)};
}

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "none";
    }
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);  // drop feature suffixes
}

// Minimal reader for the JSON this file writes: an "arch" string and an
// "entries" array of flat objects with integer or number fields.
bool read_number(const std::string& obj, const char* name, double& out) {
    const std::string k = std::string("\"") + name + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return false;
    char* end = nullptr;
    out = std::strtod(obj.c_str() + p + 1, &end);
    return end != obj.c_str() + p + 1;
}

bool read_string(const std::string& text, const char* name, std::string& out) {
    const std::string k = std::string("\"") + name + "\"";
    size_t p = text.find(k);
    if (p == std::string::npos) return false;
    p = text.find(':', p + k.size());
    if (p == std::string::npos) return false;
    const size_t q0 = text.find('"', p + 1);
    if (q0 == std::string::npos) return false;
    const size_t q1 = text.find('"', q0 + 1);
    if (q1 == std::string::npos) return false;
    out = text.substr(q0 + 1, q1 - q0 - 1);
    return true;
}

bool valid(const Schedule& s) {
    return s.tile_shift >= 3 && s.tile_shift <= 6 && s.ready_batch >= 1 && s.ready_batch <= 64;
}

}  // namespace

Schedule schedule_for(int W, int H, int C, int K, int B) {
    Schedule s{kDefaultShift, kDefaultBatch};
    std::lock_guard<std::mutex> lk(g_mu);
    const auto it = g_table.find(key_for(W, H, C, K, B));
    if (it != g_table.end()) s = it->second.s;
    if (g_forced_shift) s.tile_shift = g_forced_shift;
    if (g_forced_batch) s.ready_batch = g_forced_batch;
    return s;
}

}  // namespace host
}  // namespace irtps

using namespace irtps;
using namespace irtps::host;

extern "C" {

int irtps_set_schedule(int32_t tile_w, int32_t ready_batch) {
    int shift = 0;
    if (tile_w != 0) {
        if (tile_w < 8 || tile_w > 64 || (tile_w & (tile_w - 1))) return IRTPS_ERR_INVALID_ARG;
        while ((1 << shift) < tile_w) ++shift;
    }
    if (ready_batch < 0 || ready_batch > 64) return IRTPS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    g_forced_shift = shift;
    g_forced_batch = ready_batch;
    return IRTPS_OK;
}

int irtps_get_schedule(int32_t W, int32_t H, int32_t C, int32_t K, int32_t B, irtps_schedule* out) {
    if (!out || !dims_ok(W, H) || !channels_ok(C) || !lights_ok(K) || B < 0) return IRTPS_ERR_INVALID_ARG;
    const Schedule s = schedule_for(W, H, C, K, B);
    out->tile_w = 1 << s.tile_shift;
    out->ready_batch = s.ready_batch;
    return IRTPS_OK;
}

int irtps_set_ready_batch(int32_t lanes) {
    if (lanes < 0 || lanes > 64) return IRTPS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    g_forced_batch = lanes;
    return IRTPS_OK;
}

int irtps_get_ready_batch(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_forced_batch;
}

int irtps_tuning_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    return IRTPS_OK;
}

int irtps_tuning_entries(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    return (int)g_table.size();
}

int irtps_tuning_save(const char* path) {
    if (!path) return IRTPS_ERR_INVALID_ARG;
    const std::string arch = arch_name();
    std::lock_guard<std::mutex> lk(g_mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return IRTPS_ERR_INVALID_ARG;
    std::fprintf(f, "{\n  \"arch\": \"%s\",\n  \"entries\": [", arch.c_str());
    bool first = true;
    for (const auto& kv : g_table) {
        std::fprintf(f, "%s\n    {\"side\": %d, \"kcls\": %d, \"C\": %d, \"B\": %d, \"tile_w\": %d, "
                     "\"ready_batch\": %d, \"ms\": %.4f}",
                     first ? "" : ",", kv.first.side, kv.first.kcls, kv.first.C, kv.first.B,
                     1 << kv.second.s.tile_shift, kv.second.s.ready_batch, (double)kv.second.ms);
        first = false;
    }
    std::fprintf(f, "\n  ]\n}\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? IRTPS_OK : IRTPS_ERR_INVALID_ARG;
}

int irtps_tuning_load(const char* path, int32_t* loaded) {
    if (!path) return IRTPS_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "r");
    if (!f) return IRTPS_ERR_INVALID_ARG;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    std::fclose(f);
    std::string arch;
    if (!read_string(text, "arch", arch)) return IRTPS_ERR_INVALID_ARG;
    int count = 0;
    if (arch == arch_name()) {
        const size_t e0 = text.find("\"entries\"");
        size_t p = e0 == std::string::npos ? std::string::npos : text.find('[', e0);
        std::lock_guard<std::mutex> lk(g_mu);
        while (p != std::string::npos) {
            const size_t o0 = text.find('{', p);
            if (o0 == std::string::npos) break;
            const size_t o1 = text.find('}', o0);
            if (o1 == std::string::npos) break;
            const std::string obj = text.substr(o0, o1 - o0 + 1);
            double side, kcls, C, B, tw, rb, ms = 0.0;
            if (read_number(obj, "side", side) && read_number(obj, "kcls", kcls) && read_number(obj, "C", C) &&
                read_number(obj, "B", B) && read_number(obj, "tile_w", tw) &&
                read_number(obj, "ready_batch", rb)) {
                (void)read_number(obj, "ms", ms);
                int shift = 0;
                while ((1 << shift) < (int)tw) ++shift;
                const Schedule s{shift, (int)rb};
                if (valid(s) && (1 << shift) == (int)tw) {
                    g_table[Key{(int)side, (int)kcls, (int)C, (int)B}] = Entry{s, (float)ms};
                    ++count;
                }
            }
            p = o1 + 1;
        }
    }
    if (loaded) *loaded = count;
    return IRTPS_OK;
}

int irtps_autotune(const irtps_problem* pr, const irtps_params* pa, const irtps_outputs* out, void* ws_dev,
                   size_t ws_bytes, void* stream, irtps_schedule* best, float* ms) {
    STATUS_TRY(check_problem(pr, pa));
    if (!out || !out->normals_dev || !out->albedo_dev || !out->depth_dev || !ws_dev) return IRTPS_ERR_INVALID_ARG;
    const int W = pr->width, H = pr->height, C = pr->channels, K = pr->num_lights;
    const SolveLayout lay = solve_layout(W, H, C, K);
    if (ws_bytes < lay.total || (reinterpret_cast<uintptr_t>(ws_dev) % kAlign)) return IRTPS_ERR_INVALID_ARG;
    if (pa->bounces < 1) return IRTPS_ERR_INVALID_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws_dev);
    float* A = reinterpret_cast<float*>(base + lay.A);
    float* S = reinterpret_cast<float*>(base + lay.S);
    float* G = reinterpret_cast<float*>(base + lay.G);
    float* pyr = reinterpret_cast<float*>(base + lay.pyr);
    float* mg = reinterpret_cast<float*>(base + lay.mg);
    unsigned* tile_cost = reinterpret_cast<unsigned*>(base + lay.tile_cost);
    int* tile_order = reinterpret_cast<int*>(base + lay.tile_order);
    const long long npx = (long long)W * H;
    const int flat = (pa->flags & IRTPS_FLAG_FLAT_TRAVERSAL) ? 1 : 0;

    // t = 0: PS of the inputs, integrated
    kern::PsMatrix M;
    kern::LightSet L;
    STATUS_TRY(make_psmatrix(K, pr->light_dirs_host, pr->light_intensity_host, M));
    STATUS_TRY(make_lights(K, pr->light_dirs_host, pr->light_intensity_host, L));
    HIP_TRY(kern::ps_solve((int)npx, C, K, M, pr->images_dev, out->normals_dev, out->albedo_dev, st));
    HIP_TRY(kern::integrate(lay.plan, out->normals_dev, nullptr, pa->mg_cycles_cold ? pa->mg_cycles_cold : 8,
                            out->depth_dev, mg, st));
    const long long quad = pyramid_level_floats(pyramid_plan(W, H));
    HIP_TRY(kern::build_pyramid(W, H, out->depth_dev, pyramid_plan(W, H), pyr, quad, st));
    const kern::SurfaceArgs sa = surface(W, H, out->depth_dev, pyr);
    HIP_TRY(kern::direct(sa, out->normals_dev, L, flat, S, st));

    kern::TraceArgs ta;
    std::memset(&ta, 0, sizeof(ta));
    ta.sa = sa;
    ta.n = out->normals_dev;
    ta.rho = out->albedo_dev;
    ta.S = S;
    ta.env = pr->env_dev;
    ta.G = G;
    ta.counters = nullptr;
    ta.env_h = pr->env_h;
    ta.env_w = pr->env_w;
    ta.C = C;
    ta.K = K;
    ta.spp = pa->spp;
    ta.B = pa->bounces;
    ta.t = 0;
    ta.tag = IRTPS_TAG_SOLVE;
    ta.flags = pa->flags & (IRTPS_FLAG_QUADRATURE | IRTPS_FLAG_FLAT_TRAVERSAL);
    ta.key0 = (uint32_t)pa->seed;
    ta.key1 = (uint32_t)(pa->seed >> 32);
    ta.tile_shift = kDefaultShift;
    ta.ready_batch = kDefaultBatch;

    // One IRT iteration with the default schedule, so that the candidates are
    // timed on the state the solve's later iterations trace (H_1, n_1, rho_1):
    // its surface is much closer to the final one than H_0, and those
    // iterations are most of a solve's tracing.
    HIP_TRY(kern::trace(ta, st));
    HIP_TRY(kern::correct((int)npx, C, K, pa->rho_mode, (pa->flags & IRTPS_FLAG_LITERAL_CUMULATIVE) ? 1 : 0,
                          pr->images_dev, pr->images_dev, G, S, out->albedo_dev, nullptr, A, st));
    if (pa->flags & IRTPS_FLAG_SHADOW_AWARE_PS)
        HIP_TRY(kern::ps_solve_masked((int)npx, C, K, M, L, A, S, out->normals_dev, out->albedo_dev, st));
    else
        HIP_TRY(kern::ps_solve((int)npx, C, K, M, A, out->normals_dev, out->albedo_dev, st));
    HIP_TRY(kern::integrate(lay.plan, out->normals_dev, out->depth_dev, pa->mg_cycles_warm ? pa->mg_cycles_warm : 4,
                            out->depth_dev, mg, st));
    HIP_TRY(kern::build_pyramid(W, H, out->depth_dev, pyramid_plan(W, H), pyr, quad, st));
    HIP_TRY(kern::direct(sa, out->normals_dev, L, flat, S, st));
    ta.t = 1;
    ta.tile_cost = tile_cost;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(err);
    }
    Schedule pick{kDefaultShift, kDefaultBatch};
    float pick_ms = 0.0f;
    int cand = 0;
    for (int shift : kShifts) {
        for (int rb : kBatches) {
            if (err != hipSuccess) break;
            ta.tile_shift = shift;
            ta.ready_batch = rb;
            // as in the solve: a launch in row-major order records the chunks'
            // times, the timed launches deal the chunks heaviest first
            ta.order = nullptr;
            err = kern::trace(ta, st);
            if (err == hipSuccess) err = kern::order_tiles(tile_cost, kern::chunks_for(W, H, 1 << shift), tile_order, st);
            ta.order = tile_order;
            float t_ms = 0.0f;
            for (int rep = 0; rep < kRepeats && err == hipSuccess; ++rep) {  // the faster of two
                err = hipEventRecord(e0, st);
                if (err == hipSuccess) err = kern::trace(ta, st);
                if (err == hipSuccess) err = hipEventRecord(e1, st);
                if (err == hipSuccess) err = hipEventSynchronize(e1);
                float r_ms = 0.0f;
                if (err == hipSuccess) err = hipEventElapsedTime(&r_ms, e0, e1);
                if (rep == 0 || r_ms < t_ms) t_ms = r_ms;
            }
            if (err != hipSuccess) break;
            if (ms) ms[cand] = t_ms;
            if (cand == 0 || t_ms < pick_ms) {
                pick = Schedule{shift, rb};
                pick_ms = t_ms;
            }
            ++cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(err);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[key_for(W, H, C, K, pa->bounces)] = Entry{pick, pick_ms};
    }
    if (best) {
        best->tile_w = 1 << pick.tile_shift;
        best->ready_batch = pick.ready_batch;
    }
    return IRTPS_OK;
}

}  // extern "C"
