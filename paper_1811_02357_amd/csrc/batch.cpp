// batch.cpp -- many IRT-PS reconstructions at once.
//
// A batch is a table of jobs in device memory; every step of the paper's loop
// (Sec. IV) runs as one launch for all jobs (grid.y = job), and the tracer as
// one persistent launch over the (job, tile) pairs of all jobs.  Jobs keep their
// own sizes, light counts, sample counts, seeds and iteration counts, and each
// job's result is bit-identical to solving it alone: the per-pixel arithmetic
// and its order do not depend on the other jobs.
#include "batch.hpp"

#include <algorithm>
#include <cstring>
#include <list>
#include <mutex>
#include <numeric>

#include "host.hpp"

namespace irtps {
namespace eng {

using namespace irtps::host;

// Persistent tracer grid: eight 256-thread blocks per compute unit.
int resident_trace_blocks() {
    static int blocks = 0;
    if (blocks == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        blocks = cus * 8;
    }
    return blocks;
}

size_t job_region_bytes(const irtps_problem& pr) {
    return solve_layout(pr.width, pr.height, pr.channels, pr.num_lights).total;
}

int fill_job(kern::JobDesc& J, const irtps_problem& pr, const irtps_params& pa, const irtps_outputs& out,
             char* region) {
    STATUS_TRY(check_problem(&pr, &pa));
    if (!out.normals_dev || !out.albedo_dev || !out.depth_dev) return IRTPS_ERR_INVALID_ARG;
    // the multi-job engine runs the gather (environment map only) and least-squares integration only
    if ((pa.flags & (IRTPS_FLAG_ROBUST_INTEGRATION | IRTPS_FLAG_EXACT_R_MASK)) || pr.box) return IRTPS_ERR_INVALID_ARG;
    std::memset(&J, 0, sizeof(J));
    const int W = pr.width, H = pr.height, C = pr.channels, K = pr.num_lights;
    kern::PsMatrix M;
    kern::LightSet L;
    STATUS_TRY(make_psmatrix(K, pr.light_dirs_host, pr.light_intensity_host, M));
    STATUS_TRY(make_lights(K, pr.light_dirs_host, pr.light_intensity_host, L));
    std::memcpy(J.M, M.m, sizeof(J.M));
    std::memcpy(J.L, L.l, sizeof(J.L));
    std::memcpy(J.s, L.s, sizeof(J.s));
    J.W = W;
    J.Hh = H;
    J.C = C;
    J.K = K;
    J.spp = pa.spp;
    J.B = pa.bounces;
    J.t = 0;
    J.T = pa.iterations;
    J.stop_tol = pa.stop_tol;
    J.rho_mode = pa.rho_mode;
    J.flags = pa.flags;
    J.cycles_cold = pa.mg_cycles_cold ? pa.mg_cycles_cold : 8;
    J.cycles_warm = pa.mg_cycles_warm ? pa.mg_cycles_warm : 4;
    J.key0 = (uint32_t)pa.seed;
    J.key1 = (uint32_t)(pa.seed >> 32);
    J.active = 1;
    const Schedule sched = schedule_for(W, H, C, K, pa.bounces);
    J.tile_shift = sched.tile_shift;
    J.ready_batch = sched.ready_batch;
    const trv::Pyramid P = pyramid_plan(W, H);
    J.pyr_levels = P.levels;
    J.quad_off = (int)pyramid_level_floats(P);
    for (int l = 0; l < trv::kMaxLevels; ++l) {
        J.pyr_wc[l] = l < P.levels ? P.wc[l] : 0;
        J.pyr_hc[l] = l < P.levels ? P.hc[l] : 0;
        J.pyr_off[l] = l < P.levels ? (int)P.off[l] : 0;
    }
    const SolveLayout lay = solve_layout(W, H, C, K);
    J.mg = lay.plan;
    J.I0 = pr.images_dev;
    J.env = pr.env_dev;
    J.env_h = pr.env_h;
    J.env_w = pr.env_w;
    J.A = reinterpret_cast<float*>(region + lay.A);
    J.S = reinterpret_cast<float*>(region + lay.S);
    J.G = reinterpret_cast<float*>(region + lay.G);
    J.pyr = reinterpret_cast<float*>(region + lay.pyr);
    J.mg_ws = reinterpret_cast<float*>(region + lay.mg);
    J.n = out.normals_dev;
    J.rho = out.albedo_dev;
    J.depth = out.depth_dev;
    J.E = out.indirect_dev;
    J.counters = reinterpret_cast<unsigned long long*>(out.counters_dev);
    return IRTPS_OK;
}

// Tables of one batch: job descriptors, then the (job, tile) lists of the grey
// and of the colour jobs, then the tracer's queue counter.
size_t table_bytes(int n, int tiles) {
    return align_up(sizeof(kern::JobDesc) * (size_t)n) + align_up(sizeof(int2) * (size_t)tiles) + kAlign;
}

int max_tracer_tiles(int W, int H) {
    int m = 0;
    for (int shift = 3; shift <= 6; ++shift) m = std::max(m, kern::tiles_for(W, H, 1 << shift));
    return m;
}

void Batch::build(const std::vector<kern::JobDesc>& js) {
    jobs = js;
    tiles1.clear();
    tiles3.clear();
    // larger jobs first so that the queue ends on small tiles
    std::vector<int> order(jobs.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const double ca = (double)jobs[a].W * jobs[a].Hh * jobs[a].spp * std::max(jobs[a].B, 1);
        const double cb = (double)jobs[b].W * jobs[b].Hh * jobs[b].spp * std::max(jobs[b].B, 1);
        return ca > cb;
    });
    for (int j : order) {
        const kern::JobDesc& J = jobs[j];
        if (!J.active || J.B < 1) continue;
        const int tiles = kern::tiles_for(J.W, J.Hh, 1 << J.tile_shift);
        auto& list = J.C == 1 ? tiles1 : tiles3;
        for (int t = 0; t < tiles; ++t) list.push_back(make_int2(j, t));
    }
    std::memset(&shape, 0, sizeof(shape));
    shape.njobs = (int)jobs.size();
    // flattened grids: each job's blocks follow the previous job's
    for (kern::JobDesc& J : jobs) {
        for (int l = 0; l < kern::kMaxMgLevels; ++l) {
            const bool own = l < J.mg.tail;
            J.mg_bstart[l] = shape.mg_blocks[l];
            J.rs_bstart[l] = shape.rs_blocks[l];
            shape.mg_blocks[l] += own ? kern::flat_blocks((long long)J.mg.W[l] * J.mg.H[l]) : 0;
            shape.rs_blocks[l] += own ? kern::flat_blocks((long long)J.mg.W[l + 1] * J.mg.H[l + 1]) : 0;
        }
        J.near_bstart = shape.near_blocks;
        shape.near_blocks += kern::near_tiles(J.W, J.Hh);
    }
    for (const kern::JobDesc& J : jobs) {
        shape.max_npx = std::max(shape.max_npx, J.W * J.Hh);
        shape.max_direct_tiles = std::max(shape.max_direct_tiles, kern::tiles_for(J.W, J.Hh, kern::kDirectTileW));
        shape.max_rows = std::max(shape.max_rows, J.Hh);
        shape.max_cols = std::max(shape.max_cols, J.W);
        shape.max_pyr_levels = std::max(shape.max_pyr_levels, J.pyr_levels);
        for (int l = 0; l < J.pyr_levels; ++l)
            shape.max_pyr_cells[l] = std::max(shape.max_pyr_cells[l], J.pyr_wc[l] * J.pyr_hc[l]);
        shape.max_mg_tail = std::max(shape.max_mg_tail, J.mg.tail);
        shape.max_mg_tail_floats = std::max(shape.max_mg_tail_floats, J.mg.keyoff - J.mg.xoff[J.mg.tail]);
        shape.max_cycles_cold = std::max(shape.max_cycles_cold, J.cycles_cold);
        shape.max_cycles_warm = std::max(shape.max_cycles_warm, J.cycles_warm);
        shape.max_KCnpx = std::max(shape.max_KCnpx, J.K * J.C * J.W * J.Hh);
        if (J.C == 1) shape.max_K1 = std::max(shape.max_K1, J.K);
        else shape.max_K3 = std::max(shape.max_K3, J.K);
        max_T = std::max(max_T, J.T);
    }
}

int Batch::place(char* table_dev, size_t capacity) {
    if (table_bytes((int)jobs.size(), (int)(tiles1.size() + tiles3.size())) > capacity) return IRTPS_ERR_WORKSPACE;
    d_jobs = reinterpret_cast<kern::JobDesc*>(table_dev);
    char* p = table_dev + align_up(sizeof(kern::JobDesc) * jobs.size());
    d_tiles1 = reinterpret_cast<int2*>(p);
    d_tiles3 = d_tiles1 + tiles1.size();
    p += align_up(sizeof(int2) * (tiles1.size() + tiles3.size()));
    d_queue = reinterpret_cast<unsigned*>(p);
    return IRTPS_OK;
}

int Batch::upload_tables(hipStream_t st) {
    std::vector<char> buf(sizeof(kern::JobDesc) * jobs.size());
    std::memcpy(buf.data(), jobs.data(), buf.size());
    HIP_TRY(upload(d_jobs, buf.data(), buf.size(), st));
    std::vector<int2> tl(tiles1);
    tl.insert(tl.end(), tiles3.begin(), tiles3.end());
    HIP_TRY(upload(d_tiles1, tl.data(), sizeof(int2) * tl.size(), st));
    return IRTPS_OK;
}

int Batch::run_init(hipStream_t st) const {
    HIP_TRY(kern::batch_begin(d_jobs, shape, st));
    HIP_TRY(kern::batch_ps(d_jobs, shape, 0, st));
    HIP_TRY(kern::batch_integrate(d_jobs, shape, 1, st));
    return IRTPS_OK;
}

int Batch::run_iteration(hipStream_t st) const {
    const int resident = resident_trace_blocks();
    HIP_TRY(kern::batch_pyramid(d_jobs, shape, st));
    HIP_TRY(kern::batch_direct(d_jobs, shape, st));
    HIP_TRY(kern::trace_multi(d_jobs, 1, d_tiles1, (int)tiles1.size(), d_queue, IRTPS_TAG_SOLVE,
                              resident, st));
    HIP_TRY(kern::trace_multi(d_jobs, 3, d_tiles3, (int)tiles3.size(), d_queue, IRTPS_TAG_SOLVE,
                              resident, st));
    HIP_TRY(kern::batch_correct(d_jobs, shape, 0, st));
    HIP_TRY(kern::batch_ps(d_jobs, shape, 1, st));
    HIP_TRY(kern::batch_integrate(d_jobs, shape, 0, st));
    HIP_TRY(kern::batch_advance(d_jobs, shape.njobs, st));
    return IRTPS_OK;
}

// ---- hipGraph cache ---------------------------------------------------------
// A batch solve with IRTPS_BATCH_GRAPH is captured once into a graph keyed by
// the exact bytes of its job and tile tables and its device table address; a
// later call with the same key replays the graph.

namespace {

struct GraphEntry {
    std::vector<char> key;
    hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::list<GraphEntry> g_graphs;  // most recent first
constexpr size_t kMaxGraphs = 4;

std::vector<char> graph_key(const Batch& b) {
    std::vector<char> k(sizeof(void*) + sizeof(kern::JobDesc) * b.jobs.size() +
                        sizeof(int2) * (b.tiles1.size() + b.tiles3.size()));
    char* p = k.data();
    std::memcpy(p, &b.d_jobs, sizeof(void*));
    p += sizeof(void*);
    std::memcpy(p, b.jobs.data(), sizeof(kern::JobDesc) * b.jobs.size());
    p += sizeof(kern::JobDesc) * b.jobs.size();
    std::memcpy(p, b.tiles1.data(), sizeof(int2) * b.tiles1.size());
    p += sizeof(int2) * b.tiles1.size();
    std::memcpy(p, b.tiles3.data(), sizeof(int2) * b.tiles3.size());
    return k;
}

}  // namespace

int Batch::run_all(hipStream_t st, bool use_graph) {
    auto launches = [&](hipStream_t s) -> int {
        STATUS_TRY(run_init(s));
        for (int t = 0; t < max_T; ++t) STATUS_TRY(run_iteration(s));
        return IRTPS_OK;
    };
    (void)resident_trace_blocks();  // device queries stay outside any capture
    if (!use_graph || st == nullptr) return launches(st);
    std::vector<char> key = graph_key(*this);
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it) {
        if (it->key == key) {
            g_graphs.splice(g_graphs.begin(), g_graphs, it);
            HIP_TRY(hipGraphLaunch(g_graphs.front().exec, st));
            return IRTPS_OK;
        }
    }
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = launches(st);
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (rc != IRTPS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess) return hip_fail(ec);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return hip_fail(ei);
    g_graphs.push_front(GraphEntry{std::move(key), exec});
    while (g_graphs.size() > kMaxGraphs) {
        (void)hipGraphExecDestroy(g_graphs.back().exec);
        g_graphs.pop_back();
    }
    HIP_TRY(hipGraphLaunch(exec, st));
    return IRTPS_OK;
}

}  // namespace eng
}  // namespace irtps

using namespace irtps;
using namespace irtps::host;

namespace {

// Job regions follow the tables, each 256-byte aligned.
int batch_layout(int32_t n, const irtps_problem* problems, size_t* tables, std::vector<size_t>* offsets,
                 size_t* total) {
    size_t tiles = 0;
    for (int j = 0; j < n; ++j) {
        if (!dims_ok(problems[j].width, problems[j].height)) return IRTPS_ERR_INVALID_ARG;
        tiles += (size_t)eng::max_tracer_tiles(problems[j].width, problems[j].height);
    }
    *tables = eng::table_bytes(n, (int)tiles);
    size_t off = *tables;
    if (offsets) offsets->clear();
    for (int j = 0; j < n; ++j) {
        if (offsets) offsets->push_back(off);
        off = align_up(off + eng::job_region_bytes(problems[j]));
    }
    *total = off;
    return IRTPS_OK;
}

}  // namespace

extern "C" {

int irtps_batch_workspace_bytes(int32_t n, const irtps_problem* problems, const irtps_params* params,
                                size_t* bytes) {
    if (n < 1 || !problems || !params || !bytes) return IRTPS_ERR_INVALID_ARG;
    for (int j = 0; j < n; ++j) STATUS_TRY(check_problem(&problems[j], &params[j]));
    size_t tables = 0, total = 0;
    STATUS_TRY(batch_layout(n, problems, &tables, nullptr, &total));
    *bytes = total;
    return IRTPS_OK;
}

int irtps_batch_solve(int32_t n, const irtps_problem* problems, const irtps_params* params,
                      const irtps_outputs* outputs, int32_t options, void* ws_dev, size_t ws_bytes,
                      void* stream) {
    if (n < 1 || !problems || !params || !outputs || (options & ~IRTPS_BATCH_GRAPH)) return IRTPS_ERR_INVALID_ARG;
    size_t tables = 0, total = 0;
    std::vector<size_t> offsets;
    for (int j = 0; j < n; ++j) STATUS_TRY(check_problem(&problems[j], &params[j]));
    STATUS_TRY(batch_layout(n, problems, &tables, &offsets, &total));
    if (!ws_dev || ws_bytes < total || (reinterpret_cast<uintptr_t>(ws_dev) % kAlign)) return IRTPS_ERR_WORKSPACE;
    char* base = static_cast<char*>(ws_dev);
    std::vector<kern::JobDesc> jobs((size_t)n);
    for (int j = 0; j < n; ++j)
        STATUS_TRY(eng::fill_job(jobs[j], problems[j], params[j], outputs[j], base + offsets[j]));
    eng::Batch b;
    b.build(jobs);
    STATUS_TRY(b.place(base, tables));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    STATUS_TRY(b.upload_tables(st));
    return b.run_all(st, (options & IRTPS_BATCH_GRAPH) != 0);
}

}  // extern "C"
