// batch.hpp -- the multi-job engine behind the batched and served modes.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "irtps.h"
#include "kernels.hpp"

namespace irtps {
namespace eng {

// Blocks of the persistent tracer grid (queried once).
int resident_trace_blocks();
// Device bytes one job needs besides its caller-owned inputs and outputs.
size_t job_region_bytes(const irtps_problem& pr);
// Fill a job descriptor; `region` is the job's device workspace.
int fill_job(kern::JobDesc& J, const irtps_problem& pr, const irtps_params& pa, const irtps_outputs& out,
             char* region);
// Device bytes of the tables of a batch of n jobs with `tiles` tracer tiles.
size_t table_bytes(int n, int tiles);
// Tracer tiles a W x H job can need under any schedule (table space is sized
// for this, so a schedule change between sizing and solving cannot overflow).
int max_tracer_tiles(int W, int H);

struct Batch {
    std::vector<kern::JobDesc> jobs;
    std::vector<int2> tiles1, tiles3;  // (job, tile) of the grey and of the colour jobs
    kern::BatchShape shape{};
    int max_T = 0;
    kern::JobDesc* d_jobs = nullptr;
    int2* d_tiles1 = nullptr;
    int2* d_tiles3 = nullptr;
    unsigned* d_queue = nullptr;

    void build(const std::vector<kern::JobDesc>& js);
    // carve the tables at table_dev; IRTPS_ERR_WORKSPACE if they need more than capacity
    int place(char* table_dev, size_t capacity);
    int upload_tables(hipStream_t st);  // job descriptors and tile lists
    int run_init(hipStream_t st) const;                    // t = 0: PS of I0, cold integration
    int run_iteration(hipStream_t st) const;  // one IRT iteration of every job
    int run_all(hipStream_t st, bool use_graph);
};

}  // namespace eng
}  // namespace irtps
