// kernels.hpp -- launch interface of the IRT-PS kernels (internal to libirtps).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "traverse.hpp"

namespace irtps {
namespace kern {

constexpr int kMaxLights = 64;
constexpr int kMaxMgLevels = 32;
constexpr int kFlagQuadrature = 1;
constexpr int kFlagFlat = 4;

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
    int quad_off;      // floats from pyr to the quadrant tables
    int off[trv::kMaxLevels];
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
    uint32_t key0, key1;
};

// Multigrid levels of a W x H grid, offsets (in floats) into the workspace.
struct MgPlan {
    int levels;
    int W[kMaxMgLevels], H[kMaxMgLevels];
    long long xoff[kMaxMgLevels], boff[kMaxMgLevels];
    long long keyoff;  // one uint32 for the anchor's minimum
    long long total;   // floats
};

hipError_t ps_solve(int npx, int C, int K, const PsMatrix& M, const float* A, float* n, float* rho,
                    hipStream_t st);
hipError_t direct(const SurfaceArgs& sa, const float* n, const LightSet& L, int flat, float* S,
                  hipStream_t st);
hipError_t trace(TraceArgs a, hipStream_t st);
hipError_t correct(int npx, int C, int K, int rho_mode, int cumulative, const float* I0,
                   const float* Aprev, const float* G, const float* S, const float* rho, float* E,
                   float* Anext, hipStream_t st);
hipError_t compose(int npx, int C, int K, const float* rho, const float* S, const float* G, float* I,
                   hipStream_t st);
// Apron-max levels of P at pyr, then the quadrant maxima at pyr + quad_off.
hipError_t build_pyramid(int W, int Hh, const float* H, const trv::Pyramid& P, float* pyr,
                         long long quad_off, hipStream_t st);
hipError_t integrate(const MgPlan& plan, const float* n, const float* Hinit, int cycles, float* Hout,
                     float* ws, hipStream_t st);
hipError_t fill_f32(float* p, float v, long long n, hipStream_t st);
hipError_t fill_u64_zero(unsigned long long* p, int n, hipStream_t st);
hipError_t probe_philox(long long count, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                        hipStream_t st);
hipError_t probe_sample(long long count, const float* n, const float* u, float* d, hipStream_t st);
hipError_t probe_env(long long count, const float* d, int He, int We, int* rc, hipStream_t st);
hipError_t probe_traverse(const SurfaceArgs& sa, int flat, long long count, const int* ij,
                          const float* d, int* q, hipStream_t st);

}  // namespace kern
}  // namespace irtps
