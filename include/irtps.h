/*
 * irtps.h -- C ABI of the MI355X (gfx950) implementation of Iterative Ray-Tracing
 * Photometric Stereo (IRT-PS): Khadka, Remagnino, Argyriou, "Object 3D
 * Reconstruction based on Photometric Stereo and Inverted Rendering",
 * arXiv 1811.02357.
 *
 * The problem is the paper's: K images of a Lambertian object taken from one
 * viewpoint under calibrated distant lights (Sec. III, Eq.2-3), with the
 * surroundings known (Sec. IV, stages 0, 3, 4).  The library returns the
 * per-pixel normals and albedo (Eq.4), the integrated surface H_t (Sec. IV,
 * stage 1) and the estimated indirect light E_t (Sec. IV, stage 5).
 *
 * Conventions (all calls):
 *   - Sample (i, j) is world (x, y) = (i, j): i is the column in [0, W), j the row
 *     in [0, H); heights are in pixel units; z points towards the orthographic
 *     camera.  A light direction is a unit vector from the surface towards the
 *     light; its intensity is the irradiance it gives at normal incidence.
 *   - An image value is albedo x irradiance (Eq.2).  Environment texels are
 *     radiance on an equirectangular map: row r covers polar angle
 *     [r pi/He, (r+1) pi/He) from +z, column c covers azimuth
 *     [2 pi c/We, 2 pi (c+1)/We) from +x towards +y.
 *   - Layouts are row-major float32: images and indirect radiance
 *     [K][C][H][W]; gathered radiance G [H][W][K][C] (pixel-major: one pixel's
 *     sums are contiguous); normals [H][W][3]; albedo [C][H][W]; depth [H][W];
 *     direct irradiance [H][W][K]; environment [He][We][C].  C is 1 or 3,
 *     W and H are 2..16384 with W H <= 2^28, K is 3..64.
 *   - Pointers named *_dev are device memory (any hipMalloc'd or
 *     caching-allocator memory of the current device); pointers named *_host
 *     are host memory read before the call returns.  The caller owns every
 *     buffer; the library never frees caller memory and never keeps a pointer
 *     after the call, except the server (see below).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is enqueued on it and the call returns without waiting;
 *     device faults surface on a later call or on stream synchronisation.
 *   - Every call returns an irtps_status.  No exception or abort crosses the
 *     ABI.  NaN inputs are not checked.  Results are deterministic: the same
 *     inputs, parameters and seed give the same bits, alone, batched or served.
 */
#ifndef IRTPS_H
#define IRTPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IRTPS_ABI_VERSION 3

typedef enum irtps_status {
    IRTPS_OK = 0,
    IRTPS_ERR_INVALID_ARG = 1,     /* a size, pointer or parameter out of range */
    IRTPS_ERR_SINGULAR_LIGHTS = 2, /* K < 3 or the lights are (nearly) coplanar (Eq.4) */
    IRTPS_ERR_WORKSPACE = 3,       /* workspace missing or smaller than required */
    IRTPS_ERR_OOM = 4,             /* server: job larger than the memory budget */
    IRTPS_ERR_DEVICE = 5,          /* a HIP call failed: see irtps_last_hip_error() */
    IRTPS_ERR_CANCELLED = 6,       /* server: the job was cancelled */
    IRTPS_ERR_NOT_FOUND = 7,       /* server: unknown job id */
    IRTPS_ERR_BUSY = 8             /* server: job still queued or running */
} irtps_status;

/* Albedo used to turn the gathered radiance into the indirect image (stage 5). */
enum {
    IRTPS_RHO_FIT = 0,  /* albedo fitted per pixel to I0 = rho (S + G) over the K images */
    IRTPS_RHO_PREV = 1  /* the previous photometric-stereo albedo rho_t (literal) */
};

/* Option bits of irtps_params.flags and of irtps_trace. */
enum {
    IRTPS_FLAG_QUADRATURE = 1,         /* first segment on sqrt(spp)^2 stratum midpoints */
    IRTPS_FLAG_LITERAL_CUMULATIVE = 2, /* A_{t+1} = A_t - E_t instead of I0 - E_t */
    IRTPS_FLAG_FLAT_TRAVERSAL = 4,     /* walk every grid-line crossing (no pyramid skips) */
    IRTPS_FLAG_SHADOW_AWARE_PS = 8,    /* the PS after each correction keeps, per pixel, only the
                                          lights that reach it (irtps_ps_solve_masked with that
                                          iteration's direct irradiance); the first PS uses all */
    IRTPS_FLAG_GRAPH = 16,             /* irtps_solve only: capture the solve's launches in a
                                          hipGraph the first time, replay it on later calls with
                                          identical arguments (same pointers, lights, schedule);
                                          needs stop_tol = 0 and a stream other than the legacy
                                          default one; changes no result */
    IRTPS_FLAG_ROBUST_INTEGRATION = 32, /* irtps_solve and irtps_solve_static only (the batched and
                                           served engines refuse it): every integration is
                                           irtps_integrate_robust with delta 0.1, 6 rounds of 2
                                           V-cycles after the least-squares cycles */
    IRTPS_FLAG_EXACT_R_MASK = 0x700     /* bits of IRTPS_FLAG_EXACT_R(r) */
};
/* The paper's r-ray variant of the tracer (Sec. IV, the tracing paragraph, and
 * Fig. 5), r in 1..7, for irtps_solve and irtps_solve_static only (the batched
 * and served engines refuse it): each iteration's gather is replaced by one
 * environment image, the same for every light: irtps_trace_exact_r (one path
 * per pixel that leaves on its r-th ray), the pixels it leaves empty filled by
 * irtps_fill_missing, then stage 5 (irtps_correct) with G[p][k] = that image.
 * spp, bounces and IRTPS_FLAG_QUADRATURE are then unused; the trace counters
 * [0..3] stay 0. */
#define IRTPS_FLAG_EXACT_R(r) ((int32_t)(r) << 8)

/* Sample-stream tags (word 3 of the Philox counter). */
enum { IRTPS_TAG_SOLVE = 0, IRTPS_TAG_RENDER = 1 };

/* Counters, a device array of five uint64: [0] segments, [1] surface hits,
 * [2] escapes to the environment, [3] continuations (hits that start another
 * segment), accumulated by the trace kernels; [4] IRT iterations run (the
 * solves: T, or fewer with stop_tol). */
#define IRTPS_NUM_COUNTERS 5

/* The known environment as geometry (Sec. IV, stages 0, 3 and 4: the surface
 * sits in a Cornell box whose walls may carry textures).  Four vertical
 * Lambertian walls stand on the borders of the sample grid -- wall 0 at x = 0,
 * 1 at x = W - 1, 2 at y = 0, 3 at y = H - 1, each facing into the box -- from
 * below the surface up to height Z; above them the box is open to the
 * environment map.  Each wall is a texture of tex_h rows (heights 0..Z) by
 * tex_w columns (along the wall: y from 0 to H - 1 on walls 0 and 1, x from 0
 * to W - 1 on walls 2 and 3), nearest texel.
 *
 * With a box, (1) a shadow ray (direct light, Eq.2) is blocked too when it
 * meets a wall, i.e. when it is outside the footprint [0, W-1] x [0, H-1] on
 * reaching height Z from below; (2) each wall texel's direct irradiance
 * S_w[k] = s_k max(0, n_wall . l_k) V_k is taken at its centre, V_k = 1 when
 * the light's ray leaves through the open top (walls shade walls; the surface
 * casts no shadow on them); (3) a gathered ray that leaves the surface and
 * meets a wall below Z (the first wall plane ahead, a corner counting as the x
 * wall) adds, for every light k, the path's albedo product times the texel's
 * albedo times S_w[k] -- the wall's Lambertian reflection of its own direct
 * light, weighted like a surface hit -- and ends the path; a ray over the
 * walls takes the environment map.  Texel of a wall point at height z and
 * position u along a wall of length len: row = floor(z / Z tex_h), col =
 * floor(u / len tex_w), each clamped to the texture.  Counter [2] counts wall
 * hits with the escapes. */
typedef struct irtps_box {
    float height;             /* Z > 0, pixel units of the depth */
    int32_t tex_h, tex_w;     /* 1..4096 each */
    const float* albedo_dev;  /* [4][tex_h][tex_w][C] wall albedo */
} irtps_box;

typedef struct irtps_problem {
    int32_t width, height, channels, num_lights; /* W, H, C in {1,3}, K in 3..64 */
    const float* images_dev;          /* [K][C][H][W] input images I0 (stage 0) */
    const float* light_dirs_host;     /* [K][3] unit, towards the light, z > 0 */
    const float* light_intensity_host;/* [K] or NULL (all 1) */
    const float* env_dev;             /* [He][We][C] radiance of the known surroundings */
    int32_t env_h, env_w;             /* He, We >= 1 */
    const irtps_box* box;             /* host pointer, or NULL: the environment map alone.
                                         irtps_solve and irtps_solve_static only (the batched
                                         and served engines refuse it); not with
                                         IRTPS_FLAG_EXACT_R */
} irtps_problem;

typedef struct irtps_params {
    int32_t spp;            /* paths per pixel and iteration, >= 1 */
    int32_t bounces;        /* B: segments per path, 0..8 (Sec. IV: up to 3 reflections) */
    int32_t iterations;     /* T >= 0 tracer passes; T + 1 PS + integration passes */
    int32_t rho_mode;       /* IRTPS_RHO_FIT (default) or IRTPS_RHO_PREV */
    int32_t flags;          /* IRTPS_FLAG_* */
    int32_t mg_cycles_cold; /* V-cycles of the first integration (0 = 8) */
    int32_t mg_cycles_warm; /* V-cycles of each warm-started integration (0 = 4) */
    float stop_tol;         /* 0: run all T iterations; > 0: stop after the first iteration whose
                               surface change D_H = max_p |H_{t+1}(p) - H_t(p)| (pixel units) is
                               below stop_tol (last paragraph of Sec. IV); must be finite, >= 0 */
    uint64_t seed;          /* Philox key */
} irtps_params;

typedef struct irtps_outputs {
    float* normals_dev;   /* [H][W][3] n_T */
    float* albedo_dev;    /* [C][H][W] rho_T */
    float* depth_dev;     /* [H][W] H_T, pixel units, min(H_T) = 0 */
    float* indirect_dev;  /* [K][C][H][W] E of the last iteration run (zeros for T = 0), or NULL */
    uint64_t* counters_dev; /* IRTPS_NUM_COUNTERS uint64 accumulated over the solve (zeroed at
                               its start), or NULL */
} irtps_outputs;

/* ---- library ------------------------------------------------------------ */
int irtps_abi_version(void);
const char* irtps_status_string(int status);
/* The hipError_t of the last failed HIP call made by the library on this thread. */
int irtps_last_hip_error(void);

/* ---- Eq.4 solve matrix (host only) --------------------------------------- */
/* M = (L^T L)^-1 L^T with rows of L = s_k l_k (Sec. III, Eq.3-4), computed in
 * binary64 with the 3x3 adjugate and rounded to float.  M_host is [3][K].
 * Returns IRTPS_ERR_SINGULAR_LIGHTS when K < 3 or det(L^T L) <= 1e-7 (tr/3)^3. */
int irtps_ps_matrix(int32_t K, const float* light_dirs_host,
                    const float* light_intensity_host, float* M_host);

/* ---- whole IRT-PS solve (Sec. IV, stages 1-5 iterated) ----------------- */
/* Bytes of device workspace irtps_solve needs for this problem and params. */
int irtps_workspace_bytes(const irtps_problem* problem, const irtps_params* params,
                          size_t* bytes);
/* t = 0: PS of I0 (Eq.4) and integration; then T times: trace the current
 * surface (Eq.5-7), subtract the indirect estimate (stage 5), PS and integrate
 * warm-started from H_t.  ws_dev must hold irtps_workspace_bytes() bytes,
 * 256-byte aligned; it needs no initialisation and carries nothing between
 * calls (besides the loop's buffers it keeps the tracer's per-chunk pixel
 * times, which order the next iteration's chunks, and for problems of at most
 * 16384 pixels the per-path tracer's segment records, for larger ones the
 * sums of each pixel's escape terms, which the correction adds to the hit sums;
 * none of these changes a result). */
int irtps_solve(const irtps_problem* problem, const irtps_params* params,
                const irtps_outputs* outputs, void* ws_dev, size_t ws_bytes,
                void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): irtps_solve
 * with the workspace taken from a scratch area the library owns, a device
 * array of IRTPS_STATIC_SCRATCH_BYTES on every GPU the library runs on (held
 * until the process ends).  The call allocates nothing and frees nothing; the
 * caller still passes inputs and outputs.  Problems whose irtps_workspace_bytes
 * exceed IRTPS_STATIC_SCRATCH_BYTES are refused with IRTPS_ERR_WORKSPACE (a
 * 512 x 512 grey solve with 12 lights needs about 48 MiB).  All calls on one
 * GPU share its scratch: calls that overlap on one GPU (another stream,
 * another thread) race and must be serialised by the caller.  With stop_tol >
 * 0 the call synchronises the stream after each iteration, as irtps_solve
 * does.  Results are bit-identical to irtps_solve. */
#define IRTPS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int irtps_solve_static(const irtps_problem* problem, const irtps_params* params,
                       const irtps_outputs* outputs, void* stream);

/* ---- stages (teacher-forced parity and custom loops) -------------------- */
/* Eq.4 per pixel: g_c = M A_c, albedo_c = |g_c|, normal = sum_c g_c / |sum_c g_c|
 * ((0,0,1) where that sum is 0).  A_dev is [K][C][H][W]. */
int irtps_ps_solve(int32_t W, int32_t H, int32_t C, int32_t K,
                   const float* light_dirs_host, const float* light_intensity_host,
                   const float* A_dev, float* normals_dev, float* albedo_dev, void* stream);

/* Eq.4 restricted per pixel to the lights that reach it (Sec. III: the solve
 * needs at least three lights; a light whose direct irradiance is zero carries
 * no shading).  Light k is kept at pixel p when S_dev[p][k] > 0, S_dev being
 * the [H][W][K] direct irradiance s_k max(0, n.l_k) V_k of irtps_direct.  With
 * at least three kept lights whose normal matrix L_p^T L_p passes the test of
 * irtps_ps_matrix (det > 1e-7 (trace/3)^3), the pixel's own matrix
 * (L_p^T L_p)^-1 L_p^T is built in binary64 from the kept rows (3x3 adjugate),
 * rounded to float and applied over the kept lights in light order; other
 * pixels use the all-light matrix.  Normals and albedo then as irtps_ps_solve.
 * Returns IRTPS_ERR_SINGULAR_LIGHTS when the all-light matrix is singular. */
int irtps_ps_solve_masked(int32_t W, int32_t H, int32_t C, int32_t K,
                          const float* light_dirs_host, const float* light_intensity_host,
                          const float* A_dev, const float* S_dev, float* normals_dev,
                          float* albedo_dev, void* stream);

/* Bytes of workspace for irtps_integrate. */
int irtps_integrate_workspace_bytes(int32_t W, int32_t H, size_t* bytes);
/* Least-squares integration of the normals (Sec. IV, stage 1): edge height
 * differences fitted to the mean end-point gradients -(n_x, n_y)/max(n_z, 0.05);
 * `cycles` multigrid V-cycles (free boundaries) started from depth_init_dev
 * (or from 0 if NULL; it may equal depth_dev); result shifted to min 0. */
int irtps_integrate(int32_t W, int32_t H, const float* normals_dev,
                    const float* depth_init_dev, int32_t cycles, float* depth_dev,
                    void* ws_dev, size_t ws_bytes, void* stream);

/* Robust integration, the M-estimator of Sec. IV, stage 1: irtps_integrate's
 * `cycles` least-squares V-cycles, then `rounds` rounds of the Huber
 * M-estimator (threshold delta >= 0 on the edge residual H_b - H_a - g, g the
 * least-squares edge target, pixel units) by half-quadratic splitting: each
 * round moves every edge target to g + shrink(residual), shrink(r) being the
 * part of r beyond +-delta for the current surface, and runs `rcycles` more
 * V-cycles.  Result shifted to min 0.  rounds = 0 gives irtps_integrate.
 * Workspace as irtps_integrate_workspace_bytes. */
int irtps_integrate_robust(int32_t W, int32_t H, const float* normals_dev,
                           const float* depth_init_dev, int32_t cycles, float delta,
                           int32_t rounds, int32_t rcycles, float* depth_dev,
                           void* ws_dev, size_t ws_bytes, void* stream);

/* Bytes of the min-max pyramid of a W x H surface. */
int irtps_pyramid_bytes(int32_t W, int32_t H, size_t* bytes);
/* Per level l, cell (cx, cy) spans samples [cx 2^l, (cx+1) 2^l] x [cy 2^l, (cy+1) 2^l]
 * and stores the max over that box grown by one sample on each side, or +inf
 * when the box comes within two samples of the border (cx 2^l < 2 or
 * (cx+1) 2^l > W - 3, likewise in y).  Block tables follow the levels (from the
 * next multiple of 64 floats), over 8 x 8 sample blocks, QW = ceil(W/8),
 * QH = ceil(H/8), p4 = QW QH rounded up to a multiple of 4, s4 = the count of
 * 64 x 64 super-blocks rounded up likewise; q = (sx < 0) + 2 (sy < 0) names
 * the sign pair of a ray's travel.  In floats from the tables' start:
 *   0       escape windows float4 [4][QH][QW]
 *   16 p4   block maxima [QH][QW]
 *   17 p4   window row maxima [2][3][QH][QW] (build scratch)
 *   25 p4   quadrant maxima [4][QH][QW]: max over samples with x >= 8 bx
 *           (sx > 0) or x <= 8 bx + 7 (sx < 0), likewise along y
 *   29 p4   block minima [QH][QW]
 *   30 p4   horizon chords float4 [4][QH][QW] (a_mid, k_mid, a_far, k_far)
 *   46 p4   super-block maxima
 *   46 p4 + s4   near horizons float4 [H][W] (the four quadrants of a sample)
 * A rising ray from a sample whose slope (rise per unit of horizontal travel)
 * is at least the sample's near horizon for its quadrant and both chords
 * a + k h at the sample's height h cannot hit anything. */
int irtps_build_pyramid(int32_t W, int32_t H, const float* depth_dev, float* pyramid_dev,
                        void* stream);

/* Direct irradiance without albedo (Eq.2): S[q][k] = s_k max(0, n(q).l_k) V_k(q),
 * V_k = 1 when the shadow ray from sample q towards light k escapes the surface
 * (and, with box non-NULL, leaves through the box's open top; only
 * box->height is read).  pyramid_dev from irtps_build_pyramid of the same
 * depth.  S_dev is [H][W][K]. */
int irtps_direct(int32_t W, int32_t H, int32_t K, const float* depth_dev,
                 const float* normals_dev, const float* light_dirs_host,
                 const float* light_intensity_host, const float* pyramid_dev,
                 float* S_dev, const irtps_box* box, void* stream);

/* The box walls' direct irradiance (Eq.2 on the walls, at texel centres; see
 * irtps_box): wall_S_dev [4][tex_h][tex_w][K]. */
int irtps_box_shade(int32_t W, int32_t H, int32_t K, const irtps_box* box,
                    const float* light_dirs_host, const float* light_intensity_host,
                    float* wall_S_dev, void* stream);

/* Monte Carlo gather of indirect light (Sec. IV, Eq.5-7): per pixel, spp
 * cosine-weighted paths of up to B segments on the current surface.  A hit at
 * sample q adds beta_c albedo_c(q) S[q][k] for every light k; an escape adds
 * beta_c pi L_env,c(d) and ends the path; beta is the product of the albedos
 * met so far.  G_dev[p][k][c] = (sum over paths) / spp.  Sample s, segment b of
 * pixel p = j W + i draw Philox4x32-10(key = seed, counter = (p, s, t 256 + b,
 * tag)).  counters_dev (IRTPS_NUM_COUNTERS uint64, accumulated) may be NULL.
 * With box non-NULL, an escaping ray that meets a wall below its rim adds the
 * wall term instead (see irtps_box), wall_S_dev from irtps_box_shade. */
int irtps_trace(int32_t W, int32_t H, int32_t C, int32_t K, const float* depth_dev,
                const float* normals_dev, const float* albedo_dev, const float* S_dev,
                const float* env_dev, int32_t env_h, int32_t env_w,
                const float* pyramid_dev, int32_t spp, int32_t B, uint64_t seed,
                int32_t t, int32_t tag, int32_t flags, float* G_dev,
                uint64_t* counters_dev, const irtps_box* box, const float* wall_S_dev,
                void* stream);

/* The r-ray variant's trace (Sec. IV, the tracing paragraph; Fig. 5): per
 * pixel p = j W + i, the single path of sample 0 (the counters irtps_trace
 * gives sample 0, segments b = 1..r) that reflects r - 1 times and leaves for
 * the environment on its r-th ray.  Such a pixel gets, per channel, the product
 * of the albedos of its r - 1 hits times pi L_env,c of the texel that ray
 * reaches, and valid_dev[p] = 1; a path that escapes earlier, or whose r-th ray
 * meets the surface, leaves E_dev[p] = 0 and valid_dev[p] = 0.  E_dev is
 * [H][W][C], valid_dev [H][W] uint8 (may be NULL); flags: 0 or
 * IRTPS_FLAG_FLAT_TRAVERSAL; r in 1..7.  pyramid_dev as for irtps_trace. */
int irtps_trace_exact_r(int32_t W, int32_t H, int32_t C, const float* depth_dev,
                        const float* normals_dev, const float* albedo_dev, const float* env_dev,
                        int32_t env_h, int32_t env_w, const float* pyramid_dev, int32_t r,
                        uint64_t seed, int32_t t, int32_t tag, int32_t flags, float* E_dev,
                        unsigned char* valid_dev, void* stream);

/* Bytes of workspace for irtps_fill_missing. */
int irtps_fill_workspace_bytes(int32_t W, int32_t H, int32_t C, size_t* bytes);
/* Fill of the pixels the r-ray image leaves empty (the paper interpolates them
 * and names no method): pull-push over levels of 2 x 2 aggregates down to
 * 1 x 1 (level sizes ceil(w/2) x ceil(h/2)).  Pull: a coarse cell holds the
 * weighted mean of its children that carry weight (weights: counts of valid
 * pixels below; children taken (0,0), (1,0), (0,1), (1,1), each channel summed
 * with fused multiply-adds, then divided by the summed weight) and that weight.
 * Push: from the coarsest level down, a cell of weight 0 takes its parent's
 * value.  Pixels with valid_dev[p] != 0 keep their value; with no valid pixel
 * every pixel becomes 0.  E_dev [H][W][C] is filled in place. */
int irtps_fill_missing(int32_t W, int32_t H, int32_t C, float* E_dev, const unsigned char* valid_dev,
                       void* ws_dev, size_t ws_bytes, void* stream);

/* Stage 5: E = rho~ G and A_next = I0 - E (or A_prev - E with
 * IRTPS_FLAG_LITERAL_CUMULATIVE).  rho~ per IRTPS_RHO_*: the fit is
 * sum_k I0 (S + G) / sum_k (S + G)^2 (0 where the denominator is 0).
 * E_dev may be NULL; A_prev_dev is read only in the cumulative mode. */
int irtps_correct(int32_t W, int32_t H, int32_t C, int32_t K, int32_t rho_mode,
                  int32_t flags, const float* I0_dev, const float* A_prev_dev,
                  const float* G_dev, const float* S_dev, const float* albedo_dev,
                  float* E_dev, float* A_next_dev, void* stream);

/* Bytes of workspace for irtps_render (box may be NULL). */
int irtps_render_workspace_bytes(int32_t W, int32_t H, int32_t C, int32_t K, const irtps_box* box,
                                 size_t* bytes);
/* Forward render of a known surface (Sec. III, n-bounce sum truncated at B + 1):
 * images = albedo (S + G) with G traced under tag RENDER, t = 0.  B = 0 renders
 * direct light only.  box (may be NULL) as in irtps_problem. */
int irtps_render(int32_t W, int32_t H, int32_t C, int32_t K, const float* depth_dev,
                 const float* normals_dev, const float* albedo_dev,
                 const float* light_dirs_host, const float* light_intensity_host,
                 const float* env_dev, int32_t env_h, int32_t env_w, int32_t spp,
                 int32_t B, uint64_t seed, float* images_dev, void* ws_dev,
                 size_t ws_bytes, const irtps_box* box, void* stream);

/* ---- batched mode --------------------------------------------------------- */
/* Options of irtps_batch_solve. */
enum {
    IRTPS_BATCH_GRAPH = 1  /* capture the batch's launches in a hipGraph; a later call with
                              identical arguments and workspace replays it */
};
/* Bytes of device workspace irtps_batch_solve needs for these n jobs. */
int irtps_batch_workspace_bytes(int32_t n, const irtps_problem* problems,
                                const irtps_params* params, size_t* bytes);
/* n independent reconstructions (each as irtps_solve with its own problem,
 * params and outputs) run together: every stage of the loop is one launch for
 * all jobs and the tracer is one persistent launch over all jobs' pixel tiles.
 * Each job's outputs are bit-identical to irtps_solve of that job alone.  The
 * arrays are host arrays of n elements; the problems' device pointers and the
 * outputs must stay valid until the stream reaches the end of the call's work.
 * With IRTPS_BATCH_GRAPH the stream must not be the legacy default stream. */
int irtps_batch_solve(int32_t n, const irtps_problem* problems, const irtps_params* params,
                      const irtps_outputs* outputs, int32_t options, void* ws_dev,
                      size_t ws_bytes, void* stream);

/* ---- served mode ------------------------------------------------------------ */
/* A server runs reconstructions as they arrive (continuous batching): a
 * scheduler thread admits queued jobs in FIFO order when their workspace
 * footprint fits in the device memory the caller handed over, gives new jobs
 * their t = 0 steps, and advances resident jobs by one IRT iteration per round
 * in one set of launches (irtps_batch_solve's engine): every resident job, or,
 * with fill_pixels, the oldest and those with the least remaining work, enough
 * of them to fill the GPU.  Jobs join and leave at iteration boundaries.  Each job's outputs
 * are bit-identical to irtps_solve of that job.  The server reads the job's device inputs and writes
 * its outputs until the job is DONE, FAILED or CANCELLED; host arrays are
 * copied at submission.  All calls are thread-safe. */
typedef struct irtps_server irtps_server;

typedef struct irtps_server_cfg {
    int32_t max_resident_jobs; /* 0: limited by memory only */
    int32_t dry_run;           /* 1: schedule and time jobs without launching any kernel
                                  or touching any buffer (scheduler tests); 0: normal */
    uint64_t table_bytes;      /* head of the workspace kept for job and tile tables
                                  (0: workspace/64, at least 1 MiB) */
    int32_t reserved;          /* must be 0 */
    int32_t fill_pixels;       /* 0: every resident job advances one iteration per round;
                                  > 0: a round advances the oldest resident job, then the jobs
                                  with the least remaining work (iterations left x pixels x spp
                                  x bounces) in that order until their pixels reach fill_pixels;
                                  admission stays FIFO by footprint */
} irtps_server_cfg;

enum { IRTPS_JOB_QUEUED = 0, IRTPS_JOB_RUNNING = 1, IRTPS_JOB_DONE = 2, IRTPS_JOB_FAILED = 3,
       IRTPS_JOB_CANCELLED = 4 };

typedef struct irtps_job_status {
    int32_t state;      /* IRTPS_JOB_* (>= DONE: finished) */
    int32_t status;     /* irtps_status of a finished job */
    int32_t iteration;  /* IRT iterations completed */
    int32_t reserved;
    double submit_s, start_s, end_s;  /* steady-clock seconds; 0 until reached */
} irtps_job_status;

typedef struct irtps_server_stats {
    uint64_t submitted, completed, failed, cancelled;
    int32_t resident, queued;
    uint64_t bytes_in_use, bytes_budget;  /* job workspaces in use / available */
    uint64_t iterations;                  /* scheduling rounds run */
    double p50_latency_s, p99_latency_s;  /* submit -> done, over completed jobs */
    double jobs_per_s;                    /* completed / (last done - first submit) */
} irtps_server_statistics;

/* ws_dev: device memory the server may use (table_bytes of tables, the rest for
 * resident jobs' workspaces), 256-byte aligned; owned by the caller and used
 * until irtps_server_destroy returns. */
int irtps_server_create(const irtps_server_cfg* cfg, void* ws_dev, size_t ws_bytes,
                        irtps_server** server);
/* Queue a job.  IRTPS_ERR_OOM if it could never fit the budget alone. */
int irtps_server_submit(irtps_server* server, const irtps_problem* problem,
                        const irtps_params* params, const irtps_outputs* outputs,
                        uint64_t* job_id);
int irtps_server_poll(irtps_server* server, uint64_t job_id, irtps_job_status* status);
/* Wait until the job finishes (timeout_s < 0: no limit); IRTPS_ERR_BUSY on timeout. */
int irtps_server_wait(irtps_server* server, uint64_t job_id, double timeout_s,
                      irtps_job_status* status);
/* A queued job is dropped; a resident one stops at the next iteration boundary. */
int irtps_server_cancel(irtps_server* server, uint64_t job_id);
int irtps_server_stats(irtps_server* server, irtps_server_statistics* stats);
/* Stops the scheduler (resident jobs are abandoned), waits for the device. */
int irtps_server_destroy(irtps_server* server);

/* ---- tuning ----------------------------------------------------------------- */
/* The tracer's schedule: tile_w (8, 16, 32 or 64) is the width of the pixel
 * chunks a wave of the single-job tracer takes (tile_w x 64 / tile_w pixels)
 * and of the tiles a block of the batched tracer traces (tile_w x 256 / tile_w
 * pixels), and a 64-lane wave shades once ready_batch of its lanes hold a
 * finished segment.  A schedule changes speed only, never a result bit.  Every trace uses, field by field, the forced value
 * (irtps_set_schedule), else the tuning table's entry for its class (device
 * architecture, round(log2 sqrt(W H)), ceil(log2 K), C, B), else 16 x 16 tiles
 * and 32 lanes. */
typedef struct {
    int32_t tile_w;
    int32_t ready_batch;
} irtps_schedule;

#define IRTPS_TUNE_CANDIDATES 20

/* Force tile_w and/or ready_batch for every later trace in the process; 0
 * returns that field to the table / default.  Process-wide, thread-safe. */
int irtps_set_schedule(int32_t tile_w, int32_t ready_batch);
/* The schedule a trace of this class would use now. */
int irtps_get_schedule(int32_t W, int32_t H, int32_t C, int32_t K, int32_t B, irtps_schedule* schedule);
/* Shorthands for the ready_batch field (0..64; 0 = table / default); get
 * returns the forced value or 0. */
int irtps_set_ready_batch(int32_t lanes);
int irtps_get_ready_batch(void);

/* Autotuner: brings the problem to the state its second traced iteration
 * sees (PS of the images, integration, one IRT iteration with the default
 * schedule, then pyramid and direct light; written to outputs and the
 * workspace) and, for each of the IRTPS_TUNE_CANDIDATES schedules (tile_w in
 * 8, 16, 32, 64 times ready_batch in 24, 32, 40, 48, 56, in that order), runs
 * one trace launch that records the chunks' times and then times launches that
 * deal the chunks heaviest first, as the solve's later iterations do (the
 * faster of two; ms_out, if not NULL, receives the times in milliseconds).
 * The fastest goes into the process's tuning table for the problem's class and
 * to *best.  Workspace as for irtps_solve (irtps_workspace_bytes); the call
 * synchronises the stream. */
int irtps_autotune(const irtps_problem* problem, const irtps_params* params, const irtps_outputs* outputs,
                   void* ws_dev, size_t ws_bytes, void* stream, irtps_schedule* best, float* ms_out);
/* The tuning table as JSON: {"arch": "<gcnArchName>", "entries": [{"side",
 * "kcls", "C", "B", "tile_w", "ready_batch", "ms"}, ...]}.  Load merges the
 * entries of a file written on the same architecture (a file for another
 * architecture loads nothing and is not an error); *loaded gets the count. */
int irtps_tuning_save(const char* path);
int irtps_tuning_load(const char* path, int32_t* loaded);
int irtps_tuning_clear(void);
int irtps_tuning_entries(void);

/* ---- timing of the tracer ------------------------------------------------ */
/* irtps_profile_begin() makes this thread's later calls record a hipEvent pair
 * around every tracer launch on the call's stream; irtps_profile_end() waits for
 * those events, returns the summed elapsed milliseconds and the number of
 * launches, destroys the events and stops recording.  Either pointer may be NULL. */
int irtps_profile_begin(void);
int irtps_profile_end(double* trace_ms, int64_t* launches);

/* ---- probes of the device arithmetic (parity checks) -------------------- */
/* Issue-rate calibration (not part of the method): `blocks` blocks of 256
 * threads, each lane running `iters` rounds of 16 independent VALU
 * instructions of one kind -- 0: 32-bit integer shift and xor-add pairs, 1:
 * register moves, 2: fp32 fused multiply-adds; only lanes below active_lanes
 * (1..64) of each wave do the work, the others are masked off.  out_dev
 * receives blocks x 256 uint32 (the chains' values, so that the work is
 * kept).  Counted and timed launches measure the VALU instruction rates the
 * tracer's is compared with (the rate depends on the kind). */
int irtps_probe_valu(int32_t blocks, int32_t iters, int32_t active_lanes, int32_t kind, uint32_t* out_dev,
                     void* stream);
/* Philox4x32-10 of count counters [count][4] under key (seed lo, hi) -> out [count][4]. */
int irtps_probe_philox(int64_t count, const uint32_t* ctr_dev, uint64_t seed,
                       uint32_t* out_dev, void* stream);
/* Cosine-weighted direction about normals [count][3] from uniforms [count][2]. */
int irtps_probe_sample(int64_t count, const float* normals_dev, const float* u_dev,
                       float* dirs_dev, void* stream);
/* Equirectangular texel (row, col) of directions [count][3] -> rc [count][2]. */
int irtps_probe_env_texel(int64_t count, const float* dirs_dev, int32_t env_h,
                          int32_t env_w, int32_t* rc_dev, void* stream);
/* First hit of rays from samples ij [count][2] along dirs [count][3] on a
 * W x H surface with its pyramid (irtps_build_pyramid); q [count][2] = shading
 * sample, or (-1, -1) on escape.  flat != 0 walks every crossing, flat == 0
 * skips pyramid cells; both must give the same q. */
int irtps_probe_traverse(int32_t W, int32_t H, const float* depth_dev,
                         const float* pyramid_dev, int32_t flat, int64_t count,
                         const int32_t* ij_dev, const float* dirs_dev, int32_t* q_dev,
                         void* stream);

#ifdef __cplusplus
}
#endif
#endif /* IRTPS_H */
