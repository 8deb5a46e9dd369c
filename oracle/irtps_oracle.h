/*
 * irtps_oracle.h -- plain, slow CPU oracle of Iterative Ray-Tracing Photometric
 * Stereo (IRT-PS; Khadka, Remagnino, Argyriou, "Object 3D Reconstruction based on
 * Photometric Stereo and Inverted Rendering", arXiv 1811.02357).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent checker of the HIP
 * path: only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant generator
 * with the GPU library.
 *
 * Precision.  The paper fixes none.  Every value of the IRT loop (normals, albedo,
 * heights, gathered radiance) feeds the ray-surface hit tests of the next
 * iteration, and a hit test is a floating-point comparison that decides an
 * integer (which sample is hit).  The oracle therefore takes the loop in the
 * kernel's precision, IEEE binary32, with one stated operation order: every
 * fused multiply-add is written as fmaf, every other operation rounds on its own
 * (built with -ffp-contract=off), divisions and square roots are correctly
 * rounded, and no transcendental function enters compared arithmetic.  Closed
 * forms and exact solvers that pin this oracle are evaluated in binary64.
 *
 * Layouts (row-major, W = width = columns i, Hh = height = rows j, p = j*W + i):
 *   heights H[Hh][W], normals n[Hh][W][3], albedo rho[C][Hh][W],
 *   images / gathered radiance / indirect estimate [K][C][Hh][W],
 *   direct irradiance S[Hh][W][K], environment env[He][We][C] (radiance).
 */
#ifndef IRTPS_ORACLE_H
#define IRTPS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_TAG_SOLVE = 0, OR_TAG_RENDER = 1 };
enum { OR_RHO_FIT = 0, OR_RHO_PREV = 1 };
enum { OR_FLAG_QUADRATURE = 1, OR_FLAG_LITERAL_CUMULATIVE = 2, OR_FLAG_SHADOW_AWARE_PS = 8,
       OR_FLAG_ROBUST_INTEGRATION = 32 };
/* The paper's r-ray variant (flags bits 8-10 hold r = 1..7; 0: the gather). */
#define OR_FLAG_EXACT_R(r) ((r) << 8)
#define OR_EXACT_R_OF(flags) (((flags) >> 8) & 7)
/* The loop's robust integration: Huber threshold (pixel units of the edge
 * residual), rounds, and V-cycles per round. */
#define OR_ROBUST_DELTA 0.1f
#define OR_ROBUST_ROUNDS 6
#define OR_ROBUST_CYCLES 2
enum { OR_MISS = 0, OR_HIT = 1 };

/* counters of one trace: [0] segments, [1] hits, [2] escapes, [3] continuations */
/* segments, surface hits, escapes, continuations, IRT iterations run */
typedef struct { uint64_t v[5]; } or_counters;

/* Philox4x32-10 counter-based generator (Salmon et al., SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* sin and cos of a quarter turn times f, f in [0,1), by truncated Taylor series. */
float or_sin_quarter(float f);
float or_cos_quarter(float f);
/* atan2 in binary32 by octant reduction and the arctangent series; result in [-pi, pi]. */
float or_atan2(float y, float x);

/* Cosine-weighted direction about unit normal n from uniforms (u1,u2) (Malley). */
void or_sample_cosine(const float n[3], float u1, float u2, float d[3]);
/* Equirectangular nearest texel of direction d: row from polar angle, column from azimuth. */
void or_env_texel(const float d[3], int He, int We, int* row, int* col);

/* First crossing of a ray from sample (i0,j0) along d that lies strictly below the
 * grid-line surface.  Returns OR_HIT and the shading sample (qi,qj), or OR_MISS. */
int or_traverse(const float* H, int W, int Hh, float hmax, int i0, int j0,
                const float d[3], int* qi, int* qj);

/* Eq.4 solve matrix M = (L^T L)^-1 L^T, L rows = s_k l_k, built in binary64 and
 * rounded to binary32.  M is [3][K].  Returns 0, or -1 if K < 3 or the lights are
 * (nearly) coplanar. */
int or_ps_matrix(int K, const float* l, const float* s, float* M);

/* Eq.4 per pixel: g_c = M A_c, rho_c = |g_c|, n = (sum_c g_c)/|sum_c g_c|. */
void or_ps_solve(int W, int Hh, int C, int K, const float* M, const float* A,
                 float* n, float* rho);

/* Eq.4 per pixel over the lights that reach it: light k is kept at pixel p
 * when S[p][k] > 0 (it faces n_t and its shadow ray escapes H_t); with at least
 * three kept, well-conditioned lights the pixel's own binary64 solve matrix is
 * used, else the all-light one.  S is [Hh][W][K] from or_direct.  Returns 0, or
 * -1 if the all-light matrix is singular. */
int or_ps_solve_masked(int W, int Hh, int C, int K, const float* l, const float* s, const float* A,
                       const float* S, float* n, float* rho);

/* Direct irradiance S[q][k] = s_k max(0, n(q).l_k) V_k(q) (Eq.2 without albedo). */
void or_direct(int W, int Hh, int K, const float* H, const float* n,
               const float* l, const float* s, float* S);

/* The known environment as geometry (Sec. IV stages 0, 3, 4: a Cornell box):
 * four vertical Lambertian walls on the borders of the sample grid (wall 0 at
 * x = 0, 1 at x = W - 1, 2 at y = 0, 3 at y = Hh - 1, facing into the box) up
 * to height Z > 0, open above to the environment map.  Each wall is a texture
 * of th rows (height 0..Z) by tw columns (along the wall, 0..length). */
typedef struct {
    float Z;
    int th, tw;
    const float* albedo; /* [4][th][tw][C] */
    const float* S;      /* [4][th][tw][K] the walls' direct irradiance (or_box_shade) */
} or_box;
/* The wall a ray from sample (i0, j0) at height z0 along d meets below Z, and
 * its texel (wall th + row) tw + col; -1 when it leaves through the top. */
int or_box_wall(int W, int Hh, const or_box* b, int i0, int j0, float z0, const float d[3], int* texel);
/* Eq.2 on the walls at texel centres: Sw[wall][row][col][k] = s_k max(0, n_wall.l_k)
 * V_k, V_k = 1 when the light's ray leaves through the open top. */
void or_box_shade(int W, int Hh, int K, const or_box* b, const float* l, const float* s, float* Sw);
/* or_direct with the walls (Z > 0) as occluders too. */
void or_direct_box(int W, int Hh, int K, const float* H, const float* n, const float* l, const float* s,
                   float Z, float* S);

/* Monte Carlo gather of indirect light (Eq.5-7): G[k][c][p]. */
void or_trace(int W, int Hh, int C, int K, const float* H, const float* n,
              const float* rho, const float* S, const float* env, int He, int We,
              int spp, int B, uint64_t seed, int t, int tag, int flags,
              float* G, or_counters* cnt);
/* or_trace with the walls: a ray that leaves the surface and meets a wall
 * below Z adds the wall texel's albedo (times the path's albedo product) times
 * its direct irradiance for every light, like a surface hit, and ends; over the
 * walls it takes the environment map.  box->S must be set. */
void or_trace_box(int W, int Hh, int C, int K, const float* H, const float* n,
                  const float* rho, const float* S, const float* env, int He, int We,
                  int spp, int B, uint64_t seed, int t, int tag, int flags,
                  const or_box* box, float* G, or_counters* cnt);
/* Pixel-subset forms (same per-pixel arithmetic) for checks at full image
 * sizes: rows for the pixel indices pix[0..count). */
void or_direct_at(int W, int Hh, int K, const float* H, const float* n,
                  const float* l, const float* s, long long count, const long long* pix, float* S_sel);
void or_trace_at(int W, int Hh, int C, int K, const float* H, const float* n,
                 const float* rho, const float* S, const float* env, int He, int We,
                 int spp, int B, uint64_t seed, int t, int tag, int flags,
                 long long count, const long long* pix, float* G_sel, or_counters* cnt);

/* The paper's r-ray variant of the tracer: per pixel one path (sample 0, the
 * gather's Philox counters) that must reflect r - 1 times and leave on its r-th
 * ray; Er[c][p] = albedo product of the hits times pi L(texel) there, valid[p]
 * = 1; otherwise valid[p] = 0 and Er = 0. */
void or_trace_exact_r(int W, int Hh, int C, const float* H, const float* n, const float* rho,
                      const float* env, int He, int We, int r, uint64_t seed, int t, int tag,
                      float* Er, unsigned char* valid);
/* Pull-push fill of the pixels without a value (valid[p] = 0) of E [C][Hh][W]. */
void or_fill_missing(int W, int Hh, int C, float* E, const unsigned char* valid);

/* Stage-5 subtraction: E = rho~ G, A_next = I0 - E (or A_prev - E). */
void or_correct(int W, int Hh, int C, int K, int rho_mode, int flags,
                const float* I0, const float* Aprev, const float* G, const float* S,
                const float* rho, float* E, float* Anext);

/* Least-squares integration of the normal field into heights, min(H) = 0. */
void or_integrate(int W, int Hh, const float* n, const float* Hinit, int cycles, float* H);

/* Robust integration (Huber M-estimator): or_integrate's V-cycles, then
 * `rounds` rounds of half-quadratic splitting, each moving every edge target g
 * by shrink(H_b - H_a - g, delta) (the part of the residual beyond +-delta)
 * for the current surface and running `rcycles` more V-cycles; min(H) = 0. */
void or_integrate_robust(int W, int Hh, const float* n, const float* Hinit, int cycles, float delta,
                         int rounds, int rcycles, float* H);

/* Forward render I0 = rho (S + G) of a ground-truth surface (tag RENDER). */
int or_render(int W, int Hh, int C, int K, const float* H, const float* n,
              const float* rho, const float* l, const float* s, const float* env,
              int He, int We, int spp, int B, uint64_t seed, float* I0, or_counters* cnt);

/* or_render and or_solve with the walls (box->S is computed inside from the
 * lights; box may be NULL).  or_solve_box returns -2 for walls with the r-ray
 * variant. */
int or_render_box(int W, int Hh, int C, int K, const float* H, const float* n,
                  const float* rho, const float* l, const float* s, const float* env,
                  int He, int We, int spp, int B, uint64_t seed, const or_box* box, float* I0,
                  or_counters* cnt);
int or_solve_box(int W, int Hh, int C, int K, const float* I0, const float* l,
                 const float* s, const float* env, int He, int We, int spp, int B,
                 int T, uint64_t seed, int rho_mode, int flags, int cycles_cold,
                 int cycles_warm, float stop_tol, const or_box* box, float* n, float* rho, float* H,
                 float* E, or_counters* cnt);
void or_box_wall_n(int W, int Hh, const or_box* b, long long count, const int* ij, const float* z0,
                   const float* d, int* wall_texel);

/* The whole IRT-PS loop (Sec. IV): T iterations, or fewer when stop_tol > 0
 * and an iteration changes the surface by less than stop_tol, D_H =
 * max_p |H_{t+1}(p) - H_t(p)| < stop_tol (last paragraph of Sec. IV).  With
 * OR_FLAG_SHADOW_AWARE_PS the PS after each correction keeps, per pixel, only
 * the lights that reach it (or_ps_solve_masked with that iteration's S); the
 * first PS of the input images uses every light.  With OR_FLAG_ROBUST_INTEGRATION
 * every integration is or_integrate_robust (OR_ROBUST_DELTA, _ROUNDS, _CYCLES).
 * With OR_FLAG_EXACT_R(r) the gather is replaced by the r-ray environment image
 * (or_trace_exact_r, then or_fill_missing), the same for every light; spp and
 * B are then unused.  Returns 0 or -1 (singular lights). */
int or_solve(int W, int Hh, int C, int K, const float* I0, const float* l,
             const float* s, const float* env, int He, int We, int spp, int B,
             int T, uint64_t seed, int rho_mode, int flags, int cycles_cold,
             int cycles_warm, float stop_tol, float* n, float* rho, float* H, float* E,
             or_counters* cnt);

/* Element-wise batch forms (independent calls), used by the exhaustive checks. */
void or_sincos_quarter_n(long long count, const float* f, float* s, float* c);
void or_atan2_n(long long count, const float* y, const float* x, float* a);
void or_traverse_n(const float* H, int W, int Hh, long long count, const int* ij,
                   const float* d, int* q);
void or_sample_cosine_n(long long count, const float* n, const float* u, float* d);
void or_env_texel_n(long long count, const float* d, int He, int We, int* rc);
void or_philox_n(long long count, const uint32_t* ctr, const uint32_t key[2], uint32_t* out);

int or_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
