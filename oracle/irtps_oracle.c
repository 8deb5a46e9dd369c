/*
 * irtps_oracle.c -- plain CPU oracle of IRT-PS (arXiv 1811.02357).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It is written
 * straight from the paper's stages (Sec. IV) and equations, one plain loop per
 * step, in binary32 with the operation order spelled out (see the header for why
 * binary32).  Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp.
 * OpenMP only spreads independent pixels over threads; no result depends on it.
 */
#include "irtps_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159274f /* binary32 nearest to pi */

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11).  Each round multiplies words 0 and 2 by the two round
 * multipliers, splits the 64-bit products into high and low halves, xors the
 * high halves with the other two words and the key, and permutes; the key is
 * bumped by the two Weyl constants between rounds. */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n1 = lo1;
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    const uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* 24-bit uniform in [0,1): top 24 bits of a word times 2^-24 (exact). */
static float u24(uint32_t r) { return (float)(r >> 8) * 0x1p-24f; }

/* ------------------------------------------------------------------------- */
/* sin(pi/2 f) and cos(pi/2 f): Taylor coefficients (pi/2)^m / m! with alternating
 * signs, rounded to binary32, evaluated by Horner's rule in f^2 with fmaf. */
float or_sin_quarter(float f) {
    const float f2 = f * f;
    float p = 0x1.e8f434p-25f;
    p = fmaf(p, f2, -0x1.e30750p-19f);
    p = fmaf(p, f2, 0x1.507834p-13f);
    p = fmaf(p, f2, -0x1.32d2ccp-8f);
    p = fmaf(p, f2, 0x1.466bc6p-4f);
    p = fmaf(p, f2, -0x1.4abbcep-1f);
    p = fmaf(p, f2, 0x1.921fb6p+0f);
    return p * f;
}

float or_cos_quarter(float f) {
    const float f2 = f * f;
    float p = -0x1.b6e250p-28f;
    p = fmaf(p, f2, 0x1.f9d38ap-22f);
    p = fmaf(p, f2, -0x1.a6d1f2p-16f);
    p = fmaf(p, f2, 0x1.e1f506p-11f);
    p = fmaf(p, f2, -0x1.55d3c8p-6f);
    p = fmaf(p, f2, 0x1.03c1f0p-2f);
    p = fmaf(p, f2, -0x1.3bd3ccp+0f);
    p = fmaf(p, f2, 0x1.000000p+0f);
    return p;
}

/* arctan(u) for |u| <= tan(pi/8): the alternating odd series 1/(2m+1), through u^17. */
static float atan_series(float u) {
    const float u2 = u * u;
    float p = 0x1.e1e1e2p-5f;
    p = fmaf(p, u2, -0x1.111112p-4f);
    p = fmaf(p, u2, 0x1.3b13b2p-4f);
    p = fmaf(p, u2, -0x1.745d18p-4f);
    p = fmaf(p, u2, 0x1.c71c72p-4f);
    p = fmaf(p, u2, -0x1.24924ap-3f);
    p = fmaf(p, u2, 0x1.99999ap-3f);
    p = fmaf(p, u2, -0x1.555556p-2f);
    p = fmaf(p, u2, 0x1.000000p+0f);
    return p * u;
}

float or_atan2(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = (ax > ay) ? ax : ay;
    const float mn = (ax > ay) ? ay : ax;
    if (mx == 0.0f) return 0.0f;
    const float r = mn / mx; /* in [0,1] */
    float a;
    if (r > 0x1.a8279ap-2f) { /* tan(pi/8): atan r = pi/4 + atan((r-1)/(r+1)) */
        const float u = (r - 1.0f) / (r + 1.0f);
        a = 0x1.921fb6p-1f + atan_series(u);
    } else {
        a = atan_series(r);
    }
    if (ay > ax) a = 0x1.921fb6p+0f - a;
    if (x < 0.0f) a = OR_PI - a;
    if (y < 0.0f) a = -a;
    return a;
}

/* Element-wise forms of the three functions above, for exhaustive checks. */
void or_sincos_quarter_n(long long count, const float* f, float* s, float* c) {
    for (long long x = 0; x < count; ++x) {
        s[x] = or_sin_quarter(f[x]);
        c[x] = or_cos_quarter(f[x]);
    }
}

void or_atan2_n(long long count, const float* y, const float* x, float* a) {
    for (long long e = 0; e < count; ++e) a[e] = or_atan2(y[e], x[e]);
}

/* ------------------------------------------------------------------------- */
/* Cosine-weighted hemisphere sample (Malley's method: uniform on the unit disc,
 * lifted to the hemisphere) about the unit normal n.  The tangent frame is the
 * branchless orthonormal basis of Duff et al., "Building an Orthonormal Basis,
 * Revisited", JCGT 6(1), 2017. */
void or_sample_cosine(const float n[3], float u1, float u2, float d[3]) {
    const float rr = sqrtf(u1);
    const float lz = sqrtf(1.0f - u1);
    const int q = (int)(u2 * 4.0f);          /* quadrant 0..3 */
    const float f = u2 * 4.0f - (float)q;   /* exact, in [0,1) */
    const float c = or_cos_quarter(f), s = or_sin_quarter(f);
    float cx, sy;
    switch (q) {
        case 0: cx = c; sy = s; break;
        case 1: cx = -s; sy = c; break;
        case 2: cx = -c; sy = -s; break;
        default: cx = s; sy = -c; break;
    }
    const float lx = rr * cx;
    const float ly = rr * sy;

    const float nx = n[0], ny = n[1], nz = n[2];
    const float sg = copysignf(1.0f, nz);
    const float a = -1.0f / (sg + nz);
    const float b = (nx * ny) * a;
    const float tx = 1.0f + ((sg * nx) * nx) * a;
    const float ty = sg * b;
    const float tz = -(sg * nx);
    const float bx = b;
    const float by = sg + (ny * ny) * a;
    const float bz = -ny;
    d[0] = fmaf(lx, tx, fmaf(ly, bx, lz * nx));
    d[1] = fmaf(lx, ty, fmaf(ly, by, lz * ny));
    d[2] = fmaf(lx, tz, fmaf(ly, bz, lz * nz));
}

/* Equirectangular map: row i covers polar angle [i pi/He, (i+1) pi/He) from +z,
 * column j covers azimuth [2 pi j/We, 2 pi (j+1)/We) from +x toward +y. */
void or_env_texel(const float d[3], int He, int We, int* row, int* col) {
    const float rxy = sqrtf(fmaf(d[0], d[0], d[1] * d[1]));
    const float theta = or_atan2(rxy, d[2]);          /* [0, pi] */
    float phi = or_atan2(d[1], d[0]);                 /* [-pi, pi] */
    if (phi < 0.0f) phi = phi + 0x1.921fb6p+2f;       /* [0, 2 pi] */
    int i = (int)((theta * 0x1.45f306p-2f) * (float)He);
    int j = (int)((phi * 0x1.45f306p-3f) * (float)We);
    if (i < 0) i = 0;
    if (i > He - 1) i = He - 1;
    if (j < 0) j = 0;
    if (j > We - 1) j = We - 1;
    *row = i;
    *col = j;
}

/* ------------------------------------------------------------------------- */
/* Ray against the grid-line heightfield.  The surface is the piecewise-linear
 * interpolation of the samples along every grid line; the ray starts at a
 * sample and is tested at each crossing with a grid line, in order of t (a tie
 * goes to the x-line first).  A crossing hits when the ray lies strictly below
 * the surface there; the shading sample is the nearer end of that grid segment.
 * The ray escapes at the first crossing outside the sample domain, or as soon as
 * it is at or above the highest sample while not descending. */
int or_traverse(const float* H, int W, int Hh, float hmax, int i0, int j0,
                const float d[3], int* qi, int* qj) {
    const float dx = d[0], dy = d[1], dz = d[2];
    if (dx == 0.0f && dy == 0.0f) return OR_MISS;
    const float ox = (float)i0, oy = (float)j0, oz = H[(size_t)j0 * W + i0];
    const int sx = signbit(dx) ? -1 : 1;
    const int sy = signbit(dy) ? -1 : 1;
    const float inv_dx = 1.0f / dx;
    const float inv_dy = 1.0f / dy;
    int mx = 1, my = 1;
    float tX = (float)(sx * mx) * inv_dx;
    float tY = (float)(sy * my) * inv_dy;
    for (;;) {
        if (isinf(tX) && isinf(tY)) return OR_MISS;
        if (tX <= tY) { /* crossing with the vertical grid line x = X */
            const int X = i0 + sx * mx;
            if (X < 0 || X > W - 1) return OR_MISS;
            const float y = fmaf(tX, dy, oy);
            if (!(y >= 0.0f && y <= (float)(Hh - 1))) return OR_MISS;
            const int y0 = (int)floorf(y);
            const float f = y - (float)y0;
            float h;
            if (f == 0.0f) {
                h = H[(size_t)y0 * W + X];
            } else {
                const float h0 = H[(size_t)y0 * W + X], h1 = H[(size_t)(y0 + 1) * W + X];
                h = fmaf(f, h1 - h0, h0);
                const float lo = (h0 < h1) ? h0 : h1, hi = (h0 < h1) ? h1 : h0;
                if (h < lo) h = lo;
                if (h > hi) h = hi;
            }
            const float z = fmaf(tX, dz, oz);
            if (z < h) {
                *qi = X;
                *qj = (f < 0.5f) ? y0 : y0 + 1;
                return OR_HIT;
            }
            if (z >= hmax && dz >= 0.0f) return OR_MISS;
            ++mx;
            tX = (float)(sx * mx) * inv_dx;
        } else { /* crossing with the horizontal grid line y = Y */
            const int Y = j0 + sy * my;
            if (Y < 0 || Y > Hh - 1) return OR_MISS;
            const float x = fmaf(tY, dx, ox);
            if (!(x >= 0.0f && x <= (float)(W - 1))) return OR_MISS;
            const int x0 = (int)floorf(x);
            const float f = x - (float)x0;
            float h;
            if (f == 0.0f) {
                h = H[(size_t)Y * W + x0];
            } else {
                const float h0 = H[(size_t)Y * W + x0], h1 = H[(size_t)Y * W + x0 + 1];
                h = fmaf(f, h1 - h0, h0);
                const float lo = (h0 < h1) ? h0 : h1, hi = (h0 < h1) ? h1 : h0;
                if (h < lo) h = lo;
                if (h > hi) h = hi;
            }
            const float z = fmaf(tY, dz, oz);
            if (z < h) {
                *qi = (f < 0.5f) ? x0 : x0 + 1;
                *qj = Y;
                return OR_HIT;
            }
            if (z >= hmax && dz >= 0.0f) return OR_MISS;
            ++my;
            tY = (float)(sy * my) * inv_dy;
        }
    }
}

/* Many rays at once (independent), for the traversal checks. */
void or_traverse_n(const float* H, int W, int Hh, long long count, const int* ij,
                   const float* d, int* q) {
    float hmax = H[0];
    for (size_t p = 1; p < (size_t)W * Hh; ++p)
        if (H[p] > hmax) hmax = H[p];
    for (long long r = 0; r < count; ++r) {
        int qi = -1, qj = -1;
        const int hit = or_traverse(H, W, Hh, hmax, ij[2 * r], ij[2 * r + 1], d + 3 * r, &qi, &qj);
        q[2 * r] = hit ? qi : -1;
        q[2 * r + 1] = hit ? qj : -1;
    }
}

void or_sample_cosine_n(long long count, const float* n, const float* u, float* d) {
    for (long long r = 0; r < count; ++r) or_sample_cosine(n + 3 * r, u[2 * r], u[2 * r + 1], d + 3 * r);
}

void or_env_texel_n(long long count, const float* d, int He, int We, int* rc) {
    for (long long r = 0; r < count; ++r) or_env_texel(d + 3 * r, He, We, rc + 2 * r, rc + 2 * r + 1);
}

void or_philox_n(long long count, const uint32_t* ctr, const uint32_t key[2], uint32_t* out) {
    for (long long r = 0; r < count; ++r) or_philox4x32_10(ctr + 4 * r, key, out + 4 * r);
}

static float max_height(const float* H, size_t npx) {
    float m = H[0];
    for (size_t p = 1; p < npx; ++p)
        if (H[p] > m) m = H[p];
    return m;
}

/* ------------------------------------------------------------------------- */
/* Eq.3-4: the lights stacked row-wise, scaled by their intensities, form L; the
 * least-squares solve of A = rho L n is g = (L^T L)^-1 L^T A.  The 3x3 inverse is
 * the adjugate over the determinant, in binary64. */
int or_ps_matrix(int K, const float* l, const float* s, float* M) {
    if (K < 3) return -1;
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int k = 0; k < K; ++k) {
        const double sk = s ? (double)s[k] : 1.0;
        double Lk[3];
        for (int a = 0; a < 3; ++a) Lk[a] = sk * (double)l[3 * k + a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A[a][b] = A[a][b] + Lk[a] * Lk[b];
    }
    double cof[3][3];
    cof[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    cof[0][1] = -(A[1][0] * A[2][2] - A[1][2] * A[2][0]);
    cof[0][2] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    cof[1][0] = -(A[0][1] * A[2][2] - A[0][2] * A[2][1]);
    cof[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
    cof[1][2] = -(A[0][0] * A[2][1] - A[0][1] * A[2][0]);
    cof[2][0] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
    cof[2][1] = -(A[0][0] * A[1][2] - A[0][2] * A[1][0]);
    cof[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
    const double det = A[0][0] * cof[0][0] + A[0][1] * cof[0][1] + A[0][2] * cof[0][2];
    const double tr3 = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
    /* det / (trace/3)^3 is the ratio of the geometric to the arithmetic mean of
     * the eigenvalues, cubed: 1 for isotropic lights, 0 for coplanar ones. */
    if (!(det > 1e-7 * tr3 * tr3 * tr3)) return -1;
    double inv[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) inv[a][b] = cof[b][a] / det;
    for (int k = 0; k < K; ++k) {
        const double sk = s ? (double)s[k] : 1.0;
        double Lk[3];
        for (int a = 0; a < 3; ++a) Lk[a] = sk * (double)l[3 * k + a];
        for (int a = 0; a < 3; ++a)
            M[(size_t)a * K + k] = (float)(inv[a][0] * Lk[0] + inv[a][1] * Lk[1] + inv[a][2] * Lk[2]);
    }
    return 0;
}

/* Eq.4 per pixel and channel; the normal is the direction and the albedo the
 * length of the solved vector.  Colour: one solve per channel, normal from the
 * channel sum. */
void or_ps_solve(int W, int Hh, int C, int K, const float* M, const float* A,
                 float* n, float* rho) {
    const size_t npx = (size_t)W * Hh;
    for (size_t p = 0; p < npx; ++p) {
        float sx = 0.0f, sy = 0.0f, sz = 0.0f;
        for (int c = 0; c < C; ++c) {
            float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
            for (int k = 0; k < K; ++k) {
                const float a = A[((size_t)k * C + c) * npx + p];
                g0 = fmaf(M[0 * K + k], a, g0);
                g1 = fmaf(M[1 * K + k], a, g1);
                g2 = fmaf(M[2 * K + k], a, g2);
            }
            rho[(size_t)c * npx + p] = sqrtf(fmaf(g0, g0, fmaf(g1, g1, g2 * g2)));
            sx = sx + g0;
            sy = sy + g1;
            sz = sz + g2;
        }
        const float len = sqrtf(fmaf(sx, sx, fmaf(sy, sy, sz * sz)));
        if (len > 0.0f) {
            n[3 * p + 0] = sx / len;
            n[3 * p + 1] = sy / len;
            n[3 * p + 2] = sz / len;
        } else {
            n[3 * p + 0] = 0.0f;
            n[3 * p + 1] = 0.0f;
            n[3 * p + 2] = 1.0f;
        }
    }
}

/* Eq.4 restricted, per pixel, to the lights that reach it (the paper's shadow
 * condition: at least three lights are needed for the solve).  A light is kept
 * at pixel p when its direct irradiance S[p][k] = s_k max(0, n_t . l_k) V_k(H_t)
 * is positive, i.e. it faces the current normal and its shadow ray escapes the
 * current surface.  With at least three kept lights whose 3x3 normal matrix
 * passes the same conditioning test as or_ps_matrix, the pixel's own solve
 * matrix M_p = (L_p^T L_p)^-1 L_p^T is built in binary64 from the kept rows (in
 * light order), rounded to binary32, and applied like M; otherwise the pixel
 * takes the all-light M.  The normal and albedo then follow as in or_ps_solve. */
static int masked_matrix(int K, const float* l, const float* s, const float* Sp, float* Mp) {
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    int kept = 0;
    for (int k = 0; k < K; ++k) {
        if (!(Sp[k] > 0.0f)) continue;
        ++kept;
        const double sk = s ? (double)s[k] : 1.0;
        double Lk[3];
        for (int a = 0; a < 3; ++a) Lk[a] = sk * (double)l[3 * k + a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A[a][b] = A[a][b] + Lk[a] * Lk[b];
    }
    if (kept < 3) return -1;
    double cof[3][3];
    cof[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    cof[0][1] = -(A[1][0] * A[2][2] - A[1][2] * A[2][0]);
    cof[0][2] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    cof[1][0] = -(A[0][1] * A[2][2] - A[0][2] * A[2][1]);
    cof[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
    cof[1][2] = -(A[0][0] * A[2][1] - A[0][1] * A[2][0]);
    cof[2][0] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
    cof[2][1] = -(A[0][0] * A[1][2] - A[0][2] * A[1][0]);
    cof[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
    const double det = A[0][0] * cof[0][0] + A[0][1] * cof[0][1] + A[0][2] * cof[0][2];
    const double tr3 = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
    if (!(det > 1e-7 * tr3 * tr3 * tr3)) return -1;
    double inv[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) inv[a][b] = cof[b][a] / det;
    for (int k = 0; k < K; ++k) {
        if (!(Sp[k] > 0.0f)) {
            Mp[0 * K + k] = Mp[1 * K + k] = Mp[2 * K + k] = 0.0f;
            continue;
        }
        const double sk = s ? (double)s[k] : 1.0;
        double Lk[3];
        for (int a = 0; a < 3; ++a) Lk[a] = sk * (double)l[3 * k + a];
        for (int a = 0; a < 3; ++a)
            Mp[(size_t)a * K + k] = (float)(inv[a][0] * Lk[0] + inv[a][1] * Lk[1] + inv[a][2] * Lk[2]);
    }
    return 0;
}

int or_ps_solve_masked(int W, int Hh, int C, int K, const float* l, const float* s, const float* A,
                       const float* S, float* n, float* rho) {
    const size_t npx = (size_t)W * Hh;
    float* M = (float*)malloc(sizeof(float) * 3 * K);
    float* Mp = (float*)malloc(sizeof(float) * 3 * K);
    if (or_ps_matrix(K, l, s, M) != 0) {
        free(M);
        free(Mp);
        return -1;
    }
    for (size_t p = 0; p < npx; ++p) {
        const float* Sp = S + p * K;
        const int own = masked_matrix(K, l, s, Sp, Mp) == 0;
        const float* Mu = own ? Mp : M;
        float sx = 0.0f, sy = 0.0f, sz = 0.0f;
        for (int c = 0; c < C; ++c) {
            float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
            for (int k = 0; k < K; ++k) {
                if (own && !(Sp[k] > 0.0f)) continue; /* a dropped light adds nothing */
                const float a = A[((size_t)k * C + c) * npx + p];
                g0 = fmaf(Mu[0 * K + k], a, g0);
                g1 = fmaf(Mu[1 * K + k], a, g1);
                g2 = fmaf(Mu[2 * K + k], a, g2);
            }
            rho[(size_t)c * npx + p] = sqrtf(fmaf(g0, g0, fmaf(g1, g1, g2 * g2)));
            sx = sx + g0;
            sy = sy + g1;
            sz = sz + g2;
        }
        const float len = sqrtf(fmaf(sx, sx, fmaf(sy, sy, sz * sz)));
        if (len > 0.0f) {
            n[3 * p + 0] = sx / len;
            n[3 * p + 1] = sy / len;
            n[3 * p + 2] = sz / len;
        } else {
            n[3 * p + 0] = 0.0f;
            n[3 * p + 1] = 0.0f;
            n[3 * p + 2] = 1.0f;
        }
    }
    free(M);
    free(Mp);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The known environment as geometry (Sec. IV, stages 0, 3 and 4: the surface
 * sits in a Cornell box).  Four vertical walls stand on the borders of the
 * sample grid, x = 0, x = W - 1, y = 0 and y = Hh - 1, from below the surface
 * up to height Z; above them the box is open to the environment map. */

/* Does a ray from (x0, y0, z0) along d (d[2] > 0) leave through the open top,
 * i.e. is it still inside the walls' footprint when it reaches height Z?
 * Starting at or above Z it is out already. */
static int box_top_exit(int W, int Hh, float Z, float x0, float y0, float z0, const float d[3]) {
    if (z0 >= Z) return 1;
    const float t = (Z - z0) / d[2];
    const float x = fmaf(t, d[0], x0), y = fmaf(t, d[1], y0);
    return x >= 0.0f && x <= (float)(W - 1) && y >= 0.0f && y <= (float)(Hh - 1);
}

/* A wall coordinate scaled to texels: floor, clamped to [0, n - 1]. */
static int texel_index(float f, int n) {
    if (!(f >= 0.0f)) return 0;
    if (f >= (float)(n - 1)) return n - 1;
    return (int)f;
}

int or_box_wall(int W, int Hh, const or_box* b, int i0, int j0, float z0, const float d[3], int* texel) {
    const float xmax = (float)(W - 1), ymax = (float)(Hh - 1);
    const float x0 = (float)i0, y0 = (float)j0;
    /* travel to the wall plane ahead in x and in y */
    float tx = INFINITY, ty = INFINITY;
    if (d[0] > 0.0f) tx = (xmax - x0) / d[0];
    else if (d[0] < 0.0f) tx = -x0 / d[0];
    if (d[1] > 0.0f) ty = (ymax - y0) / d[1];
    else if (d[1] < 0.0f) ty = -y0 / d[1];
    const int xwall = tx <= ty; /* a corner counts as the x wall */
    const float t = xwall ? tx : ty;
    if (t == INFINITY) return -1; /* straight up */
    const float zw = fmaf(t, d[2], z0);
    if (!(zw < b->Z)) return -1; /* over the walls */
    const int wall = xwall ? (d[0] > 0.0f ? 1 : 0) : (d[1] > 0.0f ? 3 : 2);
    const float u = xwall ? fmaf(t, d[1], y0) : fmaf(t, d[0], x0); /* position along the wall */
    const float len = xwall ? ymax : xmax;
    const int col = texel_index((u / len) * (float)b->tw, b->tw);
    const int row = texel_index((zw / b->Z) * (float)b->th, b->th);
    *texel = (wall * b->th + row) * b->tw + col;
    return wall;
}

/* Eq.2 on the walls' inner faces at texel centres, without the albedo: a wall
 * faces into the box (normals +x, -x, +y, -y for walls 0..3), so its cosine
 * with light k is a coordinate of l_k; the light reaches the point when its
 * ray leaves through the open top (the walls shade each other; the surface
 * casts no shadow on them). */
void or_box_shade(int W, int Hh, int K, const or_box* b, const float* l, const float* s, float* Sw) {
    const float xmax = (float)(W - 1), ymax = (float)(Hh - 1);
    for (int wall = 0; wall < 4; ++wall)
        for (int row = 0; row < b->th; ++row)
            for (int col = 0; col < b->tw; ++col) {
                const float len = wall < 2 ? ymax : xmax;
                const float u = (((float)col + 0.5f) / (float)b->tw) * len;
                const float z = (((float)row + 0.5f) / (float)b->th) * b->Z;
                const float px = wall == 0 ? 0.0f : (wall == 1 ? xmax : u);
                const float py = wall == 2 ? 0.0f : (wall == 3 ? ymax : u);
                float* out = Sw + ((size_t)(wall * b->th + row) * b->tw + col) * K;
                for (int k = 0; k < K; ++k) {
                    const float* lk = l + 3 * k;
                    const float c = wall == 0 ? lk[0] : (wall == 1 ? -lk[0] : (wall == 2 ? lk[1] : -lk[1]));
                    float v = 0.0f;
                    if (c > 0.0f && box_top_exit(W, Hh, b->Z, px, py, z, lk)) v = (s ? s[k] : 1.0f) * c;
                    out[k] = v;
                }
            }
}

/* Eq.2 at every sample without the albedo: the irradiance from light k, zero
 * where the sample faces away or a shadow ray towards the light hits the
 * surface (or, with walls of height Z > 0, meets a wall). */
static void direct_pixel(int W, int Hh, int K, const float* H, float hmax, const float* n,
                         const float* l, const float* s, float Z, size_t p, float* out) {
    const int i = (int)(p % W), j = (int)(p / W);
    for (int k = 0; k < K; ++k) {
        const float* lk = l + 3 * k;
        const float c = fmaf(n[3 * p + 0], lk[0], fmaf(n[3 * p + 1], lk[1], n[3 * p + 2] * lk[2]));
        float v = 0.0f;
        if (c > 0.0f) {
            int qi, qj;
            int blocked = or_traverse(H, W, Hh, hmax, i, j, lk, &qi, &qj);
            if (Z > 0.0f && !box_top_exit(W, Hh, Z, (float)i, (float)j, H[p], lk)) blocked = 1;
            if (!blocked) v = (s ? s[k] : 1.0f) * c;
        }
        out[k] = v;
    }
}

void or_direct_box(int W, int Hh, int K, const float* H, const float* n, const float* l, const float* s,
                   float Z, float* S) {
    const size_t npx = (size_t)W * Hh;
    const float hmax = max_height(H, npx);
#pragma omp parallel for schedule(dynamic, 16)
    for (long long pp = 0; pp < (long long)npx; ++pp)
        direct_pixel(W, Hh, K, H, hmax, n, l, s, Z, (size_t)pp, S + (size_t)pp * K);
}

void or_direct(int W, int Hh, int K, const float* H, const float* n,
               const float* l, const float* s, float* S) {
    or_direct_box(W, Hh, K, H, n, l, s, 0.0f, S);
}

/* The same at the listed samples only: S_sel[m][k] for pixel index pix[m]. */
void or_direct_at(int W, int Hh, int K, const float* H, const float* n,
                  const float* l, const float* s, long long count, const long long* pix, float* S_sel) {
    const float hmax = max_height(H, (size_t)W * Hh);
#pragma omp parallel for schedule(dynamic, 4)
    for (long long m = 0; m < count; ++m)
        direct_pixel(W, Hh, K, H, hmax, n, l, s, 0.0f, (size_t)pix[m], S_sel + (size_t)m * K);
}

/* ------------------------------------------------------------------------- */
/* Eq.5-7 with a cosine-weighted pdf: for a Lambertian surface each sample
 * contributes pi times the incident radiance times the albedo.  A path from
 * pixel p picks up, at each surface hit q, the Lambertian reflection of the
 * direct irradiance there (albedo rho(q) times S[q][k]) weighted by the product
 * of the albedos met before (the colour products of Fig. 5), and at an escape the
 * environment radiance times pi.  Up to B segments per path; G is the mean over
 * spp paths of the summed contributions. */
typedef struct {
    int W, Hh, C, K;
    const float *H, *n, *rho, *S, *env;
    int He, We, spp, B, t, tag, M;
    float hmax;
    uint32_t key[2];
    const or_box* box; /* walls, or NULL */
} trace_ctx;

/* One pixel's gather: out[k][c] = mean over the spp paths; events added to ev. */
static void trace_pixel(const trace_ctx* x, size_t p, float* out, uint64_t ev[4]) {
    const int W = x->W, C = x->C, K = x->K, B = x->B, spp = x->spp, M = x->M;
    const size_t npx = (size_t)W * x->Hh;
    float hitacc[64 * 4];
    float envacc[4];
    float* acc = hitacc;
    float* big = NULL;
    if ((size_t)K * C > sizeof(hitacc) / sizeof(float)) {
        big = (float*)malloc(sizeof(float) * (size_t)K * C);
        acc = big;
    }
    for (int q = 0; q < K * C; ++q) acc[q] = 0.0f;
    for (int c = 0; c < C; ++c) envacc[c] = 0.0f;
    for (int smp = 0; smp < spp; ++smp) {
        float beta[4];
        for (int c = 0; c < C; ++c) beta[c] = 1.0f;
        int ci = (int)(p % W), cj = (int)(p / W);
        const float* N = x->n + 3 * p;
        for (int b = 1; b <= B; ++b) {
            float u1, u2;
            if (M > 0 && b == 1) {
                const int sa = smp / M, sb = smp % M;
                u1 = ((float)sa + 0.5f) / (float)M;
                u2 = ((float)sb + 0.5f) / (float)M;
            } else {
                const uint32_t ctr[4] = {(uint32_t)p, (uint32_t)smp,
                                         (uint32_t)x->t * 256u + (uint32_t)b, (uint32_t)x->tag};
                uint32_t r[4];
                or_philox4x32_10(ctr, x->key, r);
                u1 = u24(r[0]);
                u2 = u24(r[1]);
            }
            float d[3];
            or_sample_cosine(N, u1, u2, d);
            int qi, qj;
            ++ev[0];
            if (!or_traverse(x->H, W, x->Hh, x->hmax, ci, cj, d, &qi, &qj)) {
                int tex = 0;
                const int wall = x->box ? or_box_wall(W, x->Hh, x->box, ci, cj, x->H[(size_t)cj * W + ci], d, &tex)
                                        : -1;
                if (wall >= 0) {
                    /* a wall: its Lambertian reflection of its own direct light,
                     * weighted like a surface hit; the path ends there */
                    float w[4];
                    for (int c = 0; c < C; ++c) w[c] = beta[c] * x->box->albedo[(size_t)tex * C + c];
                    for (int k = 0; k < K; ++k) {
                        const float sq = x->box->S[(size_t)tex * K + k];
                        for (int c = 0; c < C; ++c) acc[k * C + c] = fmaf(w[c], sq, acc[k * C + c]);
                    }
                } else {
                    int er, ec;
                    or_env_texel(d, x->He, x->We, &er, &ec);
                    const float* L = x->env + ((size_t)er * x->We + ec) * C;
                    for (int c = 0; c < C; ++c) envacc[c] = fmaf(beta[c], OR_PI * L[c], envacc[c]);
                }
                ++ev[2];
                break;
            }
            ++ev[1];
            const size_t q = (size_t)qj * W + qi;
            float w[4];
            for (int c = 0; c < C; ++c) w[c] = beta[c] * x->rho[(size_t)c * npx + q];
            for (int k = 0; k < K; ++k) {
                const float sq = x->S[q * K + k];
                for (int c = 0; c < C; ++c) acc[k * C + c] = fmaf(w[c], sq, acc[k * C + c]);
            }
            if (b < B) {
                ++ev[3];
                for (int c = 0; c < C; ++c) beta[c] = w[c];
                ci = qi;
                cj = qj;
                N = x->n + 3 * q;
            }
        }
    }
    for (int k = 0; k < K; ++k)
        for (int c = 0; c < C; ++c) out[k * C + c] = (acc[k * C + c] + envacc[c]) / (float)spp;
    free(big);
}

static trace_ctx make_trace_ctx(int W, int Hh, int C, int K, const float* H, const float* n,
                                const float* rho, const float* S, const float* env, int He, int We,
                                int spp, int B, uint64_t seed, int t, int tag, int flags) {
    trace_ctx x;
    x.W = W; x.Hh = Hh; x.C = C; x.K = K;
    x.H = H; x.n = n; x.rho = rho; x.S = S; x.env = env;
    x.He = He; x.We = We; x.spp = spp; x.B = B; x.t = t; x.tag = tag;
    x.hmax = max_height(H, (size_t)W * Hh);
    x.key[0] = (uint32_t)seed;
    x.key[1] = (uint32_t)(seed >> 32);
    x.M = 0;
    x.box = NULL;
    if (flags & OR_FLAG_QUADRATURE) {
        x.M = 1;
        while (x.M * x.M < spp) ++x.M;
    }
    return x;
}

/* Eq.5-7 with a cosine-weighted pdf: for a Lambertian surface each sample
 * contributes pi times the incident radiance times the albedo.  A path from
 * pixel p picks up, at each surface hit q, the Lambertian reflection of the
 * direct irradiance there (albedo rho(q) times S[q][k]) weighted by the product
 * of the albedos met before (the colour products of Fig. 5), and at an escape the
 * environment radiance times pi.  Up to B segments per path; G is the mean over
 * spp paths of the summed contributions. */
void or_trace_box(int W, int Hh, int C, int K, const float* H, const float* n,
                  const float* rho, const float* S, const float* env, int He, int We,
                  int spp, int B, uint64_t seed, int t, int tag, int flags,
                  const or_box* box, float* G, or_counters* cnt) {
    const size_t npx = (size_t)W * Hh;
    trace_ctx x = make_trace_ctx(W, Hh, C, K, H, n, rho, S, env, He, We, spp, B, seed, t, tag, flags);
    x.box = box;
    uint64_t tot_seg = 0, tot_hit = 0, tot_esc = 0, tot_cont = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : tot_seg, tot_hit, tot_esc, tot_cont)
    for (long long pp = 0; pp < (long long)npx; ++pp) {
        float out[64 * 4];
        float* o = out;
        float* big = NULL;
        if ((size_t)K * C > sizeof(out) / sizeof(float)) {
            big = (float*)malloc(sizeof(float) * (size_t)K * C);
            o = big;
        }
        uint64_t ev[4] = {0, 0, 0, 0};
        trace_pixel(&x, (size_t)pp, o, ev);
        for (int k = 0; k < K; ++k)
            for (int c = 0; c < C; ++c) G[((size_t)k * C + c) * npx + (size_t)pp] = o[k * C + c];
        tot_seg += ev[0];
        tot_hit += ev[1];
        tot_esc += ev[2];
        tot_cont += ev[3];
        free(big);
    }
    if (cnt) {
        cnt->v[0] += tot_seg;
        cnt->v[1] += tot_hit;
        cnt->v[2] += tot_esc;
        cnt->v[3] += tot_cont;
    }
}

void or_trace(int W, int Hh, int C, int K, const float* H, const float* n,
              const float* rho, const float* S, const float* env, int He, int We,
              int spp, int B, uint64_t seed, int t, int tag, int flags,
              float* G, or_counters* cnt) {
    or_trace_box(W, Hh, C, K, H, n, rho, S, env, He, We, spp, B, seed, t, tag, flags, NULL, G, cnt);
}

/* The same gather at the listed pixels only: G_sel[m][k][c] for pixel pix[m];
 * cnt (may be NULL) gets the events of those pixels. */
void or_trace_at(int W, int Hh, int C, int K, const float* H, const float* n,
                 const float* rho, const float* S, const float* env, int He, int We,
                 int spp, int B, uint64_t seed, int t, int tag, int flags,
                 long long count, const long long* pix, float* G_sel, or_counters* cnt) {
    const trace_ctx x = make_trace_ctx(W, Hh, C, K, H, n, rho, S, env, He, We, spp, B, seed, t, tag, flags);
    uint64_t tot_seg = 0, tot_hit = 0, tot_esc = 0, tot_cont = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tot_seg, tot_hit, tot_esc, tot_cont)
    for (long long m = 0; m < count; ++m) {
        uint64_t ev[4] = {0, 0, 0, 0};
        trace_pixel(&x, (size_t)pix[m], G_sel + (size_t)m * K * C, ev);
        tot_seg += ev[0];
        tot_hit += ev[1];
        tot_esc += ev[2];
        tot_cont += ev[3];
    }
    if (cnt) {
        cnt->v[0] += tot_seg;
        cnt->v[1] += tot_hit;
        cnt->v[2] += tot_esc;
        cnt->v[3] += tot_cont;
    }
}

/* ------------------------------------------------------------------------- */
/* The paper's own variant of the tracer (Sec. IV, the tracing paragraph and
 * Fig. 5): a single path per pixel (sample 0) that reflects exactly r - 1
 * times and leaves for the environment on its r-th ray.  Such a pixel gets the
 * environment colour through r reflections: the albedo products of the hits
 * (c1, c1 c2, ... of Fig. 5) times pi L of the texel the r-th ray reaches.  A
 * path that escapes earlier, or whose r-th ray hits the surface, leaves its
 * pixel without a value.  The rays are the gather's sample 0, segments 1..r
 * (same Philox counters), so where the r-th ray escapes the value equals the
 * gather's with spp 1, B = r and no direct light. */
void or_trace_exact_r(int W, int Hh, int C, const float* H, const float* n, const float* rho,
                      const float* env, int He, int We, int r, uint64_t seed, int t, int tag,
                      float* Er, unsigned char* valid) {
    const size_t npx = (size_t)W * Hh;
    const float hmax = max_height(H, npx);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(dynamic, 64)
    for (long long pp = 0; pp < (long long)npx; ++pp) {
        const size_t p = (size_t)pp;
        float beta[4] = {1.0f, 1.0f, 1.0f, 1.0f};
        int ci = (int)(p % W), cj = (int)(p / W);
        const float* N = n + 3 * p;
        int ok = 0;
        for (int b = 1; b <= r; ++b) {
            const uint32_t ctr[4] = {(uint32_t)p, 0u, (uint32_t)t * 256u + (uint32_t)b, (uint32_t)tag};
            uint32_t rr[4];
            or_philox4x32_10(ctr, key, rr);
            float d[3];
            or_sample_cosine(N, u24(rr[0]), u24(rr[1]), d);
            int qi, qj;
            if (!or_traverse(H, W, Hh, hmax, ci, cj, d, &qi, &qj)) {
                if (b == r) {
                    int er, ec;
                    or_env_texel(d, He, We, &er, &ec);
                    const float* L = env + ((size_t)er * We + ec) * C;
                    for (int c = 0; c < C; ++c) Er[(size_t)c * npx + p] = beta[c] * (OR_PI * L[c]);
                    ok = 1;
                }
                break;
            }
            if (b == r) break; /* the r-th ray met the surface */
            const size_t q = (size_t)qj * W + qi;
            for (int c = 0; c < C; ++c) beta[c] = beta[c] * rho[(size_t)c * npx + q];
            ci = qi;
            cj = qj;
            N = n + 3 * q;
        }
        valid[p] = (unsigned char)ok;
        if (!ok)
            for (int c = 0; c < C; ++c) Er[(size_t)c * npx + p] = 0.0f;
    }
}

/* Non-uniform interpolation of the missing pixels (the paper interpolates the
 * pixels the r-ray images leave empty; it names no method): pull-push over a
 * pyramid of 2 x 2 aggregates.  Pull: a coarse cell holds the weighted mean of
 * its children that carry a value (weights = counts of valid pixels below them,
 * children in the order (0,0), (1,0), (0,1), (1,1), ragged edges with the
 * children that exist), and their summed weight.  Push: from the coarsest level
 * down, a cell without a value takes its parent's.  Pixels with a value keep it;
 * with no valid pixel at all every pixel gets 0.  E is [C][Hh][W]. */
void or_fill_missing(int W, int Hh, int C, float* E, const unsigned char* valid) {
    int lw[40], lh[40];
    int nl = 1;
    lw[0] = W;
    lh[0] = Hh;
    while ((lw[nl - 1] > 1 || lh[nl - 1] > 1) && nl < 40) {
        lw[nl] = (lw[nl - 1] + 1) / 2;
        lh[nl] = (lh[nl - 1] + 1) / 2;
        ++nl;
    }
    float* v[40];
    float* w[40];
    for (int l = 0; l < nl; ++l) {
        v[l] = (float*)calloc((size_t)lw[l] * lh[l] * C, sizeof(float));
        w[l] = (float*)calloc((size_t)lw[l] * lh[l], sizeof(float));
    }
    const size_t npx = (size_t)W * Hh;
    for (size_t p = 0; p < npx; ++p) {
        w[0][p] = valid[p] ? 1.0f : 0.0f;
        for (int c = 0; c < C; ++c) v[0][(size_t)c * npx + p] = valid[p] ? E[(size_t)c * npx + p] : 0.0f;
    }
    for (int l = 0; l + 1 < nl; ++l) {
        const size_t nf = (size_t)lw[l] * lh[l], ncs = (size_t)lw[l + 1] * lh[l + 1];
        for (int J = 0; J < lh[l + 1]; ++J)
            for (int I = 0; I < lw[l + 1]; ++I) {
                const size_t u = (size_t)J * lw[l + 1] + I;
                float den = 0.0f, num[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                for (int dj = 0; dj < 2; ++dj)
                    for (int di = 0; di < 2; ++di) {
                        const int fi = 2 * I + di, fj = 2 * J + dj;
                        if (fi >= lw[l] || fj >= lh[l]) continue;
                        const size_t f = (size_t)fj * lw[l] + fi;
                        const float wf = w[l][f];
                        if (!(wf > 0.0f)) continue;
                        for (int c = 0; c < C; ++c) num[c] = fmaf(wf, v[l][(size_t)c * nf + f], num[c]);
                        den = den + wf;
                    }
                w[l + 1][u] = den;
                for (int c = 0; c < C; ++c) v[l + 1][(size_t)c * ncs + u] = den > 0.0f ? num[c] / den : 0.0f;
            }
    }
    for (int l = nl - 2; l >= 0; --l) {
        const size_t nf = (size_t)lw[l] * lh[l], ncs = (size_t)lw[l + 1] * lh[l + 1];
        for (int j = 0; j < lh[l]; ++j)
            for (int i = 0; i < lw[l]; ++i) {
                const size_t f = (size_t)j * lw[l] + i;
                if (w[l][f] > 0.0f) continue;
                const size_t u = (size_t)(j / 2) * lw[l + 1] + i / 2;
                for (int c = 0; c < C; ++c) v[l][(size_t)c * nf + f] = v[l + 1][(size_t)c * ncs + u];
            }
    }
    for (size_t p = 0; p < npx; ++p)
        for (int c = 0; c < C; ++c) E[(size_t)c * npx + p] = v[0][(size_t)c * npx + p];
    for (int l = 0; l < nl; ++l) {
        free(v[l]);
        free(w[l]);
    }
}

/* ------------------------------------------------------------------------- */
/* Stage 5: the indirect estimate E = rho~ G is removed from the input images.
 * rho~ is either the albedo fitted to the model I0 = rho (S + G) over the K
 * images (default), or the previous PS albedo (literal reading). */
void or_correct(int W, int Hh, int C, int K, int rho_mode, int flags,
                const float* I0, const float* Aprev, const float* G, const float* S,
                const float* rho, float* E, float* Anext) {
    const size_t npx = (size_t)W * Hh;
    for (size_t p = 0; p < npx; ++p) {
        for (int c = 0; c < C; ++c) {
            float rt;
            if (rho_mode == OR_RHO_FIT) {
                float num = 0.0f, den = 0.0f;
                for (int k = 0; k < K; ++k) {
                    const size_t x = ((size_t)k * C + c) * npx + p;
                    const float v = S[p * K + k] + G[x];
                    num = fmaf(I0[x], v, num);
                    den = fmaf(v, v, den);
                }
                rt = (den > 0.0f) ? num / den : 0.0f;
            } else {
                rt = rho[(size_t)c * npx + p];
            }
            for (int k = 0; k < K; ++k) {
                const size_t x = ((size_t)k * C + c) * npx + p;
                const float e = rt * G[x];
                if (E) E[x] = e;
                const float base = (flags & OR_FLAG_LITERAL_CUMULATIVE) ? Aprev[x] : I0[x];
                Anext[x] = base - e;
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Integration of the normals into heights: the least-squares fit of height
 * differences along every grid edge to the mean of the two end-point gradients
 * (p, q) = -(n_x, n_y)/n_z.  Its normal equations are the graph Laplacian with
 * free (Neumann) boundaries, solved by a fixed number of multigrid V-cycles:
 * 2x2 aggregation, coarse edge weights = number of fine edges between the
 * aggregates, red-black Gauss-Seidel (2 before, 2 after), piecewise-constant
 * prolongation scaled by 2.  The result is shifted so that min(H) = 0. */
typedef struct {
    int W, H, shift; /* level size and log2 of the aggregate side */
} mg_level;

static float mg_wx(const mg_level* L, int H0, int J) { /* horizontal edges of row J */
    const int s = 1 << L->shift;
    const int rows = H0 - J * s;
    return (float)(rows < s ? rows : s);
}
static float mg_wy(const mg_level* L, int W0, int I) { /* vertical edges of column I */
    const int s = 1 << L->shift;
    const int cols = W0 - I * s;
    return (float)(cols < s ? cols : s);
}

static void mg_smooth(const mg_level* L, int W0, int H0, float* X, const float* b, int sweeps) {
    for (int sw = 0; sw < sweeps; ++sw) {
        for (int colour = 0; colour < 2; ++colour) {
            for (int J = 0; J < L->H; ++J) {
                for (int I = 0; I < L->W; ++I) {
                    if (((I + J) & 1) != colour) continue;
                    const size_t v = (size_t)J * L->W + I;
                    const float wx = mg_wx(L, H0, J), wy = mg_wy(L, W0, I);
                    float num = b[v], den = 0.0f;
                    if (I > 0) { num = fmaf(wx, X[v - 1], num); den = den + wx; }
                    if (I < L->W - 1) { num = fmaf(wx, X[v + 1], num); den = den + wx; }
                    if (J > 0) { num = fmaf(wy, X[v - L->W], num); den = den + wy; }
                    if (J < L->H - 1) { num = fmaf(wy, X[v + L->W], num); den = den + wy; }
                    if (den > 0.0f) X[v] = num / den;
                }
            }
        }
    }
}

static void mg_residual(const mg_level* L, int W0, int H0, const float* X, const float* b, float* r) {
    for (int J = 0; J < L->H; ++J) {
        for (int I = 0; I < L->W; ++I) {
            const size_t v = (size_t)J * L->W + I;
            const float wx = mg_wx(L, H0, J), wy = mg_wy(L, W0, I);
            float lx = 0.0f;
            if (I > 0) lx = fmaf(wx, X[v] - X[v - 1], lx);
            if (I < L->W - 1) lx = fmaf(wx, X[v] - X[v + 1], lx);
            if (J > 0) lx = fmaf(wy, X[v] - X[v - L->W], lx);
            if (J < L->H - 1) lx = fmaf(wy, X[v] - X[v + L->W], lx);
            r[v] = b[v] - lx;
        }
    }
}

static void mg_vcycle(const mg_level* lv, int nlev, int l, int W0, int H0,
                      float** X, float** b, float* r) {
    const mg_level* L = &lv[l];
    if (l == nlev - 1) {
        mg_smooth(L, W0, H0, X[l], b[l], 16);
        return;
    }
    const mg_level* Lc = &lv[l + 1];
    mg_smooth(L, W0, H0, X[l], b[l], 2);
    mg_residual(L, W0, H0, X[l], b[l], r);
    for (int J = 0; J < Lc->H; ++J) {
        for (int I = 0; I < Lc->W; ++I) {
            float acc = 0.0f;
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) {
                    const int fi = 2 * I + di, fj = 2 * J + dj;
                    if (fi < L->W && fj < L->H) acc = acc + r[(size_t)fj * L->W + fi];
                }
            b[l + 1][(size_t)J * Lc->W + I] = acc;
            X[l + 1][(size_t)J * Lc->W + I] = 0.0f;
        }
    }
    mg_vcycle(lv, nlev, l + 1, W0, H0, X, b, r);
    for (int J = 0; J < L->H; ++J)
        for (int I = 0; I < L->W; ++I) {
            const size_t v = (size_t)J * L->W + I;
            X[l][v] = X[l][v] + 2.0f * X[l + 1][(size_t)(J / 2) * Lc->W + I / 2];
        }
    mg_smooth(L, W0, H0, X[l], b[l], 2);
}

/* Right-hand side of the normal equations for explicit edge targets: tx at
 * [j][i] for the edge (i,j)-(i+1,j), ty at [j][i] for (i,j)-(i,j+1). */
static void rhs_from_targets(int W, int Hh, const float* tx, const float* ty, float* b) {
    for (int j = 0; j < Hh; ++j)
        for (int i = 0; i < W; ++i) {
            const size_t v = (size_t)j * W + i;
            float acc = 0.0f;
            if (i > 0) acc = acc + tx[v - 1];
            if (i < W - 1) acc = acc - tx[v];
            if (j > 0) acc = acc + ty[v - W];
            if (j < Hh - 1) acc = acc - ty[v];
            b[v] = acc;
        }
}

/* Huber shrinkage of an edge residual: the part of r beyond +-delta. */
static float shrink(float r, float delta) {
    if (r > delta) return r - delta;
    if (r < -delta) return r + delta;
    return 0.0f;
}

static void integrate_impl(int W, int Hh, const float* n, const float* Hinit, int cycles, float delta,
                           int rounds, int rcycles, float* Hout) {
    const size_t npx = (size_t)W * Hh;
    float* pg = (float*)malloc(sizeof(float) * npx);
    float* qg = (float*)malloc(sizeof(float) * npx);
    for (size_t v = 0; v < npx; ++v) {
        const float nz = n[3 * v + 2] > 0.05f ? n[3 * v + 2] : 0.05f;
        pg[v] = -(n[3 * v + 0] / nz);
        qg[v] = -(n[3 * v + 1] / nz);
    }
    mg_level lv[40];
    int nlev = 0;
    lv[0].W = W; lv[0].H = Hh; lv[0].shift = 0;
    nlev = 1;
    while ((lv[nlev - 1].W > 4 || lv[nlev - 1].H > 4) && nlev < 40) {
        lv[nlev].W = (lv[nlev - 1].W + 1) / 2;
        lv[nlev].H = (lv[nlev - 1].H + 1) / 2;
        lv[nlev].shift = lv[nlev - 1].shift + 1;
        ++nlev;
    }
    float* X[40];
    float* b[40];
    for (int l = 0; l < nlev; ++l) {
        X[l] = (float*)calloc((size_t)lv[l].W * lv[l].H, sizeof(float));
        b[l] = (float*)calloc((size_t)lv[l].W * lv[l].H, sizeof(float));
    }
    float* r = (float*)malloc(sizeof(float) * npx);
    /* right-hand side: edge targets are the means of the end-point gradients */
    for (int j = 0; j < Hh; ++j)
        for (int i = 0; i < W; ++i) {
            const size_t v = (size_t)j * W + i;
            float acc = 0.0f;
            if (i > 0) acc = acc + (pg[v - 1] + pg[v]) * 0.5f;
            if (i < W - 1) acc = acc - (pg[v] + pg[v + 1]) * 0.5f;
            if (j > 0) acc = acc + (qg[v - W] + qg[v]) * 0.5f;
            if (j < Hh - 1) acc = acc - (qg[v] + qg[v + W]) * 0.5f;
            b[0][v] = acc;
        }
    if (Hinit) memcpy(X[0], Hinit, sizeof(float) * npx);
    for (int c = 0; c < cycles; ++c) mg_vcycle(lv, nlev, 0, W, Hh, X, b, r);
    if (rounds > 0) {
        /* Huber M-estimator by half-quadratic splitting: the Huber cost of an edge
         * residual is the least, over an offset z, of (r - z)^2 / 2 + delta |z|.
         * Alternately z = shrink(r) on every edge for the current surface, and
         * more V-cycles on the least-squares problem whose edge targets are
         * moved by z.  Both steps lower the joint (convex) cost. */
        float* tx = (float*)calloc(npx, sizeof(float));
        float* ty = (float*)calloc(npx, sizeof(float));
        for (int rd = 0; rd < rounds; ++rd) {
            const float* H = X[0];
            for (int j = 0; j < Hh; ++j)
                for (int i = 0; i < W; ++i) {
                    const size_t v = (size_t)j * W + i;
                    if (i < W - 1) {
                        const float g = (pg[v] + pg[v + 1]) * 0.5f;
                        tx[v] = g + shrink((H[v + 1] - H[v]) - g, delta);
                    }
                    if (j < Hh - 1) {
                        const float g = (qg[v] + qg[v + W]) * 0.5f;
                        ty[v] = g + shrink((H[v + W] - H[v]) - g, delta);
                    }
                }
            rhs_from_targets(W, Hh, tx, ty, b[0]);
            for (int c = 0; c < rcycles; ++c) mg_vcycle(lv, nlev, 0, W, Hh, X, b, r);
        }
        free(tx);
        free(ty);
    }
    /* the minimum is taken over X + 0, so that a -0 and a +0 count as one zero */
    float mn = X[0][0] + 0.0f;
    for (size_t v = 1; v < npx; ++v) {
        const float x = X[0][v] + 0.0f;
        if (x < mn) mn = x;
    }
    for (size_t v = 0; v < npx; ++v) Hout[v] = X[0][v] - mn;
    for (int l = 0; l < nlev; ++l) {
        free(X[l]);
        free(b[l]);
    }
    free(r);
    free(pg);
    free(qg);
}

void or_integrate(int W, int Hh, const float* n, const float* Hinit, int cycles, float* Hout) {
    integrate_impl(W, Hh, n, Hinit, cycles, 0.0f, 0, 0, Hout);
}

/* Robust integration (the M-estimator of Sec. IV, stage 1): or_integrate's
 * `cycles` V-cycles, then `rounds` rounds of the Huber M-estimator (threshold
 * delta on the edge residual H_b - H_a - g, pixel units) by half-quadratic
 * splitting, each new edge targets g + shrink(residual) and `rcycles` more
 * V-cycles; then min(H) = 0. */
void or_integrate_robust(int W, int Hh, const float* n, const float* Hinit, int cycles, float delta,
                         int rounds, int rcycles, float* Hout) {
    integrate_impl(W, Hh, n, Hinit, cycles, delta, rounds, rcycles, Hout);
}

/* ------------------------------------------------------------------------- */
/* The walls' direct light for lights (l, s): a copy of *box with S set
 * (caller frees *Sw). */
static or_box shaded_box(int W, int Hh, int K, const or_box* box, const float* l, const float* s, float** Sw) {
    or_box b = *box;
    *Sw = (float*)malloc(sizeof(float) * 4 * (size_t)box->th * box->tw * K);
    or_box_shade(W, Hh, K, box, l, s, *Sw);
    b.S = *Sw;
    return b;
}

int or_render_box(int W, int Hh, int C, int K, const float* H, const float* n,
                  const float* rho, const float* l, const float* s, const float* env,
                  int He, int We, int spp, int B, uint64_t seed, const or_box* box, float* I0,
                  or_counters* cnt) {
    const size_t npx = (size_t)W * Hh;
    float* S = (float*)malloc(sizeof(float) * npx * K);
    float* G = (float*)malloc(sizeof(float) * npx * K * C);
    float* Sw = NULL;
    or_box b;
    if (box) b = shaded_box(W, Hh, K, box, l, s, &Sw);
    or_direct_box(W, Hh, K, H, n, l, s, box ? box->Z : 0.0f, S);
    or_trace_box(W, Hh, C, K, H, n, rho, S, env, He, We, spp, B, seed, 0, OR_TAG_RENDER, 0, box ? &b : NULL, G,
                 cnt);
    free(Sw);
    for (int k = 0; k < K; ++k)
        for (int c = 0; c < C; ++c)
            for (size_t p = 0; p < npx; ++p) {
                const size_t x = ((size_t)k * C + c) * npx + p;
                I0[x] = rho[(size_t)c * npx + p] * (S[p * K + k] + G[x]);
            }
    free(S);
    free(G);
    return 0;
}

int or_render(int W, int Hh, int C, int K, const float* H, const float* n,
              const float* rho, const float* l, const float* s, const float* env,
              int He, int We, int spp, int B, uint64_t seed, float* I0, or_counters* cnt) {
    return or_render_box(W, Hh, C, K, H, n, rho, l, s, env, He, We, spp, B, seed, NULL, I0, cnt);
}

/* The IRT-PS loop (Sec. IV): plain PS and integration of the input images, then
 * T passes of trace -> subtract -> PS -> integrate, each warm-started from the
 * previous surface. */
int or_solve_box(int W, int Hh, int C, int K, const float* I0, const float* l,
                 const float* s, const float* env, int He, int We, int spp, int B,
                 int T, uint64_t seed, int rho_mode, int flags, int cycles_cold,
                 int cycles_warm, float stop_tol, const or_box* box, float* n, float* rho, float* H,
                 float* E, or_counters* cnt) {
    const size_t npx = (size_t)W * Hh;
    if (box && OR_EXACT_R_OF(flags) > 0) return -2; /* the r-ray image has no per-light wall term */
    float* M = (float*)malloc(sizeof(float) * 3 * K);
    if (or_ps_matrix(K, l, s, M) != 0) {
        free(M);
        return -1;
    }
    float* Sw = NULL;
    or_box bx;
    if (box) bx = shaded_box(W, Hh, K, box, l, s, &Sw); /* the lights do not move: once per solve */
    const float Z = box ? box->Z : 0.0f;
    float* A = (float*)malloc(sizeof(float) * npx * K * C);
    float* A2 = (float*)malloc(sizeof(float) * npx * K * C);
    float* S = (float*)malloc(sizeof(float) * npx * K);
    float* G = (float*)malloc(sizeof(float) * npx * K * C);
    float* Hn = (float*)malloc(sizeof(float) * npx);
    memcpy(A, I0, sizeof(float) * npx * K * C);
    or_ps_solve(W, Hh, C, K, M, A, n, rho);
    if (flags & OR_FLAG_ROBUST_INTEGRATION)
        or_integrate_robust(W, Hh, n, NULL, cycles_cold, OR_ROBUST_DELTA, OR_ROBUST_ROUNDS, OR_ROBUST_CYCLES, H);
    else
        or_integrate(W, Hh, n, NULL, cycles_cold, H);
    if (E) memset(E, 0, sizeof(float) * npx * K * C);
    for (int t = 0; t < T; ++t) {
        or_direct_box(W, Hh, K, H, n, l, s, Z, S);
        const int r_exact = OR_EXACT_R_OF(flags);
        if (r_exact > 0) {
            /* the paper's r-ray variant: one environment image, the same for
             * every light, in place of the gather */
            float* Er = (float*)malloc(sizeof(float) * npx * C);
            unsigned char* ok = (unsigned char*)malloc(npx);
            or_trace_exact_r(W, Hh, C, H, n, rho, env, He, We, r_exact, seed, t, OR_TAG_SOLVE, Er, ok);
            or_fill_missing(W, Hh, C, Er, ok);
            for (int k = 0; k < K; ++k)
                for (int c = 0; c < C; ++c)
                    memcpy(G + ((size_t)k * C + c) * npx, Er + (size_t)c * npx, sizeof(float) * npx);
            free(Er);
            free(ok);
        } else {
            or_trace_box(W, Hh, C, K, H, n, rho, S, env, He, We, spp, B, seed, t, OR_TAG_SOLVE,
                         flags & OR_FLAG_QUADRATURE, box ? &bx : NULL, G, cnt);
        }
        or_correct(W, Hh, C, K, rho_mode, flags, I0, A, G, S, rho, E, A2);
        float* tmp = A; A = A2; A2 = tmp;
        if (flags & OR_FLAG_SHADOW_AWARE_PS)
            or_ps_solve_masked(W, Hh, C, K, l, s, A, S, n, rho);
        else
            or_ps_solve(W, Hh, C, K, M, A, n, rho);
        if (flags & OR_FLAG_ROBUST_INTEGRATION)
            or_integrate_robust(W, Hh, n, H, cycles_warm, OR_ROBUST_DELTA, OR_ROBUST_ROUNDS, OR_ROBUST_CYCLES, Hn);
        else
            or_integrate(W, Hh, n, H, cycles_warm, Hn);
        /* D_H: the largest change of the surface in this iteration */
        float dh = 0.0f;
        for (size_t p = 0; p < npx; ++p) {
            const float d = fabsf(Hn[p] - H[p]);
            if (d > dh) dh = d;
        }
        memcpy(H, Hn, sizeof(float) * npx);
        if (cnt) cnt->v[4] += 1;
        if (stop_tol > 0.0f && dh < stop_tol) break;
    }
    free(M);
    free(A);
    free(A2);
    free(S);
    free(G);
    free(Hn);
    free(Sw);
    return 0;
}

int or_solve(int W, int Hh, int C, int K, const float* I0, const float* l,
             const float* s, const float* env, int He, int We, int spp, int B,
             int T, uint64_t seed, int rho_mode, int flags, int cycles_cold,
             int cycles_warm, float stop_tol, float* n, float* rho, float* H, float* E,
             or_counters* cnt) {
    return or_solve_box(W, Hh, C, K, I0, l, s, env, He, We, spp, B, T, seed, rho_mode, flags, cycles_cold,
                        cycles_warm, stop_tol, NULL, n, rho, H, E, cnt);
}

void or_box_wall_n(int W, int Hh, const or_box* b, long long count, const int* ij, const float* z0,
                   const float* d, int* wall_texel) {
    for (long long r = 0; r < count; ++r) {
        int tex = -1;
        const int w = or_box_wall(W, Hh, b, ij[2 * r], ij[2 * r + 1], z0[r], d + 3 * r, &tex);
        wall_texel[2 * r] = w;
        wall_texel[2 * r + 1] = w >= 0 ? tex : -1;
    }
}
