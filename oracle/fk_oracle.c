/*
 * fk_oracle.c -- the oracle: a plain, slow, FP64 CPU implementation of the
 * Monte Carlo (Feynman-Kac) estimator for the gravity forward problem of
 * Donzelli, Bihlo, Kischinhevsky & Farquharson, "Massively parallel stochastic
 * solution of the geophysical gravity problem" (arXiv:1709.07469).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this file.  It shares no code,
 * header, table or constant with the HIP library; the two are written
 * independently and meet only through the seeded inputs the tests build.
 *
 * What it computes (paper section 2, eqs. 1-6 and the per-walk algorithm of
 * section 2.3), in the sign and time convention used throughout:
 *   - X is standard 3-D Brownian motion started at a station x0 and stepped by
 *     Euler-Maruyama, x_{n+1} = x_n + sqrt(dt) * Z_n, Z_n ~ N(0, I_3).  The
 *     paper's walk gamma = sqrt(2) W (eq. 2) is the same process at twice the
 *     clock, so its Delta t equals dt / 2 here.
 *   - The source integral is the trapezoid rule of section 2.3:
 *     I = (dt/2) * sum_n (rho(x_n) + rho(x_{n+1})), the exiting step included
 *     (the paper accumulates before it tests for the exit).
 *   - The walk stops at the first n with x_{n+1} on or outside the domain
 *     (exit time of eq. 3).  Dirichlet data g is read at the exit point.
 *     The domain is a box, or the ball inscribed in a cubic box (the
 *     paper's experiments use a ball of radius 10 km, section 3).
 *   - Per path u_p = g(x_e) - 2*pi*G*I, the sample of
 *     u(x0) = E[g(X_tau)] - (1/2) E[int_0^tau 4 pi G rho(X_s) ds]
 *     which solves Laplace(u) = 4 pi G rho with u = g on the boundary
 *     (eqs. 3-5 with the physical sign of the potential).
 *   - The station estimate is the sample mean of eq. 11, with the unbiased
 *     sample variance and standard error.
 *   - g_z = du/dz by the central difference of eq. 6 / section 4.2, using
 *     the same random stream at x0 + h e_z and x0 - h e_z.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), counter (k, p, s, m) = (block index,
 * path, station, problem) and key (seed low word, seed high word), mapped to
 * normals with the Box-Muller transform.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off -lm.
 * Contraction is off; every fused multiply-add is an explicit fma().
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Data types (the oracle's own; nothing here is shared with the library).   */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lo[3], hi[3];
} fko_box;

typedef struct {
    const float *rho;       /* voxel densities, x fastest: rho[(k*ny + j)*nx + i] */
    int32_t n[3];           /* nx, ny, nz (0 => no grid) */
    double origin[3];       /* corner of voxel (0,0,0) */
    double spacing[3];      /* voxel edge lengths */
    const double *prisms;   /* n_prisms x 7: lo[3], hi[3], rho */
    int32_t n_prisms;
    const double *spheres;  /* n_spheres x 5: c[3], radius, rho */
    int32_t n_spheres;
} fko_source;

enum { FKO_BC_ZERO = 0, FKO_BC_QUADRATIC = 1, FKO_BC_POINT_MASSES = 2,
       FKO_BC_PRISMS = 3, FKO_BC_FACE_GRID = 4 };
enum { FKO_EXIT_OVERSHOOT = 0, FKO_EXIT_INTERSECT = 1, FKO_EXIT_BRIDGE = 2 };
enum { FKO_STREAM_F64 = 0, FKO_STREAM_F32 = 1 };
enum { FKO_PAIR_CRN = 0, FKO_PAIR_INDEPENDENT = 1 };
enum { FKO_DOMAIN_BOX = 0, FKO_DOMAIN_BALL = 1 };

typedef struct {
    int32_t kind;
    const double *data;
    int64_t n_items;
    int32_t face_n[6][2];   /* FACE_GRID: nodes along (a, b) of each face */
} fko_bc;

typedef struct {
    double dt;
    uint64_t seed;
    double G;
    double h;               /* g_z difference step; 0 => sqrt(dt) */
    int32_t stream;         /* FKO_STREAM_F64 or FKO_STREAM_F32 */
    int32_t exit_rule;
    int32_t pairing;
    int32_t domain;         /* FKO_DOMAIN_BOX, or FKO_DOMAIN_BALL: the ball inscribed in the (cubic) box */
    int64_t max_steps;
    uint32_t problem_id;
    uint32_t pad2_;
    int64_t path_offset;
} fko_params;

typedef struct {
    double mean, var, se;
    int64_t n;
    double mean_steps;
    int64_t max_steps, n_trunc;
} fko_stat;

#define FKO_TRUNC_FLAG 0x80000000u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11).                                      */
/* One round: two 32x32->64 products of the even words with the multipliers, */
/* the high halves xor'ed with the odd words and the round key, the words    */
/* permuted; the key is bumped by the Weyl constants between rounds.         */
/* ------------------------------------------------------------------------ */

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void fko_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* ------------------------------------------------------------------------ */
/* Normal variates z_j of the stream of path (m, s, p).                      */
/*   FP64 stream: block k gives two uniforms with 53 random bits each,       */
/*     U = ((hi << 21 | lo >> 11) + 1) * 2^-53 in (0, 1], and one Box-Muller */
/*     pair: z_{2k} = R cos(2 pi U2), z_{2k+1} = R sin(2 pi U2),             */
/*     R = sqrt(-2 ln U1).                                                   */
/*   FP32 stream: block k gives four uniforms with 24 bits each,             */
/*     u_i = ((w_i >> 8) + 1) * 2^-24, and two Box-Muller pairs              */
/*     (u0,u1) -> z_{4k}, z_{4k+1}; (u2,u3) -> z_{4k+2}, z_{4k+3}.           */
/*     The oracle evaluates that transform in FP64.                          */
/* Step n of a walk uses z_{3n}, z_{3n+1}, z_{3n+2} for x, y, z.            */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t seed;
    uint32_t m, s, p;
    int32_t stream;
    int64_t cached_block;   /* block index held in z[], or -1 */
    double z[4];
} fko_stream;

static void stream_init(fko_stream *st, int stream, uint64_t seed, uint32_t m, uint32_t s, uint32_t p)
{
    st->seed = seed; st->m = m; st->s = s; st->p = p; st->stream = stream;
    st->cached_block = -1;
}

static void stream_block(fko_stream *st, int64_t k)
{
    uint32_t ctr[4] = {(uint32_t)k, st->p, st->s, st->m};
    uint32_t key[2] = {(uint32_t)st->seed, (uint32_t)(st->seed >> 32)};
    uint32_t w[4];
    fko_philox4x32_10(ctr, key, w);
    if (st->stream == FKO_STREAM_F64) {
        uint64_t a = (((uint64_t)w[1] << 21) | (uint64_t)(w[0] >> 11)) + 1u;
        uint64_t b = (((uint64_t)w[3] << 21) | (uint64_t)(w[2] >> 11)) + 1u;
        double u1 = (double)a * 0x1p-53;
        double u2 = (double)b * 0x1p-53;
        double r = sqrt(-2.0 * log(u1));
        double th = 2.0 * M_PI * u2;
        st->z[0] = r * cos(th);
        st->z[1] = r * sin(th);
    } else {
        double u[4];
        for (int i = 0; i < 4; ++i) u[i] = (double)((w[i] >> 8) + 1u) * 0x1p-24;
        double r0 = sqrt(-2.0 * log(u[0]));
        double r1 = sqrt(-2.0 * log(u[2]));
        st->z[0] = r0 * cos(2.0 * M_PI * u[1]);
        st->z[1] = r0 * sin(2.0 * M_PI * u[1]);
        st->z[2] = r1 * cos(2.0 * M_PI * u[3]);
        st->z[3] = r1 * sin(2.0 * M_PI * u[3]);
    }
    st->cached_block = k;
}

static double stream_normal(fko_stream *st, int64_t j)
{
    int per = (st->stream == FKO_STREAM_F64) ? 2 : 4;
    int64_t k = j / per;
    if (k != st->cached_block) stream_block(st, k);
    return st->z[j % per];
}

/* Uniforms of the Brownian-bridge exit test: step n uses slot n mod q of
 * block 2^31 + floor(n / q) of the walk's Philox stream, q = 2 for the FP64
 * stream (53-bit uniforms from the word pairs (w1, w0) and (w3, w2), as U1
 * and U2 above) and q = 4 for the FP32 stream (24-bit uniforms).  Block
 * indices of the normals stay below 2^31 while walks are shorter than 2^30
 * steps. */
static double bridge_uniform(const fko_stream *st, int64_t n)
{
    int q = (st->stream == FKO_STREAM_F64) ? 2 : 4;
    uint32_t ctr[4] = {0x80000000u + (uint32_t)(n / q), st->p, st->s, st->m};
    uint32_t key[2] = {(uint32_t)st->seed, (uint32_t)(st->seed >> 32)};
    uint32_t w[4];
    fko_philox4x32_10(ctr, key, w);
    int slot = (int)(n % q);
    if (st->stream == FKO_STREAM_F64) {
        uint32_t hi = w[2 * slot + 1], lo = w[2 * slot];
        return (double)((((uint64_t)hi << 21) | (uint64_t)(lo >> 11)) + 1u) * 0x1p-53;
    }
    return (double)((w[slot] >> 8) + 1u) * 0x1p-24;
}

double fko_bridge_uniform(int32_t stream, uint64_t seed, uint32_t m, uint32_t s, uint32_t p, int64_t n)
{
    fko_stream st;
    stream_init(&st, stream, seed, m, s, p);
    return bridge_uniform(&st, n);
}

double fko_normal(int32_t stream, uint64_t seed, uint32_t m, uint32_t s, uint32_t p, int64_t j)
{
    fko_stream st;
    stream_init(&st, stream, seed, m, s, p);
    return stream_normal(&st, j);
}

/* ------------------------------------------------------------------------ */
/* Source density rho(x) (paper eq. 4): a voxel grid that is zero outside   */
/* itself, plus analytic homogeneous prisms and spheres; overlaps add.       */
/* Voxel i along an axis holds [o + i d, o + (i+1) d): index = floor((x-o)/d)*/
/* Prisms are half-open [lo, hi) per axis; spheres are open balls.           */
/* ------------------------------------------------------------------------ */

static int64_t voxel_index(const fko_source *src, const double x[3])
{
    if (src->rho == NULL || src->n[0] <= 0 || src->n[1] <= 0 || src->n[2] <= 0) return -1;
    int64_t idx[3];
    for (int c = 0; c < 3; ++c) {
        double t = floor((x[c] - src->origin[c]) / src->spacing[c]);
        if (!(t >= 0.0 && t < (double)src->n[c])) return -1;
        idx[c] = (int64_t)t;
    }
    return (idx[2] * src->n[1] + idx[1]) * src->n[0] + idx[0];
}

double fko_rho(const fko_source *src, const double x[3])
{
    double r = 0.0;
    int64_t v = voxel_index(src, x);
    if (v >= 0) r = r + (double)src->rho[v];
    for (int32_t j = 0; j < src->n_prisms; ++j) {
        const double *q = src->prisms + 7 * j;
        if (x[0] >= q[0] && x[0] < q[3] && x[1] >= q[1] && x[1] < q[4] && x[2] >= q[2] && x[2] < q[5])
            r = r + q[6];
    }
    for (int32_t j = 0; j < src->n_spheres; ++j) {
        const double *q = src->spheres + 5 * j;
        double dx = x[0] - q[0], dy = x[1] - q[1], dz = x[2] - q[2];
        double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < q[3] * q[3]) r = r + q[4];
    }
    return r;
}

int64_t fko_voxel_index(const fko_source *src, const double x[3]) { return voxel_index(src, x); }

/* ------------------------------------------------------------------------ */
/* Closed forms used as boundary data and as exact test targets.             */
/* ------------------------------------------------------------------------ */

/* ln(a + r), r = sqrt(a^2 + b2), without cancellation when a < 0:           */
/* a + r = b2 / (r - a).                                                      */
static double log_a_plus_r(double a, double r, double b2)
{
    if (a >= 0.0) return log(a + r);
    return log(b2) - log(r - a);
}

/* Corner function of the homogeneous-prism Newtonian integral
 * V(P) = int_prism dV / |x - P| (Nagy 1966; Nagy, Papp & Benedek 2000):
 * F = XY ln(Z+r) + YZ ln(X+r) + ZX ln(Y+r)
 *     - X^2/2 atan(YZ/(Xr)) - Y^2/2 atan(ZX/(Yr)) - Z^2/2 atan(XY/(Zr)),
 * a term with a zero prefactor being zero. */
static double prism_F(double X, double Y, double Z)
{
    double X2 = X * X, Y2 = Y * Y, Z2 = Z * Z;
    double r = sqrt(X2 + Y2 + Z2);
    double f = 0.0;
    if (X * Y != 0.0) f += X * Y * log_a_plus_r(Z, r, X2 + Y2);
    if (Y * Z != 0.0) f += Y * Z * log_a_plus_r(X, r, Y2 + Z2);
    if (Z * X != 0.0) f += Z * X * log_a_plus_r(Y, r, Z2 + X2);
    if (X != 0.0) f -= 0.5 * X2 * atan(Y * Z / (X * r));
    if (Y != 0.0) f -= 0.5 * Y2 * atan(Z * X / (Y * r));
    if (Z != 0.0) f -= 0.5 * Z2 * atan(X * Y / (Z * r));
    return f;
}

/* d/dZ of the corner function: X ln(Y+r) + Y ln(X+r) - Z atan(XY/(Zr)). */
static double prism_Fz(double X, double Y, double Z)
{
    double X2 = X * X, Y2 = Y * Y, Z2 = Z * Z;
    double r = sqrt(X2 + Y2 + Z2);
    double f = 0.0;
    if (X != 0.0) f += X * log_a_plus_r(Y, r, Z2 + X2);
    if (Y != 0.0) f += Y * log_a_plus_r(X, r, Y2 + Z2);
    if (Z != 0.0) f -= Z * atan(X * Y / (Z * r));
    return f;
}

/* V(P) = sum over the 8 corners of (-1)^(i+j+k) F(x_i - xP, y_j - yP, z_k - zP),
 * i, j, k in {1 (lower), 2 (upper)}. */
double fko_prism_newton(const double lo[3], const double hi[3], const double P[3])
{
    double v = 0.0;
    for (int i = 1; i <= 2; ++i)
        for (int j = 1; j <= 2; ++j)
            for (int k = 1; k <= 2; ++k) {
                double X = (i == 1 ? lo[0] : hi[0]) - P[0];
                double Y = (j == 1 ? lo[1] : hi[1]) - P[1];
                double Z = (k == 1 ? lo[2] : hi[2]) - P[2];
                double s = ((i + j + k) % 2 == 0) ? 1.0 : -1.0;
                v += s * prism_F(X, Y, Z);
            }
    return v;
}

/* Potential of a homogeneous prism, Phi = -G rho V (negative, zero at infinity). */
double fko_prism_potential(const double lo[3], const double hi[3], double rho, double G, const double P[3])
{
    return -G * rho * fko_prism_newton(lo, hi, P);
}

/* g_z = dPhi/dz_P = G rho sum (-1)^(i+j+k) Fz (dZ/dz_P = -1 flips -G rho dV). */
double fko_prism_gz(const double lo[3], const double hi[3], double rho, double G, const double P[3])
{
    double v = 0.0;
    for (int i = 1; i <= 2; ++i)
        for (int j = 1; j <= 2; ++j)
            for (int k = 1; k <= 2; ++k) {
                double X = (i == 1 ? lo[0] : hi[0]) - P[0];
                double Y = (j == 1 ? lo[1] : hi[1]) - P[1];
                double Z = (k == 1 ? lo[2] : hi[2]) - P[2];
                double s = ((i + j + k) % 2 == 0) ? 1.0 : -1.0;
                v += s * prism_Fz(X, Y, Z);
            }
    return G * rho * v;
}

/* Uniform ball of radius a, density rho, centre c: Phi = -G M / r outside,
 * -2 pi G rho (a^2 - r^2/3) inside; g_z = dPhi/dz. */
double fko_sphere_potential(const double c[3], double a, double rho, double G, const double P[3])
{
    double dx = P[0] - c[0], dy = P[1] - c[1], dz = P[2] - c[2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double M = 4.0 / 3.0 * M_PI * a * a * a * rho;
    if (r >= a) return -G * M / r;
    return -2.0 * M_PI * G * rho * (a * a - r * r / 3.0);
}

double fko_sphere_gz(const double c[3], double a, double rho, double G, const double P[3])
{
    double dx = P[0] - c[0], dy = P[1] - c[1], dz = P[2] - c[2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double M = 4.0 / 3.0 * M_PI * a * a * a * rho;
    if (r >= a) return G * M * dz / (r * r * r);
    return 4.0 / 3.0 * M_PI * G * rho * dz;
}

/* ------------------------------------------------------------------------ */
/* Dirichlet data g on the boundary, read at the exit point.                 */
/*   ZERO: 0 (the paper's choice, section 2.2).                              */
/*   QUADRATIC: c0 + b.x + x^T A x, data = c0, b0..b2, A00 A01 A02 A11 A12 A22*/
/*   POINT_MASSES: -sum G m_j / |x - c_j|, data rows (cx, cy, cz, m).        */
/*   PRISMS: sum of homogeneous-prism potentials, rows (lo[3], hi[3], rho).  */
/*   FACE_GRID: bilinear interpolation of node values on the face the exit  */
/*     point is furthest beyond (ties: lower axis, then lower face), the    */
/*     point first clamped to the box.  Faces f = 2c + side, side 0 = lo.   */
/*     Face axes (a, b): x faces (y, z); y faces (x, z); z faces (x, y).    */
/*     Node (ia, ib) of face f sits at data[off_f + ib * n_a + ia], nodes   */
/*     uniformly spaced from lo to hi along each face axis.                 */
/* ------------------------------------------------------------------------ */

static double face_grid_value(const fko_bc *bc, const fko_box *box, const double xe[3])
{
    int best_c = 0, best_side = 0;
    double best = -INFINITY;
    for (int c = 0; c < 3; ++c) {
        double vlo = box->lo[c] - xe[c];
        double vhi = xe[c] - box->hi[c];
        if (vlo > best) { best = vlo; best_c = c; best_side = 0; }
        if (vhi > best) { best = vhi; best_c = c; best_side = 1; }
    }
    int f = 2 * best_c + best_side;
    int64_t off = 0;
    for (int g = 0; g < f; ++g) off += (int64_t)bc->face_n[g][0] * bc->face_n[g][1];
    int a = (best_c == 0) ? 1 : 0;
    int b = (best_c == 2) ? 1 : 2;
    int na = bc->face_n[f][0], nb = bc->face_n[f][1];
    double pa = fmin(fmax(xe[a], box->lo[a]), box->hi[a]);
    double pb = fmin(fmax(xe[b], box->lo[b]), box->hi[b]);
    double ta = (pa - box->lo[a]) / (box->hi[a] - box->lo[a]) * (double)(na - 1);
    double tb = (pb - box->lo[b]) / (box->hi[b] - box->lo[b]) * (double)(nb - 1);
    int ia = (int)floor(ta), ib = (int)floor(tb);
    if (ia > na - 2) ia = na - 2;
    if (ib > nb - 2) ib = nb - 2;
    if (ia < 0) ia = 0;
    if (ib < 0) ib = 0;
    double fa = ta - ia, fb = tb - ib;
    const double *d = bc->data + off;
    double v00 = d[(int64_t)ib * na + ia], v10 = d[(int64_t)ib * na + ia + 1];
    double v01 = d[(int64_t)(ib + 1) * na + ia], v11 = d[(int64_t)(ib + 1) * na + ia + 1];
    return (1.0 - fa) * (1.0 - fb) * v00 + fa * (1.0 - fb) * v10 + (1.0 - fa) * fb * v01 + fa * fb * v11;
}

double fko_bc_value(const fko_bc *bc, const fko_box *box, double G, const double x[3])
{
    switch (bc->kind) {
    case FKO_BC_ZERO:
        return 0.0;
    case FKO_BC_QUADRATIC: {
        const double *q = bc->data;
        return q[0] + q[1] * x[0] + q[2] * x[1] + q[3] * x[2]
             + q[4] * x[0] * x[0] + 2.0 * q[5] * x[0] * x[1] + 2.0 * q[6] * x[0] * x[2]
             + q[7] * x[1] * x[1] + 2.0 * q[8] * x[1] * x[2] + q[9] * x[2] * x[2];
    }
    case FKO_BC_POINT_MASSES: {
        double v = 0.0;
        for (int64_t j = 0; j < bc->n_items; ++j) {
            const double *q = bc->data + 4 * j;
            double dx = x[0] - q[0], dy = x[1] - q[1], dz = x[2] - q[2];
            v -= G * q[3] / sqrt(dx * dx + dy * dy + dz * dz);
        }
        return v;
    }
    case FKO_BC_PRISMS: {
        double v = 0.0;
        for (int64_t j = 0; j < bc->n_items; ++j) {
            const double *q = bc->data + 7 * j;
            v += fko_prism_potential(q, q + 3, q[6], G, x);
        }
        return v;
    }
    case FKO_BC_FACE_GRID:
        return face_grid_value(bc, box, x);
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* One walk (paper section 2.3, steps 1-4).                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    const fko_box *box;
    const fko_source *src;
    const fko_bc *bc;
    const fko_params *prm;
} fko_problem;

/* The ball domain: centre (lo + hi) / 2 and radius (hi_x - lo_x) / 2 of its
 * box. */
static void ball_of(const fko_box *box, double c[3], double *r2)
{
    for (int k = 0; k < 3; ++k) c[k] = 0.5 * (box->lo[k] + box->hi[k]);
    double r = 0.5 * (box->hi[0] - box->lo[0]);
    *r2 = r * r;
}

/* |x - c|^2 with the products of y and x fused into the running sum. */
static double dist2(const double x[3], const double c[3])
{
    double d0 = x[0] - c[0], d1 = x[1] - c[1], d2 = x[2] - c[2];
    return fma(d0, d0, fma(d1, d1, d2 * d2));
}

/* On or beyond the boundary (a point on the boundary has left, eq. 3). */
static int outside(const fko_box *box, int domain, const double x[3])
{
    if (domain == FKO_DOMAIN_BALL) {
        double c[3], r2;
        ball_of(box, c, &r2);
        return dist2(x, c) >= r2;
    }
    for (int k = 0; k < 3; ++k)
        if (x[k] <= box->lo[k] || x[k] >= box->hi[k]) return 1;
    return 0;
}

/* INTERSECT on the ball: the point of the segment x -> xn on the sphere,
 * x + t (xn - x) with t the root in (0, 1] of |x + t v - c|^2 = R^2, written
 * t = -C / (B + sqrt(B^2 - A C)) (A = |v|^2, B = (x - c).v, C = |x - c|^2 -
 * R^2 < 0), which has no cancellation. */
static void intersect_ball(const fko_box *box, const double x[3], const double xn[3], double xe[3])
{
    double c[3], r2;
    ball_of(box, c, &r2);
    double v[3], a[3];
    for (int k = 0; k < 3; ++k) { v[k] = xn[k] - x[k]; a[k] = x[k] - c[k]; }
    double A = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double B = a[0] * v[0] + a[1] * v[1] + a[2] * v[2];
    double C = (a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) - r2;
    double t = -C / (B + sqrt(B * B - A * C));
    if (t > 1.0) t = 1.0;
    for (int k = 0; k < 3; ++k) xe[k] = fma(t, v[k], x[k]);
}

/* Exit point on the segment x -> xn under the INTERSECT rule: the first face
 * crossed (smallest crossing fraction; ties: lower axis); the crossing
 * coordinate is set to the face value exactly. */
static void intersect_point(const fko_box *box, const double x[3], const double xn[3], double xe[3])
{
    double tbest = INFINITY;
    int cbest = -1;
    double face = 0.0;
    for (int c = 0; c < 3; ++c) {
        double fc;
        if (xn[c] <= box->lo[c]) fc = box->lo[c];
        else if (xn[c] >= box->hi[c]) fc = box->hi[c];
        else continue;
        double t = (fc - x[c]) / (xn[c] - x[c]);
        if (t < tbest) { tbest = t; cbest = c; face = fc; }
    }
    for (int c = 0; c < 3; ++c) xe[c] = fma(tbest, xn[c] - x[c], x[c]);
    xe[cbest] = face;
}

/* Brownian-bridge exit test (paper section 2.3, remark on the exit time;
 * Gobet 2000): a standard Brownian motion that goes from distance a to
 * distance b > 0 of a plane in time dt has touched the plane in between with
 * probability exp(-2 a b / dt).  For a step x -> xn with both ends inside,
 * every face of the box (or the tangent plane of the sphere) contributes
 * such a probability p_f; the walk is stopped in this step when its uniform
 * U satisfies U <= 1 - prod_f (1 - p_f).  The exit point is xn projected onto
 * the face with the largest p_f (ties: -x, +x, -y, +y, -z, +z order), or
 * radially onto the sphere.  Returns 1 and fills xe when the walk stops. */
static int bridge_exit(const fko_box *box, int domain, double dt, double U, const double x[3],
                       const double xn[3], double xe[3])
{
    if (domain == FKO_DOMAIN_BALL) {
        double c[3], r2;
        ball_of(box, c, &r2);
        double R = sqrt(r2);
        double a = R - sqrt(dist2(x, c)), b = R - sqrt(dist2(xn, c));
        double p = exp(-2.0 * a * b / dt);
        if (!(U <= p)) return 0;
        double r = sqrt(dist2(xn, c));
        for (int k = 0; k < 3; ++k) xe[k] = c[k] + R * ((xn[k] - c[k]) / r);
        return 1;
    }
    double keep = 1.0, pbest = -1.0;
    int fbest = 0;
    for (int f = 0; f < 6; ++f) {
        int k = f / 2;
        double a = (f % 2) ? box->hi[k] - x[k] : x[k] - box->lo[k];
        double b = (f % 2) ? box->hi[k] - xn[k] : xn[k] - box->lo[k];
        double p = exp(-2.0 * a * b / dt);
        keep *= 1.0 - p;
        if (p > pbest) { pbest = p; fbest = f; }
    }
    if (!(U <= 1.0 - keep)) return 0;
    for (int k = 0; k < 3; ++k) xe[k] = xn[k];
    xe[fbest / 2] = (fbest % 2) ? box->hi[fbest / 2] : box->lo[fbest / 2];
    return 1;
}

/* Adds the trapezoid weights of one walk to counts[voxel]: one per end of
 * every step whose end lies in the grid. */
static void add_count(const fko_source *src, uint64_t *counts, const double x[3])
{
    int64_t v = voxel_index(src, x);
    if (v >= 0) counts[v] += 1;
}

/* Runs one walk from x0 with stream (m, sctr, p).  Returns the trapezoid sum
 * S = sum (rho_n + rho_{n+1}) in *S_out, the exit point in xe, the number of
 * steps in *steps, and 1 if the walk hit max_steps without leaving the box. */
static int walk(const fko_problem *P, const double x0[3], uint32_t sctr, uint32_t p,
                double *S_out, double xe[3], int64_t *steps, uint64_t *counts)
{
    const fko_params *prm = P->prm;
    fko_stream st;
    stream_init(&st, prm->stream, prm->seed, prm->problem_id, sctr, p);
    double sdt = sqrt(prm->dt);
    double x[3] = {x0[0], x0[1], x0[2]};
    double rp = fko_rho(P->src, x);
    double S = 0.0;
    int64_t n = 0;
    for (;;) {
        double xn[3];
        for (int c = 0; c < 3; ++c) xn[c] = fma(sdt, stream_normal(&st, 3 * n + c), x[c]);
        double rn = fko_rho(P->src, xn);
        S = S + (rp + rn);
        if (counts) { add_count(P->src, counts, x); add_count(P->src, counts, xn); }
        if (outside(P->box, prm->domain, xn)) {
            n = n + 1;
            if (prm->exit_rule != FKO_EXIT_OVERSHOOT && prm->domain == FKO_DOMAIN_BALL)
                intersect_ball(P->box, x, xn, xe);
            else if (prm->exit_rule != FKO_EXIT_OVERSHOOT)
                intersect_point(P->box, x, xn, xe);
            else { xe[0] = xn[0]; xe[1] = xn[1]; xe[2] = xn[2]; }
            *S_out = S;
            *steps = n;
            return 0;
        }
        if (prm->exit_rule == FKO_EXIT_BRIDGE &&
            bridge_exit(P->box, prm->domain, prm->dt, bridge_uniform(&st, n), x, xn, xe)) {
            *S_out = S;
            *steps = n + 1;
            return 0;
        }
        x[0] = xn[0]; x[1] = xn[1]; x[2] = xn[2];
        rp = rn;
        n = n + 1;
        if (n == prm->max_steps) {
            *S_out = S;
            xe[0] = x[0]; xe[1] = x[1]; xe[2] = x[2];
            *steps = n;
            return 1;
        }
    }
}

/* Per-path sample u_p = g(x_e) - 2 pi G (dt/2) S. */
static double path_value(const fko_problem *P, double S, const double xe[3])
{
    const fko_params *prm = P->prm;
    double w = 2.0 * M_PI * prm->G * (0.5 * prm->dt);
    return fko_bc_value(P->bc, P->box, prm->G, xe) - w * S;
}

static double diff_step(const fko_params *prm)
{
    return prm->h > 0.0 ? prm->h : sqrt(prm->dt);
}

/* ------------------------------------------------------------------------ */
/* Public entry points for the tests.                                        */
/* ------------------------------------------------------------------------ */

/* Runs the paths named by items = (station index s, local path index i)
 * pairs.  kind 0: potential; u_out = u_p, steps_out = steps.
 * kind 1: g_z; u_out = (u+ - u-)/(2h), aux_out[2n], [2n+1] = u+, u- (nullable),
 * steps_out = steps+ + steps-.  The truncation flag is the top bit of
 * steps_out; a truncated sample's value is NaN.  xe_out (nullable) receives
 * the exit point (kind 0) or the + walk's exit point (kind 1).
 * Path p = path_offset + i; stream station index = s (potential and CRN) or
 * 2s / 2s+1 (independent pairing). */
int fko_run_paths(int32_t kind, const double *stations, int64_t n_stations,
                  const fko_box *box, const fko_source *src, const fko_bc *bc,
                  const fko_params *prm, const int64_t *items, int64_t n_items,
                  double *u_out, uint32_t *steps_out, double *aux_out, double *xe_out,
                  int32_t n_threads)
{
    fko_problem P = {box, src, bc, prm};
    for (int64_t t = 0; t < n_items; ++t)
        if (items[2 * t] < 0 || items[2 * t] >= n_stations) return -1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t t = 0; t < n_items; ++t) {
        int64_t s = items[2 * t];
        uint32_t p = (uint32_t)(prm->path_offset + items[2 * t + 1]);
        const double *xs = stations + 3 * s;
        if (kind == 0) {
            double S, xe[3];
            int64_t n;
            int tr = walk(&P, xs, (uint32_t)s, p, &S, xe, &n, NULL);
            u_out[t] = tr ? NAN : path_value(&P, S, xe);
            steps_out[t] = (uint32_t)n | (tr ? FKO_TRUNC_FLAG : 0u);
            if (xe_out) { xe_out[3 * t] = xe[0]; xe_out[3 * t + 1] = xe[1]; xe_out[3 * t + 2] = xe[2]; }
        } else {
            double h = diff_step(prm);
            double xp[3] = {xs[0], xs[1], xs[2] + h};
            double xm[3] = {xs[0], xs[1], xs[2] - h};
            uint32_t sp = (prm->pairing == FKO_PAIR_INDEPENDENT) ? (uint32_t)(2 * s) : (uint32_t)s;
            uint32_t sm = (prm->pairing == FKO_PAIR_INDEPENDENT) ? (uint32_t)(2 * s + 1) : (uint32_t)s;
            double Sp, Sm, xep[3], xem[3];
            int64_t np_, nm;
            int trp = walk(&P, xp, sp, p, &Sp, xep, &np_, NULL);
            int trm = walk(&P, xm, sm, p, &Sm, xem, &nm, NULL);
            double up = trp ? NAN : path_value(&P, Sp, xep);
            double um = trm ? NAN : path_value(&P, Sm, xem);
            int tr = trp || trm;
            u_out[t] = tr ? NAN : (up - um) / (2.0 * h);
            steps_out[t] = (uint32_t)(np_ + nm) | (tr ? FKO_TRUNC_FLAG : 0u);
            if (aux_out) { aux_out[2 * t] = up; aux_out[2 * t + 1] = um; }
            if (xe_out) { xe_out[3 * t] = xep[0]; xe_out[3 * t + 1] = xep[1]; xe_out[3 * t + 2] = xep[2]; }
        }
    }
    return 0;
}

/* Station statistics of eq. 11 from per-path samples, in path order:
 * n = untruncated samples, mean = sum/n, var = sum (u - mean)^2 / (n - 1),
 * se = sqrt(var / n); mean_steps and max_steps over all paths. */
void fko_station_stats(const double *u, const uint32_t *steps, int64_t n_paths, fko_stat *out)
{
    int64_t n = 0, ntr = 0, smax = 0;
    double sum = 0.0, ssteps = 0.0;
    for (int64_t i = 0; i < n_paths; ++i) {
        int64_t k = (int64_t)(steps[i] & ~FKO_TRUNC_FLAG);
        ssteps += (double)k;
        if (k > smax) smax = k;
        if (steps[i] & FKO_TRUNC_FLAG) { ntr++; continue; }
        sum += u[i];
        n++;
    }
    double mean = n > 0 ? sum / (double)n : NAN;
    double m2 = 0.0;
    for (int64_t i = 0; i < n_paths; ++i) {
        if (steps[i] & FKO_TRUNC_FLAG) continue;
        double d = u[i] - mean;
        m2 += d * d;
    }
    out->mean = mean;
    out->var = n > 1 ? m2 / (double)(n - 1) : NAN;
    out->se = n > 1 ? sqrt(out->var / (double)n) : NAN;
    out->n = n;
    out->mean_steps = n_paths > 0 ? ssteps / (double)n_paths : 0.0;
    out->max_steps = smax;
    out->n_trunc = ntr;
}

/* Occupation counts behind the adjoint: for every untruncated walk of the
 * local paths [i_begin, i_end) of each station, counts[s][v] gains the
 * trapezoid weight of voxel v (one per step end inside v).  kind 1 fills
 * counts_plus from the x0 + h e_z walks and counts_minus from the x0 - h e_z
 * walks, skipping a pair when either walk is truncated.  Then
 * d u_s / d rho_v = -2 pi G (dt/2) counts[s][v] / n_s and
 * d gz_s / d rho_v = -2 pi G (dt/2) (c+ - c-) / (2 h n_s).
 * Each walk is run twice: once to learn whether it is truncated, then once
 * to count. */
int fko_occupation(int32_t kind, const double *stations, int64_t n_stations,
                   const fko_box *box, const fko_source *src, const fko_bc *bc,
                   const fko_params *prm, int64_t i_begin, int64_t i_end,
                   uint64_t *counts_plus, uint64_t *counts_minus, int32_t n_threads)
{
    fko_problem P = {box, src, bc, prm};
    int64_t nvox = (int64_t)src->n[0] * src->n[1] * src->n[2];
    if (src->rho == NULL || nvox <= 0) return -1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t s = 0; s < n_stations; ++s) {
        const double *xs = stations + 3 * s;
        uint64_t *cp = counts_plus + s * nvox;
        uint64_t *cm = counts_minus ? counts_minus + s * nvox : NULL;
        for (int64_t i = i_begin; i < i_end; ++i) {
            uint32_t p = (uint32_t)(prm->path_offset + i);
            double S, xe[3];
            int64_t n;
            if (kind == 0) {
                if (walk(&P, xs, (uint32_t)s, p, &S, xe, &n, NULL)) continue;
                walk(&P, xs, (uint32_t)s, p, &S, xe, &n, cp);
            } else {
                double h = diff_step(prm);
                double xp[3] = {xs[0], xs[1], xs[2] + h};
                double xm[3] = {xs[0], xs[1], xs[2] - h};
                uint32_t sp = (prm->pairing == FKO_PAIR_INDEPENDENT) ? (uint32_t)(2 * s) : (uint32_t)s;
                uint32_t sm = (prm->pairing == FKO_PAIR_INDEPENDENT) ? (uint32_t)(2 * s + 1) : (uint32_t)s;
                if (walk(&P, xp, sp, p, &S, xe, &n, NULL)) continue;
                if (walk(&P, xm, sm, p, &S, xe, &n, NULL)) continue;
                walk(&P, xp, sp, p, &S, xe, &n, cp);
                walk(&P, xm, sm, p, &S, xe, &n, cm);
            }
        }
    }
    return 0;
}

/* Moving averages of a station profile (paper section 4.1): the mean over
 * the largest centred window of at most `span` points that fits; standard
 * errors of independent values combine as sqrt(sum se^2) / width. */
int fko_moving_average(const double *v, const double *se, int64_t n, int span, double *out, double *out_se)
{
    if (span < 1 || span % 2 == 0) return -1;
    for (int64_t k = 0; k < n; ++k) {
        int64_t half = span / 2;
        int64_t left = k, right = n - 1 - k;
        int64_t r = half < left ? half : left;
        r = r < right ? r : right;
        double acc = 0.0, acc2 = 0.0;
        int64_t cnt = 0;
        for (int64_t j = k - r; j <= k + r; ++j) {
            acc += v[j];
            if (se) acc2 += se[j] * se[j];
            cnt++;
        }
        out[k] = acc / (double)cnt;
        if (se) out_se[k] = sqrt(acc2) / (double)cnt;
    }
    return 0;
}

int fko_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
