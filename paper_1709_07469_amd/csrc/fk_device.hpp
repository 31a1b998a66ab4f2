// fk_device.hpp -- device-side building blocks of the walk kernels for gfx950:
// the Philox4x32-10 counter generator, the Box-Muller maps of the two random
// streams, the density lookup, the exit test and exit point, and the
// Dirichlet data read at the exit (arXiv:1709.07469, section 2.3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fk_internal.hpp"

namespace fk {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Each round multiplies
// words 0 and 2 by the Philox multipliers (32x32 -> 64), mixes the high halves
// into words 1 and 3 with the round key and permutes; the key advances by the
// Weyl increments.  The key is wave-uniform (it is the seed), so the key
// schedule is scalar work.
// ---------------------------------------------------------------------------
struct Block {
    uint32_t w0, w1, w2, w3;
};

// a ^ b ^ c in one instruction: gfx950's three-input bitwise operation with
// the truth table of a three-way exclusive or (0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Block philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Block{c0, c1, c2, c3};
}

// ---------------------------------------------------------------------------
// FP64 elementary functions for the Box-Muller transform, written for the
// argument ranges it needs (gfx950 has no FP64 transcendental unit, and the
// general library routines handle ranges and cases that never occur here).
// ---------------------------------------------------------------------------

// -2 ln u for u in (0, 1].  u = m 2^e with m in [sqrt(1/2), sqrt(2)), and
// ln m = 2 atanh(s) with s = (m - 1)/(m + 1), |s| <= 0.1716, summed as
// s * sum_k s^(2k) / (2k + 1) for k = 0..10 (truncation below 1e-18
// relative); ln 2 in a high part with trailing zeros (so e * ln2_hi is exact)
// and a low part.  Error about 1 ulp.
__device__ __forceinline__ double neg2_log(double u)
{
    double m = __builtin_amdgcn_frexp_mant(u);   // [0.5, 1)
    int e = __builtin_amdgcn_frexp_exp(u);
    if (m < 0x1.6a09e667f3bcdp-1) {             // sqrt(1/2)
        m = 2.0 * m;
        e -= 1;
    }
    const double d = m + 1.0;
    double r = __builtin_amdgcn_rcp(d);          // estimate of 1/d, refined twice
    double t = fma(-d, r, 1.0);
    r = fma(r, t, r);
    t = fma(-d, r, 1.0);
    r = fma(r, t, r);
    const double n = m - 1.0;                    // exact
    double q = n * r;
    q = fma(fma(-d, q, n), r, q);                // s = (m - 1)/(m + 1)
    const double z = q * q;
    double p = 0x1.8618618618618p-5;             // 1/21
    p = fma(p, z, 0x1.af286bca1af28p-5);         // 1/19
    p = fma(p, z, 0x1.e1e1e1e1e1e1ep-5);         // 1/17
    p = fma(p, z, 0x1.1111111111111p-4);         // 1/15
    p = fma(p, z, 0x1.3b13b13b13b14p-4);         // 1/13
    p = fma(p, z, 0x1.745d1745d1746p-4);         // 1/11
    p = fma(p, z, 0x1.c71c71c71c71cp-4);         // 1/9
    p = fma(p, z, 0x1.2492492492492p-3);         // 1/7
    p = fma(p, z, 0x1.999999999999ap-3);         // 1/5
    p = fma(p, z, 0x1.5555555555555p-2);         // 1/3
    p = fma(p, z, 1.0);
    const double ts = (4.0 * q) * p;             // -2 ln m = -4 atanh(s)
    const double fe = -2.0 * (double)e;
    return fma(fe, 0x1.62e42fee00000p-1, fma(fe, 0x1.a39ef35793c76p-33, -ts));
}

// sqrt(x) for x >= 0: hardware reciprocal square-root estimate, FK_SQRT_ITERS
// Goldschmidt iterations on (g = x y, h = y/2), and a final residual
// correction.  Each step roughly doubles the correct bits of the estimate;
// with one iteration the Box-Muller normals still agree with a correctly
// rounded reference to 2e-15 of max(1, |z|), within the 4e-15 the reference
// angle's own rounding allows.
#ifndef FK_SQRT_ITERS
#define FK_SQRT_ITERS 1
#endif
__device__ __forceinline__ double sqrt_nonneg(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
#pragma unroll
    for (int i = 0; i < FK_SQRT_ITERS; ++i) {
        const double r = fma(-g, h, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
    }
    g = fma(fma(-g, g, x), h, g);
    return x > 0.0 ? g : 0.0;
}

// sin and cos of 2 pi u for u in (0, 1].  x = 2u is reduced exactly to
// r = x - q/2 in [-1/4, 1/4] (q = nearest integer to 2x); sin(pi r) and
// cos(pi r) are their Taylor series to r^17 and r^18 (truncation below
// 1e-17); the quadrant q mod 4 swaps and negates them.
__device__ __forceinline__ void sincos_2pi(double u, double& s, double& c)
{
    const double x = 2.0 * u;
    const double q = __builtin_rint(2.0 * x);
    const double r = fma(-0.5, q, x);
    const double z = r * r;
    double ps = 0x1.aaec32af93359p-21;
    ps = fma(ps, z, -0x1.6fadb9f155744p-16);
    ps = fma(ps, z, 0x1.e8f434d018d63p-12);
    ps = fma(ps, z, -0x1.e3074fde8871fp-8);
    ps = fma(ps, z, 0x1.50783487ee782p-4);
    ps = fma(ps, z, -0x1.32d2cce62bd86p-1);
    ps = fma(ps, z, 0x1.466bc6775aae2p+1);
    ps = fma(ps, z, -0x1.4abbce625be53p+2);
    ps = fma(ps, z, 0x1.921fb54442d18p+1);      // pi
    const double sv = r * ps;
    double pc = -0x1.2a0c591af8314p-23;
    pc = fma(pc, z, 0x1.20c62c2f2d7f5p-18);
    pc = fma(pc, z, -0x1.b6e24f44b128fp-14);
    pc = fma(pc, z, 0x1.f9d38a3763cc3p-10);
    pc = fma(pc, z, -0x1.a6d1f2a204a8cp-6);
    pc = fma(pc, z, 0x1.e1f506891babbp-3);
    pc = fma(pc, z, -0x1.55d3c7e3cbffap+0);
    pc = fma(pc, z, 0x1.03c1f081b5ac4p+2);
    pc = fma(pc, z, -0x1.3bd3cc9be45dep+2);
    const double cv = fma(pc, z, 1.0);
    const int qi = (int)q & 3;
    const double ss = (qi & 1) ? cv : sv;
    const double cc = (qi & 1) ? sv : cv;
    s = (qi & 2) ? -ss : ss;
    c = ((qi + 1) & 2) ? -cc : cc;
}

// Tables that shorten the two FP64 transcendentals of the walk loop, held in
// LDS and filled at the start of every launch by the table-free routines
// above (so they carry those routines' ~1 ulp accuracy):
//   sc[k] = (sin, cos)(2 pi k / 256), k = 0..255;
//   lg[j] = (v, -ln v) with v = 1/c rounded, c = 1 + (j - 37)/128, j = 0..90,
//           the grid of c over [sqrt(1/2), sqrt(2)).
struct BmTables {
    static constexpr int kSc = 256;
    static constexpr int kLg = 91;
    static constexpr int kLgOff = 37;
    double2 sc[kSc];
    double2 lg[kLg];
};

// The block's table, in LDS (one instance per kernel that uses it).
__device__ __forceinline__ BmTables* bm_tables()
{
    __shared__ BmTables t;
    return &t;
}

// Fills T with every thread of the block; ends with a block barrier.
__device__ __forceinline__ void fill_bm_tables(BmTables& T)
{
    for (int i = threadIdx.x; i < BmTables::kSc + BmTables::kLg; i += blockDim.x) {
        if (i < BmTables::kSc) {
            double s, c;
            sincos_2pi((double)i * (1.0 / BmTables::kSc), s, c);
            T.sc[i] = make_double2(s, c);
        } else {
            const int j = i - BmTables::kSc;
            const double v = 1.0 / (1.0 + (double)(j - BmTables::kLgOff) * (1.0 / 128.0));
            T.lg[j] = make_double2(v, 0.5 * neg2_log(v));
        }
    }
    __syncthreads();
}

// -2 ln u for u in (0, 1] with the table: u = m 2^e, m in [sqrt(1/2),
// sqrt(2)); c = 1 + j/128 the nearest grid point, v = 1/c rounded; then
// ln m = -ln v + ln(1 + r) with r = m v - 1 (one rounding, |r| < 0.0056), and
// ln(1 + r) is its series to r^7 (truncation below 2.2e-17 relative).  Near
// u = 1 the grid point is c = v = 1 and r = m - 1 exactly.
__device__ __forceinline__ double neg2_log_t(double u, const BmTables& T)
{
    double m = __builtin_amdgcn_frexp_mant(u);   // [0.5, 1)
    int e = __builtin_amdgcn_frexp_exp(u);
    if (m < 0x1.6a09e667f3bcdp-1) {
        m = 2.0 * m;
        e -= 1;
    }
    const int j = (int)__builtin_rint((m - 1.0) * 128.0) + BmTables::kLgOff;   // both exact
    const double2 g = T.lg[j];
    const double r = fma(m, g.x, -1.0);
    double p = 0x1.2492492492492p-3;             // 1/7
    p = fma(p, r, -0x1.5555555555555p-3);        // -1/6
    p = fma(p, r, 0x1.999999999999ap-3);         // 1/5
    p = fma(p, r, -0x1.0000000000000p-2);        // -1/4
    p = fma(p, r, 0x1.5555555555555p-2);         // 1/3
    p = fma(p, r, -0.5);
    const double l1p = fma(p, r * r, r);         // ln(1 + r)
    const double fe = -2.0 * (double)e;
    return fma(fe, 0x1.62e42fee00000p-1, fma(fe, 0x1.a39ef35793c76p-33, -2.0 * (g.y + l1p)));
}

// sin and cos of 2 pi u, u in (0, 1], with the table: k = nearest integer
// to 256 u, t = u - k/256 (exact, |t| <= 1/512), theta = 2 pi t; sin and cos
// of theta by their series to theta^7 and theta^6 (truncation below 7e-18
// relative and 2e-20 absolute), rotated by the table's angle 2 pi k / 256.
__device__ __forceinline__ void sincos_2pi_t(double u, const BmTables& T, double& s, double& c)
{
    const double q = __builtin_rint(256.0 * u);
    const double t = fma(-q, 1.0 / 256.0, u);
    const double th = t * 0x1.921fb54442d18p+2;  // 2 pi
    const double z = th * th;
    double ps = fma(-0x1.a01a01a01a01ap-13, z, 0x1.1111111111111p-7);   // -1/5040, 1/120
    ps = fma(ps, z, -0x1.5555555555555p-3);                              // -1/6
    const double st = fma(th * z, ps, th);
    double pc = fma(-0x1.6c16c16c16c17p-10, z, 0x1.5555555555555p-5);  // -1/720, 1/24
    pc = fma(pc, z, -0.5);
    const double ct = fma(pc, z, 1.0);
    const double2 a = T.sc[(int)q & (BmTables::kSc - 1)];
    s = fma(a.x, ct, a.y * st);
    c = fma(a.y, ct, -(a.x * st));
}

// FP64 stream: one block -> two 53-bit uniforms in (0, 1] -> one Box-Muller
// pair (cosine branch first): z0 = R cos(2 pi U2), z1 = R sin(2 pi U2),
// R = sqrt(-2 ln U1).
// ((hi << 21 | lo >> 11) + 1) * 2^-53, formed without a 64-bit integer: both
// terms below are exact doubles and so is their sum (a 53-bit integer times
// 2^-53), so the one rounding of the fma changes nothing.
__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo)
{
    return fma((double)hi, 0x1p-32, (double)((lo >> 11) + 1u) * 0x1p-53);
}

__device__ __forceinline__ void normals_f64(const Block& b, const BmTables& T, double& z0, double& z1)
{
    const double u1 = uniform53(b.w1, b.w0);
    const double u2 = uniform53(b.w3, b.w2);
    const double r = sqrt_nonneg(neg2_log_t(u1, T));
    double s, co;
    sincos_2pi_t(u2, T, s, co);
    z0 = r * co;
    z1 = r * s;
}

// FP32 uniform in (0, 1] from the top 24 bits of a word: (k + 1) 2^-24 with
// k = w >> 8, formed as k 2^-24 + 2^-24 in one fma (exact, like the product
// of the integer k + 1 and 2^-24).
__device__ __forceinline__ float uniform24(uint32_t w)
{
    return fmaf((float)(w >> 8), 0x1p-24f, 0x1p-24f);
}

// FP32 stream: two 24-bit uniforms in (0, 1] -> one Box-Muller pair, on the
// hardware transcendental unit: v_log_f32 is log2, and v_sin_f32 / v_cos_f32
// take their argument in revolutions, so sin(2 pi u) is one instruction.
__device__ __forceinline__ void normals_f32(uint32_t wa, uint32_t wb, float& z0, float& z1)
{
    const float u1 = uniform24(wa);
    const float u2 = uniform24(wb);
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));  // -2 ln 2 log2 u
    z0 = r * __builtin_amdgcn_cosf(u2);
    z1 = r * __builtin_amdgcn_sinf(u2);
}

// ---------------------------------------------------------------------------
// Density rho(x): voxel grid (zero outside), then analytic prisms [lo, hi),
// then open balls; contributions add in that order.
// ---------------------------------------------------------------------------
// floor((x - o) / d), the quotient rounded as a division rounds it.  When d
// is a power of two the reciprocal product is that quotient.  Otherwise the
// product q with the rounded reciprocal inv lies within 3 ulp of it (one
// rounding in inv, one in the product, one in the division), so floor(q) is
// the quotient's floor unless q lies within 2^-50 |q| (8 ulp) of an
// integer; only then (for a fraction of about 2^-49 |q| of the
// coordinates) the division runs.
__device__ __forceinline__ double grid_axis_f64(double x, double o, double d, double inv, int exact)
{
    const double a = x - o;
    const double q = a * inv;
    double t = floor(q);
    if (!exact) {
        const double f = q - t;   // exact
        const double e = fabs(q) * 0x1p-50;
        if (__builtin_expect((f < e) | (f > 1.0 - e), 0)) t = floor(a / d);
    }
    return t;
}

// Voxel holding (x, y, z), or -1 outside the grid (or without a grid).
__device__ __forceinline__ int64_t voxel_f64(const SourceF64& s, double x, double y, double z)
{
    if (!s.has_grid) return -1;
    const double tx = grid_axis_f64(x, s.origin[0], s.spacing[0], s.inv[0], s.exact[0]);
    const double ty = grid_axis_f64(y, s.origin[1], s.spacing[1], s.inv[1], s.exact[1]);
    const double tz = grid_axis_f64(z, s.origin[2], s.spacing[2], s.inv[2], s.exact[2]);
    // tested without short-circuiting (the bounds load together)
    const bool in = (tx >= 0.0) & (tx < (double)s.n[0]) & (ty >= 0.0) & (ty < (double)s.n[1]) & (tz >= 0.0) &
                    (tz < (double)s.n[2]);
    return in ? ((int64_t)(int)tz * s.n[1] + (int)ty) * s.n[0] + (int)tx : -1;
}

// Density of the analytic bodies at (x, y, z), added to r in body order.
// The membership tests are combined without short-circuiting and the sum is
// selected, not branched on: a body's bounds then load together (one wait
// instead of one per bound) and no lane diverges.
__device__ __forceinline__ double bodies_f64(const SourceF64& s, double r, double x, double y, double z, int j0 = 0)
{
    for (int j = j0; j < s.n_prisms; ++j) {
        const double* q = s.prisms[j];
        const bool in = (x >= q[0]) & (x < q[3]) & (y >= q[1]) & (y < q[4]) & (z >= q[2]) & (z < q[5]);
        r = in ? r + q[6] : r;
    }
    for (int j = 0; j < s.n_spheres; ++j) {
        const double* q = s.spheres[j];
        const double dx = x - q[0], dy = y - q[1], dz = z - q[2];
        const bool in = dx * dx + dy * dy + dz * dz < q[3] * q[3];
        r = in ? r + q[4] : r;
    }
    return r;
}

// A floored coordinate as an int (v_cvt_i32_f64): exact for integers in the
// int range, saturating to INT_MIN or INT_MAX beyond it, which in_axis reads
// as outside.
__device__ __forceinline__ int floor_to_i32(double t)
{
    int i;
    asm("v_cvt_i32_f64 %0, %1" : "=v"(i) : "v"(t));
    return i;
}

// 0 <= i < n as one unsigned compare.
__device__ __forceinline__ bool in_axis(int i, int n) { return (uint32_t)i < (uint32_t)n; }

// The voxel grid's density at (x, y, z): zero outside the grid or without one
// (the same voxel as voxel_f64).  Branch-free, and in two halves so that a
// run of lookups has all its loads in flight before the first value is used:
// fetch floors the coordinates to ints and loads the voxel's value, each
// index clamped into the grid so that the load always reads one of its
// voxels; keep drops the value unless all three indices lie in the grid (one
// unsigned compare each).  A voxel value of -0 may come back as -0 where the
// other paths give +0: no sum of densities can tell them apart (the walk's
// sums start at +0).  Positions are finite (walks start at finite stations
// and take bounded steps inside the box).  LEVELS: the grid is given by
// levels, the voxel's density levels[idx[v]]; fetch loads the level and keep
// its density (the index grid is a quarter of the FP32 grid's size).
// grid_in_* need a grid (has_grid); grid_* check for one.
struct GridProbe {
    float r;      // the voxel's density (FP32 grid)
    uint32_t b;   // or its level (grid by levels)
    int i[3];     // the floored indices, possibly outside the grid
};

// The flat index of indices i clamped into the grid; an index outside it
// becomes some voxel of the grid.  The row offset is a 24-bit multiply-add
// (the host limits each axis to fewer than 2^24 voxels) and the layer offset
// a 64-bit one.
template <class Src>
__device__ __forceinline__ uint64_t probe_index(const Src& s, const int* i)
{
    const uint32_t cx = min((uint32_t)i[0], (uint32_t)s.n[0] - 1u);
    const uint32_t cy = min((uint32_t)i[1], (uint32_t)s.n[1] - 1u);
    const uint32_t cz = min((uint32_t)i[2], (uint32_t)s.n[2] - 1u);
    uint64_t v = (uint64_t)cz * s.nxy + (__umul24(cy, (uint32_t)s.n[0]) + cx);
    asm("" : "+v"(v));   // one index, one address: the sum is not split
    return v;
}

template <bool LEVELS, class Src>
__device__ __forceinline__ void probe_load(const Src& s, GridProbe& p)
{
    const uint64_t v = probe_index(s, p.i);
    if (LEVELS)
        p.b = s.idx[v];
    else
        p.r = s.rho[v];
}

template <bool LEVELS, class Src>
__device__ __forceinline__ float probe_keep(const Src& s, const GridProbe& p)
{
    const bool in = in_axis(p.i[0], s.n[0]) & in_axis(p.i[1], s.n[1]) & in_axis(p.i[2], s.n[2]);
    const float r = LEVELS ? s.levels[p.b] : p.r;
    return in ? r : 0.0f;
}

template <bool LEVELS = false>
__device__ __forceinline__ GridProbe grid_fetch_f64(const SourceF64& s, double x, double y, double z)
{
    GridProbe p;
    p.i[0] = floor_to_i32(grid_axis_f64(x, s.origin[0], s.spacing[0], s.inv[0], s.exact[0]));
    p.i[1] = floor_to_i32(grid_axis_f64(y, s.origin[1], s.spacing[1], s.inv[1], s.exact[1]));
    p.i[2] = floor_to_i32(grid_axis_f64(z, s.origin[2], s.spacing[2], s.inv[2], s.exact[2]));
    probe_load<LEVELS>(s, p);
    return p;
}

template <bool LEVELS = false>
__device__ __forceinline__ double grid_keep_f64(const SourceF64& s, const GridProbe& p)
{
    return (double)probe_keep<LEVELS>(s, p);
}

template <bool LEVELS = false>
__device__ __forceinline__ double grid_in_f64(const SourceF64& s, double x, double y, double z)
{
    return grid_keep_f64<LEVELS>(s, grid_fetch_f64<LEVELS>(s, x, y, z));
}

// LEVELS: the kernel's grids are given by levels (a compile-time property
// of the launch, like the stepping loop's lookup).
template <bool LEVELS = false>
__device__ __forceinline__ double grid_f64(const SourceF64& s, double x, double y, double z)
{
    return s.has_grid ? grid_in_f64<LEVELS>(s, x, y, z) : 0.0;
}

template <bool LEVELS = false>
__device__ __forceinline__ double rho_f64(const SourceF64& s, double x, double y, double z)
{
    return bodies_f64(s, grid_f64<LEVELS>(s, x, y, z), x, y, z);
}

// floor(x) as an int in one instruction (v_cvt_flr_i32_f32 rounds toward
// -infinity while it converts).  Equal to (int)floorf(x) for finite x in the
// int range; beyond it the result saturates to INT_MIN or INT_MAX, which the
// unsigned compare of in_axis reads as outside.
__device__ __forceinline__ int floor_i32(float x)
{
    int i;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(i) : "v"(x));
    return i;
}

// FP32 voxel index along one axis: floor(x / spacing - origin / spacing)
// from one fma with both constants rounded to FP32 (inv = 1/spacing, ob =
// -origin/spacing).  Within an ulp of floor((x - origin) / spacing); the FP32
// walks' lookups and the mixed adjoint's voxels use this same formula.
// Positions are finite: walks start at finite stations and take bounded
// steps inside the box.
__device__ __forceinline__ int axis_f32(float x, float inv, float ob) { return floor_i32(fmaf(x, inv, ob)); }

__device__ __forceinline__ int voxel_f32(const SourceF32& s, float x, float y, float z)
{
    if (!s.has_grid) return -1;
    const int ix = axis_f32(x, s.inv[0], s.ob[0]);
    const int iy = axis_f32(y, s.inv[1], s.ob[1]);
    const int iz = axis_f32(z, s.inv[2], s.ob[2]);
    const bool in = in_axis(ix, s.n[0]) & in_axis(iy, s.n[1]) & in_axis(iz, s.n[2]);
    return in ? (iz * s.n[1] + iy) * s.n[0] + ix : -1;
}

__device__ __forceinline__ float bodies_f32(const SourceF32& s, float r, float x, float y, float z, int j0 = 0)
{
    for (int j = j0; j < s.n_prisms; ++j) {
        const float* q = s.prisms[j];
        const bool in = (x >= q[0]) & (x < q[3]) & (y >= q[1]) & (y < q[4]) & (z >= q[2]) & (z < q[5]);
        r = in ? r + q[6] : r;
    }
    for (int j = 0; j < s.n_spheres; ++j) {
        const float* q = s.spheres[j];
        const float dx = x - q[0], dy = y - q[1], dz = z - q[2];
        const bool in = dx * dx + dy * dy + dz * dz < q[3] * q[3];
        r = in ? r + q[4] : r;
    }
    return r;
}

// FP32 stepping's grid lookup, branch-free like grid_in_f64 (the same voxel
// as voxel_f32).
template <bool LEVELS = false>
__device__ __forceinline__ GridProbe grid_fetch_f32(const SourceF32& s, float x, float y, float z)
{
    GridProbe p;
    p.i[0] = axis_f32(x, s.inv[0], s.ob[0]);
    p.i[1] = axis_f32(y, s.inv[1], s.ob[1]);
    p.i[2] = axis_f32(z, s.inv[2], s.ob[2]);
    probe_load<LEVELS>(s, p);
    return p;
}

template <bool LEVELS = false>
__device__ __forceinline__ float grid_keep_f32(const SourceF32& s, const GridProbe& p)
{
    return probe_keep<LEVELS>(s, p);
}

template <bool LEVELS = false>
__device__ __forceinline__ float grid_in_f32(const SourceF32& s, float x, float y, float z)
{
    return grid_keep_f32<LEVELS>(s, grid_fetch_f32<LEVELS>(s, x, y, z));
}

template <bool LEVELS = false>
__device__ __forceinline__ float grid_f32(const SourceF32& s, float x, float y, float z)
{
    return s.has_grid ? grid_in_f32<LEVELS>(s, x, y, z) : 0.0f;
}

template <bool LEVELS = false>
__device__ __forceinline__ float rho_f32(const SourceF32& s, float x, float y, float z)
{
    return bodies_f32(s, grid_f32<LEVELS>(s, x, y, z), x, y, z);
}

// ---------------------------------------------------------------------------
// Exit test (the boundary counts as outside) and the INTERSECT exit point.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool outside(const T* lo, const T* hi, T x, T y, T z)
{
    return x <= lo[0] || x >= hi[0] || y <= lo[1] || y >= hi[1] || z <= lo[2] || z >= hi[2];
}

// First face met on the segment a -> b (b outside, a inside): the crossing
// fraction t_c = (face_c - a_c) / (b_c - a_c) is smallest (ties: lower axis);
// the point is a + t (b - a) with the crossing coordinate set to the face.
__device__ __forceinline__ void intersect_exit(const double* lo, const double* hi, const double a[3],
                                               const double b[3], double e[3])
{
    double tmin = 2.0;
    int cmin = 0;
    double fmin = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const bool below = b[c] <= lo[c];
        const bool above = b[c] >= hi[c];
        if (below || above) {
            const double f = below ? lo[c] : hi[c];
            const double t = (f - a[c]) / (b[c] - a[c]);
            if (t < tmin) {
                tmin = t;
                cmin = c;
                fmin = f;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) e[c] = fma(tmin, b[c] - a[c], a[c]);
    e[cmin] = fmin;
}

// Squared distance |x - c|^2, the products of the first two axes fused into
// the running sum (the ball domain's exit test).
template <typename T>
__device__ __forceinline__ T dist2(T x0, T x1, T x2, T c0, T c1, T c2)
{
    const T d0 = x0 - c0, d1 = x1 - c1, d2 = x2 - c2;
    return fma(d0, d0, fma(d1, d1, d2 * d2));
}

// INTERSECT on the ball |x - c| = R: a + t (b - a) with t the root in (0, 1]
// of |a + t v - c|^2 = R^2, written t = -C / (B + sqrt(B^2 - A C)) with
// A = |v|^2, B = (a - c).v and C = |a - c|^2 - R^2 < 0 (no cancellation).
__device__ __forceinline__ void intersect_ball(const double* c, double r2, const double a[3], const double b[3],
                                               double e[3])
{
    double v[3], q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = b[k] - a[k];
        q[k] = a[k] - c[k];
    }
    const double A = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double B = q[0] * v[0] + q[1] * v[1] + q[2] * v[2];
    const double C = (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) - r2;
    double t = -C / (B + sqrt(B * B - A * C));
    if (t > 1.0) t = 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) e[k] = fma(t, v[k], a[k]);
}

// ---------------------------------------------------------------------------
// Dirichlet data.
// ---------------------------------------------------------------------------

// Tables of the prism closed form, in LDS: the log grid of BmTables and
// atan(k/64), k = 0..64 (library atan, filled at the start of the launch).
struct AtanTable {
    static constexpr int kN = 64;
    double at[kN + 1];
};

struct DataTables {
    const BmTables* bm;
    const AtanTable* at;
};

__device__ __forceinline__ AtanTable* atan_table()
{
    __shared__ AtanTable t;
    return &t;
}

// Fills both tables with every thread of the block; ends with a barrier.
__device__ __forceinline__ DataTables fill_data_tables()
{
    BmTables* bm = bm_tables();
    AtanTable* at = atan_table();
    for (int i = threadIdx.x; i <= AtanTable::kN; i += blockDim.x) at->at[i] = atan((double)i / AtanTable::kN);
    fill_bm_tables(*bm);
    return DataTables{bm, at};
}

// ln x for a positive finite x, from the table-driven -2 ln x.
__device__ __forceinline__ double ln_t(double x, const BmTables& T) { return -0.5 * neg2_log_t(x, T); }

// 1/q for a positive normal q: the hardware estimate and two Newton steps
// (each squares the relative error), within about 1 ulp.
__device__ __forceinline__ double recip(double q)
{
    double y = __builtin_amdgcn_rcp(q);
    y = fma(fma(-q, y, 1.0), y, y);
    return fma(fma(-q, y, 1.0), y, y);
}

// atan(n / d) for finite n and d != 0.  With u = min(|n|, |d|) and
// v = max(|n|, |d|), t = u / v lies in [0, 1]; c = k/64 is a grid point near
// t (k from the reciprocal estimate, any k with |t - c| <= 1/128 + 1e-9 does)
// and atan t = atan c + atan(delta) with delta = (u - c v)/(v + c u) (the
// quotient from the refined reciprocal of its positive denominator and one
// residual correction, within about an ulp), its series to delta^9
// (truncation below 1e-24); pi/2 - atan t when |n| > |d|, and the sign of
// n/d.  No branches.
__device__ __forceinline__ double atan_q(double n, double d, const AtanTable& A)
{
    const double an = fabs(n), ad = fabs(d);
    const bool swap = an > ad;
    const double u = swap ? ad : an, v = swap ? an : ad;
    double k = __builtin_rint(u * __builtin_amdgcn_rcp(v) * (double)AtanTable::kN);
    k = fmin(fmax(k, 0.0), (double)AtanTable::kN);
    const double c = k * (1.0 / AtanTable::kN);
    const double num = fma(-c, v, u), den = fma(c, u, v);
    const double rd = recip(den);
    double dl = num * rd;
    dl = fma(fma(-den, dl, num), rd, dl);
    const double z = dl * dl;
    double p = fma(z, 0x1.c71c71c71c71cp-4, -0x1.2492492492492p-3);   // 1/9, -1/7
    p = fma(p, z, 0x1.999999999999ap-3);                                // 1/5
    p = fma(p, z, -0x1.5555555555555p-2);                               // -1/3
    double a = A.at[(int)k] + fma(dl * z, p, dl);
    a = swap ? 0x1.921fb54442d18p+0 - a : a;                            // pi/2
    return ((n < 0.0) != (d < 0.0)) ? -a : a;
}

// The argument of ln(w + r), r = sqrt(w^2 + s), as a quotient n / d free
// of cancellation: (w + r) / 1 for w >= 0, and s / (r - w) for w < 0, where
// the sum would cancel.
struct Quot {
    double n, d;
};

__device__ __forceinline__ Quot shift_quot(double w, double r, double s)
{
    const bool pos = w >= 0.0;
    return Quot{pos ? w + r : s, pos ? 1.0 : r - w};
}

// ln(A / B) for A = a.n / a.d and B = b.n / b.d, as one logarithm of
// (a.n b.d) / (a.d b.n).  An argument that is not positive and finite --
// only in terms the caller discards, whose prefactor is zero -- is replaced by
// 1 so that the table lookup stays in range.
__device__ __forceinline__ double ln_ratio(const Quot& a, const Quot& b, const BmTables& T)
{
    double x = (a.n * b.d) * recip(a.d * b.n);
    x = (x > 0.0 && x <= 0x1.fffffffffffffp+1023) ? x : 1.0;
    return ln_t(x, T);
}

// atan2(n, d), the angle of the point (d, n) in (-pi, pi]: atan(n / d) moved
// by pi to the left half-plane.  n = d = 0 occurs only in discarded terms.
__device__ __forceinline__ double atan2_q(double n, double d, const AtanTable& A)
{
    const double a = atan_q(n, d, A);
    const double pi = 0x1.921fb54442d18p+1;
    return d < 0.0 ? (n < 0.0 ? a - pi : a + pi) : a;
}

// F(X, Y, Z) below has the cyclic form sum over (u, v, w) of
// u v ln(w + r) - (u^2 / 2) atan(v w / (u r)), (u, v, w) = (X, Y, Z), (Y, Z, X),
// (Z, X, Y).  Along a prism edge only w changes, so the difference of the
// logarithmic term between the edge's upper corner (w_u, r_u) and lower
// corner (w_l, r_l) takes one logarithm, u v ln((w_u + r_u) / (w_l + r_l));
// it vanishes when u v = 0.  s = u^2 + v^2.
__device__ __forceinline__ double edge_log(double u, double v, double wl, double wu, double rl, double ru, double s,
                                           const BmTables& T)
{
    const double uv = u * v;
    const double l = uv * ln_ratio(shift_quot(wu, ru, s), shift_quot(wl, rl, s), T);
    return (uv != 0.0) ? l : 0.0;
}

// The arctangent terms of one face of the prism, the plane u = U with corners
// (v_j, w_k): sum_jk (-1)^(j+k) atan(v_j w_k / (|U| r_jk)), the solid angle
// the face subtends from p for U > 0.  Each term is the argument of
// c_jk = |U| r_jk + i v_j w_k, inside (-pi/2, pi/2).  The two edge products
// E0 = c00 conj(c01) and E1 = c11 conj(c10) have arguments inside (-pi, pi)
// whose sum, inside (-2 pi, 2 pi), is the face's: the argument of E0 E1 (one
// atan2), plus 2 pi when both edge arguments are positive and the product's
// is negative, minus 2 pi in the mirrored case.  au = |U|; vw[j][k] = v_j w_k.
__device__ __forceinline__ double face_angle(double au, const double (&r)[2][2], const double (&vw)[2][2],
                                             const AtanTable& A)
{
    double p[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int k = 0; k < 2; ++k) p[j][k] = au * r[j][k];
    const double e0r = fma(p[0][0], p[0][1], vw[0][0] * vw[0][1]);      // c00 conj(c01)
    const double e0i = fma(vw[0][0], p[0][1], -(p[0][0] * vw[0][1]));
    const double e1r = fma(p[1][1], p[1][0], vw[1][1] * vw[1][0]);      // c11 conj(c10)
    const double e1i = fma(vw[1][1], p[1][0], -(p[1][1] * vw[1][0]));
    const double pr = fma(e0r, e1r, -(e0i * e1i));
    const double pi = fma(e0r, e1i, e0i * e1r);
    const double two_pi = 0x1.921fb54442d18p+2;
    const double wrap = ((e0i > 0.0) & (e1i > 0.0) & (pi < 0.0))   ? two_pi
                        : ((e0i < 0.0) & (e1i < 0.0) & (pi > 0.0)) ? -two_pi
                                                                   : 0.0;
    return atan2_q(pi, pr, A) + wrap;
}

// Newtonian integral of the unit-density prism [lo, hi] seen from p: the
// alternating corner sum of
//   XY ln(Z+r) + YZ ln(X+r) + ZX ln(Y+r)
//   - X^2/2 atan(YZ/(Xr)) - Y^2/2 atan(ZX/(Yr)) - Z^2/2 atan(XY/(Zr))
// with corner (X, Y, Z) = corner - p and sign + at the corners with an odd
// number of upper coordinates (Nagy, Papp & Benedek 2000); a term whose
// prefactor is zero vanishes.  The logarithms are taken in pairs along each
// of the 12 edges (edge_log) and the arctangents by face: the face U = U_a
// contributes (-1)^a U_a |U_a| / 2 times its angle (face_angle).  That is 8
// corner distances (sqrt_nonneg, from the hardware reciprocal square root:
// a distance is zero or far above the subnormal range), 12 logarithms and 6
// arctangents instead of 24 of each, with no cancellation between the two
// corners' large logarithms.  Every term is evaluated and the vanishing ones
// selected away (their logarithm or quotient may be infinite), so the lanes
// of a wavefront -- whose exit points differ -- take no branches.  The face
// products are of degree 8 in the coordinates: exact for |coordinates| up
// to about 1e37.
__device__ inline double prism_newton(const double* q, double px, double py, double pz, const DataTables& tb)
{
    const BmTables& T = *tb.bm;
    const AtanTable& A = *tb.at;
    const double X[2] = {q[0] - px, q[3] - px};
    const double Y[2] = {q[1] - py, q[4] - py};
    const double Z[2] = {q[2] - pz, q[5] - pz};
    const double X2[2] = {X[0] * X[0], X[1] * X[1]};
    const double Y2[2] = {Y[0] * Y[0], Y[1] * Y[1]};
    const double Z2[2] = {Z[0] * Z[0], Z[1] * Z[1]};
    double r[2][2][2];                    // r[i][j][k] at corner (X[i], Y[j], Z[k])
    double xy[2][2], yz[2][2], zx[2][2];  // xy[i][j] = X[i] Y[j], ...
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            xy[i][j] = X[i] * Y[j];
            yz[i][j] = Y[i] * Z[j];
            zx[i][j] = Z[i] * X[j];
#pragma unroll
            for (int k = 0; k < 2; ++k) r[i][j][k] = sqrt_nonneg(X2[i] + Y2[j] + Z2[k]);
        }
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            // an edge's upper corner has a + b + 1 upper coordinates: sign + when that is odd
            double e = edge_log(X[a], Y[b], Z[0], Z[1], r[a][b][0], r[a][b][1], X2[a] + Y2[b], T);   // along z
            e += edge_log(Y[a], Z[b], X[0], X[1], r[0][a][b], r[1][a][b], Y2[a] + Z2[b], T);          // along x
            e += edge_log(Z[a], X[b], Y[0], Y[1], r[b][0][a], r[b][1][a], Z2[a] + X2[b], T);          // along y
            v += ((a + b) & 1) ? -e : e;
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        // the faces x = X[a] (corners (Y_j, Z_k)), y = Y[a] (corners (Z_k, X_i))
        // and z = Z[a] (corners (X_i, Y_j))
        const double rx[2][2] = {{r[a][0][0], r[a][0][1]}, {r[a][1][0], r[a][1][1]}};
        const double ry[2][2] = {{r[0][a][0], r[1][a][0]}, {r[0][a][1], r[1][a][1]}};
        const double rz[2][2] = {{r[0][0][a], r[0][1][a]}, {r[1][0][a], r[1][1][a]}};
        const double tx = X[a] * fabs(X[a]) * face_angle(fabs(X[a]), rx, yz, A);
        const double ty = Y[a] * fabs(Y[a]) * face_angle(fabs(Y[a]), ry, zx, A);
        const double tz = Z[a] * fabs(Z[a]) * face_angle(fabs(Z[a]), rz, xy, A);
        const double t = ((X[a] != 0.0) ? tx : 0.0) + ((Y[a] != 0.0) ? ty : 0.0) + ((Z[a] != 0.0) ? tz : 0.0);
        v += a ? -0.5 * t : 0.5 * t;
    }
    return v;
}

__device__ inline double face_grid(const BoundaryArgs& bc, const double* lo, const double* hi, const double e[3])
{
    int fc = 0, side = 0;
    double best = -1.0 / 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double dl = lo[c] - e[c];
        const double dh = e[c] - hi[c];
        if (dl > best) { best = dl; fc = c; side = 0; }
        if (dh > best) { best = dh; fc = c; side = 1; }
    }
    const int f = 2 * fc + side;
    const int ax = (fc == 0) ? 1 : 0;
    const int bx = (fc == 2) ? 1 : 2;
    const int na = bc.face_n[f][0], nb = bc.face_n[f][1];
    const double pa = fmin(fmax(e[ax], lo[ax]), hi[ax]);
    const double pb = fmin(fmax(e[bx], lo[bx]), hi[bx]);
    const double ta = (pa - lo[ax]) / (hi[ax] - lo[ax]) * (double)(na - 1);
    const double tb = (pb - lo[bx]) / (hi[bx] - lo[bx]) * (double)(nb - 1);
    int ia = (int)floor(ta), ib = (int)floor(tb);
    ia = ia < 0 ? 0 : (ia > na - 2 ? na - 2 : ia);
    ib = ib < 0 ? 0 : (ib > nb - 2 ? nb - 2 : ib);
    const double fa = ta - ia, fb = tb - ib;
    const double* d = bc.face_data + bc.face_off[f];
    const double v00 = d[(int64_t)ib * na + ia], v10 = d[(int64_t)ib * na + ia + 1];
    const double v01 = d[(int64_t)(ib + 1) * na + ia], v11 = d[(int64_t)(ib + 1) * na + ia + 1];
    return (1.0 - fa) * (1.0 - fb) * v00 + fa * (1.0 - fb) * v10 + (1.0 - fa) * fb * v01 + fa * fb * v11;
}

__device__ inline double boundary_value(const BoundaryArgs& bc, const double* lo, const double* hi, double G,
                                        const double e[3], const DataTables& tb)
{
    const double x = e[0], y = e[1], z = e[2];
    switch (bc.kind) {
    case 1: {  // quadratic c0 + b.x + x^T A x, A from its upper triangle
        const double* q = bc.quad;
        return q[0] + q[1] * x + q[2] * y + q[3] * z + q[4] * x * x + 2.0 * q[5] * x * y +
               2.0 * q[6] * x * z + q[7] * y * y + 2.0 * q[8] * y * z + q[9] * z * z;
    }
    case 2: {  // point masses
        double v = 0.0;
        for (int j = 0; j < bc.n_items; ++j) {
            const double* q = bc.items[j];
            const double dx = x - q[0], dy = y - q[1], dz = z - q[2];
            v -= G * q[3] / sqrt(dx * dx + dy * dy + dz * dz);
        }
        return v;
    }
    case 3: {  // homogeneous prisms
        double v = 0.0;
        for (int j = 0; j < bc.n_items; ++j) {
            const double* q = bc.items[j];
            v += -G * q[6] * prism_newton(q, x, y, z, tb);
        }
        return v;
    }
    case 4:
        return face_grid(bc, lo, hi, e);
    default:
        return 0.0;
    }
}

}  // namespace fk
