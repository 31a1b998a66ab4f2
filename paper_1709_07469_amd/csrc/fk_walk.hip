// fk_walk.hip -- the walk kernels: every lane steps one Brownian walk at a
// time by Euler-Maruyama, accumulates the trapezoid sum of the density along
// it, detects the exit from the box and stores the exit point and the sum
// (arXiv:1709.07469, section 2.3, steps 1-4).  The Dirichlet data is read at
// the stored exit points by the reduction pass, where every lane evaluates it
// at once instead of one lane at a time inside the stepping loop.
//
// Scheduling (gfx950, wave64):
//   - persistent blocks, sized from the occupancy calculator;
//   - a wavefront claims a run of consecutive walks from one global counter
//     (one atomic per claim; the run shrinks as the queue drains so the last
//     walks spread over all wavefronts);
//   - lanes whose walk has ended are refilled at macro-step boundaries, where
//     every active lane is at the start of a Philox block triple: FP64 walks
//     take 2 steps (6 normals = 3 blocks), mixed walks take 4 steps
//     (12 normals = 3 blocks) per macro-step;
//   - a walk's sample is written to its own slot (task index), so the result
//     does not depend on which lane or wavefront ran it.
#include <hip/hip_runtime.h>

#include "fk_device.hpp"

namespace fk {

namespace {

constexpr uint32_t kCapFlag = 0x80000000u;

__global__ void zero_queue_kernel(unsigned long long* q)
{
    if (threadIdx.x == 0) q[0] = 0ull;
}

__device__ __forceinline__ uint64_t first_lane_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Wave-uniform claim state.
struct Pool {
    uint64_t next;
    uint64_t end;
    uint64_t left;
    bool exhausted;
};

// Refills idle lanes from the wavefront's claimed run, claiming a new run
// when it is empty.  Returns the task of this lane if it was idle and got
// one, else ~0.
__device__ __forceinline__ uint64_t refill(Pool& pool, const WalkCommon& C, bool active)
{
    const uint64_t idle = __ballot(!active);
    if (idle == 0) return ~0ull;
    const uint32_t n_idle = (uint32_t)__popcll(idle);
    if (pool.next == pool.end && !pool.exhausted) {
        uint64_t want = pool.left / (4ull * C.total_waves);
        if (want < n_idle) want = n_idle;
        if (want > (uint64_t)C.grab) want = (uint64_t)C.grab;
        unsigned long long old = 0ull;
        if (__lane_id() == 0) old = atomicAdd(C.queue, (unsigned long long)want);
        old = first_lane_u64(__shfl(old, 0));
        if (old >= (uint64_t)C.n_tasks) {
            pool.exhausted = true;
        } else {
            pool.next = old;
            pool.end = old + want < (uint64_t)C.n_tasks ? old + want : (uint64_t)C.n_tasks;
            pool.left = (uint64_t)C.n_tasks - pool.end;
        }
    }
    const uint64_t avail = pool.end - pool.next;
    const uint32_t rank = (uint32_t)__popcll(idle & __lanemask_lt());
    uint64_t mine = ~0ull;
    if (!active && rank < avail) mine = pool.next + rank;
    pool.next += (n_idle < avail) ? n_idle : avail;
    return mine;
}

struct TaskInfo {
    double x0[3];
    uint64_t s;      // station
    uint32_t w;      // 0: the walk from x0 (+h e_z for g_z), 1: from x0 - h e_z
    uint32_t sctr;   // station word of the Philox counter
    uint32_t pctr;   // path word
};

__device__ __forceinline__ TaskInfo decode(const WalkCommon& C, uint64_t t)
{
    TaskInfo ti;
    const uint64_t q = (C.npair == 2) ? (t >> 1) : t;
    const uint32_t w = (C.npair == 2) ? (uint32_t)(t & 1ull) : 0u;
    const uint64_t s = q / (uint64_t)C.N;
    const uint64_t i = q - s * (uint64_t)C.N;
    const double* st = C.stations + 3 * s;
    ti.x0[0] = st[0];
    ti.x0[1] = st[1];
    ti.x0[2] = st[2];
    if (C.npair == 2) ti.x0[2] = (w == 0) ? st[2] + C.h : st[2] - C.h;
    ti.sctr = (C.npair == 2 && C.pairing == FK_PAIR_INDEPENDENT) ? (uint32_t)(2 * s + w) : (uint32_t)s;
    ti.pctr = (uint32_t)((uint64_t)C.path_offset + i);
    ti.s = s;
    ti.w = w;
    return ti;
}

// Adjoint replay: a walk whose sample (or pair) the forward solve excluded
// is skipped.
__device__ __forceinline__ bool forward_capped(const WalkCommon& C, uint64_t t)
{
    if (C.npair == 2) {
        const uint64_t j = t & ~1ull;
        return ((C.fwd_steps[j] | C.fwd_steps[j + 1]) & kCapFlag) != 0;
    }
    return (C.fwd_steps[t] & kCapFlag) != 0;
}

// Run-length coalesced scatter of signed trapezoid weights.
struct Scatter {
    int64_t* base;   // counts of this walk's station
    int64_t v;       // pending voxel (-1: none)
    int64_t c;       // pending weight
    int64_t sign;
    __device__ __forceinline__ void flush()
    {
        if (v >= 0 && c != 0) atomicAdd(reinterpret_cast<unsigned long long*>(base + v), (unsigned long long)c);
        c = 0;
    }
    __device__ __forceinline__ void add(int64_t voxel, int64_t weight)
    {
        if (voxel != v) {
            flush();
            v = voxel;
        }
        c += sign * weight;
    }
};

__device__ __forceinline__ bool strictly_inside(const WalkCommon& C, const double x[3])
{
    return x[0] > C.lo[0] && x[0] < C.hi[0] && x[1] > C.lo[1] && x[1] < C.hi[1] && x[2] > C.lo[2] &&
           x[2] < C.hi[2];
}

// ---------------------------------------------------------------------------
// FP64 walks: FP64 stream (53-bit uniforms), FP64 position and trapezoid sum.
// ---------------------------------------------------------------------------
template <bool ADJ>
__global__ void __launch_bounds__(256) walk_f64_kernel(const WalkArgsF64 A)
{
    const WalkCommon& C = A.c;
    Pool pool{0ull, 0ull, (uint64_t)C.n_tasks, false};

    bool active = false;
    uint64_t task = 0;
    double x0 = 0.0, x1 = 0.0, x2 = 0.0, rp = 0.0, S = 0.0;
    uint32_t n = 0, k = 0, sctr = 0, pctr = 0;
    Scatter sc{nullptr, -1, 0, 1};

    for (;;) {
        const uint64_t got = refill(pool, C, active);
        if (got != ~0ull) {
            const TaskInfo ti = decode(C, got);
            task = got;
            if (ADJ && (!strictly_inside(C, ti.x0) || forward_capped(C, task))) {
                // excluded in the forward solve: contributes nothing
            } else if (ADJ) {
                x0 = ti.x0[0];
                x1 = ti.x0[1];
                x2 = ti.x0[2];
                sctr = ti.sctr;
                pctr = ti.pctr;
                n = 0;
                k = 0;
                sc.base = C.counts + ti.s * C.nvox;
                sc.v = -1;
                sc.c = 0;
                sc.sign = ti.w ? -1 : 1;
                sc.add(voxel_f64(A.src, x0, x1, x2), 1);
                active = true;
            } else if (!strictly_inside(C, ti.x0)) {
                // a start point on or outside the boundary yields no sample
                const double q = __builtin_nan("");
                C.exits[task] = ExitRecord{q, q, q, q};
                C.steps[task] = kCapFlag;
            } else {
                x0 = ti.x0[0];
                x1 = ti.x0[1];
                x2 = ti.x0[2];
                sctr = ti.sctr;
                pctr = ti.pctr;
                rp = rho_f64(A.src, x0, x1, x2);
                S = 0.0;
                n = 0;
                k = 0;
                active = true;
            }
        }
        if (__ballot(active) == 0ull) {
            if (pool.exhausted) break;
            continue;
        }
        if (!active) continue;

        double z[6];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const Block bl = philox10(k + b, pctr, sctr, C.problem_id, C.key0, C.key1);
            normals_f64(bl, z[2 * b], z[2 * b + 1]);
        }
        k += 3;

        bool done = false, capped = false;
        double e[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            if (!done) {
                const double y0 = fma(C.sdt, z[3 * st + 0], x0);
                const double y1 = fma(C.sdt, z[3 * st + 1], x1);
                const double y2 = fma(C.sdt, z[3 * st + 2], x2);
                double rn = 0.0;
                if (!ADJ) {
                    rn = rho_f64(A.src, y0, y1, y2);
                    S = S + (rp + rn);
                }
                n += 1;
                const bool out = outside(C.lo, C.hi, y0, y1, y2);
                if (ADJ) sc.add(voxel_f64(A.src, y0, y1, y2), out ? 1 : 2);
                if (out) {
                    done = true;
                    if (ADJ) {
                    } else if (C.exit_rule == FK_EXIT_INTERSECT) {
                        const double a[3] = {x0, x1, x2};
                        const double b[3] = {y0, y1, y2};
                        intersect_exit(C.lo, C.hi, a, b, e);
                    } else {
                        e[0] = y0;
                        e[1] = y1;
                        e[2] = y2;
                    }
                } else {
                    x0 = y0;
                    x1 = y1;
                    x2 = y2;
                    rp = rn;
                    if ((int64_t)n == C.max_steps) {
                        done = true;
                        capped = true;
                    }
                }
            }
        }
        if (done) {
            if (ADJ) {
                sc.flush();
            } else {
                C.exits[task] = ExitRecord{e[0], e[1], e[2], S};
                C.steps[task] = n | (capped ? kCapFlag : 0u);
            }
            active = false;
        }
    }
}

// ---------------------------------------------------------------------------
// Mixed walks: FP32 stream and FP32 position; the trapezoid sum in FP64 or
// as a Kahan-compensated FP32 pair; exit point and data in FP64.
// ---------------------------------------------------------------------------
template <bool KAHAN, bool ADJ>
__global__ void __launch_bounds__(256) walk_f32_kernel(const WalkArgsF32 A)
{
    const WalkCommon& C = A.c;
    Pool pool{0ull, 0ull, (uint64_t)C.n_tasks, false};

    bool active = false;
    uint64_t task = 0;
    float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f, rp = 0.0f;
    double S = 0.0;            // FP64 accumulation
    float Sf = 0.0f, Sc = 0.0f;  // Kahan sum and compensation
    uint32_t n = 0, k = 0, sctr = 0, pctr = 0;
    Scatter sc{nullptr, -1, 0, 1};

    for (;;) {
        const uint64_t got = refill(pool, C, active);
        if (got != ~0ull) {
            const TaskInfo ti = decode(C, got);
            task = got;
            if (ADJ && (!strictly_inside(C, ti.x0) || forward_capped(C, task))) {
                // excluded in the forward solve: contributes nothing
            } else if (ADJ) {
                x0 = (float)ti.x0[0];
                x1 = (float)ti.x0[1];
                x2 = (float)ti.x0[2];
                sctr = ti.sctr;
                pctr = ti.pctr;
                n = 0;
                k = 0;
                sc.base = C.counts + ti.s * C.nvox;
                sc.v = -1;
                sc.c = 0;
                sc.sign = ti.w ? -1 : 1;
                sc.add(voxel_f32(A.src, x0, x1, x2), 1);
                active = true;
            } else if (!strictly_inside(C, ti.x0)) {
                // a start point on or outside the boundary yields no sample
                const double q = __builtin_nan("");
                C.exits[task] = ExitRecord{q, q, q, q};
                C.steps[task] = kCapFlag;
            } else {
                x0 = (float)ti.x0[0];
                x1 = (float)ti.x0[1];
                x2 = (float)ti.x0[2];
                sctr = ti.sctr;
                pctr = ti.pctr;
                rp = rho_f32(A.src, x0, x1, x2);
                S = 0.0;
                Sf = 0.0f;
                Sc = 0.0f;
                n = 0;
                k = 0;
                active = true;
            }
        }
        if (__ballot(active) == 0ull) {
            if (pool.exhausted) break;
            continue;
        }
        if (!active) continue;

        float z[12];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const Block bl = philox10(k + b, pctr, sctr, C.problem_id, C.key0, C.key1);
            normals_f32(bl.w0, bl.w1, z[4 * b + 0], z[4 * b + 1]);
            normals_f32(bl.w2, bl.w3, z[4 * b + 2], z[4 * b + 3]);
        }
        k += 3;

        bool done = false, capped = false;
        float ex = 0.0f, ey = 0.0f, ez = 0.0f;   // last inside point (INTERSECT)
        float fx = 0.0f, fy = 0.0f, fz = 0.0f;   // first outside point
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            if (!done) {
                const float y0 = fmaf(C.sdt_f, z[3 * st + 0], x0);
                const float y1 = fmaf(C.sdt_f, z[3 * st + 1], x1);
                const float y2 = fmaf(C.sdt_f, z[3 * st + 2], x2);
                float rn = 0.0f;
                if (!ADJ) {
                    rn = rho_f32(A.src, y0, y1, y2);
                    if (KAHAN) {
                        const float y = (rp + rn) - Sc;
                        const float t = Sf + y;
                        Sc = (t - Sf) - y;
                        Sf = t;
                    } else {
                        S = S + ((double)rp + (double)rn);
                    }
                }
                n += 1;
                const bool out = outside(C.lo_f, C.hi_f, y0, y1, y2);
                if (ADJ) sc.add(voxel_f32(A.src, y0, y1, y2), out ? 1 : 2);
                if (out) {
                    done = true;
                    ex = x0; ey = x1; ez = x2;
                    fx = y0; fy = y1; fz = y2;
                } else {
                    x0 = y0;
                    x1 = y1;
                    x2 = y2;
                    rp = rn;
                    if ((int64_t)n == C.max_steps) {
                        done = true;
                        capped = true;
                    }
                }
            }
        }
        if (done && ADJ) {
            sc.flush();
            active = false;
        } else if (done) {
            double e[3] = {(double)fx, (double)fy, (double)fz};
            if (!capped && C.exit_rule == FK_EXIT_INTERSECT) {
                const double a[3] = {(double)ex, (double)ey, (double)ez};
                const double b[3] = {(double)fx, (double)fy, (double)fz};
                intersect_exit(C.lo, C.hi, a, b, e);
            }
            const double sum = KAHAN ? ((double)Sf - (double)Sc) : S;
            C.exits[task] = ExitRecord{e[0], e[1], e[2], sum};
            C.steps[task] = n | (capped ? kCapFlag : 0u);
            active = false;
        }
    }
}

}  // namespace

hipError_t launch_zero_queue(unsigned long long* queue, hipStream_t stream)
{
    hipLaunchKernelGGL(zero_queue_kernel, dim3(1), dim3(64), 0, stream, queue);
    return hipGetLastError();
}

hipError_t launch_walk_f64(const WalkArgsF64& a, const LaunchCfg& cfg, hipStream_t stream, bool adjoint)
{
    if (adjoint)
        hipLaunchKernelGGL(walk_f64_kernel<true>, dim3(cfg.grid), dim3(cfg.block), 0, stream, a);
    else
        hipLaunchKernelGGL(walk_f64_kernel<false>, dim3(cfg.grid), dim3(cfg.block), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_walk_f32(const WalkArgsF32& a, bool kahan, const LaunchCfg& cfg, hipStream_t stream, bool adjoint)
{
    if (adjoint) {
        if (kahan)
            hipLaunchKernelGGL((walk_f32_kernel<true, true>), dim3(cfg.grid), dim3(cfg.block), 0, stream, a);
        else
            hipLaunchKernelGGL((walk_f32_kernel<false, true>), dim3(cfg.grid), dim3(cfg.block), 0, stream, a);
    } else {
        if (kahan)
            hipLaunchKernelGGL((walk_f32_kernel<true, false>), dim3(cfg.grid), dim3(cfg.block), 0, stream, a);
        else
            hipLaunchKernelGGL((walk_f32_kernel<false, false>), dim3(cfg.grid), dim3(cfg.block), 0, stream, a);
    }
    return hipGetLastError();
}

hipError_t walk_occupancy(int precision, int block, int* blocks_per_cu)
{
    const void* fn = precision == FK_F64 ? (const void*)walk_f64_kernel<false>
                   : precision == FK_MIXED_KAHAN ? (const void*)walk_f32_kernel<true, false>
                                                 : (const void*)walk_f32_kernel<false, false>;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, 0);
}

// ---------------------------------------------------------------------------
// Adjoint helpers.
// ---------------------------------------------------------------------------
namespace {

__global__ void fill_zero_kernel(int64_t* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// grad_rho[v] = sum_s coef_s counts[s][v], s in order, with
// coef_s = grad_out[s] * scale / n_s (n_s = untruncated samples of station s).
__global__ void combine_kernel(const int64_t* counts, int64_t n_stations, int64_t nvox, const double* grad_out,
                               const fk_stat* fwd, double scale, double* grad_rho)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int64_t s = 0; s < n_stations; ++s) {
            const int64_t ns = fwd[s].n;
            if (ns <= 0) continue;
            const double coef = grad_out[s] * scale / (double)ns;
            acc += coef * (double)counts[s * nvox + v];
        }
        grad_rho[v] = acc;
    }
}

}  // namespace

hipError_t launch_fill_zero(int64_t* p, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_adjoint_combine(const int64_t* counts, int64_t n_stations, int64_t nvox, const double* grad_out,
                                  const fk_stat* fwd, double scale, double* grad_rho, hipStream_t stream)
{
    const int64_t blocks = (nvox + 255) / 256 < 8192 ? (nvox + 255) / 256 : 8192;
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, counts, n_stations, nvox,
                       grad_out, fwd, scale, grad_rho);
    return hipGetLastError();
}

}  // namespace fk
