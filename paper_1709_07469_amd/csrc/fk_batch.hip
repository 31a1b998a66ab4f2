// fk_batch.hip -- many independent problems (density models, station sets,
// walk counts, parameters) solved in one persistent launch with one
// work-stealing queue, so that problems of very uneven cost share the GPU
// without a launch per problem and without idle tails between problems.
//
//   - Problem descriptors live in the workspace; they are written by small
//     kernels that carry the bytes in their arguments, so a captured HIP graph
//     replays the upload together with the solve.
//   - A wavefront claims runs of consecutive global tasks; a lane finds the
//     problem of its task by binary search over the task prefix sums and
//     caches that problem's stepping parameters in registers for the walk.
//   - Per-walk arithmetic is the same as the single-problem kernels', task
//     for task, so a problem solved in a batch gives the same bits as the
//     same problem solved alone.
#include <hip/hip_runtime.h>

#include "fk_device.hpp"

namespace fk {

namespace {

constexpr uint32_t kCapFlag = 0x80000000u;
constexpr int kWords = 256;   // 2 KiB of payload per write launch

struct Words {
    uint64_t v[kWords];
};

__global__ void write_words_kernel(uint64_t* dst, const Words w, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = w.v[i];
}

__device__ __forceinline__ uint64_t first_lane_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

struct Pool {
    uint64_t next, end, left;
    bool exhausted;
};

__device__ __forceinline__ uint64_t refill(Pool& pool, const BatchArgs& B, bool active)
{
    const uint64_t idle = __ballot(!active);
    if (idle == 0) return ~0ull;
    const uint32_t n_idle = (uint32_t)__popcll(idle);
    if (pool.next == pool.end && !pool.exhausted) {
        uint64_t want = pool.left / (4ull * B.total_waves);
        if (want < n_idle) want = n_idle;
        if (want > (uint64_t)B.grab) want = (uint64_t)B.grab;
        unsigned long long old = 0ull;
        if (__lane_id() == 0) old = atomicAdd(B.queue, (unsigned long long)want);
        old = first_lane_u64(__shfl(old, 0));
        if (old >= (uint64_t)B.n_tasks) {
            pool.exhausted = true;
        } else {
            pool.next = old;
            pool.end = old + want < (uint64_t)B.n_tasks ? old + want : (uint64_t)B.n_tasks;
            pool.left = (uint64_t)B.n_tasks - pool.end;
        }
    }
    const uint64_t avail = pool.end - pool.next;
    const uint32_t rank = (uint32_t)__popcll(idle & __lanemask_lt());
    uint64_t mine = ~0ull;
    if (!active && rank < avail) mine = pool.next + rank;
    pool.next += (n_idle < avail) ? n_idle : avail;
    return mine;
}

// Largest m with off[m] <= t (off[0] = 0, off[n] = total > t).
__device__ __forceinline__ int find_problem(const int64_t* off, int n, int64_t t)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The start of local task t of a problem: station point (shifted by +-h for
// g_z walks) and the station / path words of the Philox counter.
__device__ __forceinline__ void task_start(const WalkCommon& C, uint64_t t, double x0[3], uint32_t& sctr,
                                           uint32_t& pctr)
{
    const uint64_t q = (C.npair == 2) ? (t >> 1) : t;
    const uint32_t w = (C.npair == 2) ? (uint32_t)(t & 1ull) : 0u;
    const uint64_t s = q / (uint64_t)C.N;
    const uint64_t i = q - s * (uint64_t)C.N;
    const double* st = C.stations + 3 * s;
    x0[0] = st[0];
    x0[1] = st[1];
    x0[2] = st[2];
    if (C.npair == 2) x0[2] = (w == 0) ? st[2] + C.h : st[2] - C.h;
    sctr = (C.npair == 2 && C.pairing == FK_PAIR_INDEPENDENT) ? (uint32_t)(2 * s + w) : (uint32_t)s;
    pctr = (uint32_t)((uint64_t)C.path_offset + i);
}

__device__ __forceinline__ bool inside_open(const WalkCommon& C, const double x[3])
{
    return x[0] > C.lo[0] && x[0] < C.hi[0] && x[1] > C.lo[1] && x[1] < C.hi[1] && x[2] > C.lo[2] &&
           x[2] < C.hi[2];
}

// ---------------------------------------------------------------------------
// FP64 batch walks.  Lane registers hold the problem's parameters; the
// density goes through the problem's descriptor (rho_f64 on device memory).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) batch_f64_kernel(const BatchArgs B)
{
    Pool pool{0ull, 0ull, (uint64_t)B.n_tasks, false};
    bool active = false;
    const BatchDesc* D = nullptr;
    uint64_t task = 0;
    double x0 = 0.0, x1 = 0.0, x2 = 0.0, rp = 0.0, S = 0.0;
    double sdt = 0.0, lo0 = 0, lo1 = 0, lo2 = 0, hi0 = 0, hi1 = 0, hi2 = 0;
    uint32_t n = 0, k = 0, sctr = 0, pctr = 0, key0 = 0, key1 = 0, pid = 0;
    int64_t max_steps = 0;

    for (;;) {
        const uint64_t got = refill(pool, B, active);
        if (got != ~0ull) {
            const int m = find_problem(B.task_off, B.n_problems, (int64_t)got);
            D = B.desc + m;
            const WalkCommon& C = D->c;
            task = got - (uint64_t)B.task_off[m];
            double xs[3];
            task_start(C, task, xs, sctr, pctr);
            if (!inside_open(C, xs)) {
                const double q = __builtin_nan("");
                C.exits[task] = ExitRecord{q, q, q, q};
                C.steps[task] = kCapFlag;
            } else {
                x0 = xs[0];
                x1 = xs[1];
                x2 = xs[2];
                sdt = C.sdt;
                lo0 = C.lo[0]; lo1 = C.lo[1]; lo2 = C.lo[2];
                hi0 = C.hi[0]; hi1 = C.hi[1]; hi2 = C.hi[2];
                key0 = C.key0;
                key1 = C.key1;
                pid = C.problem_id;
                max_steps = C.max_steps;
                rp = rho_f64(D->s64, x0, x1, x2);
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
            const Block bl = philox10(k + b, pctr, sctr, pid, key0, key1);
            normals_f64(bl, z[2 * b], z[2 * b + 1]);
        }
        k += 3;

        bool done = false, capped = false;
        double e0 = 0.0, e1 = 0.0, e2 = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            if (!done) {
                const double y0 = fma(sdt, z[3 * st + 0], x0);
                const double y1 = fma(sdt, z[3 * st + 1], x1);
                const double y2 = fma(sdt, z[3 * st + 2], x2);
                const double rn = rho_f64(D->s64, y0, y1, y2);
                S = S + (rp + rn);
                n += 1;
                if (y0 <= lo0 || y0 >= hi0 || y1 <= lo1 || y1 >= hi1 || y2 <= lo2 || y2 >= hi2) {
                    done = true;
                    a0 = x0; a1 = x1; a2 = x2;
                    e0 = y0; e1 = y1; e2 = y2;
                } else {
                    x0 = y0;
                    x1 = y1;
                    x2 = y2;
                    rp = rn;
                    if ((int64_t)n == max_steps) {
                        done = true;
                        capped = true;
                    }
                }
            }
        }
        if (done) {
            const WalkCommon& C = D->c;
            double e[3] = {e0, e1, e2};
            if (capped) {
                e[0] = e[1] = e[2] = 0.0;
            } else if (C.exit_rule == FK_EXIT_INTERSECT) {
                const double a[3] = {a0, a1, a2};
                const double b[3] = {e0, e1, e2};
                intersect_exit(C.lo, C.hi, a, b, e);
            }
            C.exits[task] = ExitRecord{e[0], e[1], e[2], S};
            C.steps[task] = n | (capped ? kCapFlag : 0u);
            active = false;
        }
    }
}

// ---------------------------------------------------------------------------
// Mixed-precision batch walks (FP32 stream and stepping).
// ---------------------------------------------------------------------------
template <bool KAHAN>
__global__ void __launch_bounds__(256) batch_f32_kernel(const BatchArgs B)
{
    Pool pool{0ull, 0ull, (uint64_t)B.n_tasks, false};
    bool active = false;
    const BatchDesc* D = nullptr;
    uint64_t task = 0;
    float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f, rp = 0.0f;
    double S = 0.0;
    float Sf = 0.0f, Sc = 0.0f;
    float sdt = 0.0f, lo0 = 0, lo1 = 0, lo2 = 0, hi0 = 0, hi1 = 0, hi2 = 0;
    uint32_t n = 0, k = 0, sctr = 0, pctr = 0, key0 = 0, key1 = 0, pid = 0;
    int64_t max_steps = 0;

    for (;;) {
        const uint64_t got = refill(pool, B, active);
        if (got != ~0ull) {
            const int m = find_problem(B.task_off, B.n_problems, (int64_t)got);
            D = B.desc + m;
            const WalkCommon& C = D->c;
            task = got - (uint64_t)B.task_off[m];
            double xs[3];
            task_start(C, task, xs, sctr, pctr);
            if (!inside_open(C, xs)) {
                const double q = __builtin_nan("");
                C.exits[task] = ExitRecord{q, q, q, q};
                C.steps[task] = kCapFlag;
            } else {
                x0 = (float)xs[0];
                x1 = (float)xs[1];
                x2 = (float)xs[2];
                sdt = C.sdt_f;
                lo0 = C.lo_f[0]; lo1 = C.lo_f[1]; lo2 = C.lo_f[2];
                hi0 = C.hi_f[0]; hi1 = C.hi_f[1]; hi2 = C.hi_f[2];
                key0 = C.key0;
                key1 = C.key1;
                pid = C.problem_id;
                max_steps = C.max_steps;
                rp = rho_f32(D->s32, x0, x1, x2);
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
            const Block bl = philox10(k + b, pctr, sctr, pid, key0, key1);
            normals_f32(bl.w0, bl.w1, z[4 * b + 0], z[4 * b + 1]);
            normals_f32(bl.w2, bl.w3, z[4 * b + 2], z[4 * b + 3]);
        }
        k += 3;

        bool done = false, capped = false;
        float ex = 0.0f, ey = 0.0f, ez = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            if (!done) {
                const float y0 = fmaf(sdt, z[3 * st + 0], x0);
                const float y1 = fmaf(sdt, z[3 * st + 1], x1);
                const float y2 = fmaf(sdt, z[3 * st + 2], x2);
                const float rn = rho_f32(D->s32, y0, y1, y2);
                if (KAHAN) {
                    const float y = (rp + rn) - Sc;
                    const float t = Sf + y;
                    Sc = (t - Sf) - y;
                    Sf = t;
                } else {
                    S = S + ((double)rp + (double)rn);
                }
                n += 1;
                if (y0 <= lo0 || y0 >= hi0 || y1 <= lo1 || y1 >= hi1 || y2 <= lo2 || y2 >= hi2) {
                    done = true;
                    ex = x0; ey = x1; ez = x2;
                    fx = y0; fy = y1; fz = y2;
                } else {
                    x0 = y0;
                    x1 = y1;
                    x2 = y2;
                    rp = rn;
                    if ((int64_t)n == max_steps) {
                        done = true;
                        capped = true;
                    }
                }
            }
        }
        if (done) {
            const WalkCommon& C = D->c;
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

// ---------------------------------------------------------------------------
// Batched reduction: the blocks of all problems in one launch; block b finds
// its problem by binary search over the block prefix sums.  Same arithmetic
// and order as the single-problem reduction.
// ---------------------------------------------------------------------------
constexpr int kReduceBlock = 256;

struct Acc {
    double n, mean, m2;
    int64_t sum_steps, max_steps, n_trunc;
};

__device__ __forceinline__ void merge(Acc& a, const Acc& b)
{
    a.sum_steps += b.sum_steps;
    a.max_steps = b.max_steps > a.max_steps ? b.max_steps : a.max_steps;
    a.n_trunc += b.n_trunc;
    if (b.n == 0.0) return;
    if (a.n == 0.0) {
        a.n = b.n;
        a.mean = b.mean;
        a.m2 = b.m2;
        return;
    }
    const double n = a.n + b.n;
    const double d = b.mean - a.mean;
    const double f = b.n / n;
    a.mean = a.mean + d * f;
    a.m2 = a.m2 + b.m2 + d * d * a.n * f;
    a.n = n;
}

__device__ __forceinline__ double batch_sample(const BatchDesc& D, int64_t j, uint32_t steps)
{
    double v = __builtin_nan("");
    if ((steps & kCapFlag) == 0) {
        const ExitRecord r = D.c.exits[j];
        const double e[3] = {r.x, r.y, r.z};
        v = boundary_value(D.bc, D.c.lo, D.c.hi, D.c.G, e) - D.c.w * r.S;
    }
    D.values[j] = v;
    return v;
}

__global__ void __launch_bounds__(kReduceBlock) batch_chunk_kernel(const BatchArgs B)
{
    const int64_t gb = blockIdx.x;
    const int m = find_problem(B.block_off, B.n_problems, gb);
    const BatchDesc& D = B.desc[m];
    const int64_t b = gb - B.block_off[m];
    const int64_t N = D.c.N;
    const int64_t s = b / D.n_chunks;
    const int64_t c = b - s * D.n_chunks;
    const int64_t i0 = c * B.chunk;
    const int64_t i1 = (i0 + B.chunk < N) ? i0 + B.chunk : N;
    const double two_h = 2.0 * D.c.h;

    Acc a{0.0, 0.0, 0.0, 0, 0, 0};
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kReduceBlock) {
        double v;
        uint32_t st;
        bool capped;
        if (D.c.npair == 2) {
            const int64_t j = 2 * (s * N + i);
            const uint32_t sp = D.c.steps[j], sm = D.c.steps[j + 1];
            capped = ((sp | sm) & kCapFlag) != 0;
            st = (sp & ~kCapFlag) + (sm & ~kCapFlag);
            const double up = batch_sample(D, j, sp);
            const double um = batch_sample(D, j + 1, sm);
            v = (up - um) / two_h;
        } else {
            const int64_t j = s * N + i;
            const uint32_t sp = D.c.steps[j];
            capped = (sp & kCapFlag) != 0;
            st = sp & ~kCapFlag;
            v = batch_sample(D, j, sp);
        }
        a.sum_steps += st;
        a.max_steps = (int64_t)st > a.max_steps ? (int64_t)st : a.max_steps;
        if (capped) {
            a.n_trunc += 1;
        } else {
            a.n += 1.0;
            const double d = v - a.mean;
            a.mean += d / a.n;
            a.m2 += d * (v - a.mean);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Acc o;
        o.n = __shfl_down(a.n, off);
        o.mean = __shfl_down(a.mean, off);
        o.m2 = __shfl_down(a.m2, off);
        o.sum_steps = __shfl_down(a.sum_steps, off);
        o.max_steps = __shfl_down(a.max_steps, off);
        o.n_trunc = __shfl_down(a.n_trunc, off);
        if ((int)__lane_id() < off) merge(a, o);
    }
    __shared__ Acc waves[kReduceBlock / 64];
    if (__lane_id() == 0) waves[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc t = waves[0];
        for (int w = 1; w < kReduceBlock / 64; ++w) merge(t, waves[w]);
        Partial& p = D.partials[b];
        p.n = t.n;
        p.mean = t.mean;
        p.m2 = t.m2;
        p.sum_steps = t.sum_steps;
        p.max_steps = t.max_steps;
        p.n_trunc = t.n_trunc;
    }
}

// Thread g handles station g of the concatenated station list (problems in
// order, each problem's stations in order).
__global__ void __launch_bounds__(64) batch_station_kernel(const BatchArgs B, int64_t n_total)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_total) return;
    int lo = 0, hi = B.n_problems;       // last problem with station_base <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (B.desc[mid].station_base <= g) lo = mid;
        else hi = mid;
    }
    const BatchDesc& D = B.desc[lo];
    const int64_t s = g - D.station_base;
    Acc a{0.0, 0.0, 0.0, 0, 0, 0};
    for (int64_t c = 0; c < D.n_chunks; ++c) {
        const Partial& p = D.partials[s * D.n_chunks + c];
        const Acc b{p.n, p.mean, p.m2, p.sum_steps, p.max_steps, p.n_trunc};
        merge(a, b);
    }
    fk_stat o;
    o.n = (int64_t)a.n;
    o.mean = a.n > 0.0 ? a.mean : __builtin_nan("");
    o.var = a.n > 1.0 ? a.m2 / (a.n - 1.0) : __builtin_nan("");
    o.se = a.n > 1.0 ? sqrt(o.var / a.n) : __builtin_nan("");
    o.sum_steps = a.sum_steps;
    o.max_steps = a.max_steps;
    o.n_trunc = a.n_trunc;
    o.mean_steps = (double)a.sum_steps / (double)D.c.N;
    D.out[s] = o;
}

}  // namespace

hipError_t launch_write_words(uint64_t* dst, const uint64_t* host_words, int64_t n_words, hipStream_t stream)
{
    for (int64_t at = 0; at < n_words; at += kWords) {
        Words w;
        const int n = (int)((n_words - at) < kWords ? (n_words - at) : kWords);
        for (int i = 0; i < n; ++i) w.v[i] = host_words[at + i];
        hipLaunchKernelGGL(write_words_kernel, dim3(1), dim3(256), 0, stream, dst + at, w, n);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batch_walk(const BatchArgs& a, const LaunchCfg& cfg, hipStream_t stream)
{
    if (a.precision == FK_F64)
        hipLaunchKernelGGL(batch_f64_kernel, dim3(cfg.grid), dim3(cfg.block), 0, stream, a);
    else if (a.precision == FK_MIXED_KAHAN)
        hipLaunchKernelGGL(batch_f32_kernel<true>, dim3(cfg.grid), dim3(cfg.block), 0, stream, a);
    else
        hipLaunchKernelGGL(batch_f32_kernel<false>, dim3(cfg.grid), dim3(cfg.block), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_batch_reduce(const BatchArgs& a, int64_t n_blocks, int64_t n_station_threads, hipStream_t stream)
{
    hipLaunchKernelGGL(batch_chunk_kernel, dim3((unsigned)n_blocks), dim3(kReduceBlock), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_station_kernel, dim3((unsigned)((n_station_threads + 63) / 64)), dim3(64), 0, stream, a,
                       n_station_threads);
    return hipGetLastError();
}

hipError_t batch_occupancy(int precision, int block, int* blocks_per_cu)
{
    const void* fn = precision == FK_F64 ? (const void*)batch_f64_kernel
                   : precision == FK_MIXED_KAHAN ? (const void*)batch_f32_kernel<true>
                                                 : (const void*)batch_f32_kernel<false>;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, 0);
}

}  // namespace fk
