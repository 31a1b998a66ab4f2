// fk_batch.hip -- support of batched solves, where many independent problems
// (density models, station sets, walk counts, parameters) are solved in one
// persistent walk launch with one work-stealing queue (the batch instance of
// the walk kernel template in fk_walk.hip):
//   - problem descriptors live in the workspace; they are written by small
//     kernels that carry the bytes in their arguments, so a captured HIP graph
//     replays the upload together with the solve;
//   - the batched reduction forms every problem's per-walk samples and
//     station statistics in one launch, with the same arithmetic and order as
//     the single-problem reduction.
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

__device__ __forceinline__ double batch_sample(const BatchDesc& D, int64_t j, uint32_t steps, const DataTables& tb)
{
    double v = __builtin_nan("");
    if ((steps & kCapFlag) == 0) {
        const ExitRecord r = D.c.exits[j];
        const double e[3] = {r.x, r.y, r.z};
        v = boundary_value(D.bc, D.c.lo, D.c.hi, D.c.G, e, tb) - D.c.w * r.S;
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

    DataTables tb{nullptr, nullptr};
    if (D.bc.kind == FK_BC_PRISMS) tb = fill_data_tables();     // one problem per block: uniform

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
            const double up = batch_sample(D, j, sp, tb);
            const double um = batch_sample(D, j + 1, sm, tb);
            v = (up - um) / two_h;
        } else {
            const int64_t j = s * N + i;
            const uint32_t sp = D.c.steps[j];
            capped = (sp & kCapFlag) != 0;
            st = sp & ~kCapFlag;
            v = batch_sample(D, j, sp, tb);
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

hipError_t launch_batch_reduce(const BatchArgs& a, int64_t n_blocks, int64_t n_station_threads, hipStream_t stream)
{
    hipLaunchKernelGGL(batch_chunk_kernel, dim3((unsigned)n_blocks), dim3(kReduceBlock), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_station_kernel, dim3((unsigned)((n_station_threads + 63) / 64)), dim3(64), 0, stream, a,
                       n_station_threads);
    return hipGetLastError();
}

}  // namespace fk
