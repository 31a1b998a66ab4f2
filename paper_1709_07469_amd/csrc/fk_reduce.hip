// fk_reduce.hip -- the per-walk samples u_p = g(x_e) - 2 pi G (dt/2) S from the
// walks' exit records (Dirichlet data read at the exit point, FP64), and the
// per-station statistics of the samples (the sample mean of arXiv:1709.07469
// eq. 11, with the unbiased variance and standard error), with the paired
// central difference of eq. 6 for g_z.
//
// Deterministic two-level reduction: the N samples of a station are cut into
// fixed chunks; a block turns its chunk into a (count, mean, M2) triple with
// per-lane Welford updates, a wavefront shuffle tree and an LDS merge across
// wavefronts, all in a fixed order; a second kernel merges a station's chunk
// triples in chunk order (Chan, Golub & LeVeque pairwise update).
#include <hip/hip_runtime.h>

#include "fk_device.hpp"

namespace fk {

namespace {

constexpr int kReduceBlock = 256;
constexpr uint32_t kCapFlag = 0x80000000u;

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

__device__ __forceinline__ Acc shfl_down_acc(const Acc& a, int off)
{
    Acc b;
    b.n = __shfl_down(a.n, off);
    b.mean = __shfl_down(a.mean, off);
    b.m2 = __shfl_down(a.m2, off);
    b.sum_steps = __shfl_down(a.sum_steps, off);
    b.max_steps = __shfl_down(a.max_steps, off);
    b.n_trunc = __shfl_down(a.n_trunc, off);
    return b;
}

// The sample of walk j, stored for inspection: NaN for a capped walk.
__device__ __forceinline__ double sample(const ReduceArgs& R, int64_t j, uint32_t steps, const DataTables& tb)
{
    double v = __builtin_nan("");
    if ((steps & kCapFlag) == 0) {
        const ExitRecord r = R.exits[j];
        const double e[3] = {r.x, r.y, r.z};
        v = boundary_value(R.bc, R.lo, R.hi, R.G, e, tb) - R.w * r.S;
    }
    R.values[j] = v;
    return v;
}

__global__ void __launch_bounds__(kReduceBlock) chunk_kernel(const ReduceArgs R)
{
    const int64_t b = blockIdx.x;
    const int64_t s = b / R.n_chunks;
    const int64_t c = b - s * R.n_chunks;
    const int64_t i0 = c * R.chunk;
    const int64_t i1 = (i0 + R.chunk < R.N) ? i0 + R.chunk : R.N;

    DataTables tb{nullptr, nullptr};
    if (R.bc.kind == FK_BC_PRISMS) tb = fill_data_tables();     // uniform: every thread takes it

    Acc a{0.0, 0.0, 0.0, 0, 0, 0};
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kReduceBlock) {
        double v;
        uint32_t st;
        bool capped;
        if (R.npair == 2) {
            const int64_t j = 2 * (s * R.N + i);
            const uint32_t sp = R.steps[j], sm = R.steps[j + 1];
            capped = ((sp | sm) & kCapFlag) != 0;
            st = (sp & ~kCapFlag) + (sm & ~kCapFlag);
            const double up = sample(R, j, sp, tb);
            const double um = sample(R, j + 1, sm, tb);
            v = (up - um) / R.two_h;
        } else {
            const int64_t j = s * R.N + i;
            const uint32_t sp = R.steps[j];
            capped = (sp & kCapFlag) != 0;
            st = sp & ~kCapFlag;
            v = sample(R, j, sp, tb);
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
    // wavefront tree: lane l takes lane l + off, off = 32 .. 1
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const Acc o = shfl_down_acc(a, off);
        if ((int)__lane_id() < off) merge(a, o);
    }
    __shared__ Acc waves[kReduceBlock / 64];
    const int wave = threadIdx.x >> 6;
    if (__lane_id() == 0) waves[wave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc t = waves[0];
        for (int w = 1; w < kReduceBlock / 64; ++w) merge(t, waves[w]);
        Partial& p = R.partials[b];
        p.n = t.n;
        p.mean = t.mean;
        p.m2 = t.m2;
        p.sum_steps = t.sum_steps;
        p.max_steps = t.max_steps;
        p.n_trunc = t.n_trunc;
    }
}

__global__ void __launch_bounds__(64) station_kernel(const ReduceArgs R)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= R.n_stations) return;
    Acc a{0.0, 0.0, 0.0, 0, 0, 0};
    for (int64_t c = 0; c < R.n_chunks; ++c) {
        const Partial& p = R.partials[s * R.n_chunks + c];
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
    o.mean_steps = (double)a.sum_steps / (double)R.N;
    R.out[s] = o;
}

}  // namespace

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t stream)
{
    const int64_t blocks = a.n_stations * a.n_chunks;
    hipLaunchKernelGGL(chunk_kernel, dim3((unsigned)blocks), dim3(kReduceBlock), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(station_kernel, dim3((unsigned)((a.n_stations + 63) / 64)), dim3(64), 0, stream, a);
    return hipGetLastError();
}

}  // namespace fk
