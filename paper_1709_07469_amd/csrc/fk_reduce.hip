// fk_reduce.hip -- the per-walk samples u_p = g(x_e) - 2 pi G (dt/2) S from the
// walks' exit records (Dirichlet data read at the exit point, FP64), and the
// per-station statistics of the samples (the sample mean of arXiv:1709.07469
// eq. 11, with the unbiased variance and standard error), with the paired
// central difference of eq. 6 for g_z.
//
// Deterministic two-level reduction (fk_stats.hpp): one block per (station,
// chunk) pair turns the pair's samples into a (count, mean, M2) partial in a
// fixed order; a second kernel merges a station's partials in chunk order.
// A bounded workspace runs the first kernel once per slice of pairs, as soon
// as the slice's walks are done, and the second once at the end.
#include <hip/hip_runtime.h>

#include "fk_stats.hpp"

namespace fk {

namespace {

__global__ void __launch_bounds__(kReduceBlock) chunk_kernel(const ReduceArgs R)
{
    const int64_t q = R.q0 + blockIdx.x;
    const int64_t s = q / R.n_chunks;
    const int64_t c = q - s * R.n_chunks;
    const int64_t i0 = c * R.chunk;
    const int64_t i1 = (i0 + R.chunk < R.N) ? i0 + R.chunk : R.N;

    DataTables tb{nullptr, nullptr};
    if (R.bc.kind == FK_BC_PRISMS) tb = fill_data_tables();     // uniform: every thread takes it

    const PairSpan P{R.exits, R.steps, R.values, s * R.N * R.npair - R.task0, i0, i1, R.npair, R.two_h};
    auto data = [&](const ExitRecord& r) {
        const double e[3] = {r.x, r.y, r.z};
        return boundary_value(R.bc, R.lo, R.hi, R.G, e, tb) - R.w * r.S;
    };
    reduce_pair(P, data, R.partials + q, R.status);
}

__global__ void __launch_bounds__(64) station_kernel(const ReduceArgs R)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= R.n_stations) return;
    R.out[s] = finish_station(R.partials + s * R.n_chunks, R.n_chunks, R.N);
}

}  // namespace

hipError_t launch_reduce(const ReduceArgs& a, int64_t n_pairs, bool finish, hipStream_t stream)
{
    if (n_pairs > 0) {
        hipLaunchKernelGGL(chunk_kernel, dim3((unsigned)n_pairs), dim3(kReduceBlock), 0, stream, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!finish) return hipSuccess;
    hipLaunchKernelGGL(station_kernel, dim3((unsigned)((a.n_stations + 63) / 64)), dim3(64), 0, stream, a);
    return hipGetLastError();
}

}  // namespace fk
