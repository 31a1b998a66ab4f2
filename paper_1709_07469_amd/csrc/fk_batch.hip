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

#include "fk_stats.hpp"

namespace fk {

namespace {

constexpr int kWords = 256;   // 2 KiB of payload per write launch

struct Words {
    uint64_t v[kWords];
};

__global__ void write_words_kernel(uint64_t* dst, const Words w, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = w.v[i];
}

// ---------------------------------------------------------------------------
// Batched reduction: the pairs of all problems in one launch; block b takes
// global pair q0 + b and finds its problem by binary search over the pair
// prefix sums.  Same arithmetic and order as the single-problem reduction.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kReduceBlock) batch_chunk_kernel(const BatchArgs B)
{
    const int64_t gq = B.q0 + blockIdx.x;
    const int m = find_problem(B.block_off, B.n_problems, gq);
    const BatchDesc& D = B.desc[m];
    const int64_t b = gq - B.block_off[m];
    const int64_t N = D.c.N;
    const int64_t s = b / D.n_chunks;
    const int64_t c = b - s * D.n_chunks;
    const int64_t i0 = c * B.chunk;
    const int64_t i1 = (i0 + B.chunk < N) ? i0 + B.chunk : N;

    DataTables tb{nullptr, nullptr};
    if (D.bc.kind == FK_BC_PRISMS) tb = fill_data_tables();     // one problem per block: uniform

    const int64_t rec0 = B.task_off[m] + s * N * D.c.npair - B.task0;
    const PairSpan P{B.exits, B.steps, B.values ? B.values + B.task0 : nullptr, rec0, i0, i1, D.c.npair,
                     2.0 * D.c.h};
    auto data = [&](const ExitRecord& r) {
        const double e[3] = {r.x, r.y, r.z};
        return boundary_value(D.bc, D.c.lo, D.c.hi, D.c.G, e, tb) - D.c.w * r.S;
    };
    reduce_pair(P, data, B.partials + gq, B.status);
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
    D.out[s] = finish_station(B.partials + D.block_base + s * D.n_chunks, D.n_chunks, D.c.N);
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

hipError_t launch_batch_chunks(const BatchArgs& a, int64_t n_pairs, hipStream_t stream)
{
    if (n_pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_chunk_kernel, dim3((unsigned)n_pairs), dim3(kReduceBlock), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_batch_stations(const BatchArgs& a, int64_t n_stations, hipStream_t stream)
{
    hipLaunchKernelGGL(batch_station_kernel, dim3((unsigned)((n_stations + 63) / 64)), dim3(64), 0, stream, a,
                       n_stations);
    return hipGetLastError();
}

}  // namespace fk
