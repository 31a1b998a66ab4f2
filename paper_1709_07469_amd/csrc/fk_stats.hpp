// fk_stats.hpp -- the per-station statistics of the walk samples, shared by
// the single-problem and the batched reductions: the sample mean of
// arXiv:1709.07469 eq. 11 with the unbiased variance, accumulated per lane
// by Welford's update and merged by the pairwise update of Chan, Golub &
// LeVeque, always in the same order, so results do not depend on the
// schedule that produced the walks.
//
// A (station, chunk) pair is the unit of the reduction: the samples of one
// station's local paths [c K, min(N, (c+1) K)) (K = the chunk size).  One
// block turns a pair into a Partial -- lane Welford over a strided share,
// a wavefront shuffle tree, then the wavefronts merged in order through
// LDS -- and a station's partials are merged in chunk order at the end.
// The walks' records of a pair are contiguous: walk w of local path i of
// station s is task (s N + i) npair + w, stored at that index minus the
// first task the records hold (record mode: 0; a slice of a bounded
// workspace: the slice's first task).
#pragma once

#include "fk_device.hpp"

namespace fk {

constexpr uint32_t kCapFlag = 0x80000000u;   // bit 31 of a step count: the walk was capped
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

// Where the walks of one (station, chunk) pair are and how their samples
// combine.  rec0 = (s N) npair - first task held, so local path i, walk w
// is at rec0 + i npair + w.
struct PairSpan {
    const ExitRecord* exits;
    const uint32_t* steps;
    double* values;           // per-walk samples written here; null: not kept
    int64_t rec0;
    int64_t i0, i1;
    int32_t npair;
    double two_h;
};

// The sample of one walk, NaN for a capped walk; stored when values are kept.
template <class Data>
__device__ __forceinline__ double pair_sample(const PairSpan& P, int64_t j, uint32_t steps, const Data& data)
{
    double v = __builtin_nan("");
    if ((steps & kCapFlag) == 0) v = data(P.exits[j]);
    if (P.values) P.values[j] = v;
    return v;
}

// Reduces one pair into *out with the whole block (kReduceBlock threads) and
// ORs the anomaly flags of its walks into *status: FK_FLAG_TRUNCATED when a
// walk was capped (max_steps, or a start point not strictly inside),
// FK_FLAG_NONFINITE when an uncapped sample is not finite (a NaN or infinite
// density, position or datum).  data(record) gives a walk's sample
// u_p = g(x_e) - 2 pi G (dt/2) S.
template <class Data>
__device__ __forceinline__ void reduce_pair(const PairSpan& P, const Data& data, Partial* out, uint32_t* status)
{
    Acc a{0.0, 0.0, 0.0, 0, 0, 0};
    uint32_t flags = 0;
    for (int64_t i = P.i0 + threadIdx.x; i < P.i1; i += kReduceBlock) {
        double v;
        uint32_t st;
        bool capped;
        if (P.npair == 2) {
            const int64_t j = P.rec0 + 2 * i;
            const uint32_t sp = P.steps[j], sm = P.steps[j + 1];
            capped = ((sp | sm) & kCapFlag) != 0;
            st = (sp & ~kCapFlag) + (sm & ~kCapFlag);
            const double up = pair_sample(P, j, sp, data);
            const double um = pair_sample(P, j + 1, sm, data);
            v = (up - um) / P.two_h;
        } else {
            const int64_t j = P.rec0 + i;
            const uint32_t sp = P.steps[j];
            capped = (sp & kCapFlag) != 0;
            st = sp & ~kCapFlag;
            v = pair_sample(P, j, sp, data);
        }
        a.sum_steps += st;
        a.max_steps = (int64_t)st > a.max_steps ? (int64_t)st : a.max_steps;
        if (capped) {
            a.n_trunc += 1;
            flags |= FK_FLAG_TRUNCATED;
        } else {
            if (!isfinite(v)) flags |= FK_FLAG_NONFINITE;
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
    __shared__ uint32_t wave_flags[kReduceBlock / 64];
    const int wave = threadIdx.x >> 6;
    const uint32_t wf = (__ballot((flags & FK_FLAG_TRUNCATED) != 0) ? FK_FLAG_TRUNCATED : 0u) |
                        (__ballot((flags & FK_FLAG_NONFINITE) != 0) ? FK_FLAG_NONFINITE : 0u);
    if (__lane_id() == 0) {
        waves[wave] = a;
        wave_flags[wave] = wf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc t = waves[0];
        uint32_t f = wave_flags[0];
        for (int w = 1; w < kReduceBlock / 64; ++w) {
            merge(t, waves[w]);
            f |= wave_flags[w];
        }
        Partial& p = *out;
        p.n = t.n;
        p.mean = t.mean;
        p.m2 = t.m2;
        p.sum_steps = t.sum_steps;
        p.max_steps = t.max_steps;
        p.n_trunc = t.n_trunc;
        if (f) atomicOr(status, f);
    }
}

// A station's partials merged in chunk order into its result.
__device__ __forceinline__ fk_stat finish_station(const Partial* parts, int64_t n_chunks, int64_t N)
{
    Acc a{0.0, 0.0, 0.0, 0, 0, 0};
    for (int64_t c = 0; c < n_chunks; ++c) {
        const Partial& p = parts[c];
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
    o.mean_steps = (double)a.sum_steps / (double)N;
    return o;
}

}  // namespace fk
