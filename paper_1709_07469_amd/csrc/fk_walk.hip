// fk_walk.hip -- the walk kernels: every lane steps one Brownian walk at a
// time by Euler-Maruyama, accumulates the trapezoid sum of the density along
// it, detects the exit from the box and stores the exit point and the sum
// (arXiv:1709.07469, section 2.3, steps 1-4).  The Dirichlet data is read at
// the stored exit points by the reduction pass, where every lane evaluates it
// at once instead of one lane at a time inside the stepping loop.
//
// One kernel template covers FP64 and mixed precision, single problems and
// batches of problems, and the adjoint replay (which walks the same paths and
// scatters trapezoid weights instead of storing exit records).
//
// Scheduling (gfx950, wave64):
//   - persistent blocks, sized from the occupancy calculator;
//   - a wavefront claims a run of consecutive walks from one global counter
//     (one atomic per claim; the run shrinks as the queue drains so the last
//     walks spread over all wavefronts);
//   - lanes whose walk has ended are refilled at macro-step boundaries, where
//     every active lane is at the start of a Philox block triple: FP64 walks
//     take 2 steps (6 normals = 3 blocks), mixed walks take 4 steps
//     (12 normals = 3 blocks) per macro-step; a wavefront whose walks end
//     often waits for several idle lanes and starts their walks together;
//   - a macro-step in which no walk of the wavefront ends runs its steps as
//     straight-line code;
//   - drain rounds: once the queue is empty, all 64 lanes of a wavefront
//     generate Philox blocks and normals for its remaining live walks into
//     LDS (any lane can compute any walk's block, the generator being
//     counter based), and the live lanes step through that buffer -- up to
//     128 (FP64) or 256 (mixed) steps per round for a lone walk.  The longest
//     walks, which decide when the launch ends, then cost a move and a test
//     per step instead of a full random-number generation each, and partly
//     idle wavefronts keep all lanes busy generating;
//   - a walk's record is written to its own slot (task index), so the result
//     does not depend on which lane or wavefront ran it, nor on the mode.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fk_stats.hpp"

namespace fk {

namespace {

constexpr int kMaxWaves = 4;        // 256 threads per block at most

// The task queue can be split into contiguous stripes with a claim counter
// each (the queue slot of a workspace holds kMaxStripes counters).  Block b
// starts on stripe b mod stripes -- consecutive blocks are placed on the 8
// XCDs in turn, so with 8 stripes each XCD walks its own contiguous range of
// tasks and, in a batch of problems with separate sources, its wavefronts
// hold walks of one problem at a time (the problem-uniform fast path applies,
// and an XCD's L2 serves one problem's grid) -- and a wavefront whose stripe
// runs out takes the next.  The launch settings choose the count: 8 for
// batches of separate sources, 1 for other launches (their lanes share a
// source anyway, and stripes that end on long walks lengthen the drain).
constexpr uint32_t kMaxStripes = 32;

__global__ void zero_queue_kernel(unsigned long long* q, uint32_t* status, uint32_t flags)
{
    if (threadIdx.x < kMaxStripes) q[threadIdx.x] = 0ull;
    if (status && threadIdx.x == 0) *status = flags;
}

__device__ __forceinline__ uint64_t first_lane_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-uniform claim state over the striped task queue.
struct Queue {
    unsigned long long* counter;   // one claim counter per stripe
    uint64_t n_tasks;
    uint32_t grab;
    uint32_t total_waves;
    uint32_t stripes;              // 1 .. kMaxStripes
    uint32_t refill_cost;          // 128 R of the refill rule below
};

struct Pool {
    uint64_t next, end, left;
    bool exhausted;
    uint32_t stripe, tried;
    uint64_t rounds;    // refill calls (one per macro-step or drain round)
    int64_t started;    // walks started after the first fill
};

__device__ __forceinline__ Pool start_pool(const Queue& Q)
{
    return Pool{0ull, 0ull, Q.n_tasks, false, blockIdx.x % Q.stripes, 0u, 0ull, -64};
}

// Starting walks costs the wavefront about half a macro-step however many
// lanes take one (the set-up code runs once for all of them), while a lane
// left idle loses its share of every macro-step.  With walks ending at a rate
// of lambda per macro-step, waiting for k idle lanes costs (k - 1)/(128 lambda)
// + R/k macro-steps per walk (R = 1/2 the set-up), least for the smallest k
// with k (k + 1) >= 128 R lambda.  lambda is the wavefront's own count of
// walks started over its macro-steps so far: long walks (rare ends) refill
// every lane at once, short ones wait for several.  The launch settings give
// 128 R (default 64: R = 1/2; R = 1/4 measured the same).

// Refills idle lanes from the wavefront's claimed run, claiming a new run
// from its stripe when it is empty (and moving to the next stripe when that
// one is used up).  Returns the task of this lane if it was idle and got
// one, else ~0.  Called by the whole wavefront once per macro-step.
__device__ __forceinline__ uint64_t refill(Pool& pool, const Queue& Q, bool active)
{
    pool.rounds += 1;
    const uint64_t idle = __ballot(!active);
    if (idle == 0) return ~0ull;
    const uint32_t n_idle = (uint32_t)__popcll(idle);
    // an all-idle wavefront always passes: started <= 64 rounds
    if (!pool.exhausted && pool.started > 0 &&
        (uint64_t)n_idle * (n_idle + 1) * pool.rounds < (uint64_t)Q.refill_cost * (uint64_t)pool.started)
        return ~0ull;
    const uint32_t stripes = Q.stripes;
    // each pass claims a run or uses up one stripe: stripes passes at most
    for (uint32_t pass = 0; pass < stripes && pool.next == pool.end && !pool.exhausted; ++pass) {
        const uint64_t lo = Q.n_tasks * pool.stripe / stripes;
        const uint64_t hi = Q.n_tasks * (pool.stripe + 1) / stripes;
        uint64_t want = pool.left / (4ull * Q.total_waves);
        if (want < n_idle) want = n_idle;
        if (want > (uint64_t)Q.grab) want = (uint64_t)Q.grab;
        unsigned long long old = 0ull;
        if (__lane_id() == 0) old = atomicAdd(Q.counter + pool.stripe, (unsigned long long)want);
        old = first_lane_u64(__shfl(old, 0));
        if (old < hi - lo) {
            pool.next = lo + old;
            pool.end = lo + old + want < hi ? lo + old + want : hi;
            pool.left = (hi - pool.end) * stripes;   // the whole queue's, estimated
        } else if (stripes == 1 || ++pool.tried == stripes) {
            pool.exhausted = true;
        } else {
            pool.stripe = (pool.stripe + 1) % stripes;
        }
    }
    const uint64_t avail = pool.end - pool.next;
    const uint32_t rank = (uint32_t)__popcll(idle & __lanemask_lt());
    uint64_t mine = ~0ull;
    if (!active && rank < avail) mine = pool.next + rank;
    const uint64_t taken = (n_idle < avail) ? n_idle : avail;
    pool.next += taken;
    pool.started += (int64_t)taken;
    return mine;
}

struct TaskInfo {
    double x0[3];
    uint64_t s;      // station
    uint32_t w;      // 0: the walk from x0 (+h e_z for g_z), 1: from x0 - h e_z
    uint32_t sctr;   // station word of the Philox counter
    uint32_t pctr;   // path word
};

// Local task t of a problem: (station s, local path i, walk w) with
// t = (s * N + i) * npair + w.
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

__device__ __forceinline__ bool strictly_inside(const WalkCommon& C, const double x[3])
{
    if (C.domain == FK_DOMAIN_BALL) return dist2(x[0], x[1], x[2], C.ctr[0], C.ctr[1], C.ctr[2]) < C.r2;
    return (x[0] > C.lo[0]) & (x[0] < C.hi[0]) & (x[1] > C.lo[1]) & (x[1] < C.hi[1]) & (x[2] > C.lo[2]) &
           (x[2] < C.hi[2]);
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

// The adjoint's signed trapezoid weights are gathered in a block-shared LDS
// table before they reach the global int64 counts.  A walk crosses a voxel
// face on most steps of a fine grid, and every global atomic on device memory
// is performed at the memory side (hundreds of cycles, limited in flight), so
// the walks of a block -- which start from the same stations and crowd the
// same voxels -- first add into the table.  Each slot is one 32-bit word,
// (index + 1) << 11 | 11-bit signed count, updated by compare-and-swap only,
// so it is atomic across the block's wavefronts; a different index evicts the
// slot's entry to the global counts, a count that would leave +-1024 goes
// there as well, and so does every weight whose index + 1 needs more than 21
// bits or whose size is 1024 or more.  The table is flushed when the block's
// walks are done.  Integer sums in any order: the counts are exact and the
// same as without the table.
constexpr int kAdjTableBits = 13;
constexpr int kAdjSlots = 1 << kAdjTableBits;    // 32 KiB of LDS per block
constexpr int kAdjCountBits = 11;
constexpr uint32_t kAdjKeyLimit = 1u << (32 - kAdjCountBits);
constexpr int64_t kAdjBound = 1ll << (kAdjCountBits - 1);

__device__ __forceinline__ void global_add(int64_t* counts, int64_t idx, int64_t w)
{
    atomicAdd(reinterpret_cast<unsigned long long*>(counts + idx), (unsigned long long)w);
}

// The key (index + 1, 0 = empty) and the signed count of a table word.
__device__ __forceinline__ uint32_t adj_key(uint32_t e) { return e >> kAdjCountBits; }
__device__ __forceinline__ int64_t adj_count(uint32_t e)
{
    return (int64_t)((int32_t)(e << (32 - kAdjCountBits)) >> (32 - kAdjCountBits));
}

__device__ __forceinline__ void adj_emit(uint32_t* tab, int64_t* counts, int64_t idx, int64_t w)
{
    if ((uint64_t)idx + 1 >= kAdjKeyLimit || w >= kAdjBound || w <= -kAdjBound) {
        global_add(counts, idx, w);
        return;
    }
    const uint32_t k1 = (uint32_t)idx + 1u;
    const uint32_t slot = ((uint32_t)idx * 2654435761u) >> (32 - kAdjTableBits);
    uint32_t cur = __hip_atomic_load(&tab[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        const uint32_t ck = adj_key(cur);
        const int64_t cc = adj_count(cur);
        int64_t keep = w, out_idx = -1, out_c = 0;   // out: what leaves the table if this swap wins
        if (ck == k1) {
            keep = cc + w;
            if (keep >= kAdjBound || keep <= -kAdjBound) {
                out_idx = idx;
                out_c = keep;
                keep = 0;
            }
        } else if (ck != 0) {
            out_idx = (int64_t)ck - 1;
            out_c = cc;
        }
        const uint32_t want = (k1 << kAdjCountBits) | ((uint32_t)keep & ((1u << kAdjCountBits) - 1u));
        const uint32_t prev = atomicCAS(&tab[slot], cur, want);
        if (prev == cur) {
            if (out_c != 0) global_add(counts, out_idx, out_c);
            return;
        }
        cur = prev;
    }
}

// Dense station tables: when a grid has at most kDenseVoxels voxels, each
// block of the adjoint works on one station at a time and adds its walks'
// weights into a plain int32 count per voxel in LDS (128 KiB: an LDS atomic
// add, no key, no eviction), flushed to the global counts when the block
// moves on to another station.  A weight of 2^19 or more goes straight to
// the global counts; a count that reaches +-2^30 is taken out of the table by
// an atomic exchange and moved there too (concurrent adds of the block's
// 1024 threads, each below 2^19, cannot carry it past 2^31 meanwhile).
constexpr int kDenseVoxels = (int)kAdjDenseVoxels;
constexpr int64_t kDenseDirect = 1ll << 19;
constexpr int64_t kDenseLimit = 1ll << 30;
static_assert(kAdjDenseBlock * kDenseDirect + kDenseLimit < (1ll << 31), "a dense count must stay within int32");

__device__ __forceinline__ void dense_emit(int* tab, int64_t* counts, int64_t row, int64_t v, int64_t w)
{
    if (w >= kDenseDirect || w <= -kDenseDirect) {
        global_add(counts, row + v, w);
        return;
    }
    const int old = atomicAdd(&tab[v], (int)w);
    const int64_t now = (int64_t)old + w;
    if (now >= kDenseLimit || now <= -kDenseLimit) global_add(counts, row + v, (int64_t)atomicExch(&tab[v], 0));
}

// Run-length coalesced scatter of one walk's signed trapezoid weights, into
// the block's hashed table or (DENSE) its dense station table.
template <bool DENSE>
struct Scatter {
    int64_t* counts;            // the problem's counts
    void* tab;                  // the block's table
    int64_t row;                // station offset into counts
    int64_t v;                  // pending voxel (-1: none)
    int64_t c;                  // pending weight
    int64_t sign;
    __device__ __forceinline__ void flush()
    {
        if (v >= 0 && c != 0) {
            if constexpr (DENSE)
                dense_emit(static_cast<int*>(tab), counts, row, v, c);
            else
                adj_emit(static_cast<uint32_t*>(tab), counts, row + v, c);
        }
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

// ---------------------------------------------------------------------------
// Precision traits.
// ---------------------------------------------------------------------------
template <bool F64>
struct Prec;

// x, from here on held in a vector register (an empty asm with a vector
// operand: no instruction is emitted)
template <class T>
__device__ __forceinline__ T in_vgpr(T x)
{
    asm("" : "+v"(x));
    return x;
}

template <>
struct Prec<true> {
    using T = double;
    using Src = SourceF64;
    static constexpr int kNormals = 2;   // per Philox block
    static constexpr int kMacro = 2;     // steps per 3 blocks
    __device__ static void normals(const Block& b, T* z, const BmTables* t) { normals_f64(b, *t, z[0], z[1]); }
    __device__ static T fmat(T a, T b, T c) { return fma(a, b, c); }
    template <bool LEVELS>
    __device__ static T rho(const Src& s, T x, T y, T z) { return rho_f64<LEVELS>(s, x, y, z); }
    template <bool LEVELS>
    __device__ static T grid_in(const Src& s, T x, T y, T z) { return grid_in_f64<LEVELS>(s, x, y, z); }
    template <bool LEVELS>
    __device__ static GridProbe grid_fetch(const Src& s, T x, T y, T z) { return grid_fetch_f64<LEVELS>(s, x, y, z); }
    template <bool LEVELS>
    __device__ static T grid_keep(const Src& s, const GridProbe& p) { return grid_keep_f64<LEVELS>(s, p); }
    __device__ static T bodies(const Src& s, T g, T x, T y, T z, int j0 = 0) { return bodies_f64(s, g, x, y, z, j0); }
    __device__ static int64_t voxel(const Src& s, T x, T y, T z) { return voxel_f64(s, x, y, z); }
    __device__ static T lo(const WalkCommon& C, int c) { return C.lo[c]; }
    __device__ static T hi(const WalkCommon& C, int c) { return C.hi[c]; }
    __device__ static T ctr(const WalkCommon& C, int c) { return C.ctr[c]; }
    __device__ static T r2(const WalkCommon& C) { return C.r2; }
    __device__ static T radius(const WalkCommon& C) { return C.R; }
    __device__ static T dt(const WalkCommon& C) { return C.dt; }
    __device__ static T delta(const WalkCommon& C) { return C.delta; }
    __device__ static T deep2(const WalkCommon& C) { return C.deep2; }
    __device__ static T uniform(const Block& b, int j)
    {
        const uint32_t hi = j ? b.w3 : b.w1, lo = j ? b.w2 : b.w0;
        return uniform53(hi, lo);
    }
    __device__ static T sdt(const WalkCommon& C) { return C.sdt; }
};

template <>
struct Prec<false> {
    using T = float;
    using Src = SourceF32;
    static constexpr int kNormals = 4;
    static constexpr int kMacro = 4;
    __device__ static void normals(const Block& b, T* z, const BmTables*)
    {
        normals_f32(b.w0, b.w1, z[0], z[1]);
        normals_f32(b.w2, b.w3, z[2], z[3]);
    }
    __device__ static T fmat(T a, T b, T c) { return fmaf(a, b, c); }
    template <bool LEVELS>
    __device__ static T rho(const Src& s, T x, T y, T z) { return rho_f32<LEVELS>(s, x, y, z); }
    template <bool LEVELS>
    __device__ static T grid_in(const Src& s, T x, T y, T z) { return grid_in_f32<LEVELS>(s, x, y, z); }
    template <bool LEVELS>
    __device__ static GridProbe grid_fetch(const Src& s, T x, T y, T z) { return grid_fetch_f32<LEVELS>(s, x, y, z); }
    template <bool LEVELS>
    __device__ static T grid_keep(const Src& s, const GridProbe& p) { return grid_keep_f32<LEVELS>(s, p); }
    __device__ static T bodies(const Src& s, T g, T x, T y, T z, int j0 = 0) { return bodies_f32(s, g, x, y, z, j0); }
    __device__ static int64_t voxel(const Src& s, T x, T y, T z) { return voxel_f32(s, x, y, z); }
    __device__ static T lo(const WalkCommon& C, int c) { return C.lo_f[c]; }
    __device__ static T hi(const WalkCommon& C, int c) { return C.hi_f[c]; }
    __device__ static T ctr(const WalkCommon& C, int c) { return C.ctr_f[c]; }
    __device__ static T r2(const WalkCommon& C) { return C.r2_f; }
    __device__ static T radius(const WalkCommon& C) { return C.R_f; }
    __device__ static T dt(const WalkCommon& C) { return C.dt_f; }
    __device__ static T delta(const WalkCommon& C) { return C.delta_f; }
    __device__ static T deep2(const WalkCommon& C) { return C.deep2_f; }
    __device__ static T uniform(const Block& b, int j)
    {
        const uint32_t w = j == 0 ? b.w0 : j == 1 ? b.w1 : j == 2 ? b.w2 : b.w3;
        return uniform24(w);
    }
    __device__ static T sdt(const WalkCommon& C) { return C.sdt_f; }
};

template <bool F64>
struct SourceOf;
template <>
struct SourceOf<true> {
    __device__ static const SourceF64& get(const BatchDesc& D) { return D.s64; }
};
template <>
struct SourceOf<false> {
    __device__ static const SourceF32& get(const BatchDesc& D) { return D.s32; }
};

// The batch's shared source, in the kernel arguments.
template <bool F64>
__device__ __forceinline__ const typename std::conditional<F64, SourceF64, SourceF32>::type& shared_source(
    const BatchArgs& A)
{
    if constexpr (F64)
        return A.src64;
    else
        return A.src32;
}

// The lanes' common source when every live lane of the wavefront points at
// the same one (a wavefront claims consecutive walks, so it almost always
// works on one problem), re-addressed through the constant address space so
// that its fields load with scalar instructions into scalar registers; null
// when the lanes' problems differ.  Called with only the live lanes active.
template <class Src>
__device__ __forceinline__ const Src* wave_uniform(const Src* p)
{
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const uint64_t f = ((uint64_t)hi << 32) | lo;
    if (!__all(a == f)) return nullptr;
    return (const Src*)(const __attribute__((address_space(4))) Src*)f;
}

// Stepping parameters of the problem a lane is walking.  In single-problem
// launches they are the same for every lane; in a batch each lane loads its
// problem's at the start of a walk.
template <bool F64>
struct LaneProblem {
    using T = typename Prec<F64>::T;
    const WalkCommon* C;
    const typename Prec<F64>::Src* src;
    T sdt;
    // box domain: the bounds; ball domain: (lo0, lo1, lo2) = centre,
    // hi0 = squared radius, hi1 = radius, hi2 = (R - delta)^2 (the two never
    // coexist, so they share registers)
    T lo0, lo1, lo2, hi0, hi1, hi2;
    T dt, delta;               // Brownian-bridge test
    bool ball, bridge;
    uint32_t key0, key1, pid;
    int64_t max_steps;

    // keys = false leaves key0 and key1 as they are (a batch whose problems
    // share the generator key holds it in scalar registers, set once).
    __device__ __forceinline__ void load(const WalkCommon& c, const typename Prec<F64>::Src& s, bool keys = true)
    {
        C = &c;
        src = &s;
        sdt = Prec<F64>::sdt(c);
        lo0 = Prec<F64>::lo(c, 0);
        lo1 = Prec<F64>::lo(c, 1);
        lo2 = Prec<F64>::lo(c, 2);
        hi0 = Prec<F64>::hi(c, 0);
        hi1 = Prec<F64>::hi(c, 1);
        hi2 = Prec<F64>::hi(c, 2);
        ball = c.domain == FK_DOMAIN_BALL;
        bridge = c.exit_rule == FK_EXIT_BRIDGE;
        dt = Prec<F64>::dt(c);
        delta = Prec<F64>::delta(c);
        if (ball) {
            lo0 = Prec<F64>::ctr(c, 0);
            lo1 = Prec<F64>::ctr(c, 1);
            lo2 = Prec<F64>::ctr(c, 2);
            hi0 = Prec<F64>::r2(c);
            hi1 = Prec<F64>::radius(c);
            hi2 = Prec<F64>::deep2(c);
        }
        if (keys) {
            key0 = c.key0;
            key1 = c.key1;
        }
        pid = c.problem_id;
        max_steps = c.max_steps;
    }
};

// The stepping loop a kernel instance is built for.  Bits 0-1: 0 = the box
// domain's loop with the step-end exit test only; 1 = with the ball domain's
// exit test; 2 = also with the Brownian-bridge test.  Bit 2: the density
// source has a voxel grid, whose values each macro-step loads ahead; bit 3
// (with bit 2): the grids are given by levels (an index grid and its
// densities).  A launch uses the least general loop its problems need.
constexpr int kLoopGrid = 4;
constexpr int kLoopLevels = 8;
constexpr int loop_exit(int loop) { return loop & 3; }
constexpr bool loop_grid(int loop) { return (loop & kLoopGrid) != 0; }
constexpr bool loop_levels(int loop) { return (loop & kLoopLevels) != 0; }

// One lane's walk.
template <bool F64, bool KAHAN, bool ADJ, int LOOP, bool DENSE = false>
struct Walker {
    using T = typename Prec<F64>::T;
    uint64_t rec;    // the walk's record slot (its task minus the launch's first task)
    ExitRecord* exits;
    uint32_t* steps_out;
    T x0, x1, x2, rp;
    double S;        // trapezoid sum (FP64 accumulation)
    float Sf, Sc;    // Kahan sum and compensation
    uint32_t n, k, sctr, pctr;
    bool active;
    bool deep;       // the current point lies delta inside every face (bridge test)
    Scatter<DENSE> sc;

    // delta inside every face (ball: |x - c|^2 <= (R - delta)^2)
    __device__ __forceinline__ static bool deep_inside(const LaneProblem<F64>& P, T y0, T y1, T y2, T d2)
    {
        if (P.ball) return d2 <= P.hi2;
        return y0 - P.lo0 >= P.delta && P.hi0 - y0 >= P.delta && y1 - P.lo1 >= P.delta && P.hi1 - y1 >= P.delta &&
               y2 - P.lo2 >= P.delta && P.hi2 - y2 >= P.delta;
    }

    // Brownian-bridge test of step m from (x0, x1, x2) to y (both inside):
    // returns the face the walk stopped at (0..5; 6 = the sphere) or -1.
    __device__ __forceinline__ int bridge_stop(const LaneProblem<F64>& P, uint32_t m, T x0, T x1, T x2, T y0, T y1,
                                               T y2) const
    {
        constexpr int q = Prec<F64>::kNormals;
        const Block b = philox10(0x80000000u + m / q, pctr, sctr, P.pid, P.key0, P.key1);
        const T U = Prec<F64>::uniform(b, (int)(m % q));
        if (P.ball) {
            const T a = P.hi1 - sqrt(dist2(x0, x1, x2, P.lo0, P.lo1, P.lo2));
            const T c = P.hi1 - sqrt(dist2(y0, y1, y2, P.lo0, P.lo1, P.lo2));
            const T p = exp(T(-2) * a * c / P.dt);
            return U <= p ? 6 : -1;
        }
        const T lo[3] = {P.lo0, P.lo1, P.lo2}, hi[3] = {P.hi0, P.hi1, P.hi2};
        const T x[3] = {x0, x1, x2}, y[3] = {y0, y1, y2};
        T keep = T(1), pbest = T(-1);
        int fbest = 0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int j = f >> 1;
            const T a = (f & 1) ? hi[j] - x[j] : x[j] - lo[j];
            const T c = (f & 1) ? hi[j] - y[j] : y[j] - lo[j];
            const T p = exp(T(-2) * a * c / P.dt);
            keep *= T(1) - p;
            if (p > pbest) {
                pbest = p;
                fbest = f;
            }
        }
        return U <= T(1) - keep ? fbest : -1;
    }

    // Turns the normals of the next MACRO steps into the points those steps
    // reach (as if none ended the walk) and, with a grid, loads the grid
    // density at each, all loads issued before the first is used.  Points past
    // the walk's end are never used.
    template <int MACRO = Prec<F64>::kMacro>
    __device__ __forceinline__ void advance(const LaneProblem<F64>& P, const typename Prec<F64>::Src& src, T* z,
                                            T* g) const
    {
        T p0 = x0, p1 = x1, p2 = x2;
#pragma unroll
        for (int s = 0; s < MACRO; ++s) {
            p0 = Prec<F64>::fmat(P.sdt, z[3 * s], p0);
            p1 = Prec<F64>::fmat(P.sdt, z[3 * s + 1], p1);
            p2 = Prec<F64>::fmat(P.sdt, z[3 * s + 2], p2);
            z[3 * s] = p0;
            z[3 * s + 1] = p1;
            z[3 * s + 2] = p2;
            g[s] = T(0);
        }
        // A launch takes the grid loop when any of its problems has a grid,
        // but a batch may mix sources with and without one: the lane's own
        // source is checked, once for all the macro-step's loads.
        if (!ADJ && loop_grid(LOOP) && src.has_grid) {
            GridProbe pr[MACRO];
#pragma unroll
            for (int s = 0; s < MACRO; ++s)
                pr[s] = Prec<F64>::template grid_fetch<loop_levels(LOOP)>(src, z[3 * s], z[3 * s + 1], z[3 * s + 2]);
#pragma unroll
            for (int s = 0; s < MACRO; ++s) g[s] = Prec<F64>::template grid_keep<loop_levels(LOOP)>(src, pr[s]);
        }
    }

    // Adds one trapezoid term rho(a) + rho(b) to the walk's sum.
    __device__ __forceinline__ void add_trapezoid(T a, T b)
    {
        if (F64) {
            S = S + (double)(a + b);
        } else if (KAHAN) {
            const float t0 = (float)(a + b) - Sc;
            const float t = Sf + t0;
            Sc = (t - Sf) - t0;
            Sf = t;
        } else {
            S = S + ((double)a + (double)b);
        }
    }

    // Whether y has left the domain (on the boundary counts as left); d2 is
    // the squared distance from the ball's centre (ball domains only).
    __device__ __forceinline__ static bool leaves(const LaneProblem<F64>& P, T y0, T y1, T y2, T& d2)
    {
        if (loop_exit(LOOP) >= 1 && P.ball) {
            d2 = dist2(y0, y1, y2, P.lo0, P.lo1, P.lo2);
            return d2 >= P.hi0;
        }
        d2 = T(0);
        return (y0 <= P.lo0) | (y0 >= P.hi0) | (y1 <= P.lo1) | (y1 >= P.hi1) | (y2 <= P.lo2) | (y2 >= P.hi2);
    }

    // The macro-step's Euler-Maruyama steps through the points y (advance),
    // each with its density and exit test, up to the first that ends the
    // walk.  Returns true when the walk ended, at step at, with how = 0: it
    // left the domain; how = 1: it reached max_steps; how = 2 + f: the bridge
    // test stopped it at face f.  The walk's point x and density rp move to
    // the macro-step's last point only when the walk goes on, so a walk that
    // ended keeps them at the macro-step's start (finish recovers the step's
    // two ends from x and y).  g holds the grid density at each point.
    // The source's density at y: the grid value g, then the analytic bodies
    // in their order.  With HELD the first prism comes from hq (registers;
    // lo = +inf when the source has none) and the rest from the source.
    template <bool HELD>
    __device__ __forceinline__ static T density(const typename Prec<F64>::Src& src, const T* hq, T g, T y0, T y1, T y2)
    {
        if constexpr (HELD) {
            const bool in = (y0 >= hq[0]) & (y0 < hq[3]) & (y1 >= hq[1]) & (y1 < hq[4]) & (y2 >= hq[2]) & (y2 < hq[5]);
            return Prec<F64>::bodies(src, in ? g + hq[6] : g, y0, y1, y2, 1);
        } else {
            return Prec<F64>::bodies(src, g, y0, y1, y2);
        }
    }

    template <bool HELD = false, int MACRO = Prec<F64>::kMacro>
    __device__ __forceinline__ bool steps(const LaneProblem<F64>& P, const typename Prec<F64>::Src& src, const T* y,
                                          const T* g, int& at, int& how, const T* hq = nullptr)
    {
        bool done = false;
        T r = rp;   // the density at the step's start
        if constexpr (!ADJ && loop_exit(LOOP) < 2) {
            // Densities and exit tests of all the points first.  When no
            // walk of the wavefront ends in this macro-step -- nearly always
            // for walks of hundreds of steps -- the steps run as straight-line
            // code, without the per-step masking of walks that ended.
            T rn[MACRO];
            bool out[MACRO];
            bool end = (int64_t)n + MACRO >= P.max_steps;
#pragma unroll
            for (int s = 0; s < MACRO; ++s) {
                T d2;
                rn[s] = density<HELD>(src, hq, g[s], y[3 * s], y[3 * s + 1], y[3 * s + 2]);
                out[s] = leaves(P, y[3 * s], y[3 * s + 1], y[3 * s + 2], d2);
                end = end | out[s];
            }
            if (__ballot(end) == 0ull) {
#pragma unroll
                for (int s = 0; s < MACRO; ++s) {
                    add_trapezoid(r, rn[s]);
                    r = rn[s];
                }
                n += MACRO;
            } else {
#pragma unroll
                for (int s = 0; s < MACRO; ++s) {
                    if (done) break;
                    add_trapezoid(r, rn[s]);
                    n += 1;
                    if (out[s]) {
                        how = 0;
                        at = s;
                        done = true;
                    } else if ((int64_t)n == P.max_steps) {
                        how = 1;
                        at = s;
                        done = true;
                    }
                    r = rn[s];
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < MACRO; ++s) {
                if (done) break;
                const T y0 = y[3 * s], y1 = y[3 * s + 1], y2 = y[3 * s + 2];
                T rn = T(0);
                if (!ADJ) {
                    rn = density<HELD>(src, hq, g[s], y0, y1, y2);
                    add_trapezoid(r, rn);
                }
                n += 1;
                T d2;
                const bool out = leaves(P, y0, y1, y2, d2);
                int stop = -1;
                if (loop_exit(LOOP) == 2 && P.bridge && !out) {
                    const bool deep_y = deep_inside(P, y0, y1, y2, d2);
                    if (!(deep && deep_y)) {
                        const T p0 = s ? y[3 * s - 3] : x0, p1 = s ? y[3 * s - 2] : x1, p2 = s ? y[3 * s - 1] : x2;
                        stop = bridge_stop(P, n - 1, p0, p1, p2, y0, y1, y2);
                    }
                    deep = deep_y;
                }
                if (ADJ) sc.add(Prec<F64>::voxel(src, y0, y1, y2), (out || stop >= 0) ? 1 : 2);
                if (out || stop >= 0) {
                    how = out ? 0 : 2 + stop;
                    at = s;
                    done = true;
                } else if ((int64_t)n == P.max_steps) {
                    how = 1;
                    at = s;
                    done = true;
                }
                r = rn;
            }
        }
        if (!done) {
            x0 = y[3 * MACRO - 3];
            x1 = y[3 * MACRO - 2];
            x2 = y[3 * MACRO - 1];
            rp = r;
        }
        return done;
    }

    // Stores the walk's exit record (or flushes its scatter) and frees the
    // lane.  y holds the macro-step's points (advance) and the walk ended at
    // step at of them: the end point is y[at], the last point inside the one
    // before it (x for the first step).
    template <int MACRO = Prec<F64>::kMacro>
    __device__ __forceinline__ void finish(const LaneProblem<F64>& P, const T* y, int at, int how)
    {
        T a0 = x0, a1 = x1, a2 = x2, e0 = y[0], e1 = y[1], e2 = y[2];
#pragma unroll
        for (int s = 1; s < MACRO; ++s) {
            if (at == s) {
                a0 = y[3 * s - 3];
                a1 = y[3 * s - 2];
                a2 = y[3 * s - 1];
                e0 = y[3 * s];
                e1 = y[3 * s + 1];
                e2 = y[3 * s + 2];
            }
        }
        const bool capped = how == 1;
        if (ADJ) {
            sc.flush();
        } else {
            const WalkCommon& C = *P.C;
            double e[3] = {0.0, 0.0, 0.0};
            if (loop_exit(LOOP) == 2 && how >= 2) {
                // bridge stop: the step's end projected onto the face
                e[0] = (double)e0;
                e[1] = (double)e1;
                e[2] = (double)e2;
                const int f = how - 2;
                if (f == 6) {
                    const double r = sqrt(dist2(e[0], e[1], e[2], C.ctr[0], C.ctr[1], C.ctr[2]));
#pragma unroll
                    for (int j = 0; j < 3; ++j) e[j] = C.ctr[j] + C.R * ((e[j] - C.ctr[j]) / r);
                } else {
                    e[f >> 1] = (f & 1) ? C.hi[f >> 1] : C.lo[f >> 1];
                }
            } else if (!capped) {
                e[0] = (double)e0;
                e[1] = (double)e1;
                e[2] = (double)e2;
                if (C.exit_rule != FK_EXIT_OVERSHOOT) {
                    const double a[3] = {(double)a0, (double)a1, (double)a2};
                    const double b[3] = {(double)e0, (double)e1, (double)e2};
                    if (C.domain == FK_DOMAIN_BALL)
                        intersect_ball(C.ctr, C.r2, a, b, e);
                    else
                        intersect_exit(C.lo, C.hi, a, b, e);
                }
            }
            const double sum = (!F64 && KAHAN) ? ((double)Sf - (double)Sc) : S;
            exits[rec] = ExitRecord{e[0], e[1], e[2], sum};
            steps_out[rec] = n | (capped ? kCapFlag : 0u);
        }
        active = false;
    }
};

// ---------------------------------------------------------------------------
// The kernel body.
// ---------------------------------------------------------------------------
// DENSE (adjoint only): blocks of kAdjDenseBlock threads with a dense
// per-station table,
// working through the stations one at a time (each station's tasks have
// their own claim counter; a block starts on station blockIdx mod S and,
// when its station's tasks are all claimed and its walks done, flushes the
// table and moves on to the next station with unclaimed tasks).
// UKEY (batches): every problem has the same generator key, passed in the
// launch arguments, so the Philox key schedule is scalar work.
template <bool F64, bool KAHAN, bool ADJ, bool BATCH, int LOOP, bool SHARED, bool DENSE, bool UKEY, class Args>
__device__ __forceinline__ void walk_body(const Args& A)
{
    using T = typename Prec<F64>::T;
    constexpr int NPB = Prec<F64>::kNormals;
    constexpr int MACRO = Prec<F64>::kMacro;
    // Drain rounds need a buffer per wavefront; the dense instance runs
    // without them (its LDS holds the table), so its last walks of a station
    // step in ordinary macro-steps.
    constexpr bool DRAIN = !DENSE;
    constexpr int TAIL_WAVES = DRAIN ? kMaxWaves : 1;
    static_assert(!DENSE || (ADJ && !BATCH), "dense tables are the adjoint's");

    __shared__ int tail_lane[TAIL_WAVES][64];
    __shared__ T tail_z[TAIL_WAVES][3 * 64][NPB];
    const BmTables* bmt = nullptr;
    if constexpr (F64) {
        BmTables* t = bm_tables();
        fill_bm_tables(*t);
        bmt = t;
    }

    Queue Q;
    LaneProblem<F64> P;
    if constexpr (BATCH) {
        Q = Queue{A.queue, (uint64_t)A.n_tasks, (uint32_t)A.grab, A.total_waves, A.stripes, A.refill_cost};
        P.C = nullptr;
        P.src = nullptr;
        P.sdt = T(0);
        P.lo0 = P.lo1 = P.lo2 = P.hi0 = P.hi1 = P.hi2 = T(0);
        P.ball = false;
        P.key0 = P.key1 = P.pid = 0;
        if constexpr (UKEY) {
            P.key0 = A.key0;
            P.key1 = A.key1;
        }
        P.max_steps = 0;
    } else {
        Q = Queue{A.c.queue, (uint64_t)A.c.n_tasks, (uint32_t)A.c.grab, A.c.total_waves, A.c.stripes,
                  A.c.refill_cost};
        P.load(A.c, A.src);
        // held in vector registers, as a batch holds them: kept in scalar
        // registers beside the source's bodies they overflow the scalar file,
        // and every step then reloads them from spill lanes
        P.sdt = in_vgpr(P.sdt);
        P.lo0 = in_vgpr(P.lo0);
        P.lo1 = in_vgpr(P.lo1);
        P.lo2 = in_vgpr(P.lo2);
        P.hi0 = in_vgpr(P.hi0);
        P.hi1 = in_vgpr(P.hi1);
        P.hi2 = in_vgpr(P.hi2);
    }
    // the density source of the lane's walk: the launch's (kernel arguments),
    // the batch's shared one (kernel arguments), or the lane's problem's
    auto source = [&]() -> const typename Prec<F64>::Src& {
        if constexpr (!BATCH) return A.src;
        else if constexpr (SHARED) return shared_source<F64>(A);
        else return *P.src;
    };
    // runs f on the source of the live lanes' walks (called with only those
    // lanes active): in a batch of separate sources, through wave_uniform when
    // the wavefront's walks share one
    auto with_source = [&](auto&& f) {
        if constexpr (BATCH && !SHARED) {
            if (const auto* u = wave_uniform(P.src))
                f(*u);
            else
                f(*P.src);
        } else if constexpr (!BATCH) {
            // the source in the kernel arguments (the launch's one argument,
            // at the start of the argument segment), re-addressed through an
            // opaque scalar pointer each macro-step: its bodies are reloaded
            // with scalar loads instead of being held live (and spilled)
            // across the loop
            uint64_t a = (uint64_t)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(Args, src);
            asm volatile("" : "+s"(a));
            f(*(const typename Prec<F64>::Src*)(const __attribute__((address_space(4))) typename Prec<F64>::Src*)a);
        } else {
            f(source());
        }
    };
    // drain rounds hold the first prism in registers (below); not in grid
    // loops, whose sources are mostly grids, nor in FP64 batches, whose
    // registers it costs more than it gains (both measured)
    constexpr bool kHeld = !loop_grid(LOOP) && !(F64 && BATCH);
    Pool pool = start_pool(Q);
    Walker<F64, KAHAN, ADJ, LOOP, DENSE> W;
    W.active = false;
    W.rec = 0;
    if constexpr (BATCH) {
        W.exits = A.exits;
        W.steps_out = A.steps;
    } else {
        W.exits = A.c.exits;
        W.steps_out = A.c.steps;
    }
    W.x0 = W.x1 = W.x2 = W.rp = T(0);
    W.S = 0.0;
    W.Sf = W.Sc = 0.0f;
    W.n = W.k = W.sctr = W.pctr = 0;
    W.deep = false;
    W.sc = Scatter<DENSE>{nullptr, nullptr, 0, -1, 0, 1};
    void* adj_tab = nullptr;
    int* dirty = nullptr;       // dense: set when the block starts a walk of its station
    if constexpr (ADJ && !DENSE) {
        static_assert(!BATCH, "the adjoint runs single-problem launches");
        __shared__ uint32_t tab[kAdjSlots];
        for (int i = threadIdx.x; i < kAdjSlots; i += blockDim.x) tab[i] = 0u;
        __syncthreads();
        adj_tab = tab;
    }
    if constexpr (DENSE) {
        __shared__ int dtab[kDenseVoxels];
        __shared__ int dflag;
        for (int i = threadIdx.x; i < kDenseVoxels; i += blockDim.x) dtab[i] = 0;
        if (threadIdx.x == 0) dflag = 0;
        __syncthreads();
        adj_tab = dtab;
        dirty = &dflag;
    }
    const int wave = threadIdx.x >> 6;
    const int lane = (int)__lane_id();
    uint64_t task_base = 0;   // task of queue index 0
    if constexpr (!BATCH) task_base = (uint64_t)A.c.task0;

    // The wavefront's walks until its queue is used up and they are done.
    auto run_waves = [&]() {
    for (;;) {
        const uint64_t got = refill(pool, Q, W.active);
        if (got != ~0ull) {
            const WalkCommon* Cp;
            uint64_t t;
            if constexpr (BATCH) {
                const int64_t T = A.task0 + (int64_t)got;
                const int m = find_problem(A.task_off, A.n_problems, T);
                const BatchDesc& D = A.desc[m];
                t = (uint64_t)(T - A.task_off[m]);
                if constexpr (SHARED)
                    P.load(D.c, shared_source<F64>(A), !UKEY);
                else
                    P.load(D.c, SourceOf<F64>::get(D), !UKEY);
                Cp = &D.c;
            } else {
                t = task_base + got;
                Cp = &A.c;
            }
            const WalkCommon& C = *Cp;
            const TaskInfo ti = decode(C, t);
            W.rec = got;
            const bool inside = strictly_inside(C, ti.x0);
            if (ADJ && (!inside || forward_capped(C, t))) {
                // excluded in the forward solve: contributes nothing
            } else if (!ADJ && !inside) {
                // a start point on or outside the boundary yields no sample
                const double q = __builtin_nan("");
                W.exits[got] = ExitRecord{q, q, q, q};
                W.steps_out[got] = kCapFlag;
            } else {
                W.x0 = (T)ti.x0[0];
                W.x1 = (T)ti.x0[1];
                W.x2 = (T)ti.x0[2];
                W.sctr = ti.sctr;
                W.pctr = ti.pctr;
                W.n = 0;
                W.k = 0;
                W.S = 0.0;
                W.Sf = W.Sc = 0.0f;
                if (ADJ) {
                    if (DENSE) __hip_atomic_store(dirty, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    W.sc.counts = C.counts;
                    W.sc.tab = adj_tab;
                    W.sc.row = (int64_t)ti.s * C.nvox;
                    W.sc.v = -1;
                    W.sc.c = 0;
                    W.sc.sign = ti.w ? -1 : 1;
                    W.sc.add(Prec<F64>::voxel(source(), W.x0, W.x1, W.x2), 1);
                } else {
                    // a launch without the grid loop has no grid in any source
                    if constexpr (loop_grid(LOOP))
                        W.rp = Prec<F64>::template rho<loop_levels(LOOP)>(source(), W.x0, W.x1, W.x2);
                    else
                        W.rp = Prec<F64>::bodies(source(), T(0), W.x0, W.x1, W.x2);
                }
                W.deep = false;
                if (loop_exit(LOOP) == 2 && P.bridge) {
                    const T d2 = P.ball ? dist2(W.x0, W.x1, W.x2, P.lo0, P.lo1, P.lo2) : T(0);
                    W.deep = W.deep_inside(P, W.x0, W.x1, W.x2, d2);
                }
                W.active = true;
            }
        }
        const uint64_t live = __ballot(W.active);
        if (live == 0ull) {
            if (pool.exhausted) break;
            continue;
        }
        const int m = __popcll(live);

        if (DRAIN && pool.exhausted) {
            // ---- drain round: the queue is empty, so every lane generates
            // three Philox blocks for the live walks of its wavefront (block
            // slot g = r * m + w holds block r of live walk w), and each live
            // walk then takes 2 * 64/m (FP64) or 4 * 64/m (mixed) steps from
            // LDS.  With m = 64 this costs what a macro-step costs; with few
            // live walks it spreads their random-number generation over all
            // lanes instead of leaving most lanes idle.
            const int rank = __popcll(live & __lanemask_lt());
            if (W.active) tail_lane[wave][rank] = lane;
            wave_sync_lds();
            const int B = 3 * (64 / m);                // blocks per live walk this round
#pragma unroll 1
            for (int i = 0; i < 3; ++i) {
                const int g = lane + 64 * i;
                const int w = g % m;
                const int r = g / m;
                const int src = tail_lane[wave][w];
                const uint32_t ks = (uint32_t)__shfl((int)W.k, src);
                const uint32_t ps = (uint32_t)__shfl((int)W.pctr, src);
                const uint32_t ss = (uint32_t)__shfl((int)W.sctr, src);
                uint32_t key0 = P.key0, key1 = P.key1, pid = P.pid;
                if constexpr (BATCH) {
                    if constexpr (!UKEY) {
                        key0 = (uint32_t)__shfl((int)P.key0, src);
                        key1 = (uint32_t)__shfl((int)P.key1, src);
                    }
                    pid = (uint32_t)__shfl((int)P.pid, src);
                }
                if (r < B) {
                    const Block bl = philox10(ks + (uint32_t)r, ps, ss, pid, key0, key1);
                    T z[NPB];
                    Prec<F64>::normals(bl, z, bmt);
#pragma unroll
                    for (int j = 0; j < NPB; ++j) tail_z[wave][g][j] = z[j];
                }
            }
            wave_sync_lds();
            if (W.active) {
                const int n_steps = B * NPB / 3;      // a multiple of MACRO
                bool done = false;
                int how = 0;
                if constexpr (kHeld) {
                    // A walk stepping alone here has no other wavefronts to
                    // hide the latency of re-reading the source's bodies at
                    // every step: the first prism is held in registers for
                    // the round.
                    with_source([&](const typename Prec<F64>::Src& src) {
                        const bool any = src.n_prisms > 0;
                        T hq[7];
#pragma unroll
                        for (int c = 0; c < 7; ++c)
                            hq[c] = in_vgpr(any ? (T)src.prisms[0][c] : (c == 0 ? (T)__builtin_inf() : T(0)));
                        // FP64: two macro-steps at a time while the round has
                        // them, so that their densities and exit tests overlap
                        // (mixed walks measured slower so: registers)
                        constexpr int DRAIN = F64 ? 2 * MACRO : MACRO;
                        int s0 = 0;
                        for (; s0 + DRAIN <= n_steps && !done; s0 += DRAIN) {
                            T zz[3 * DRAIN];
#pragma unroll
                            for (int c = 0; c < 3 * DRAIN; ++c) {
                                const int q = 3 * s0 + c;
                                zz[c] = tail_z[wave][(q / NPB) * m + rank][q % NPB];
                            }
                            int at = 0;
                            T g[DRAIN];
                            W.template advance<DRAIN>(P, src, zz, g);
                            done = W.template steps<true, DRAIN>(P, src, zz, g, at, how, hq);
                            if (done) W.template finish<DRAIN>(P, zz, at, how);
                        }
                        if constexpr (DRAIN != MACRO) {
                            for (; s0 < n_steps && !done; s0 += MACRO) {
                                T zz[3 * MACRO];
#pragma unroll
                                for (int c = 0; c < 3 * MACRO; ++c) {
                                    const int q = 3 * s0 + c;
                                    zz[c] = tail_z[wave][(q / NPB) * m + rank][q % NPB];
                                }
                                int at = 0;
                                T g[MACRO];
                                W.advance(P, src, zz, g);
                                done = W.template steps<true>(P, src, zz, g, at, how, hq);
                                if (done) W.finish(P, zz, at, how);
                            }
                        }
                    });
                } else {
                    for (int s0 = 0; s0 < n_steps && !done; s0 += MACRO) {
                        T zz[3 * MACRO];
#pragma unroll
                        for (int c = 0; c < 3 * MACRO; ++c) {
                            const int q = 3 * s0 + c;
                            zz[c] = tail_z[wave][(q / NPB) * m + rank][q % NPB];
                        }
                        int at = 0;
                        with_source([&](const typename Prec<F64>::Src& src) {
                            T g[MACRO];
                            W.advance(P, src, zz, g);
                            done = W.steps(P, src, zz, g, at, how);
                        });
                        if (done) W.finish(P, zz, at, how);
                    }
                }
                W.k += (uint32_t)B;
            }
            wave_sync_lds();
            continue;
        }

        if (!W.active) continue;

        // ---- macro-step: 3 blocks of this lane's own walk ----
        T z[3 * NPB];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const Block bl = philox10(W.k + b, W.pctr, W.sctr, P.pid, P.key0, P.key1);
            Prec<F64>::normals(bl, z + NPB * b, bmt);
        }
        W.k += 3;
        bool done = false;
        int how = 0, at = 0;
        with_source([&](const typename Prec<F64>::Src& src) {
            T g[MACRO];
            W.advance(P, src, z, g);
            done = W.steps(P, src, z, g, at, how);
        });
        if (done) W.finish(P, z, at, how);
    }
    };

    if constexpr (DENSE) {
        __shared__ int next_station;
        const int64_t S = A.c.n_stations;
        const uint64_t per = (uint64_t)A.c.N * (uint64_t)A.c.npair;   // tasks of one station
        const int64_t nvox = A.c.nvox;
        int* tab = static_cast<int*>(adj_tab);
        const uint32_t waves_per_station = A.c.total_waves / (uint32_t)S > 0 ? A.c.total_waves / (uint32_t)S : 1u;
        if (threadIdx.x == 0) next_station = (int)(blockIdx.x % (uint32_t)S);
        __syncthreads();
        for (;;) {
            const int s = next_station;
            if (s < 0) break;
            Q = Queue{A.c.queue + s, per, (uint32_t)A.c.grab, waves_per_station, 1u, A.c.refill_cost};
            pool = start_pool(Q);
            task_base = (uint64_t)s * per;
            run_waves();
            __syncthreads();    // the block's walks of station s are done
            if (*dirty) {
                for (int64_t v = threadIdx.x; v < nvox; v += blockDim.x) {
                    const int c = tab[v];
                    if (c != 0) {
                        global_add(A.c.counts, (int64_t)s * nvox + v, c);
                        tab[v] = 0;
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                *dirty = 0;
                int nxt = -1;
                for (int64_t k = 1; k <= S; ++k) {
                    const int c = (int)((s + k) % S);
                    if (__hip_atomic_load(A.c.queue + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < per) {
                        nxt = c;
                        break;
                    }
                }
                next_station = nxt;
            }
            __syncthreads();
        }
    } else {
        run_waves();
    }
    if constexpr (ADJ && !DENSE) {
        // every wavefront has left the loop: the table's entries go out
        __syncthreads();
        const uint32_t* tab = static_cast<const uint32_t*>(adj_tab);
        for (int i = threadIdx.x; i < kAdjSlots; i += blockDim.x) {
            const uint32_t e = tab[i];
            const int64_t c = adj_count(e);
            if (adj_key(e) != 0 && c != 0) global_add(A.c.counts, (int64_t)adj_key(e) - 1, c);
        }
    }
}

// Minimum resident 256-thread blocks per CU the compiler must allow (this
// bounds the VGPRs per lane: 4 blocks = 4 wavefronts per SIMD = 128 VGPRs).
// FP64 walks are held to 4 wavefronts per SIMD: measured faster than 3
// wavefronts without the limit, despite a small spill.
#ifndef FK_F64_BLOCKS_PER_CU
#define FK_F64_BLOCKS_PER_CU 4
#endif
// Mixed-precision walks are held to 6 (80 VGPRs).
#ifndef FK_F32_BLOCKS_PER_CU
#define FK_F32_BLOCKS_PER_CU 6
#endif
// Batches (box loop): 4 blocks for FP64 (128 VGPRs, no spill) and 5 for
// mixed precision (96 VGPRs, a 12-byte spill) measured 7-10 % faster than the
// unconstrained 3 and 4.  The ball and bridge loops are left free.
#ifndef FK_BATCH_F64_BLOCKS_PER_CU
#define FK_BATCH_F64_BLOCKS_PER_CU 4
#endif
#ifndef FK_BATCH_F32_BLOCKS_PER_CU
#define FK_BATCH_F32_BLOCKS_PER_CU 5
#endif

// Grid loops keep several grid loads in flight, which takes registers: mixed
// single-problem walks measured best at 5 blocks (96 VGPRs), mixed batches of
// separate sources at 4 (128 VGPRs; per-lane source fields), while a batch
// sharing one source stays at 5.
#ifndef FK_F32_GRID_BLOCKS_PER_CU
#define FK_F32_GRID_BLOCKS_PER_CU 5
#endif
#ifndef FK_BATCH_F32_GRID_BLOCKS_PER_CU
#define FK_BATCH_F32_GRID_BLOCKS_PER_CU 4
#endif
// FP64 batches of separate grids: 3 blocks (up to 170 VGPRs) hold the walk
// without the 28-register spill that 4 blocks cost (whose stores reached
// memory at about 130 GB/s), and measured 3 % faster.
#ifndef FK_BATCH_F64_GRID_BLOCKS_PER_CU
#define FK_BATCH_F64_GRID_BLOCKS_PER_CU 3
#endif

// The adjoint's blocks are held to 3 per CU by their LDS (the 32 KiB table
// and the drain buffers), so their registers are bounded for 3.
constexpr int kAdjBlocksPerCu = 3;

template <bool F64, bool KAHAN, bool ADJ, int LOOP>
__global__ void __launch_bounds__(256, ADJ                ? kAdjBlocksPerCu
                                       : F64             ? FK_F64_BLOCKS_PER_CU
                                       : loop_grid(LOOP) ? FK_F32_GRID_BLOCKS_PER_CU
                                                         : FK_F32_BLOCKS_PER_CU)
    walk_kernel(const typename std::conditional<F64, WalkArgsF64, WalkArgsF32>::type A)
{
    walk_body<F64, KAHAN, ADJ, false, LOOP, false, false, false>(A);
}

// The adjoint with dense station tables: one block of kAdjDenseBlock threads
// per CU (the 128 KiB table takes most of the CU's 160 KiB of LDS).
template <bool F64, bool KAHAN, int LOOP>
__global__ void __launch_bounds__(kAdjDenseBlock, 1)
    adjoint_dense_kernel(const typename std::conditional<F64, WalkArgsF64, WalkArgsF32>::type A)
{
    walk_body<F64, KAHAN, true, false, LOOP, false, true, false>(A);
}

template <bool F64, bool KAHAN, int LOOP, bool SHARED, bool UKEY>
__global__ void __launch_bounds__(256, loop_exit(LOOP)   ? 1
                                       : (F64 && loop_grid(LOOP) && !SHARED) ? FK_BATCH_F64_GRID_BLOCKS_PER_CU
                                       : F64             ? FK_BATCH_F64_BLOCKS_PER_CU
                                       : (loop_grid(LOOP) && !SHARED) ? FK_BATCH_F32_GRID_BLOCKS_PER_CU
                                                                      : FK_BATCH_F32_BLOCKS_PER_CU)
    batch_walk_kernel(const BatchArgs A)
{
    walk_body<F64, KAHAN, false, true, LOOP, SHARED, false, UKEY>(A);
}

}  // namespace

hipError_t launch_zero_queue(unsigned long long* queue, hipStream_t stream, uint32_t* status, uint32_t flags)
{
    hipLaunchKernelGGL(zero_queue_kernel, dim3(1), dim3(64), 0, stream, queue, status, flags);
    return hipGetLastError();
}

namespace {

// Calls f with the loop variant as a compile-time constant.
template <class F>
void with_loop(int loop, F&& f)
{
    switch (loop) {
    case 14: f(std::integral_constant<int, 14>{}); break;
    case 13: f(std::integral_constant<int, 13>{}); break;
    case 12: f(std::integral_constant<int, 12>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    default: f(std::integral_constant<int, 0>{});
    }
}

// The adjoint samples no density (it counts voxel visits), so its loop never
// carries the grid bit.
template <bool F64, bool KAHAN, bool ADJ, class A>
void launch_walk(const A& a, int loop, const LaunchCfg& cfg, hipStream_t stream, bool dense)
{
    with_loop(ADJ ? loop_exit(loop) : loop, [&](auto L) {
        if (ADJ && dense)
            hipLaunchKernelGGL((adjoint_dense_kernel<F64, KAHAN, loop_exit(decltype(L)::value)>), dim3(cfg.grid),
                               dim3(cfg.block), 0, stream, a);
        else
            hipLaunchKernelGGL((walk_kernel<F64, KAHAN, ADJ, decltype(L)::value>), dim3(cfg.grid), dim3(cfg.block),
                               0, stream, a);
    });
}

template <int LOOP, bool ADJ>
const void* walk_fn(int precision, bool dense)
{
    if (ADJ && dense)
        return precision == FK_F64 ? (const void*)adjoint_dense_kernel<true, false, loop_exit(LOOP)>
             : precision == FK_MIXED_KAHAN ? (const void*)adjoint_dense_kernel<false, true, loop_exit(LOOP)>
                                           : (const void*)adjoint_dense_kernel<false, false, loop_exit(LOOP)>;
    return precision == FK_F64 ? (const void*)walk_kernel<true, false, ADJ, LOOP>
         : precision == FK_MIXED_KAHAN ? (const void*)walk_kernel<false, true, ADJ, LOOP>
                                       : (const void*)walk_kernel<false, false, ADJ, LOOP>;
}

// FP64 batches take the uniform key only with one shared source (+2 % on
// the SI-prism FP64 batch).  Batches of separate sources keep the per-lane
// key: their walks already fill the scalar registers, and with the key
// schedule there too they spill more and measured 1.6 % slower (the
// 32-model FP64 grid batch).
template <bool SHARED, bool UKEY>
constexpr bool kF64Ukey = SHARED && UKEY;

template <int LOOP, bool SHARED, bool UKEY>
const void* batch_fn(int precision)
{
    return precision == FK_F64 ? (const void*)batch_walk_kernel<true, false, LOOP, SHARED, kF64Ukey<SHARED, UKEY>>
         : precision == FK_MIXED_KAHAN ? (const void*)batch_walk_kernel<false, true, LOOP, SHARED, UKEY>
                                       : (const void*)batch_walk_kernel<false, false, LOOP, SHARED, UKEY>;
}

template <int LOOP, bool SHARED, bool UKEY>
void launch_batch(const BatchArgs& a, const LaunchCfg& cfg, hipStream_t stream)
{
    if (a.precision == FK_F64)
        hipLaunchKernelGGL((batch_walk_kernel<true, false, LOOP, SHARED, kF64Ukey<SHARED, UKEY>>), dim3(cfg.grid),
                           dim3(cfg.block), 0, stream, a);
    else if (a.precision == FK_MIXED_KAHAN)
        hipLaunchKernelGGL((batch_walk_kernel<false, true, LOOP, SHARED, UKEY>), dim3(cfg.grid), dim3(cfg.block), 0,
                           stream, a);
    else
        hipLaunchKernelGGL((batch_walk_kernel<false, false, LOOP, SHARED, UKEY>), dim3(cfg.grid), dim3(cfg.block), 0,
                           stream, a);
}

// Calls f with (shared source, uniform key) as compile-time constants.
template <class F>
void with_batch_mode(bool shared, bool ukey, F&& f)
{
    if (shared) {
        if (ukey) f(std::true_type{}, std::true_type{});
        else f(std::true_type{}, std::false_type{});
    } else {
        if (ukey) f(std::false_type{}, std::true_type{});
        else f(std::false_type{}, std::false_type{});
    }
}

// The loop variant of a single problem's launch (see loop_exit, loop_grid,
// loop_levels).
template <class Src>
int loop_of(const WalkCommon& c, const Src& s)
{
    const int e = c.exit_rule == FK_EXIT_BRIDGE ? 2 : c.domain == FK_DOMAIN_BALL ? 1 : 0;
    return e | (s.has_grid ? kLoopGrid : 0) | (s.has_grid && s.idx ? kLoopLevels : 0);
}

}  // namespace

hipError_t launch_walk_f64(const WalkArgsF64& a, const LaunchCfg& cfg, hipStream_t stream, bool adjoint, bool dense)
{
    const int loop = loop_of(a.c, a.src);
    if (adjoint)
        launch_walk<true, false, true>(a, loop, cfg, stream, dense);
    else
        launch_walk<true, false, false>(a, loop, cfg, stream, false);
    return hipGetLastError();
}

hipError_t launch_walk_f32(const WalkArgsF32& a, bool kahan, const LaunchCfg& cfg, hipStream_t stream, bool adjoint,
                           bool dense)
{
    const int loop = loop_of(a.c, a.src);
    if (adjoint) {
        if (kahan)
            launch_walk<false, true, true>(a, loop, cfg, stream, dense);
        else
            launch_walk<false, false, true>(a, loop, cfg, stream, dense);
    } else {
        if (kahan)
            launch_walk<false, true, false>(a, loop, cfg, stream, false);
        else
            launch_walk<false, false, false>(a, loop, cfg, stream, false);
    }
    return hipGetLastError();
}

hipError_t walk_occupancy(int precision, int block, int* blocks_per_cu, int loop, bool adjoint, bool dense)
{
    const void* fn = nullptr;
    if (adjoint)
        with_loop(loop_exit(loop), [&](auto L) { fn = walk_fn<decltype(L)::value, true>(precision, dense); });
    else
        with_loop(loop, [&](auto L) { fn = walk_fn<decltype(L)::value, false>(precision, false); });
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, 0);
}

hipError_t launch_batch_walk(const BatchArgs& a, const LaunchCfg& cfg, hipStream_t stream, int loop, bool shared)
{
    with_loop(loop, [&](auto L) {
        with_batch_mode(shared, a.uniform_key != 0, [&](auto S, auto U) {
            launch_batch<decltype(L)::value, decltype(S)::value, decltype(U)::value>(a, cfg, stream);
        });
    });
    return hipGetLastError();
}

hipError_t batch_occupancy(int precision, int block, int* blocks_per_cu, int loop, bool shared, bool ukey)
{
    const void* fn = nullptr;
    with_loop(loop, [&](auto L) {
        with_batch_mode(shared, ukey, [&](auto S, auto U) {
            fn = batch_fn<decltype(L)::value, decltype(S)::value, decltype(U)::value>(precision);
        });
    });
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, 0);
}

// ---------------------------------------------------------------------------
// Diagnostic: the random stream as the walk kernels compute it.
// ---------------------------------------------------------------------------
namespace {

__global__ void stream_blocks_kernel(const uint32_t* ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t* words,
                                     double* z64, float* z32)
{
    BmTables* bmt = bm_tables();
    fill_bm_tables(*bmt);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Block b = philox10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key0, key1);
    if (words) {
        words[4 * i] = b.w0;
        words[4 * i + 1] = b.w1;
        words[4 * i + 2] = b.w2;
        words[4 * i + 3] = b.w3;
    }
    if (z64) normals_f64(b, *bmt, z64[2 * i], z64[2 * i + 1]);
    if (z32) {
        normals_f32(b.w0, b.w1, z32[4 * i], z32[4 * i + 1]);
        normals_f32(b.w2, b.w3, z32[4 * i + 2], z32[4 * i + 3]);
    }
}

}  // namespace

hipError_t launch_stream_blocks(const uint32_t* ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t* words,
                                double* z64, float* z32, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(stream_blocks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, ctr, n, key0,
                       key1, words, z64, z32);
    return hipGetLastError();
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
