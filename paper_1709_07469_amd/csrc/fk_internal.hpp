// fk_internal.hpp -- launch-argument blocks shared by the host runtime and the
// kernels of the library.  Everything a walk needs travels by value in the
// kernel argument block (analytic bodies and coefficient sets included), so a
// solve reads no host memory after it is enqueued and can be captured in a
// HIP graph.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "fkgrav.h"

namespace fk {

struct SourceF64 {
    const float* rho;          // device voxel grid or nullptr
    const uint8_t* idx;        // or the grid by levels: device index grid
    const float* levels;       // and its 256 densities
    int32_t n[3];
    int32_t has_grid;
    double origin[3];
    double spacing[3];
    double inv[3];             // 1 / spacing
    int32_t exact[3];          // spacing is a power of two: (x - o) * inv == (x - o) / spacing
    int32_t n_prisms;
    int32_t n_spheres;
    uint32_t nxy;              // n[0] n[1], the voxels of one layer
    double prisms[FK_MAX_PRISMS][7];
    double spheres[FK_MAX_SPHERES][5];
};

struct SourceF32 {
    const float* rho;
    const uint8_t* idx;
    const float* levels;
    int32_t n[3];
    int32_t has_grid;
    float ob[3];               // -origin / spacing
    float inv[3];              // 1 / spacing
    uint32_t nxy;              // n[0] n[1], the voxels of one layer
    int32_t n_prisms;
    int32_t n_spheres;
    int32_t pad0;
    float prisms[FK_MAX_PRISMS][7];
    float spheres[FK_MAX_SPHERES][5];
};

struct BoundaryArgs {
    int32_t kind;
    int32_t n_items;
    double quad[10];
    double items[FK_MAX_BC_ITEMS][7];
    const double* face_data;   // device, FACE_GRID only
    int64_t face_off[6];
    int32_t face_n[6][2];
};

// What a walk leaves for the reduction pass: its exit point and its
// trapezoid sum S = sum_n (rho_n + rho_{n+1}).
struct ExitRecord {
    double x, y, z, S;
};

// Task t of a solve is (station s, local path i, walk w):
//   t = (s * N + i) * npair + w,  npair = 1 (potential) or 2 (g_z walks +h, -h).
// A launch runs the tasks task0 .. task0 + n_tasks - 1 (all of them, or one
// slice of a bounded workspace) and stores task t's record at t - task0.
struct WalkCommon {
    const double* stations;    // device, n_stations x 3
    ExitRecord* exits;         // device, the launch's exit records
    uint32_t* steps;           // device, the launch's step counts (bit 31: capped)
    unsigned long long* queue; // device, next unclaimed task
    int64_t n_stations;
    int64_t N;
    int64_t n_tasks;           // tasks of this launch
    int64_t task0;             // first task of this launch
    int64_t path_offset;
    int64_t max_steps;
    double lo[3], hi[3];
    float lo_f[3], hi_f[3];
    double sdt;                // sqrt(dt)
    double w;                  // 2 pi G (dt / 2), weight of the trapezoid sum
    double G;
    double h;                  // g_z difference step
    float sdt_f;
    uint32_t key0, key1;       // Philox key (seed)
    uint32_t problem_id;
    int32_t npair;
    int32_t pairing;
    int32_t exit_rule;
    int32_t grab;              // largest queue claim per wavefront
    uint32_t total_waves;      // resident wavefronts of the launch
    uint32_t stripes;          // claim counters of the queue (1 .. 32)
    uint32_t refill_cost;      // 128 x the start-up cost of the refill rule, in macro-steps
    int32_t domain;            // FK_DOMAIN_BOX / FK_DOMAIN_BALL
    double ctr[3];             // ball domain: centre, squared radius, radius
    double r2;
    double R;
    double dt;
    double delta;              // Brownian bridge: a step whose ends both lie at least delta
    double deep2;              // inside every face cannot be stopped; ball: (R - delta)^2 or -1
    float ctr_f[3];
    float r2_f, R_f, dt_f, delta_f, deep2_f;
    // adjoint replay only: signed trapezoid weights per (station, voxel), and
    // the forward solve's step counts (walks capped there are skipped)
    int64_t* counts;
    const uint32_t* fwd_steps;
    int64_t nvox;
};

struct WalkArgsF64 {
    WalkCommon c;
    SourceF64 src;
};

struct WalkArgsF32 {
    WalkCommon c;
    SourceF32 src;
};

// Per-chunk partial statistics of one station: count, mean and sum of
// squared deviations (Chan et al. merge), and step tallies.
struct Partial {
    double n;
    double mean;
    double m2;
    int64_t sum_steps;
    int64_t max_steps;
    int64_t n_trunc;
};

// The reduction of the (station, chunk) pairs q0 .. q0 + gridDim - 1 (pair
// q = s * n_chunks + c) whose walks' records start at task task0.
struct ReduceArgs {
    const ExitRecord* exits;
    double* values;            // per-walk samples written here (record mode), or null
    const uint32_t* steps;
    Partial* partials;         // one per pair, all pairs of the solve
    fk_stat* out;
    uint32_t* status;          // the workspace's status word (FK_FLAG_* bits)
    int64_t n_stations;
    int64_t N;
    int64_t chunk;             // samples per partial
    int64_t n_chunks;          // partials per station
    int64_t q0;                // first pair of this launch
    int64_t task0;             // task of the first record
    int32_t npair;
    int32_t pad0;
    double two_h;
    double w;                  // 2 pi G (dt / 2)
    double G;
    double lo[3], hi[3];
    BoundaryArgs bc;
};

// One problem of a batched solve, as the batch kernels see it (in device
// memory, written by the descriptor kernels).  Tasks and (station, chunk) pairs of a batch are numbered across its
// problems in order: global task T = task_off[m] + t, global pair
// Q = block_off[m] + q.  Records, per-walk values and partials are indexed
// by these global numbers (records from the launch's first task).
struct BatchDesc {
    WalkCommon c;              // queue, exits, steps, n_tasks, task0 unused
    SourceF64 s64;
    SourceF32 s32;
    BoundaryArgs bc;
    fk_stat* out;              // this problem's first station result
    int64_t n_chunks;
    int64_t task_base;
    int64_t block_base;        // first reduction block (pair) of this problem
    int64_t station_base;      // first station of this problem in the batch's station numbering
};

struct BatchArgs {
    BatchDesc* desc;           // device, n_problems
    const int64_t* task_off;   // device, n_problems + 1 prefix sums of tasks
    const int64_t* block_off;  // device, n_problems + 1 prefix sums of (station, chunk) pairs
    unsigned long long* queue;
    ExitRecord* exits;         // device, records of tasks task0 .. task0 + n_tasks - 1
    uint32_t* steps;
    double* values;            // device, per-walk samples by global task (record mode), or null
    Partial* partials;         // device, one per global pair
    uint32_t* status;          // the workspace's status word
    int64_t n_tasks;           // tasks of this launch
    int64_t task0;             // first global task of this launch
    int64_t q0;                // first global pair of this reduction launch
    int32_t n_problems;
    int32_t grab;
    uint32_t total_waves;
    int32_t precision;
    uint32_t stripes;
    uint32_t refill_cost;
    // uniform_key: every problem's generator key is (key0, key1)
    uint32_t key0, key1;
    int32_t uniform_key;
    int64_t chunk;
    // when every problem of the batch has the same source, that source (the
    // walk kernel then reads it from the kernel arguments, as a single
    // problem's launch does)
    SourceF64 src64;
    SourceF32 src32;
};

struct LaunchCfg {
    int block;
    int grid;
    int grab;
    uint32_t stripes;
    uint32_t refill_cost;
};

// Host launchers (one translation unit per kernel family).
// Clears the queue's claim counters; with status non-null also sets the
// status word to `flags` (the start of a solve).
hipError_t launch_zero_queue(unsigned long long* queue, hipStream_t stream, uint32_t* status = nullptr,
                             uint32_t flags = 0);
// adjoint: the replay that scatters occupation weights; dense: its instance
// with per-station dense LDS tables (grids of at most kAdjDenseVoxels voxels,
// blocks of kAdjDenseBlock threads, one claim counter per station in the
// queue region).
constexpr int64_t kAdjDenseVoxels = 32768;
constexpr int64_t kAdjDenseMaxStations = 65536;
constexpr int kAdjDenseBlock = 1024;
hipError_t launch_walk_f64(const WalkArgsF64& a, const LaunchCfg& cfg, hipStream_t stream, bool adjoint = false,
                           bool dense = false);
hipError_t launch_walk_f32(const WalkArgsF32& a, bool kahan, const LaunchCfg& cfg, hipStream_t stream,
                           bool adjoint = false, bool dense = false);
// Adjoint helpers: zero the count array; combine counts into the
// vector-Jacobian product grad_rho[v] = sum_s coef_s * counts[s][v].
hipError_t launch_fill_zero(int64_t* p, int64_t n, hipStream_t stream);
hipError_t launch_adjoint_combine(const int64_t* counts, int64_t n_stations, int64_t nvox, const double* grad_out,
                                  const fk_stat* fwd, double scale, double* grad_rho, hipStream_t stream);
// The chunk partials of pairs a.q0 .. a.q0 + n_pairs - 1; then, when
// finish is set, every station's result from all its partials.
hipError_t launch_reduce(const ReduceArgs& a, int64_t n_pairs, bool finish, hipStream_t stream);
// loop: 0 box stepping loop, 1 with the ball exit test, 2 with the
// Brownian-bridge test too
hipError_t walk_occupancy(int precision, int block, int* blocks_per_cu, int loop = 0, bool adjoint = false,
                          bool dense = false);
hipError_t launch_stream_blocks(const uint32_t* ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t* words,
                                double* z64, float* z32, hipStream_t stream);

// Batched solve: descriptor upload (by value through kernel arguments, so a
// captured graph replays it), the persistent walk kernel over all problems,
// and the batched reduction.
hipError_t launch_write_words(uint64_t* dst, const uint64_t* host_words, int64_t n_words, hipStream_t stream);
hipError_t launch_batch_walk(const BatchArgs& a, const LaunchCfg& cfg, hipStream_t stream, int loop, bool shared);
hipError_t launch_batch_chunks(const BatchArgs& a, int64_t n_pairs, hipStream_t stream);
hipError_t launch_batch_stations(const BatchArgs& a, int64_t n_stations, hipStream_t stream);
hipError_t batch_occupancy(int precision, int block, int* blocks_per_cu, int loop = 0, bool shared = false,
                           bool ukey = false);

}  // namespace fk
