/*
 * fkgrav.h -- C interface of the MI355X (gfx950) Monte Carlo solver for the
 * gravity forward problem by the Feynman-Kac formula, after Donzelli, Bihlo,
 * Kischinhevsky & Farquharson, "Massively parallel stochastic solution of the
 * geophysical gravity problem" (arXiv:1709.07469).
 *
 * What a solve computes (paper section 2.1 eqs. 3-6, section 2.3):
 *   For every station x0 strictly inside the box, N walks of standard 3-D
 *   Brownian motion are stepped by Euler-Maruyama, x_{n+1} = x_n + sqrt(dt) Z_n,
 *   Z_n ~ N(0, I_3), until the first n with x_{n+1} on or outside the box.
 *   Along each walk the source is integrated with the trapezoid rule,
 *   I = (dt/2) sum_n (rho(x_n) + rho(x_{n+1})), the exiting step included, and
 *   the Dirichlet data g is read at the exit point x_e.  The path sample is
 *       u_p = g(x_e) - 2 pi G I,
 *   whose mean estimates the potential u(x0) solving Laplace(u) = 4 pi G rho,
 *   u = g on the boundary (u < 0 for positive mass; the paper's walk
 *   gamma = sqrt(2) W of eq. 2 is the same process run twice as fast, so its
 *   Delta t equals dt/2).  Station results are the sample mean (eq. 11), the
 *   unbiased sample variance and the standard error.
 *   fk_solve_gz estimates g_z = du/dz (eq. 6) by the central difference of
 *   section 4.2, (u(x0 + h e_z) - u(x0 - h e_z)) / (2h), with both walks of a
 *   pair driven by the same random numbers unless FK_PAIR_INDEPENDENT.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11).  Block k of path p of
 * station s of problem m is Philox(counter = (k, p, s, m), key = (seed mod
 * 2^32, seed >> 32)).  FK_F64 draws two 53-bit uniforms per block
 * U = ((w_hi << 21 | w_lo >> 11) + 1) 2^-53 and one Box-Muller pair; the
 * mixed precisions draw four 24-bit uniforms u = ((w >> 8) + 1) 2^-24 and two
 * pairs.  Step n uses normals 3n, 3n+1, 3n+2.  p = path_offset + i for local
 * path i; s is the station index (or 2s / 2s+1 for independent g_z pairs).
 *
 * Conventions for every entry point:
 *   - "device" pointers address GPU memory (e.g. a torch tensor's data_ptr());
 *     "host" pointers address CPU memory and are read before the call returns.
 *   - Calls are asynchronous and ordered on hip_stream (a hipStream_t; NULL is
 *     the null stream).  Device inputs must stay valid until the stream has
 *     passed the call.  The library keeps no pointer after it returns and
 *     allocates no device memory: scratch comes from the caller's workspace.
 *   - A solve's workspace begins with a 256-byte status block whose first
 *     word collects the FK_FLAG_* anomaly bits of the solve's walks (set on
 *     the device, read by fk_workspace_status without a synchronisation
 *     inside the solve).
 *   - All argument checks run on the host before any launch.  On an error
 *     nothing is launched, outputs are untouched and fk_last_error() holds a
 *     message.  No C++ exception crosses this interface.
 *   - Identical inputs, seed and launch settings give bitwise-identical
 *     outputs: per-path samples are stored by path index and reduced in a
 *     fixed order.
 */
#ifndef FKGRAV_H
#define FKGRAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FK_OK = 0,
    FK_EINVAL = -1,        /* malformed argument (dt <= 0, N < 2, NULL pointer, bad enum, ...) */
    FK_EDOMAIN = -2,       /* a station (or station +- h e_z) is not strictly inside the box */
    FK_EWORKSPACE = -3,    /* workspace smaller than fk_workspace_bytes() or misaligned */
    FK_EDEVICE = -4,       /* a HIP runtime call failed */
    FK_ETRUNC = -5,        /* fk_workspace_status: a strict solve capped walks at max_steps */
    FK_EUNSUPPORTED = -6,  /* a size limit of the library is exceeded (see FK_MAX_*) */
    FK_ENONFINITE = -7     /* fk_workspace_status: a walk sample was NaN or infinite */
} fk_status;

/* Anomaly bits of a solve's status word (fk_workspace_status).  The
 * reduction ORs them in on the device as it forms the walk samples. */
typedef enum {
    FK_FLAG_TRUNCATED = 1,  /* a walk hit max_steps, or started on or outside the boundary; it is
                             * excluded from mean and variance and counted in fk_stat.n_trunc */
    FK_FLAG_NONFINITE = 2,  /* an uncapped walk's sample is NaN or infinite (a NaN or infinite density,
                             * position or boundary datum); it enters mean and variance as it is */
    FK_FLAG_STRICT = 256    /* the solve ran with fk_params.strict set */
} fk_flag;

typedef enum {
    FK_F64 = 0,            /* FP64 stream, FP64 stepping and accumulation */
    FK_MIXED_F64ACC = 1,   /* FP32 stream and stepping, FP64 path integral, FP64 exit/data */
    FK_MIXED_KAHAN = 2     /* FP32 stream and stepping, Kahan-compensated FP32 path integral */
} fk_precision;

typedef enum {
    FK_EXIT_OVERSHOOT = 0, /* data read at the first point on/outside the box (unbiased for harmonic data) */
    FK_EXIT_INTERSECT = 1, /* data read where the last step's segment first meets the boundary */
    FK_EXIT_BRIDGE = 2     /* INTERSECT plus the Brownian-bridge test of the paper's remark on the exit
                            * time (section 2.3; Gobet 2000): a step whose two ends lie inside is a stop
                            * with probability 1 - prod_f (1 - exp(-2 a_f b_f / dt)), a_f and b_f the
                            * distances of its ends to face f (ball: to the sphere, one term).  The
                            * walk's uniform for step n is slot n mod q of Philox block 2^31 + n / q of
                            * its stream (q = 2 FP64: 53-bit uniforms from word pairs (w1,w0), (w3,w2);
                            * q = 4 FP32: 24-bit uniforms (w >> 8) + 1) * 2^-24); it stops when
                            * U <= that probability, and the data is read at the step's end projected
                            * onto the face with the largest probability (ties: -x, +x, -y, +y, -z, +z)
                            * or radially onto the sphere.  Needs max_steps <= 2^30. */
} fk_exit_rule;

typedef enum {
    FK_BC_ZERO = 0,        /* g = 0 (the paper's truncated-domain choice, section 2.2) */
    FK_BC_QUADRATIC = 1,   /* g = c0 + b.x + x^T A x; data (host) = c0, b0..b2, A00 A01 A02 A11 A12 A22 */
    FK_BC_POINT_MASSES = 2,/* g = -sum_j G m_j / |x - c_j|; data (host) rows (cx, cy, cz, m) */
    FK_BC_PRISMS = 3,      /* g = sum_j -G rho_j V_j(x), homogeneous prisms; data (host) rows (lo[3], hi[3], rho) */
    FK_BC_FACE_GRID = 4    /* bilinear node grids on the six faces; data (DEVICE), see fk_boundary */
} fk_bc_kind;

typedef enum { FK_PAIR_CRN = 0, FK_PAIR_INDEPENDENT = 1 } fk_pairing;

enum {
    FK_MAX_PRISMS = 16,    /* analytic prisms in a source */
    FK_MAX_SPHERES = 16,   /* analytic balls in a source */
    FK_MAX_BC_ITEMS = 16,  /* rows of POINT_MASSES / PRISMS boundary data */
    FK_MAX_BATCH = 256     /* problems in one fk_solve_batch call */
};

/* Box domain [lo, hi] (paper section 2.1: Omega; here an axis-aligned box). */
typedef struct {
    double lo[3], hi[3];
} fk_box;

/* Density rho(x) (paper eq. 4), the sum of
 *   - a voxel grid: rho (DEVICE, float, [n[2]][n[1]][n[0]], x fastest; NULL
 *     for none); voxel (i,j,k) is [origin + (i,j,k)*spacing, origin +
 *     (i+1,j+1,k+1)*spacing), zero outside the grid; each n[c] at most
 *     2^24 - 1 and the grid at most 2^31 - 1 voxels (FK_EUNSUPPORTED
 *     beyond).  Or the same grid given
 *     by levels: rho_index (DEVICE, uint8, the same layout) selects the
 *     voxel's density rho_levels[rho_index] (DEVICE, 256 floats: any byte
 *     indexes inside it; entries no voxel selects are never read), with rho
 *     NULL.  A model of at most 256 distinct densities (a few units, each
 *     of one density) then takes a quarter of the memory and cache of the
 *     FP32 grid; the densities, so the results, are the same;
 *   - analytic homogeneous prisms (HOST, n_prisms rows lo[3], hi[3], rho),
 *     half-open [lo, hi) per axis;
 *   - analytic homogeneous balls (HOST, n_spheres rows c[3], radius, rho),
 *     open. */
typedef struct {
    const float *rho;
    int32_t n[3];
    int32_t pad0;
    double origin[3];
    double spacing[3];
    const double *prisms;
    int32_t n_prisms;
    int32_t pad1;
    const double *spheres;
    int32_t n_spheres;
    int32_t pad2;
    const uint8_t *rho_index;
    const float *rho_levels;
} fk_source;

/* Dirichlet data g (paper eq. 1).  For FK_BC_FACE_GRID, data is DEVICE memory
 * holding the node values of faces f = 0..5 (-x, +x, -y, +y, -z, +z) one after
 * the other; face f has face_n[f][0] x face_n[f][1] (>= 2 each) nodes spread
 * uniformly from lo to hi along its axes (a, b) = (y, z) for x faces, (x, z)
 * for y faces, (x, y) for z faces; node (ia, ib) is at offset ib*n_a + ia.  The
 * exit point is clamped to the box and read on the face it lies furthest
 * beyond (ties: lower axis, then the lower face).  For the other kinds data
 * is HOST memory with n_items rows as listed in fk_bc_kind. */
typedef struct {
    int32_t kind;
    int32_t pad0;
    const double *data;
    int64_t n_items;
    int32_t face_n[6][2];
} fk_boundary;

/* The domain Omega of eq. 1.  FK_DOMAIN_BOX: the box itself.  FK_DOMAIN_BALL:
 * the ball inscribed in the box, centre (lo + hi) / 2 and radius
 * (hi[0] - lo[0]) / 2 -- the box must be a cube (edges equal to 1e-12
 * relative) -- as in the experiments of section 3 (a ball of radius 10 km).
 * A point x has left the ball when |x - c|^2 >= R^2, with |x - c|^2 =
 * fma(d0, d0, fma(d1, d1, d2 * d2)).  FK_BC_FACE_GRID needs a box domain. */
typedef enum { FK_DOMAIN_BOX = 0, FK_DOMAIN_BALL = 1 } fk_domain;

/* Run parameters (paper section 3: N walks per station and time step Delta t). */
typedef struct {
    int64_t paths_per_station;   /* N >= 2, path_offset + N <= 2^32 */
    double dt;                   /* > 0; standard deviation per coordinate and step sqrt(dt) */
    uint64_t seed;               /* Philox key */
    double G;                    /* gravitational constant */
    double h;                    /* g_z difference step; 0 selects sqrt(dt) */
    int32_t precision;           /* fk_precision */
    int32_t exit_rule;           /* fk_exit_rule */
    int32_t pairing;             /* fk_pairing (g_z only) */
    int32_t strict;              /* nonzero: fk_workspace_status reports capped walks as FK_ETRUNC */
    int64_t max_steps;           /* cap per walk, 1 .. 2^31-1; capped walks are excluded and counted */
    uint32_t problem_id;         /* counter word m */
    int32_t domain;              /* fk_domain */
    int64_t path_offset;         /* first path index p */
    int64_t slice_walks;         /* 0: the workspace keeps every walk's record (the per-walk samples stay
                                  * inspectable, fk_workspace_layout).  > 0: bounded workspace -- the walks
                                  * run in slices of at most this many (at least 8192 per walk of a pair,
                                  * i.e. 8192 for a potential, 16384 for g_z), each slice a run of whole
                                  * (station, 8192-path chunk) pairs reduced before the next starts, so the
                                  * workspace holds one slice's records and every pair's partial
                                  * statistics; results are bit for bit those of record mode */
} fk_params;

/* Per-station result.  For fk_solve_gz the samples are the pair differences
 * and the step counts are those of both walks of a pair. */
typedef struct {
    double mean;                 /* sample mean of the untruncated samples (eq. 11) */
    double var;                  /* unbiased sample variance */
    double se;                   /* standard error sqrt(var / n) */
    int64_t n;                   /* untruncated samples */
    int64_t sum_steps;           /* Euler-Maruyama steps taken, all samples, exiting steps included */
    int64_t max_steps;           /* longest sample in steps */
    int64_t n_trunc;             /* samples that hit max_steps (excluded from mean/var) */
    double mean_steps;           /* sum_steps / N */
} fk_stat;

/* One problem of a batch. */
typedef struct {
    int32_t kind;                /* 0 = potential, 1 = g_z */
    int32_t pad0;
    const double *stations;      /* DEVICE, n_stations x 3 */
    int64_t n_stations;
    fk_box box;
    fk_source source;
    fk_boundary bc;
    fk_params params;
    int64_t out_offset;          /* first fk_stat of this problem in the batch output */
} fk_problem;

/* Bytes of device workspace a solve needs (host, pure).  kind 0 = potential,
 * 1 = g_z.  With params->slice_walks = 0 the workspace holds every walk's
 * record (about 44 bytes per walk) and keeps the per-path samples of the last
 * solve, laid out as described by fk_workspace_layout; with slice_walks > 0 it
 * holds 36 bytes per walk of one slice plus 48 bytes per (station, chunk)
 * pair, whatever the walk count.  0 for invalid parameters. */
size_t fk_workspace_bytes(int32_t kind, int64_t n_stations, const fk_params *params);

/* Offsets (bytes from the workspace start) of the per-path arrays a solve
 * leaves behind: values (double) and steps (uint32, bit 31 set for a walk that
 * hit max_steps).  Potential: index s*N + i.  g_z: index (s*N + i)*2 + w with
 * w = 0 for the walk from x0 + h e_z and 1 for x0 - h e_z.  Values of capped
 * walks are NaN.  Record mode only (slice_walks = 0; else FK_EINVAL). */
fk_status fk_workspace_layout(int32_t kind, int64_t n_stations, const fk_params *params,
                              size_t *values_offset, size_t *steps_offset, size_t *total_bytes);

/* Anomaly report of the last solve (single or batched) run in a workspace:
 * waits for hip_stream, copies the status word to *flags (HOST, nullable;
 * FK_FLAG_* bits) and returns FK_ENONFINITE if some sample was not finite,
 * else FK_ETRUNC if the solve was strict and capped some walk, else FK_OK.
 * workspace: DEVICE, the solve's workspace (its first 256 bytes). */
fk_status fk_workspace_status(const void *workspace, uint32_t *flags, void *hip_stream);

/* Host-side check that every station (HOST, n_stations x 3) lies strictly
 * inside the box -- for kind 1 also x0 +- h e_z.  Returns FK_EDOMAIN naming the
 * first offender.  The solvers take device station arrays and cannot read
 * them on the host; a walk whose start point is not strictly inside yields no
 * sample and is counted in fk_stat.n_trunc with a step count of 0. */
fk_status fk_check_stations(const double *stations_host, int64_t n_stations, const fk_box *box, int32_t kind,
                            const fk_params *params);

/* Potential u at n_stations stations (DEVICE, n_stations x 3 doubles).
 * out: DEVICE, n_stations fk_stat.  workspace: DEVICE, 256-byte aligned,
 * at least fk_workspace_bytes(0, ...) bytes.  Paper section 2.3. */
fk_status fk_solve_potential(const double *stations, int64_t n_stations, const fk_box *box,
                             const fk_source *source, const fk_boundary *bc, const fk_params *params,
                             fk_stat *out, void *workspace, size_t workspace_bytes, void *hip_stream);

/* Vertical acceleration g_z = du/dz by paired central differences at x0 +- h
 * e_z (paper eq. 6, section 4.2).  Same arguments as fk_solve_potential;
 * workspace at least fk_workspace_bytes(1, ...). */
fk_status fk_solve_gz(const double *stations, int64_t n_stations, const fk_box *box,
                      const fk_source *source, const fk_boundary *bc, const fk_params *params,
                      fk_stat *out, void *workspace, size_t workspace_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * potential (kind 0) or g_z (kind 1) solve of fk_solve_potential /
 * fk_solve_gz without a workspace argument.  Its scratch is a device array of
 * 64 MiB inside the library, one per GPU, allocated with the library's code
 * object and held until the process ends; the call itself allocates nothing.
 * It runs as a bounded-workspace solve (no per-walk records are kept) with
 * slices as large as the array allows (at most params->slice_walks when that
 * is set), and gives the results of fk_solve_potential / fk_solve_gz bit for
 * bit.  The array holds every (station, chunk) pair's 48-byte partial, so a
 * solve with more than about 1.38 million pairs (n_stations *
 * ceil(N / 8192)) is rejected with FK_EUNSUPPORTED before anything is
 * launched.  Every call on a GPU uses the same array: calls that overlap on
 * one GPU (on different streams, or from several threads) race and must not
 * be issued; each call clears the claim counters it needs.  The status word
 * of fk_workspace_status is not reachable for these solves; fk_stat.n_trunc
 * and NaN means carry the same information. */
fk_status fk_solve_static(int32_t kind, const double *stations, int64_t n_stations, const fk_box *box,
                          const fk_source *source, const fk_boundary *bc, const fk_params *params,
                          fk_stat *out, void *hip_stream);

/* Batched solve (one persistent launch): n_problems independent problems --
 * each with its own stations (DEVICE), box, density, boundary data and
 * parameters -- share one work queue, so problems of very different cost keep
 * the whole GPU busy until the last walk.  All problems must use the same
 * precision.  Problem m writes its n_stations results to out[out_offset ...]
 * (DEVICE; ranges of different problems must not overlap).  The problem
 * descriptors are uploaded into the workspace by kernels that carry them in
 * their arguments, so the call can be captured into a HIP graph and replayed;
 * a replay re-solves the problems as they were at capture time.  Each
 * problem's results equal those of the same problem solved alone, bit for
 * bit.  Host arrays of the problems are read before the call returns. */
size_t fk_batch_workspace_bytes(const fk_problem *problems, int32_t n_problems);

/* Offsets (bytes from the workspace start) of problem m's per-walk values and
 * step counts after fk_solve_batch, laid out as in fk_workspace_layout.
 * Record mode only.  A batch's slice_walks (the same for every problem) works
 * as for a single solve: slices are runs of whole (station, chunk) pairs of
 * the problems in order. */
fk_status fk_batch_layout(const fk_problem *problems, int32_t n_problems, int32_t m, size_t *values_offset,
                          size_t *steps_offset);

fk_status fk_solve_batch(const fk_problem *problems, int32_t n_problems, fk_stat *out, void *workspace,
                         size_t workspace_bytes, void *hip_stream);

/* Adjoint: the vector-Jacobian product of a forward solve with respect to the
 * voxel densities, grad_rho[v] = sum_s grad_out[s] * d mean_s / d rho_v.
 * For fixed random streams every walk is independent of rho, and its sample
 * is affine in rho: u_p = g(x_e) - 2 pi G (dt/2) (S_bodies + sum_v rho_v c_pv),
 * where c_pv counts the trapezoid weights of voxel v along walk p (one per
 * step end inside v).  The adjoint replays exactly the forward walks (same
 * streams, same stepping code), accumulates integer weights per station and
 * voxel (signed +/- for the two walks of a g_z pair), and combines
 *   d mean_s / d rho_v = -2 pi G (dt/2) C_sv / n_s        (potential)
 *   d mean_s / d rho_v = -2 pi G (dt/2) C_sv / (2 h n_s)  (g_z)
 * in a fixed order, so the result is deterministic.  The boundary data is held
 * fixed (it does not depend on rho).
 *   forward_out, forward_workspace: DEVICE results and workspace of the forward
 *     solve with the same arguments, run in record mode (slice_walks = 0;
 *     walks capped there are skipped here);
 *   grad_out: DEVICE, n_stations doubles; grad_rho: DEVICE, one double per
 *     voxel, overwritten; workspace: DEVICE, fk_adjoint_workspace_bytes().
 * The source must have a voxel grid. */
size_t fk_adjoint_workspace_bytes(int64_t n_stations, const fk_source *source);

fk_status fk_potential_adjoint(const double *stations, int64_t n_stations, const fk_box *box,
                               const fk_source *source, const fk_boundary *bc, const fk_params *params,
                               const fk_stat *forward_out, const void *forward_workspace,
                               size_t forward_workspace_bytes, const double *grad_out, double *grad_rho,
                               void *workspace, size_t workspace_bytes, void *hip_stream);

fk_status fk_gz_adjoint(const double *stations, int64_t n_stations, const fk_box *box, const fk_source *source,
                        const fk_boundary *bc, const fk_params *params, const fk_stat *forward_out,
                        const void *forward_workspace, size_t forward_workspace_bytes, const double *grad_out,
                        double *grad_rho, void *workspace, size_t workspace_bytes, void *hip_stream);

/* Diagnostic: the random stream exactly as the walk kernels compute it.  For
 * n_items Philox counters (DEVICE, 4 uint32 words each: block k, path p,
 * station s, problem m) and the key taken from seed, writes (each output
 * DEVICE and nullable) the Philox4x32-10 words (4 per item), the two normals
 * of the FP64 stream and the four normals of the mixed-precision stream that
 * the block yields. */
fk_status fk_stream_blocks(const uint32_t *counters, int64_t n_items, uint64_t seed, uint32_t *words,
                           double *normals_f64, float *normals_f32, void *hip_stream);

/* Merges per-station results of two disjoint walk ranges of the same
 * stations (e.g. path_offset ranges run separately, on one GPU or several):
 * the sample mean of eq. 11 and the unbiased variance of the union (Chan's
 * pairwise update), its standard error, and the summed step tallies.  a, b,
 * out: HOST arrays of n fk_stat (out may alias a or b). */
fk_status fk_merge_stats(const fk_stat *a, const fk_stat *b, int64_t n, fk_stat *out);

/* Moving-average smoothing of a station profile (paper section 4.1): value k
 * is replaced by the mean of the values in the widest window of at most
 * `span` (odd) points centred on k that fits in the profile, so the window
 * shrinks symmetrically near the ends.  With standard errors se (HOST,
 * nullable) of independent stations, out_se[k] = sqrt(sum se_j^2) / w.  All
 * arrays HOST, length n. */
fk_status fk_moving_average(const double *values, const double *se, int64_t n, int32_t span, double *out_values,
                            double *out_se);

/* Launch settings of the walk kernels (the autotuner's knobs).  block: threads
 * per block (64..256, multiple of 64); blocks_per_cu: resident blocks per
 * compute unit (0 = as many as fit); grab: largest number of walks a
 * wavefront takes from the global queue at once (1..64); adjoint_table: how
 * the adjoint gathers its occupation weights in LDS before they reach the
 * global counts -- 0: a dense per-station table when the grid has at most
 * 32768 voxels (1024-thread blocks working through the stations one at a
 * time), else the hashed block table; 1: the hashed block table always;
 * stripes: claim counters the task queue is split into, each a contiguous
 * run of tasks that blocks b = s mod stripes start on (1..32; 0 = 8 for
 * batches of problems with separate sources, 1 otherwise); refill_cost: the
 * start-up cost R of a wavefront's walk refill, as 128 R macro-steps (a
 * wavefront waits for k idle lanes, the smallest k with k (k + 1) >= 128 R
 * times its walk-end rate per macro-step; 1..8192; 0 = 64).  Settings never
 * change results. */
typedef struct {
    int32_t block;
    int32_t blocks_per_cu;
    int32_t grab;
    int32_t adjoint_table;
    int32_t stripes;
    int32_t refill_cost;
} fk_launch;

fk_status fk_set_launch(int32_t precision, const fk_launch *launch);

/* Autotuner: solves the given problem (kind 0 = potential, 1 = g_z; same
 * arguments as fk_solve_potential) once untimed and once timed with HIP
 * events for every candidate launch setting -- block 64/128/256 threads,
 * resident blocks per CU at the occupancy limit or half of it, queue runs of
 * 16/32/64 walks -- installs the fastest for params->precision (as
 * fk_set_launch) and returns it in *best (and its time in *best_ms,
 * nullable).  Every setting gives the same results bit for bit; only the
 * time differs.  Waits for the stream.  Tune on a reduced walk count of the
 * target workload: a call runs 36 solves. */
fk_status fk_autotune(int32_t kind, const double *stations, int64_t n_stations, const fk_box *box,
                      const fk_source *source, const fk_boundary *bc, const fk_params *params, fk_stat *out,
                      void *workspace, size_t workspace_bytes, void *hip_stream, fk_launch *best, double *best_ms);
fk_status fk_get_launch(int32_t precision, fk_launch *launch);

/* Kernel timing (tracing aid).  fk_timing_enable(1) makes every later solve
 * on the calling thread record a pair of HIP events on its stream right before
 * and right after its walk kernel (at most 256 pairs are kept; older ones are
 * dropped).  fk_timing_read waits for the recorded pairs, writes up to max_n
 * elapsed times in milliseconds (launch order) to ms_out, their count to
 * *n_out, and forgets them.  fk_timing_enable(0) stops recording. */
fk_status fk_timing_enable(int32_t on);
fk_status fk_timing_read(double *ms_out, int32_t max_n, int32_t *n_out);

/* Human-readable text of a status code, and the message of the calling
 * thread's last failed call (empty if none). */
const char *fk_status_string(int32_t status);
const char *fk_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t fk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FKGRAV_H */
