// fk_api.cpp -- host runtime behind the C interface of fkgrav.h: argument
// checks, workspace layout, launch planning and the enqueueing of the walk
// and reduction kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fk_internal.hpp"

namespace {

thread_local std::string g_last_error;

fk_status fail(fk_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fk_status fail(fk_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

constexpr int64_t kChunk = 8192;             // samples per reduction partial
constexpr int64_t kMaxPathIndex = 1ll << 32; // the path word of the counter is 32 bits

std::mutex g_mu;

// Walk-kernel timing: per-thread event pairs recorded around walk launches.
struct Timing {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spare;
    ~Timing()
    {
        for (auto& p : pending) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
        for (auto& p : spare) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
    }
};
thread_local Timing g_timing;
constexpr size_t kMaxTimed = 256;

bool timing_pair(std::pair<hipEvent_t, hipEvent_t>* out)
{
    if (!g_timing.spare.empty()) {
        *out = g_timing.spare.back();
        g_timing.spare.pop_back();
        return true;
    }
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) return false;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return false;
    }
    *out = {a, b};
    return true;
}
fk_launch g_launch[3] = {{256, 0, 32, 0, 0, 0}, {256, 0, 32, 0, 0, 0}, {256, 0, 32, 0, 0, 0}};

int g_cus[64] = {0};

int compute_units(int dev)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev < 0 || dev >= 64) return 0;
    if (g_cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        g_cus[dev] = n;
    }
    return g_cus[dev];
}

bool timing_begin(std::pair<hipEvent_t, hipEvent_t>* ev, hipStream_t stream)
{
    if (!g_timing.on || !timing_pair(ev)) return false;
    (void)hipEventRecord(ev->first, stream);
    return true;
}

void timing_end(const std::pair<hipEvent_t, hipEvent_t>& ev, hipStream_t stream)
{
    (void)hipEventRecord(ev.second, stream);
    if (g_timing.pending.size() >= kMaxTimed) {
        g_timing.spare.push_back(g_timing.pending.front());
        g_timing.pending.erase(g_timing.pending.begin());
    }
    g_timing.pending.push_back(ev);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of a single solve (256-byte aligned regions):
//   status    the status word (FK_FLAG_* bits) in a 256-byte block
//   values    per-walk samples, record mode only (8 B per task)
//   steps     step counts of the records held at once (4 B each)
//   exits     exit records of the records held at once (32 B each)
//   partials  one Partial per (station, chunk) pair
//   queue     the claim counters
// Record mode holds every task's record; a bounded workspace holds the
// records of one slice (at most slice_walks tasks).
struct Layout {
    int64_t n_tasks;
    int64_t n_chunks;
    int64_t n_pairs;
    int64_t held;            // records held at once
    bool records;            // record mode
    size_t status, values, steps, exits, partials, queue, total;
};

constexpr size_t kStatusBytes = 256;

bool is_finite(double v) { return std::isfinite(v); }

fk_status check_params(int32_t kind, int64_t n_stations, const fk_params* p)
{
    if (kind != 0 && kind != 1) return fail(FK_EINVAL, "kind must be 0 (potential) or 1 (g_z), got %d", kind);
    if (!p) return fail(FK_EINVAL, "params is NULL");
    if (n_stations < 0) return fail(FK_EINVAL, "n_stations < 0");
    if (p->paths_per_station < 2) return fail(FK_EINVAL, "paths_per_station must be >= 2");
    if (p->path_offset < 0 || p->path_offset + p->paths_per_station > kMaxPathIndex)
        return fail(FK_EUNSUPPORTED, "path_offset + paths_per_station must lie in [0, 2^32]");
    if (!(is_finite(p->dt) && p->dt > 0.0)) return fail(FK_EINVAL, "dt must be finite and > 0");
    if (!is_finite(p->G)) return fail(FK_EINVAL, "G must be finite");
    if (!(is_finite(p->h) && p->h >= 0.0)) return fail(FK_EINVAL, "h must be finite and >= 0");
    if (p->precision < 0 || p->precision > 2) return fail(FK_EINVAL, "unknown precision %d", p->precision);
    if (p->exit_rule < 0 || p->exit_rule > 2) return fail(FK_EINVAL, "unknown exit_rule %d", p->exit_rule);
    if (p->exit_rule == FK_EXIT_BRIDGE && p->max_steps > (1ll << 30))
        return fail(FK_EUNSUPPORTED, "the bridge exit test needs max_steps <= 2^30");
    if (p->pairing < 0 || p->pairing > 1) return fail(FK_EINVAL, "unknown pairing %d", p->pairing);
    if (p->domain != FK_DOMAIN_BOX && p->domain != FK_DOMAIN_BALL) return fail(FK_EINVAL, "unknown domain %d", p->domain);
    if (p->max_steps < 1 || p->max_steps > 0x7fffffffll) return fail(FK_EINVAL, "max_steps must lie in [1, 2^31-1]");
    const int64_t npair = kind == 1 ? 2 : 1;
    if (n_stations > 0 && p->paths_per_station > (INT64_MAX / 16) / (npair * n_stations))
        return fail(FK_EUNSUPPORTED, "n_stations * paths_per_station too large");
    if (kind == 1 && p->pairing == FK_PAIR_INDEPENDENT && n_stations > (1ll << 31))
        return fail(FK_EUNSUPPORTED, "independent pairing needs 2 * n_stations < 2^32");
    if (n_stations > (1ll << 32)) return fail(FK_EUNSUPPORTED, "n_stations must be < 2^32");
    if (p->slice_walks < 0) return fail(FK_EINVAL, "slice_walks must be >= 0");
    if (p->slice_walks > 0 && p->slice_walks < kChunk * npair)
        return fail(FK_EINVAL, "slice_walks must be 0 or at least %lld (8192 per walk of a pair)",
                    (long long)(kChunk * npair));
    const int64_t n_chunks = (p->paths_per_station + kChunk - 1) / kChunk;
    if (n_stations > 0 && n_chunks > ((1ll << 31) - 1) / n_stations)
        return fail(FK_EUNSUPPORTED, "n_stations * ceil(paths_per_station / 8192) must be < 2^31");
    return FK_OK;
}

// slice_walks: 0 = record mode, else the bound on the records held at once.
Layout make_layout(int32_t kind, int64_t n_stations, const fk_params* p, int64_t slice_walks)
{
    Layout L{};
    L.n_tasks = n_stations * p->paths_per_station * (kind == 1 ? 2 : 1);
    L.n_chunks = (p->paths_per_station + kChunk - 1) / kChunk;
    L.n_pairs = n_stations * L.n_chunks;
    L.records = slice_walks == 0;
    L.held = L.records ? L.n_tasks : std::min(L.n_tasks, slice_walks);
    L.status = 0;
    L.values = kStatusBytes;
    L.steps = align256(L.values + (L.records ? sizeof(double) * (size_t)L.n_tasks : 0));
    L.exits = align256(L.steps + sizeof(uint32_t) * (size_t)L.held);
    L.partials = align256(L.exits + sizeof(fk::ExitRecord) * (size_t)L.held);
    L.queue = align256(L.partials + sizeof(fk::Partial) * (size_t)L.n_pairs);
    L.total = align256(L.queue + 256);
    return L;
}

Layout make_layout(int32_t kind, int64_t n_stations, const fk_params* p)
{
    return make_layout(kind, n_stations, p, p->slice_walks);
}

// A slice: the tasks [t0, t1) and the (station, chunk) pairs [q0, q1) they
// make up, numbered across the problems of a solve in order.
struct Slice {
    int64_t t0, t1, q0, q1;
};

// One problem's shape: stations, walks per station and pair, chunks per
// station.
struct Shape {
    int64_t S, N, npair, n_chunks;
};

// Cuts the tasks of the problems into slices of at most `budget` tasks
// (budget >= kChunk * npair of every problem), each a run of whole
// (station, chunk) pairs, and calls fn(slice) on each in order until fn
// returns an error.  Stations that fit go into a slice whole, as many as fit;
// a station larger than the budget is cut into runs of chunks.
template <class F>
fk_status for_each_slice(const std::vector<Shape>& shapes, int64_t budget, F&& fn)
{
    Slice cur{0, 0, 0, 0};
    fk_status st = FK_OK;
    auto close = [&]() {
        if (cur.t1 > cur.t0 && st == FK_OK) st = fn(cur);
        cur = Slice{cur.t1, cur.t1, cur.q1, cur.q1};
    };
    for (const Shape& p : shapes) {
        if (p.S == 0) continue;
        const int64_t per_station = p.N * p.npair;
        if (per_station <= budget) {
            int64_t s = 0;
            while (s < p.S && st == FK_OK) {
                const int64_t k = std::min(p.S - s, (budget - (cur.t1 - cur.t0)) / per_station);
                if (k == 0) {
                    close();
                    continue;
                }
                cur.t1 += k * per_station;
                cur.q1 += k * p.n_chunks;
                s += k;
            }
        } else {
            close();
            const int64_t run = budget / (kChunk * p.npair);
            if (run < 1) return fail(FK_EINVAL, "a slice must hold one chunk of 8192 paths per walk of a pair");
            for (int64_t s = 0; s < p.S && st == FK_OK; ++s)
                for (int64_t c0 = 0; c0 < p.n_chunks && st == FK_OK; c0 += run) {
                    const int64_t c1 = std::min(p.n_chunks, c0 + run);
                    const int64_t i1 = std::min(p.N, c1 * kChunk);
                    cur.t1 = cur.t0 + (i1 - c0 * kChunk) * p.npair;
                    cur.q1 = cur.q0 + (c1 - c0);
                    close();
                }
        }
        if (st != FK_OK) return st;
    }
    close();
    return st;
}

fk_status check_box(const fk_box* b)
{
    if (!b) return fail(FK_EINVAL, "box is NULL");
    for (int c = 0; c < 3; ++c) {
        if (!is_finite(b->lo[c]) || !is_finite(b->hi[c])) return fail(FK_EINVAL, "box bounds must be finite");
        if (!(b->lo[c] < b->hi[c])) return fail(FK_EINVAL, "box lo[%d] must be < hi[%d]", c, c);
    }
    return FK_OK;
}

// The ball domain is the ball inscribed in a cubic box; face-grid data is
// defined on box faces only.
fk_status check_domain(const fk_box* b, const fk_params* p, const fk_boundary* bc)
{
    if (p->domain != FK_DOMAIN_BALL) return FK_OK;
    const double w = b->hi[0] - b->lo[0];
    for (int c = 1; c < 3; ++c)
        if (std::fabs((b->hi[c] - b->lo[c]) - w) > 1e-12 * w)
            return fail(FK_EINVAL, "a ball domain needs a cubic box (edge %d differs)", c);
    if (bc && bc->kind == FK_BC_FACE_GRID) return fail(FK_EUNSUPPORTED, "face-grid data needs a box domain");
    return FK_OK;
}

// Ball centre and squared radius, computed as the oracle defines them.
void ball_of(const fk_box* b, double c[3], double* r2)
{
    for (int k = 0; k < 3; ++k) c[k] = 0.5 * (b->lo[k] + b->hi[k]);
    const double r = 0.5 * (b->hi[0] - b->lo[0]);
    *r2 = r * r;
}

double dist2(const double x[3], const double c[3])
{
    const double d0 = x[0] - c[0], d1 = x[1] - c[1], d2 = x[2] - c[2];
    return std::fma(d0, d0, std::fma(d1, d1, d2 * d2));
}

fk_status check_source(const fk_source* s)
{
    if (!s) return fail(FK_EINVAL, "source is NULL");
    if (s->rho && s->rho_index) return fail(FK_EINVAL, "give the grid as rho or as rho_index, not both");
    if (s->rho_index && !s->rho_levels) return fail(FK_EINVAL, "rho_levels is NULL (rho_index needs 256 levels)");
    if (s->rho || s->rho_index) {
        int64_t nv = 1;
        for (int c = 0; c < 3; ++c) {
            if (s->n[c] < 1) return fail(FK_EINVAL, "grid size n[%d] must be >= 1", c);
            if (s->n[c] >= (1 << 24)) return fail(FK_EUNSUPPORTED, "grid size n[%d] must be < 2^24", c);
            if (!(is_finite(s->spacing[c]) && s->spacing[c] > 0.0)) return fail(FK_EINVAL, "grid spacing must be > 0");
            if (!is_finite(s->origin[c])) return fail(FK_EINVAL, "grid origin must be finite");
            nv *= s->n[c];
        }
        if (nv > (1ll << 31) - 1) return fail(FK_EUNSUPPORTED, "grid has more than 2^31-1 voxels");
    }
    if (s->n_prisms < 0 || s->n_prisms > FK_MAX_PRISMS)
        return fail(FK_EUNSUPPORTED, "n_prisms must lie in [0, %d]", FK_MAX_PRISMS);
    if (s->n_spheres < 0 || s->n_spheres > FK_MAX_SPHERES)
        return fail(FK_EUNSUPPORTED, "n_spheres must lie in [0, %d]", FK_MAX_SPHERES);
    if (s->n_prisms > 0 && !s->prisms) return fail(FK_EINVAL, "prisms is NULL");
    if (s->n_spheres > 0 && !s->spheres) return fail(FK_EINVAL, "spheres is NULL");
    for (int j = 0; j < s->n_prisms * 7; ++j)
        if (!is_finite(s->prisms[j])) return fail(FK_EINVAL, "prism rows must be finite");
    for (int j = 0; j < s->n_spheres * 5; ++j)
        if (!is_finite(s->spheres[j])) return fail(FK_EINVAL, "sphere rows must be finite");
    return FK_OK;
}

fk_status check_bc(const fk_boundary* bc)
{
    if (!bc) return fail(FK_EINVAL, "bc is NULL");
    switch (bc->kind) {
    case FK_BC_ZERO:
        return FK_OK;
    case FK_BC_QUADRATIC:
        if (!bc->data) return fail(FK_EINVAL, "quadratic data is NULL");
        for (int j = 0; j < 10; ++j)
            if (!is_finite(bc->data[j])) return fail(FK_EINVAL, "quadratic coefficients must be finite");
        return FK_OK;
    case FK_BC_POINT_MASSES:
    case FK_BC_PRISMS: {
        if (bc->n_items < 1 || bc->n_items > FK_MAX_BC_ITEMS)
            return fail(FK_EUNSUPPORTED, "boundary rows must lie in [1, %d]", FK_MAX_BC_ITEMS);
        if (!bc->data) return fail(FK_EINVAL, "boundary data is NULL");
        const int w = bc->kind == FK_BC_PRISMS ? 7 : 4;
        for (int64_t j = 0; j < bc->n_items * w; ++j)
            if (!is_finite(bc->data[j])) return fail(FK_EINVAL, "boundary rows must be finite");
        return FK_OK;
    }
    case FK_BC_FACE_GRID:
        if (!bc->data) return fail(FK_EINVAL, "face grid data is NULL");
        for (int f = 0; f < 6; ++f)
            if (bc->face_n[f][0] < 2 || bc->face_n[f][1] < 2)
                return fail(FK_EINVAL, "face grids need at least 2 x 2 nodes (face %d)", f);
        return FK_OK;
    default:
        return fail(FK_EINVAL, "unknown boundary kind %d", bc->kind);
    }
}

bool power_of_two(double v)
{
    int e = 0;
    return std::frexp(v, &e) == 0.5;
}

void fill_common(fk::WalkCommon& C, int32_t kind, const double* stations, int64_t n_stations, const fk_box* box,
                 const fk_params* p, const Layout& L, char* ws)
{
    std::memset(&C, 0, sizeof C);
    C.stations = stations;
    if (ws) {
        C.exits = reinterpret_cast<fk::ExitRecord*>(ws + L.exits);
        C.steps = reinterpret_cast<uint32_t*>(ws + L.steps);
        C.queue = reinterpret_cast<unsigned long long*>(ws + L.queue);
    }
    C.n_stations = n_stations;
    C.N = p->paths_per_station;
    C.n_tasks = L.n_tasks;
    C.task0 = 0;
    C.path_offset = p->path_offset;
    C.max_steps = p->max_steps;
    for (int c = 0; c < 3; ++c) {
        C.lo[c] = box->lo[c];
        C.hi[c] = box->hi[c];
        C.lo_f[c] = (float)box->lo[c];
        C.hi_f[c] = (float)box->hi[c];
    }
    C.sdt = std::sqrt(p->dt);
    C.sdt_f = (float)C.sdt;
    C.w = 2.0 * M_PI * p->G * (0.5 * p->dt);
    C.G = p->G;
    C.h = p->h > 0.0 ? p->h : std::sqrt(p->dt);
    C.key0 = (uint32_t)(p->seed & 0xffffffffull);
    C.key1 = (uint32_t)(p->seed >> 32);
    C.problem_id = p->problem_id;
    C.npair = kind == 1 ? 2 : 1;
    C.pairing = p->pairing;
    C.exit_rule = p->exit_rule;
    C.domain = p->domain;
    C.dt = p->dt;
    C.dt_f = (float)p->dt;
    // Bridge stops are skipped when both step ends lie delta = sqrt(K dt)
    // inside every face: then each crossing probability is below exp(-2K)
    // and their sum below the smallest uniform (2^-53 with K = 20 for the
    // FP64 stream, 2^-24 with K = 10 for the FP32 one), so no stop is lost.
    C.delta = std::sqrt((p->precision == FK_F64 ? 20.0 : 10.0) * p->dt);
    C.delta_f = (float)C.delta;
    if (p->domain == FK_DOMAIN_BALL) {
        ball_of(box, C.ctr, &C.r2);
        C.R = std::sqrt(C.r2);
        C.deep2 = C.delta < C.R ? (C.R - C.delta) * (C.R - C.delta) : -1.0;
        for (int c = 0; c < 3; ++c) C.ctr_f[c] = (float)C.ctr[c];
        C.r2_f = (float)C.r2;
        C.R_f = (float)C.R;
        C.deep2_f = C.delta_f < C.R_f ? (C.R_f - C.delta_f) * (C.R_f - C.delta_f) : -1.0f;
    }
}

void fill_bc(fk::BoundaryArgs& B, const fk_boundary* bc)
{
    std::memset(&B, 0, sizeof B);
    B.kind = bc->kind;
    if (bc->kind == FK_BC_QUADRATIC) {
        for (int j = 0; j < 10; ++j) B.quad[j] = bc->data[j];
    } else if (bc->kind == FK_BC_POINT_MASSES || bc->kind == FK_BC_PRISMS) {
        const int w = bc->kind == FK_BC_PRISMS ? 7 : 4;
        B.n_items = (int32_t)bc->n_items;
        for (int64_t j = 0; j < bc->n_items; ++j)
            for (int c = 0; c < w; ++c) B.items[j][c] = bc->data[j * w + c];
    } else if (bc->kind == FK_BC_FACE_GRID) {
        B.face_data = bc->data;
        int64_t off = 0;
        for (int f = 0; f < 6; ++f) {
            B.face_n[f][0] = bc->face_n[f][0];
            B.face_n[f][1] = bc->face_n[f][1];
            B.face_off[f] = off;
            off += (int64_t)bc->face_n[f][0] * bc->face_n[f][1];
        }
    }
}

// Whether the source has a voxel grid (as FP32 densities or by levels).
bool has_grid(const fk_source* s) { return s && (s->rho || s->rho_index); }

void fill_source_f64(fk::SourceF64& S, const fk_source* s)
{
    std::memset(&S, 0, sizeof S);
    const bool grid = has_grid(s);
    S.rho = s->rho;
    S.idx = s->rho_index;
    S.levels = s->rho_index ? s->rho_levels : nullptr;
    S.has_grid = grid;
    for (int c = 0; c < 3; ++c) {
        S.n[c] = grid ? s->n[c] : 0;
        S.origin[c] = s->origin[c];
        S.spacing[c] = grid ? s->spacing[c] : 1.0;
        S.inv[c] = 1.0 / S.spacing[c];
        S.exact[c] = power_of_two(S.spacing[c]);
    }
    S.nxy = grid ? (uint32_t)((int64_t)S.n[0] * S.n[1]) : 0u;
    S.n_prisms = s->n_prisms;
    S.n_spheres = s->n_spheres;
    for (int j = 0; j < s->n_prisms; ++j)
        for (int c = 0; c < 7; ++c) S.prisms[j][c] = s->prisms[7 * j + c];
    for (int j = 0; j < s->n_spheres; ++j)
        for (int c = 0; c < 5; ++c) S.spheres[j][c] = s->spheres[5 * j + c];
}

void fill_source_f32(fk::SourceF32& S, const fk_source* s)
{
    std::memset(&S, 0, sizeof S);
    const bool grid = has_grid(s);
    S.rho = s->rho;
    S.idx = s->rho_index;
    S.levels = s->rho_index ? s->rho_levels : nullptr;
    S.has_grid = grid;
    for (int c = 0; c < 3; ++c) {
        S.n[c] = grid ? s->n[c] : 0;
        S.ob[c] = grid ? (float)(-s->origin[c] / s->spacing[c]) : 0.0f;
        S.inv[c] = grid ? (float)(1.0 / s->spacing[c]) : 1.0f;
    }
    S.nxy = grid ? (uint32_t)((int64_t)S.n[0] * S.n[1]) : 0u;
    S.n_prisms = s->n_prisms;
    S.n_spheres = s->n_spheres;
    for (int j = 0; j < s->n_prisms; ++j)
        for (int c = 0; c < 7; ++c) S.prisms[j][c] = (float)s->prisms[7 * j + c];
    for (int j = 0; j < s->n_spheres; ++j)
        for (int c = 0; c < 5; ++c) S.spheres[j][c] = (float)s->spheres[5 * j + c];
}

// The stepping loop a problem needs: 0 box, 1 ball exit test, 2 bridge test;
// plus 4 when its source has a voxel grid (the loop then loads grid values
// ahead), and 8 more when that grid is given by levels.  A batch takes the
// most general exit test and the grid bits of any (its grids must all be of
// one kind, which check_batch ensures).
int loop_kind(const fk_params* p, const fk_source* s)
{
    const int e = p->exit_rule == FK_EXIT_BRIDGE ? 2 : p->domain == FK_DOMAIN_BALL ? 1 : 0;
    return e | (has_grid(s) ? 4 : 0) | (s && s->rho_index ? 8 : 0);
}

int merge_loops(int a, int b)
{
    return std::max(a & 3, b & 3) | ((a | b) & 12);
}

fk_status plan_launch(int precision, int64_t n_tasks, fk::LaunchCfg* cfg, bool batch = false, int loop = 0,
                      bool shared = false, bool adjoint = false, bool ukey = false)
{
    fk_launch l;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        l = g_launch[precision];
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FK_EDEVICE, "hipGetDevice failed");
    const int cus = compute_units(dev);
    if (cus <= 0) return fail(FK_EDEVICE, "could not query the compute-unit count");
    int bpc = l.blocks_per_cu;
    if (bpc <= 0) {
        const hipError_t oe = batch ? fk::batch_occupancy(precision, l.block, &bpc, loop, shared, ukey)
                                    : fk::walk_occupancy(precision, l.block, &bpc, loop, adjoint);
        if (oe != hipSuccess || bpc <= 0)
            return fail(FK_EDEVICE, "occupancy query failed for block %d", l.block);
    }
    int64_t grid = (int64_t)cus * bpc;
    const int64_t need = (n_tasks + l.block - 1) / l.block;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    cfg->block = l.block;
    cfg->grid = (int)grid;
    cfg->grab = l.grab;
    // claim counters: by default 8 (one run of tasks per XCD) for batches
    // whose problems have separate sources, else one
    cfg->stripes = l.stripes > 0 ? (uint32_t)l.stripes : (batch && !shared ? 8u : 1u);
    cfg->refill_cost = l.refill_cost > 0 ? (uint32_t)l.refill_cost : 64u;
    return FK_OK;
}

// Checks every argument of a single solve except the workspace.
fk_status check_solve(int32_t kind, const double* stations, int64_t n_stations, const fk_box* box,
                      const fk_source* src, const fk_boundary* bc, const fk_params* p, const fk_stat* out)
{
    fk_status st;
    if ((st = check_params(kind, n_stations, p)) != FK_OK) return st;
    if ((st = check_box(box)) != FK_OK) return st;
    if ((st = check_source(src)) != FK_OK) return st;
    if ((st = check_bc(bc)) != FK_OK) return st;
    if ((st = check_domain(box, p, bc)) != FK_OK) return st;
    if (n_stations == 0) return FK_OK;
    if (!stations) return fail(FK_EINVAL, "stations is NULL");
    if (!out) return fail(FK_EINVAL, "out is NULL");
    return FK_OK;
}

// Enqueues a checked single solve in the workspace ws laid out as L: the
// status word set, then per slice the walks and the partials of its pairs,
// then the station results.  timing: the walk launches may be event-timed.
fk_status run_solve(int32_t kind, const double* stations, int64_t n_stations, const fk_box* box, const fk_source* src,
                    const fk_boundary* bc, const fk_params* p, fk_stat* out, char* ws, const Layout& L,
                    hipStream_t stream, bool timing)
{
    fk::WalkCommon C;
    fill_common(C, kind, stations, n_stations, box, p, L, ws);
    fk::WalkArgsF64 A64;
    fk::WalkArgsF32 A32;
    if (p->precision == FK_F64) fill_source_f64(A64.src, src);
    else fill_source_f32(A32.src, src);
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + L.status);

    fk::ReduceArgs R;
    std::memset(&R, 0, sizeof R);
    R.exits = C.exits;
    R.values = L.records ? reinterpret_cast<double*>(ws + L.values) : nullptr;
    R.steps = C.steps;
    R.partials = reinterpret_cast<fk::Partial*>(ws + L.partials);
    R.out = out;
    R.status = status;
    R.n_stations = n_stations;
    R.N = p->paths_per_station;
    R.chunk = kChunk;
    R.n_chunks = L.n_chunks;
    R.npair = C.npair;
    R.two_h = 2.0 * C.h;
    R.w = C.w;
    R.G = C.G;
    for (int c = 0; c < 3; ++c) {
        R.lo[c] = C.lo[c];
        R.hi[c] = C.hi[c];
    }
    fill_bc(R.bc, bc);

    const int loop = loop_kind(p, src);
    bool first = true;
    const std::vector<Shape> shapes{Shape{n_stations, p->paths_per_station, C.npair, L.n_chunks}};
    fk_status st = for_each_slice(shapes, L.held, [&](const Slice& sl) -> fk_status {
        hipError_t e = first ? fk::launch_zero_queue(C.queue, stream, status, p->strict ? FK_FLAG_STRICT : 0u)
                             : fk::launch_zero_queue(C.queue, stream);
        first = false;
        if (e != hipSuccess) return fail(FK_EDEVICE, "queue reset launch failed: %s", hipGetErrorString(e));
        fk::LaunchCfg cfg;
        fk_status ps = plan_launch(p->precision, sl.t1 - sl.t0, &cfg, false, loop);
        if (ps != FK_OK) return ps;
        C.task0 = sl.t0;
        C.n_tasks = sl.t1 - sl.t0;
        C.grab = cfg.grab;
        C.total_waves = (uint32_t)((int64_t)cfg.grid * cfg.block / 64);
        C.stripes = cfg.stripes;
        C.refill_cost = cfg.refill_cost;
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        const bool timed = timing && timing_begin(&ev, stream);
        if (p->precision == FK_F64) {
            A64.c = C;
            e = fk::launch_walk_f64(A64, cfg, stream);
        } else {
            A32.c = C;
            e = fk::launch_walk_f32(A32, p->precision == FK_MIXED_KAHAN, cfg, stream);
        }
        if (timed) timing_end(ev, stream);
        if (e != hipSuccess) return fail(FK_EDEVICE, "walk launch failed: %s", hipGetErrorString(e));
        R.q0 = sl.q0;
        R.task0 = sl.t0;
        e = fk::launch_reduce(R, sl.q1 - sl.q0, false, stream);
        if (e != hipSuccess) return fail(FK_EDEVICE, "reduction launch failed: %s", hipGetErrorString(e));
        return FK_OK;
    });
    if (st != FK_OK) return st;
    const hipError_t e = fk::launch_reduce(R, 0, true, stream);
    if (e != hipSuccess) return fail(FK_EDEVICE, "reduction launch failed: %s", hipGetErrorString(e));
    return FK_OK;
}

fk_status solve(int32_t kind, const double* stations, int64_t n_stations, const fk_box* box, const fk_source* src,
                const fk_boundary* bc, const fk_params* p, fk_stat* out, void* workspace, size_t workspace_bytes,
                void* hip_stream)
{
    fk_status st = check_solve(kind, stations, n_stations, box, src, bc, p, out);
    if (st != FK_OK || n_stations == 0) return st;
    const Layout L = make_layout(kind, n_stations, p);
    if (!workspace) return fail(FK_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(FK_EWORKSPACE, "workspace must be 256-byte aligned");
    if (workspace_bytes < L.total)
        return fail(FK_EWORKSPACE, "workspace has %zu bytes, %zu needed", workspace_bytes, L.total);
    return run_solve(kind, stations, n_stations, box, src, bc, p, out, static_cast<char*>(workspace), L,
                     reinterpret_cast<hipStream_t>(hip_stream), true);
}

// ---------------------------------------------------------------------------
// Batched solves.
// ---------------------------------------------------------------------------
// Workspace of a batched solve: the status block, the problem descriptors,
// the task and pair prefix sums, one Partial per global pair, the per-walk
// samples by global task (record mode), the records held at once (all tasks,
// or one slice), and the claim counters.
struct BatchLayout {
    size_t status, desc, task_off, block_off, partials, values, steps, exits, queue, total;
    std::vector<Shape> shapes;
    std::vector<int64_t> tasks;    // prefix sums of tasks over the problems
    std::vector<int64_t> pairs;    // prefix sums of (station, chunk) pairs
    int64_t n_tasks = 0, n_pairs = 0, n_stations = 0, held = 0;
    bool records = true;
};

static_assert(sizeof(fk::BatchDesc) % 8 == 0, "descriptor must be whole 64-bit words");

fk_status check_batch(const fk_problem* probs, int32_t n)
{
    if (n < 0 || n > FK_MAX_BATCH) return fail(FK_EUNSUPPORTED, "n_problems must lie in [0, %d]", FK_MAX_BATCH);
    if (n > 0 && !probs) return fail(FK_EINVAL, "problems is NULL");
    fk_status st;
    int64_t pairs = 0;
    int levels_grid = 0;   // 1: the grids seen so far are given by levels, -1: FP32, 0: none yet
    for (int32_t m = 0; m < n; ++m) {
        const fk_problem& P = probs[m];
        if ((st = check_params(P.kind, P.n_stations, &P.params)) != FK_OK) return st;
        if ((st = check_box(&P.box)) != FK_OK) return st;
        if ((st = check_source(&P.source)) != FK_OK) return st;
        if ((st = check_bc(&P.bc)) != FK_OK) return st;
        if ((st = check_domain(&P.box, &P.params, &P.bc)) != FK_OK) return st;
        if (P.n_stations > 0 && !P.stations) return fail(FK_EINVAL, "problem %d: stations is NULL", m);
        if (P.out_offset < 0) return fail(FK_EINVAL, "problem %d: out_offset < 0", m);
        if (P.params.precision != probs[0].params.precision)
            return fail(FK_EINVAL, "problem %d: all problems of a batch need the same precision", m);
        if (P.params.slice_walks != probs[0].params.slice_walks)
            return fail(FK_EINVAL, "problem %d: all problems of a batch need the same slice_walks", m);
        // one kernel instance looks the grids up: all FP32 or all by levels
        if (P.source.rho_index && levels_grid < 0) return fail(FK_EINVAL, "problem %d: a batch's grids must all be "
                                                               "FP32 densities or all given by levels", m);
        if (P.source.rho && levels_grid > 0) return fail(FK_EINVAL, "problem %d: a batch's grids must all be "
                                                        "FP32 densities or all given by levels", m);
        if (P.source.rho_index) levels_grid = 1;
        else if (P.source.rho) levels_grid = -1;
        pairs += P.n_stations * ((P.params.paths_per_station + kChunk - 1) / kChunk);
        if (pairs > (1ll << 31) - 1) return fail(FK_EUNSUPPORTED, "a batch must have fewer than 2^31 (station, chunk) pairs");
    }
    return FK_OK;
}

BatchLayout make_batch_layout(const fk_problem* probs, int32_t n)
{
    BatchLayout B;
    B.tasks.assign(1, 0);
    B.pairs.assign(1, 0);
    for (int32_t m = 0; m < n; ++m) {
        const fk_problem& P = probs[m];
        const int64_t npair = P.kind == 1 ? 2 : 1;
        const int64_t nch = (P.params.paths_per_station + kChunk - 1) / kChunk;
        B.shapes.push_back(Shape{P.n_stations, P.params.paths_per_station, npair, nch});
        B.n_tasks += P.n_stations * P.params.paths_per_station * npair;
        B.n_pairs += P.n_stations * nch;
        B.n_stations += P.n_stations;
        B.tasks.push_back(B.n_tasks);
        B.pairs.push_back(B.n_pairs);
    }
    const int64_t sw = n > 0 ? probs[0].params.slice_walks : 0;
    B.records = sw == 0;
    B.held = B.records ? B.n_tasks : std::min(B.n_tasks, sw);
    B.status = 0;
    B.desc = kStatusBytes;
    B.task_off = align256(B.desc + sizeof(fk::BatchDesc) * (size_t)n);
    B.block_off = align256(B.task_off + sizeof(int64_t) * (size_t)(n + 1));
    B.partials = align256(B.block_off + sizeof(int64_t) * (size_t)(n + 1));
    B.values = align256(B.partials + sizeof(fk::Partial) * (size_t)B.n_pairs);
    B.steps = align256(B.values + (B.records ? sizeof(double) * (size_t)B.n_tasks : 0));
    B.exits = align256(B.steps + sizeof(uint32_t) * (size_t)B.held);
    B.queue = align256(B.exits + sizeof(fk::ExitRecord) * (size_t)B.held);
    B.total = align256(B.queue + 256);
    return B;
}

fk_status solve_batch(const fk_problem* probs, int32_t n, fk_stat* out, void* workspace, size_t workspace_bytes,
                      void* hip_stream)
{
    fk_status st;
    if ((st = check_batch(probs, n)) != FK_OK) return st;
    const BatchLayout BL = make_batch_layout(probs, n);
    if (BL.n_tasks == 0) return FK_OK;
    if (!out) return fail(FK_EINVAL, "out is NULL");
    if (!workspace) return fail(FK_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(FK_EWORKSPACE, "workspace must be 256-byte aligned");
    if (workspace_bytes < BL.total)
        return fail(FK_EWORKSPACE, "workspace has %zu bytes, %zu needed", workspace_bytes, BL.total);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    char* ws = static_cast<char*>(workspace);
    const int precision = probs[0].params.precision;

    int loop = 0;
    bool strict = false;
    for (int32_t m = 0; m < n; ++m) {
        loop = merge_loops(loop, loop_kind(&probs[m].params, &probs[m].source));
        strict = strict || probs[m].params.strict;
    }
    // one source for the whole batch (e.g. u and g_z of one model): the walk
    // kernel then reads it from its arguments instead of per-lane descriptors
    fk::BatchArgs A;
    std::memset(&A, 0, sizeof A);
    bool shared = true;
    if (precision == FK_F64) {
        fill_source_f64(A.src64, &probs[0].source);
        for (int32_t m = 1; m < n && shared; ++m) {
            fk::SourceF64 o;
            fill_source_f64(o, &probs[m].source);
            shared = std::memcmp(&o, &A.src64, sizeof o) == 0;
        }
    } else {
        fill_source_f32(A.src32, &probs[0].source);
        for (int32_t m = 1; m < n && shared; ++m) {
            fk::SourceF32 o;
            fill_source_f32(o, &probs[m].source);
            shared = std::memcmp(&o, &A.src32, sizeof o) == 0;
        }
    }
    // one generator key for the whole batch (the usual case: the problems'
    // streams differ by problem id): the walk kernel holds it in scalar
    // registers
    A.uniform_key = 1;
    for (int32_t m = 1; m < n; ++m)
        if (probs[m].params.seed != probs[0].params.seed) A.uniform_key = 0;
    A.key0 = (uint32_t)(probs[0].params.seed & 0xffffffffull);
    A.key1 = (uint32_t)(probs[0].params.seed >> 32);

    int64_t station_base = 0;
    auto* descs = reinterpret_cast<fk::BatchDesc*>(ws + BL.desc);
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + BL.status);
    auto* queue = reinterpret_cast<unsigned long long*>(ws + BL.queue);
    hipError_t e = fk::launch_zero_queue(queue, stream, status, strict ? FK_FLAG_STRICT : 0u);
    if (e != hipSuccess) return fail(FK_EDEVICE, "queue reset launch failed: %s", hipGetErrorString(e));
    for (int32_t m = 0; m < n; ++m) {
        const fk_problem& P = probs[m];
        const Layout L = make_layout(P.kind, P.n_stations, &P.params, 0);
        fk::BatchDesc D;
        std::memset(&D, 0, sizeof D);
        fill_common(D.c, P.kind, P.stations, P.n_stations, &P.box, &P.params, L, nullptr);
        if (precision == FK_F64) fill_source_f64(D.s64, &P.source);
        else fill_source_f32(D.s32, &P.source);
        fill_bc(D.bc, &P.bc);
        D.out = out + P.out_offset;
        D.n_chunks = L.n_chunks;
        D.task_base = BL.tasks[m];
        D.block_base = BL.pairs[m];
        D.station_base = station_base;
        station_base += P.n_stations;
        e = fk::launch_write_words(reinterpret_cast<uint64_t*>(descs + m), reinterpret_cast<const uint64_t*>(&D),
                                   (int64_t)(sizeof D / 8), stream);
        if (e != hipSuccess) return fail(FK_EDEVICE, "descriptor upload failed: %s", hipGetErrorString(e));
    }
    e = fk::launch_write_words(reinterpret_cast<uint64_t*>(ws + BL.task_off),
                               reinterpret_cast<const uint64_t*>(BL.tasks.data()), n + 1, stream);
    if (e == hipSuccess)
        e = fk::launch_write_words(reinterpret_cast<uint64_t*>(ws + BL.block_off),
                                   reinterpret_cast<const uint64_t*>(BL.pairs.data()), n + 1, stream);
    if (e != hipSuccess) return fail(FK_EDEVICE, "offset upload failed: %s", hipGetErrorString(e));

    A.desc = descs;
    A.task_off = reinterpret_cast<const int64_t*>(ws + BL.task_off);
    A.block_off = reinterpret_cast<const int64_t*>(ws + BL.block_off);
    A.queue = queue;
    A.exits = reinterpret_cast<fk::ExitRecord*>(ws + BL.exits);
    A.steps = reinterpret_cast<uint32_t*>(ws + BL.steps);
    A.values = BL.records ? reinterpret_cast<double*>(ws + BL.values) : nullptr;
    A.partials = reinterpret_cast<fk::Partial*>(ws + BL.partials);
    A.status = status;
    A.n_problems = n;
    A.precision = precision;
    A.chunk = kChunk;

    bool first = true;
    st = for_each_slice(BL.shapes, BL.held, [&](const Slice& sl) -> fk_status {
        hipError_t le = hipSuccess;
        if (!first) le = fk::launch_zero_queue(queue, stream);
        first = false;
        if (le != hipSuccess) return fail(FK_EDEVICE, "queue reset launch failed: %s", hipGetErrorString(le));
        fk::LaunchCfg cfg;
        fk_status ps = plan_launch(precision, sl.t1 - sl.t0, &cfg, true, loop, shared, false, A.uniform_key != 0);
        if (ps != FK_OK) return ps;
        A.task0 = sl.t0;
        A.n_tasks = sl.t1 - sl.t0;
        A.q0 = sl.q0;
        A.grab = cfg.grab;
        A.total_waves = (uint32_t)((int64_t)cfg.grid * cfg.block / 64);
        A.stripes = cfg.stripes;
        A.refill_cost = cfg.refill_cost;
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        const bool timed = timing_begin(&ev, stream);
        le = fk::launch_batch_walk(A, cfg, stream, loop, shared);
        if (timed) timing_end(ev, stream);
        if (le != hipSuccess) return fail(FK_EDEVICE, "batch walk launch failed: %s", hipGetErrorString(le));
        le = fk::launch_batch_chunks(A, sl.q1 - sl.q0, stream);
        if (le != hipSuccess) return fail(FK_EDEVICE, "batch reduction launch failed: %s", hipGetErrorString(le));
        return FK_OK;
    });
    if (st != FK_OK) return st;
    e = fk::launch_batch_stations(A, BL.n_stations, stream);
    if (e != hipSuccess) return fail(FK_EDEVICE, "batch reduction launch failed: %s", hipGetErrorString(e));
    return FK_OK;
}

// ---------------------------------------------------------------------------
// Adjoint (vector-Jacobian product with respect to the voxel densities).
// ---------------------------------------------------------------------------
struct AdjLayout {
    int64_t nvox;
    size_t counts, queue, total;
};

// The counts [S][nvox], then the claim counters: the queue's stripes, or
// one per station for the dense-table instance.
AdjLayout make_adj_layout(int64_t n_stations, const fk_source* src)
{
    AdjLayout A{};
    A.nvox = (int64_t)src->n[0] * src->n[1] * src->n[2];
    A.counts = 0;
    A.queue = align256(sizeof(int64_t) * (size_t)(n_stations * A.nvox));
    A.total = align256(A.queue + std::max<size_t>(256, sizeof(uint64_t) * (size_t)n_stations));
    return A;
}

bool adjoint_dense(int precision, int64_t n_stations, int64_t nvox)
{
    int table = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        table = g_launch[precision].adjoint_table;
    }
    return table == 0 && nvox <= fk::kAdjDenseVoxels && n_stations <= fk::kAdjDenseMaxStations;
}

fk_status adjoint(int32_t kind, const double* stations, int64_t n_stations, const fk_box* box, const fk_source* src,
                  const fk_boundary* bc, const fk_params* p, const fk_stat* fwd_out, const void* fwd_workspace,
                  size_t fwd_workspace_bytes, const double* grad_out, double* grad_rho, void* workspace,
                  size_t workspace_bytes, void* hip_stream)
{
    fk_status st;
    if ((st = check_params(kind, n_stations, p)) != FK_OK) return st;
    if ((st = check_box(box)) != FK_OK) return st;
    if ((st = check_source(src)) != FK_OK) return st;
    if ((st = check_bc(bc)) != FK_OK) return st;
    if ((st = check_domain(box, p, bc)) != FK_OK) return st;
    if (!has_grid(src)) return fail(FK_EINVAL, "the adjoint needs a voxel grid (source.rho and rho_index are NULL)");
    if (p->slice_walks != 0)
        return fail(FK_EINVAL, "the adjoint replays a record-mode forward solve (slice_walks must be 0)");
    if (!grad_rho) return fail(FK_EINVAL, "grad_rho is NULL");
    const AdjLayout AL = make_adj_layout(n_stations, src);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (n_stations == 0) {
        hipError_t e = fk::launch_fill_zero(reinterpret_cast<int64_t*>(grad_rho), AL.nvox, stream);
        return e == hipSuccess ? FK_OK : fail(FK_EDEVICE, "fill launch failed: %s", hipGetErrorString(e));
    }
    if (!stations || !fwd_out || !fwd_workspace || !grad_out) return fail(FK_EINVAL, "NULL input pointer");
    const Layout L = make_layout(kind, n_stations, p);
    if (fwd_workspace_bytes < L.total)
        return fail(FK_EWORKSPACE, "forward workspace has %zu bytes, %zu expected", fwd_workspace_bytes, L.total);
    if (!workspace) return fail(FK_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(FK_EWORKSPACE, "workspace must be 256-byte aligned");
    if (workspace_bytes < AL.total)
        return fail(FK_EWORKSPACE, "workspace has %zu bytes, %zu needed", workspace_bytes, AL.total);
    char* ws = static_cast<char*>(workspace);
    int64_t* counts = reinterpret_cast<int64_t*>(ws + AL.counts);

    fk::LaunchCfg cfg;
    const bool dense = adjoint_dense(p->precision, n_stations, AL.nvox);
    if (dense) {
        // 512-thread blocks, as many as the LDS allows per compute unit
        int dev = 0, bpc = 0;
        if (hipGetDevice(&dev) != hipSuccess) return fail(FK_EDEVICE, "hipGetDevice failed");
        const int cus = compute_units(dev);
        if (fk::walk_occupancy(p->precision, fk::kAdjDenseBlock, &bpc, loop_kind(p, nullptr), true, true) !=
                hipSuccess || bpc <= 0 || cus <= 0)
            return fail(FK_EDEVICE, "occupancy query failed for the dense adjoint");
        fk_launch l;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            l = g_launch[p->precision];
        }
        cfg.block = fk::kAdjDenseBlock;
        cfg.grid = cus * bpc;
        cfg.grab = l.grab;
        cfg.stripes = 1;
        cfg.refill_cost = l.refill_cost > 0 ? (uint32_t)l.refill_cost : 64u;
    } else if ((st = plan_launch(p->precision, L.n_tasks, &cfg, false, loop_kind(p, nullptr), false, true)) != FK_OK) {
        return st;
    }
    fk::WalkCommon C;
    fill_common(C, kind, stations, n_stations, box, p, L, nullptr);
    C.exits = nullptr;
    C.steps = nullptr;
    C.queue = reinterpret_cast<unsigned long long*>(ws + AL.queue);
    C.grab = cfg.grab;
    C.total_waves = (uint32_t)((int64_t)cfg.grid * cfg.block / 64);
    C.stripes = cfg.stripes;
    C.refill_cost = cfg.refill_cost;
    C.counts = counts;
    C.fwd_steps = reinterpret_cast<const uint32_t*>(static_cast<const char*>(fwd_workspace) + L.steps);
    C.nvox = AL.nvox;

    hipError_t e = fk::launch_fill_zero(counts, n_stations * AL.nvox, stream);
    if (e == hipSuccess)
        e = dense ? fk::launch_fill_zero(reinterpret_cast<int64_t*>(C.queue), n_stations, stream)
                  : fk::launch_zero_queue(C.queue, stream);
    if (e != hipSuccess) return fail(FK_EDEVICE, "adjoint set-up launch failed: %s", hipGetErrorString(e));
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    const bool timed = timing_begin(&ev, stream);
    if (p->precision == FK_F64) {
        fk::WalkArgsF64 A;
        A.c = C;
        fill_source_f64(A.src, src);
        e = fk::launch_walk_f64(A, cfg, stream, true, dense);
    } else {
        fk::WalkArgsF32 A;
        A.c = C;
        fill_source_f32(A.src, src);
        e = fk::launch_walk_f32(A, p->precision == FK_MIXED_KAHAN, cfg, stream, true, dense);
    }
    if (timed) timing_end(ev, stream);
    if (e != hipSuccess) return fail(FK_EDEVICE, "adjoint walk launch failed: %s", hipGetErrorString(e));
    // d u_p / d rho_v = -2 pi G (dt/2) c_v; a g_z sample divides by 2h
    const double scale = -C.w / (kind == 1 ? 2.0 * C.h : 1.0);
    e = fk::launch_adjoint_combine(counts, n_stations, AL.nvox, grad_out, fwd_out, scale, grad_rho, stream);
    if (e != hipSuccess) return fail(FK_EDEVICE, "adjoint combine launch failed: %s", hipGetErrorString(e));
    return FK_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Solves without a workspace argument: their scratch is this file's device
// array, one per GPU, held until the process ends.
// ---------------------------------------------------------------------------
static constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// The device address of scratch on each device (the array's host-side name
// is not a device address), looked up once per device with it current.
void* g_scratch[64] = {nullptr};

fk_status scratch_of_current_device(char** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FK_EDEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= 64) return fail(FK_EUNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(FK_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = static_cast<char*>(g_scratch[dev]);
    return FK_OK;
}

// The bounded layout that fits kScratchBytes: every pair's partial, the
// status and queue blocks, and as many records as the rest holds (no more
// than params->slice_walks when that is set).
fk_status static_layout(int32_t kind, int64_t n_stations, const fk_params* p, Layout* L)
{
    const int64_t npair = kind == 1 ? 2 : 1;
    const Layout base = make_layout(kind, n_stations, p, 1);       // one record held
    const size_t fixed = base.total - 2 * 256;                     // minus the record arrays' rounding slack
    const size_t per = sizeof(uint32_t) + sizeof(fk::ExitRecord);
    if (fixed + per * (size_t)(kChunk * npair) > kScratchBytes)
        return fail(FK_EUNSUPPORTED, "solve too large for the %zu-byte scratch: %lld (station, chunk) pairs "
                                     "(at most about %zu)", kScratchBytes, (long long)base.n_pairs,
                    (kScratchBytes - per * (size_t)(kChunk * npair)) / sizeof(fk::Partial));
    int64_t held = (int64_t)((kScratchBytes - fixed) / per);
    if (p->slice_walks > 0 && p->slice_walks < held) held = p->slice_walks;
    for (; held >= kChunk * npair; held -= 64) {   // the regions' 256-byte rounding may take a few records
        *L = make_layout(kind, n_stations, p, held);
        if (L->total <= kScratchBytes) return FK_OK;
    }
    return fail(FK_EUNSUPPORTED, "solve too large for the %zu-byte scratch", kScratchBytes);
}

fk_status solve_static(int32_t kind, const double* stations, int64_t n_stations, const fk_box* box,
                       const fk_source* src, const fk_boundary* bc, const fk_params* p, fk_stat* out,
                       void* hip_stream)
{
    fk_status st = check_solve(kind, stations, n_stations, box, src, bc, p, out);
    if (st != FK_OK || n_stations == 0) return st;
    Layout L;
    if ((st = static_layout(kind, n_stations, p, &L)) != FK_OK) return st;
    char* ws = nullptr;
    if ((st = scratch_of_current_device(&ws)) != FK_OK) return st;
    return run_solve(kind, stations, n_stations, box, src, bc, p, out, ws, L,
                     reinterpret_cast<hipStream_t>(hip_stream), false);
}

}  // namespace

extern "C" {

fk_status fk_solve_static(int32_t kind, const double* stations, int64_t n_stations, const fk_box* box,
                          const fk_source* source, const fk_boundary* bc, const fk_params* params, fk_stat* out,
                          void* hip_stream)
{
    if (kind != 0 && kind != 1) return fail(FK_EINVAL, "kind must be 0 (potential) or 1 (g_z), got %d", kind);
    return solve_static(kind, stations, n_stations, box, source, bc, params, out, hip_stream);
}

size_t fk_adjoint_workspace_bytes(int64_t n_stations, const fk_source* source)
{
    if (n_stations < 0 || !source || check_source(source) != FK_OK || !has_grid(source)) return 0;
    return make_adj_layout(n_stations, source).total;
}

fk_status fk_potential_adjoint(const double* stations, int64_t n_stations, const fk_box* box,
                               const fk_source* source, const fk_boundary* bc, const fk_params* params,
                               const fk_stat* forward_out, const void* forward_workspace,
                               size_t forward_workspace_bytes, const double* grad_out, double* grad_rho,
                               void* workspace, size_t workspace_bytes, void* hip_stream)
{
    return adjoint(0, stations, n_stations, box, source, bc, params, forward_out, forward_workspace,
                   forward_workspace_bytes, grad_out, grad_rho, workspace, workspace_bytes, hip_stream);
}

fk_status fk_gz_adjoint(const double* stations, int64_t n_stations, const fk_box* box, const fk_source* source,
                        const fk_boundary* bc, const fk_params* params, const fk_stat* forward_out,
                        const void* forward_workspace, size_t forward_workspace_bytes, const double* grad_out,
                        double* grad_rho, void* workspace, size_t workspace_bytes, void* hip_stream)
{
    return adjoint(1, stations, n_stations, box, source, bc, params, forward_out, forward_workspace,
                   forward_workspace_bytes, grad_out, grad_rho, workspace, workspace_bytes, hip_stream);
}

size_t fk_batch_workspace_bytes(const fk_problem* problems, int32_t n_problems)
{
    if (check_batch(problems, n_problems) != FK_OK) return 0;
    return make_batch_layout(problems, n_problems).total;
}

fk_status fk_batch_layout(const fk_problem* problems, int32_t n_problems, int32_t m, size_t* values_offset,
                          size_t* steps_offset)
{
    fk_status st = check_batch(problems, n_problems);
    if (st != FK_OK) return st;
    if (m < 0 || m >= n_problems) return fail(FK_EINVAL, "problem index %d out of range", m);
    const BatchLayout B = make_batch_layout(problems, n_problems);
    if (!B.records) return fail(FK_EINVAL, "per-walk records are kept only with slice_walks = 0");
    if (values_offset) *values_offset = B.values + sizeof(double) * (size_t)B.tasks[m];
    if (steps_offset) *steps_offset = B.steps + sizeof(uint32_t) * (size_t)B.tasks[m];
    return FK_OK;
}

fk_status fk_solve_batch(const fk_problem* problems, int32_t n_problems, fk_stat* out, void* workspace,
                         size_t workspace_bytes, void* hip_stream)
{
    return solve_batch(problems, n_problems, out, workspace, workspace_bytes, hip_stream);
}


size_t fk_workspace_bytes(int32_t kind, int64_t n_stations, const fk_params* params)
{
    if (check_params(kind, n_stations, params) != FK_OK) return 0;
    return make_layout(kind, n_stations, params).total;
}

fk_status fk_workspace_layout(int32_t kind, int64_t n_stations, const fk_params* params, size_t* values_offset,
                              size_t* steps_offset, size_t* total_bytes)
{
    fk_status st = check_params(kind, n_stations, params);
    if (st != FK_OK) return st;
    const Layout L = make_layout(kind, n_stations, params);
    if (!L.records) return fail(FK_EINVAL, "per-walk records are kept only with slice_walks = 0");
    if (values_offset) *values_offset = L.values;
    if (steps_offset) *steps_offset = L.steps;
    if (total_bytes) *total_bytes = L.total;
    return FK_OK;
}

fk_status fk_workspace_status(const void* workspace, uint32_t* flags, void* hip_stream)
{
    if (!workspace) return fail(FK_EINVAL, "workspace is NULL");
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    uint32_t word = 0;
    hipError_t e = hipMemcpyAsync(&word, workspace, sizeof word, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(FK_EDEVICE, "reading the status word failed: %s", hipGetErrorString(e));
    if (flags) *flags = word;
    if (word & FK_FLAG_NONFINITE) return fail(FK_ENONFINITE, "a walk sample was NaN or infinite (flags 0x%x)", word);
    if ((word & FK_FLAG_STRICT) && (word & FK_FLAG_TRUNCATED))
        return fail(FK_ETRUNC, "strict solve: walks hit max_steps or started outside (flags 0x%x)", word);
    return FK_OK;
}

fk_status fk_check_stations(const double* stations_host, int64_t n_stations, const fk_box* box, int32_t kind,
                            const fk_params* params)
{
    fk_status st;
    if ((st = check_params(kind, n_stations, params)) != FK_OK) return st;
    if ((st = check_box(box)) != FK_OK) return st;
    if ((st = check_domain(box, params, nullptr)) != FK_OK) return st;
    if (n_stations > 0 && !stations_host) return fail(FK_EINVAL, "stations is NULL");
    const double h = kind == 1 ? (params->h > 0.0 ? params->h : std::sqrt(params->dt)) : 0.0;
    double ctr[3], r2 = 0.0;
    if (params->domain == FK_DOMAIN_BALL) ball_of(box, ctr, &r2);
    for (int64_t s = 0; s < n_stations; ++s) {
        const double* x = stations_host + 3 * s;
        if (params->domain == FK_DOMAIN_BALL) {
            for (int w = 0; w < (kind == 1 ? 2 : 1); ++w) {
                const double y[3] = {x[0], x[1], kind == 1 ? (w == 0 ? x[2] + h : x[2] - h) : x[2]};
                if (!is_finite(x[0]) || !is_finite(x[1]) || !is_finite(x[2]) || !(dist2(y, ctr) < r2))
                    return fail(FK_EDOMAIN, "station %lld is not strictly inside the ball%s", (long long)s,
                                kind == 1 ? " (with +-h along z)" : "");
            }
            continue;
        }
        for (int c = 0; c < 3; ++c) {
            const double d = c == 2 ? h : 0.0;
            if (!is_finite(x[c]) || !(x[c] - d > box->lo[c] && x[c] + d < box->hi[c]))
                return fail(FK_EDOMAIN, "station %lld is not strictly inside the box%s", (long long)s,
                            kind == 1 ? " (with +-h along z)" : "");
        }
    }
    return FK_OK;
}

fk_status fk_solve_potential(const double* stations, int64_t n_stations, const fk_box* box, const fk_source* source,
                             const fk_boundary* bc, const fk_params* params, fk_stat* out, void* workspace,
                             size_t workspace_bytes, void* hip_stream)
{
    return solve(0, stations, n_stations, box, source, bc, params, out, workspace, workspace_bytes, hip_stream);
}

fk_status fk_solve_gz(const double* stations, int64_t n_stations, const fk_box* box, const fk_source* source,
                      const fk_boundary* bc, const fk_params* params, fk_stat* out, void* workspace,
                      size_t workspace_bytes, void* hip_stream)
{
    return solve(1, stations, n_stations, box, source, bc, params, out, workspace, workspace_bytes, hip_stream);
}

fk_status fk_stream_blocks(const uint32_t* counters, int64_t n_items, uint64_t seed, uint32_t* words,
                           double* normals_f64, float* normals_f32, void* hip_stream)
{
    if (n_items < 0) return fail(FK_EINVAL, "n_items < 0");
    if (n_items == 0) return FK_OK;
    if (!counters) return fail(FK_EINVAL, "counters is NULL");
    if (n_items > (1ll << 31)) return fail(FK_EUNSUPPORTED, "at most 2^31 items");
    hipError_t e = fk::launch_stream_blocks(counters, n_items, (uint32_t)(seed & 0xffffffffull),
                                            (uint32_t)(seed >> 32), words, normals_f64, normals_f32,
                                            reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? FK_OK : fail(FK_EDEVICE, "stream launch failed: %s", hipGetErrorString(e));
}

fk_status fk_autotune(int32_t kind, const double* stations, int64_t n_stations, const fk_box* box,
                      const fk_source* source, const fk_boundary* bc, const fk_params* params, fk_stat* out,
                      void* workspace, size_t workspace_bytes, void* hip_stream, fk_launch* best, double* best_ms)
{
    fk_status st = check_params(kind, n_stations, params);
    if (st != FK_OK) return st;
    if (!best) return fail(FK_EINVAL, "best is NULL");
    const int precision = params->precision;
    fk_launch keep;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        keep = g_launch[precision];
    }
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(FK_EDEVICE, "hipEventCreate failed");
    const int blocks[3] = {64, 128, 256};
    const int grabs[3] = {16, 32, 64};
    double best_t = 1e300;
    fk_launch best_l = keep;
    st = FK_OK;
    for (int bi = 0; bi < 3 && st == FK_OK; ++bi) {
        int occ = 0;
        if (fk::walk_occupancy(precision, blocks[bi], &occ, loop_kind(params, source)) != hipSuccess || occ <= 0)
            continue;
        const int bpcs[2] = {0, occ > 1 ? occ / 2 : 1};
        for (int pi = 0; pi < 2 && st == FK_OK; ++pi) {
            for (int gi = 0; gi < 3 && st == FK_OK; ++gi) {
                {
                    std::lock_guard<std::mutex> lk(g_mu);
                    g_launch[precision] = fk_launch{blocks[bi], bpcs[pi], grabs[gi], keep.adjoint_table, keep.stripes,
                                                    keep.refill_cost};
                }
                float ms = 0.0f;
                // one untimed run, then one timed run
                for (int rep = 0; rep < 2 && st == FK_OK; ++rep) {
                    if (rep == 1) (void)hipEventRecord(e0, stream);
                    st = solve(kind, stations, n_stations, box, source, bc, params, out, workspace, workspace_bytes,
                               hip_stream);
                    if (rep == 1) (void)hipEventRecord(e1, stream);
                }
                if (st != FK_OK) break;
                if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    st = fail(FK_EDEVICE, "timing failed");
                    break;
                }
                if (ms < best_t) {
                    best_t = ms;
                    best_l = fk_launch{blocks[bi], bpcs[pi], grabs[gi], keep.adjoint_table, keep.stripes,
                                       keep.refill_cost};
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_launch[precision] = st == FK_OK ? best_l : keep;
    }
    if (st != FK_OK) return st;
    *best = best_l;
    if (best_ms) *best_ms = best_t;
    return FK_OK;
}

fk_status fk_merge_stats(const fk_stat* a, const fk_stat* b, int64_t n, fk_stat* out)
{
    if (n < 0) return fail(FK_EINVAL, "n < 0");
    if (n > 0 && (!a || !b || !out)) return fail(FK_EINVAL, "NULL statistics");
    for (int64_t s = 0; s < n; ++s) {
        const fk_stat x = a[s], y = b[s];
        fk_stat r{};
        r.n = x.n + y.n;
        r.n_trunc = x.n_trunc + y.n_trunc;
        r.sum_steps = x.sum_steps + y.sum_steps;
        r.max_steps = x.max_steps > y.max_steps ? x.max_steps : y.max_steps;
        const double walks = (double)(x.n + x.n_trunc + y.n + y.n_trunc);
        r.mean_steps = walks > 0.0 ? (double)r.sum_steps / walks : 0.0;
        if (r.n == 0) {
            r.mean = r.var = r.se = std::nan("");
        } else if (x.n == 0 || y.n == 0) {
            const fk_stat& z = x.n ? x : y;
            r.mean = z.mean;
            r.var = z.var;
            r.se = z.se;
        } else {
            const double na = (double)x.n, nb = (double)y.n, nn = (double)r.n;
            const double d = y.mean - x.mean;
            r.mean = x.mean + d * (nb / nn);
            const double m2a = x.n > 1 ? x.var * (na - 1.0) : 0.0;
            const double m2b = y.n > 1 ? y.var * (nb - 1.0) : 0.0;
            const double m2 = m2a + m2b + d * d * (na * nb / nn);
            r.var = r.n > 1 ? m2 / (nn - 1.0) : std::nan("");
            r.se = r.n > 1 ? std::sqrt(r.var / nn) : std::nan("");
        }
        out[s] = r;
    }
    return FK_OK;
}

fk_status fk_moving_average(const double* values, const double* se, int64_t n, int32_t span, double* out_values,
                            double* out_se)
{
    if (n < 0) return fail(FK_EINVAL, "n < 0");
    if (span < 1 || span % 2 == 0) return fail(FK_EINVAL, "span must be a positive odd number, got %d", span);
    if (n > 0 && (!values || !out_values)) return fail(FK_EINVAL, "NULL values");
    if (se && !out_se) return fail(FK_EINVAL, "se given without out_se");
    const int64_t half = span / 2;
    for (int64_t k = 0; k < n; ++k) {
        // the widest window centred on k that fits: k - r .. k + r
        int64_t r = half;
        if (k < r) r = k;
        if (n - 1 - k < r) r = n - 1 - k;
        double sum = 0.0, var = 0.0;
        for (int64_t j = k - r; j <= k + r; ++j) {
            sum += values[j];
            if (se) var += se[j] * se[j];
        }
        const double w = (double)(2 * r + 1);
        out_values[k] = sum / w;
        if (se) out_se[k] = std::sqrt(var) / w;
    }
    return FK_OK;
}

fk_status fk_set_launch(int32_t precision, const fk_launch* launch)
{
    if (precision < 0 || precision > 2) return fail(FK_EINVAL, "unknown precision %d", precision);
    if (!launch) return fail(FK_EINVAL, "launch is NULL");
    if (launch->block < 64 || launch->block > 256 || launch->block % 64 != 0)
        return fail(FK_EINVAL, "block must be a multiple of 64 in [64, 256]");
    if (launch->blocks_per_cu < 0 || launch->blocks_per_cu > 64) return fail(FK_EINVAL, "blocks_per_cu must lie in [0, 64]");
    if (launch->grab < 1 || launch->grab > 64) return fail(FK_EINVAL, "grab must lie in [1, 64]");
    if (launch->adjoint_table < 0 || launch->adjoint_table > 1) return fail(FK_EINVAL, "adjoint_table must be 0 or 1");
    if (launch->stripes < 0 || launch->stripes > 32) return fail(FK_EINVAL, "stripes must lie in [0, 32]");
    if (launch->refill_cost < 0 || launch->refill_cost > 8192) return fail(FK_EINVAL, "refill_cost must lie in [0, 8192]");
    std::lock_guard<std::mutex> lk(g_mu);
    g_launch[precision] = *launch;

    return FK_OK;
}

fk_status fk_get_launch(int32_t precision, fk_launch* launch)
{
    if (precision < 0 || precision > 2) return fail(FK_EINVAL, "unknown precision %d", precision);
    if (!launch) return fail(FK_EINVAL, "launch is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    *launch = g_launch[precision];
    return FK_OK;
}

fk_status fk_timing_enable(int32_t on)
{
    g_timing.on = on != 0;
    return FK_OK;
}

fk_status fk_timing_read(double* ms_out, int32_t max_n, int32_t* n_out)
{
    if (max_n < 0) return fail(FK_EINVAL, "max_n < 0");
    if (max_n > 0 && !ms_out) return fail(FK_EINVAL, "ms_out is NULL");
    int32_t n = 0;
    fk_status st = FK_OK;
    for (auto& p : g_timing.pending) {
        if (hipEventSynchronize(p.second) != hipSuccess) st = fail(FK_EDEVICE, "hipEventSynchronize failed");
        float ms = 0.0f;
        if (st == FK_OK && hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess)
            st = fail(FK_EDEVICE, "hipEventElapsedTime failed");
        if (n < max_n) ms_out[n] = ms;
        ++n;
        g_timing.spare.push_back(p);
    }
    g_timing.pending.clear();
    if (n_out) *n_out = n < max_n ? n : max_n;
    return st;
}

const char* fk_status_string(int32_t status)
{
    switch (status) {
    case FK_OK: return "ok";
    case FK_EINVAL: return "invalid argument";
    case FK_EDOMAIN: return "station not strictly inside the box";
    case FK_EWORKSPACE: return "workspace too small or misaligned";
    case FK_EDEVICE: return "HIP runtime error";
    case FK_ETRUNC: return "walks hit max_steps";
    case FK_EUNSUPPORTED: return "size limit exceeded";
    case FK_ENONFINITE: return "a walk sample was not finite";
    default: return "unknown status";
    }
}

const char* fk_last_error(void) { return g_last_error.c_str(); }

int32_t fk_version(void) { return 100; }

}  // extern "C"
