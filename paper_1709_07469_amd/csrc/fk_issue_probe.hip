// fk_issue_probe.hip -- measures, on the GPU it runs on, the VALU issue cost
// of the operations one Euler-Maruyama step of the walk kernels is made of:
// a Philox4x32-10 block, an FP64 and an FP32 Box-Muller pair (uniform bits to
// two normals), the rest of a step (position update, density of one analytic
// prism, trapezoid sum, exit test) in FP64 and in FP32 with an FP64 sum, and
// FP64 / FP32 fused multiply-adds.  Each lane runs 8
// independent dependency chains whose every result feeds the next input, so
// nothing folds; the cost is reported in full-rate lane-slots (one slot = one
// lane-operation at the chip's peak VALU issue rate, CUs x 64 x clock).
//
// These costs define the algorithmic work per step used for the walk
// kernels' ALU roofline.  Build and run: see paper_1709_07469_amd/build.py
// (target "probe").  Prints one JSON object.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <type_traits>

#include "fk_device.hpp"

#define CHK(x)                                                                              \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) {                                                             \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                       \
        }                                                                                   \
    } while (0)

namespace {

constexpr int kChains = 8;
constexpr int kIter = 512;

__global__ void __launch_bounds__(256) philox_probe(uint32_t* out, uint32_t seed)
{
    uint32_t c[kChains][4];
    for (int j = 0; j < kChains; ++j) {
        c[j][0] = threadIdx.x + j;
        c[j][1] = blockIdx.x;
        c[j][2] = seed;
        c[j][3] = j;
    }
    for (int i = 0; i < kIter; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            const fk::Block b = fk::philox10(c[j][0], c[j][1], c[j][2], c[j][3], seed, 0x1234u);
            c[j][0] = b.w0;
            c[j][1] = b.w1;
            c[j][2] = b.w2;
            c[j][3] = b.w3;
        }
    }
    uint32_t s = 0;
    for (int j = 0; j < kChains; ++j) s ^= c[j][0] ^ c[j][1] ^ c[j][2] ^ c[j][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Box-Muller pairs; the next pair's uniform words are the low bits of the
// previous normals (2-3 extra integer ops per pair, included in the cost).
__global__ void __launch_bounds__(256) bm64_probe(uint32_t* out, uint32_t seed)
{
    fk::BmTables* tab = fk::bm_tables();
    fk::fill_bm_tables(*tab);
    uint32_t w[kChains][4];
    for (int j = 0; j < kChains; ++j) {
        w[j][0] = threadIdx.x * 2654435761u + j;
        w[j][1] = seed ^ blockIdx.x;
        w[j][2] = w[j][0] * 7u + 3u;
        w[j][3] = w[j][1] * 5u + 1u;
    }
    for (int i = 0; i < kIter / 8; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            double z0, z1;
            fk::normals_f64(fk::Block{w[j][0], w[j][1], w[j][2], w[j][3]}, *tab, z0, z1);
            const uint64_t a = (uint64_t)__double_as_longlong(z0), b = (uint64_t)__double_as_longlong(z1);
            w[j][0] = (uint32_t)a;
            w[j][1] = (uint32_t)(a >> 32) ^ (uint32_t)b;
            w[j][2] = (uint32_t)b + w[j][0];
            w[j][3] = (uint32_t)(b >> 32) ^ w[j][2];
        }
    }
    uint32_t s = 0;
    for (int j = 0; j < kChains; ++j) s ^= w[j][0] ^ w[j][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) bm32_probe(uint32_t* out, uint32_t seed)
{
    uint32_t w[kChains][2];
    for (int j = 0; j < kChains; ++j) {
        w[j][0] = threadIdx.x * 2654435761u + j;
        w[j][1] = seed ^ blockIdx.x;
    }
    for (int i = 0; i < kIter; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            float z0, z1;
            fk::normals_f32(w[j][0], w[j][1], z0, z1);
            w[j][0] = __float_as_uint(z0) * 2654435761u;
            w[j][1] = __float_as_uint(z1) ^ w[j][0];
        }
    }
    uint32_t s = 0;
    for (int j = 0; j < kChains; ++j) s ^= w[j][0] ^ w[j][1];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) fma64_probe(uint32_t* out, uint32_t seed)
{
    double a[kChains];
    for (int j = 0; j < kChains; ++j) a[j] = (double)(seed + threadIdx.x + j);
    const double m = 0.999999, c = 1e-7;
    for (int i = 0; i < kIter * 8; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = fma(a[j], m, c);
    }
    double s = 0.0;
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)s;
}

__global__ void __launch_bounds__(256) fma32_probe(uint32_t* out, uint32_t seed)
{
    float a[kChains];
    for (int j = 0; j < kChains; ++j) a[j] = (float)(seed + threadIdx.x + j);
    const float m = 0.999999f, c = 1e-7f;
    for (int i = 0; i < kIter * 8; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = fmaf(a[j], m, c);
    }
    float s = 0.0f;
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)s;
}

// The step body of the walk kernels for one analytic prism, normals read
// from LDS (not VALU work); a walk that leaves the box restarts at its start.
template <bool F64>
__global__ void __launch_bounds__(256) step_probe(uint32_t* out, uint32_t seed)
{
    using T = typename std::conditional<F64, double, float>::type;
    __shared__ T zs[192];
    for (int i = threadIdx.x; i < 192; i += blockDim.x) zs[i] = (T)((int)((i * 37 + seed) % 97) - 48) * (T)0.04;
    __syncthreads();
    const T lo[3] = {T(0), T(0), T(-500)}, hi[3] = {T(1000), T(1000), T(100)};
    const T q[6] = {T(400), T(450), T(-300), T(600), T(550), T(-150)};
    const T sdt = T(2), rho0 = T(300);
    T x[kChains][3], rp[kChains];
    double S[kChains];
    for (int j = 0; j < kChains; ++j) {
        x[j][0] = T(62.5) + T(125) * (T)((threadIdx.x + j) & 7);
        x[j][1] = T(62.5) + T(125) * (T)(blockIdx.x & 7);
        x[j][2] = T(0);
        rp[j] = T(0);
        S[j] = 0.0;
    }
    for (int i = 0; i < kIter * 4; ++i) {
        const int b = (i * 3) % 189;
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            const T y0 = fma(sdt, zs[b + (j & 3)], x[j][0]);
            const T y1 = fma(sdt, zs[b + 1], x[j][1]);
            const T y2 = fma(sdt, zs[b + 2], x[j][2]);
            const bool in = y0 >= q[0] && y0 < q[3] && y1 >= q[1] && y1 < q[4] && y2 >= q[2] && y2 < q[5];
            const T rn = in ? rho0 : T(0);
            S[j] = S[j] + (F64 ? (double)(rp[j] + rn) : ((double)rp[j] + (double)rn));
            const bool o = y0 <= lo[0] || y0 >= hi[0] || y1 <= lo[1] || y1 >= hi[1] || y2 <= lo[2] || y2 >= hi[2];
            x[j][0] = o ? T(500) : y0;
            x[j][1] = o ? T(500) : y1;
            x[j][2] = o ? T(0) : y2;
            rp[j] = o ? T(0) : rn;
        }
    }
    double s = 0.0;
    for (int j = 0; j < kChains; ++j) s += S[j] + (double)x[j][0] + (double)x[j][2];
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(int64_t)s;
}

typedef void (*Probe)(uint32_t*, uint32_t);

}  // namespace

int main()
{
    int dev = 0, cus = 0, khz = 0;
    CHK(hipGetDevice(&dev));
    CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev));
    const int block = 256, grid = cus * 8;
    uint32_t* buf = nullptr;
    CHK(hipMalloc(&buf, sizeof(uint32_t) * (size_t)grid * block));
    struct Item {
        const char* name;
        Probe f;
        double units_per_chain;
    } items[] = {{"philox_block", philox_probe, (double)kIter},
                 {"box_muller_pair_f64", bm64_probe, (double)(kIter / 8)},
                 {"box_muller_pair_f32", bm32_probe, (double)kIter},
                 {"step_f64", step_probe<true>, (double)(kIter * 4)},
                 {"step_f32_f64sum", step_probe<false>, (double)(kIter * 4)},
                 {"fma_f64", fma64_probe, (double)(kIter * 8)},
                 {"fma_f32", fma32_probe, (double)(kIter * 8)}};
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    const double slots_per_s = (double)cus * 64.0 * (double)khz * 1e3;
    std::printf("{\"cus\": %d, \"clock_mhz\": %.0f, \"lane_slots_per_s\": %.4e", cus, khz / 1e3, slots_per_s);
    for (const Item& it : items) {
        hipLaunchKernelGGL(it.f, dim3(grid), dim3(block), 0, 0, buf, 1u);
        CHK(hipGetLastError());
        CHK(hipDeviceSynchronize());
        // the fastest of 7 timings of 5 launches: the clock drifts by about a
        // percent between runs, and the part's cost is its best issue rate
        float ms = 0.0f;
        for (int t = 0; t < 7; ++t) {
            CHK(hipEventRecord(e0, 0));
            for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(it.f, dim3(grid), dim3(block), 0, 0, buf, 2u + r);
            CHK(hipGetLastError());
            CHK(hipEventRecord(e1, 0));
            CHK(hipEventSynchronize(e1));
            float m = 0.0f;
            CHK(hipEventElapsedTime(&m, e0, e1));
            if (t == 0 || m < ms) ms = m;
        }
        const double units = 5.0 * grid * block * (double)kChains * it.units_per_chain;
        const double slots = slots_per_s * (ms * 1e-3) / units;
        std::printf(", \"%s\": {\"ms\": %.3f, \"slots\": %.3f}", it.name, ms, slots);
    }
    std::printf("}\n");
    CHK(hipFree(buf));
    return 0;
}
