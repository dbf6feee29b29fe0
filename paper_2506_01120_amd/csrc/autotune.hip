// Autotuner for the saturated-phase block step.
//
// Once acceptances are rare (the saturated phase of Algorithm 4, where nearly all
// of a full certification's candidates are decided), a block step is dominated
// by the two projection GEMMs: the coefficients C = H V^T of a candidate block
// against the basis and the residual R = H - C V with its fused norm epilogue.
// Their speed depends on the block size (the GEMMs' M extent) and, for the FP32
// and split-BF16 screens, on the workgroup tile.  The tuner times every
// admissible (block, tile_dot, tile_sub) on the device at the problem's real
// shape -- the basis at the ambient bound, D = d^2 -- with HIP events, and keeps
// the one with the lowest time per candidate.  Choices are cached in memory for
// the process and, optionally, in a text file (one line per device, precision,
// d and ambient bound) so that later runs skip the timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lie_internal.h"

namespace lie {
namespace {

constexpr int kTuneReps = 3;

__global__ void k_fill(float *p, int64_t n, float a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = a * (float)((i * 2654435761ll) % 1024 - 512) / 512.0f;
}

__global__ void k_fill64(double *p, int64_t n, double a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = a * (double)((i * 2654435761ll) % 1024 - 512) / 512.0;
}

__global__ void k_fill_bf16(__bf16 *p, int64_t n, float a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (__bf16)(a * (float)((i * 2654435761ll) % 1024 - 512) / 512.0f);
}

struct Key {
    std::string arch;
    int precision;
    int d;
    int64_t ambient;
    bool operator==(const Key &o) const
    {
        return arch == o.arch && precision == o.precision && d == o.d && ambient == o.ambient;
    }
};

std::mutex g_mu;
std::vector<std::pair<Key, TuneChoice>> g_mem;  // process-wide cache

std::string device_arch(int dev)
{
    hipDeviceProp_t p{};
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = p.gcnArchName;
    const size_t colon = a.find(':');
    if (colon != std::string::npos)
        a = a.substr(0, colon);
    return a + "-cu" + std::to_string(p.multiProcessorCount);
}

bool file_lookup(const char *path, const Key &k, TuneChoice *out)
{
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    char line[512], arch[128];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        int prec = -1, d = -1, b = 0, td = 0, ts = 0;
        long long amb = -1;
        double us = 0;
        if (std::sscanf(line, "lie-tune v2 arch=%127s precision=%d d=%d ambient=%lld block_sat=%d tile_dot=%d "
                              "tile_sub=%d us_per_candidate=%lf",
                        arch, &prec, &d, &amb, &b, &td, &ts, &us) == 8 &&
            k.arch == arch && prec == k.precision && d == k.d && amb == k.ambient && b > 0) {
            *out = TuneChoice{b, td, ts, us};
            found = true;  // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void file_append(const char *path, const Key &k, const TuneChoice &c)
{
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f,
                 "lie-tune v2 arch=%s precision=%d d=%d ambient=%lld block_sat=%d tile_dot=%d tile_sub=%d "
                 "us_per_candidate=%.6g\n",
                 k.arch.c_str(), k.precision, k.d, (long long)k.ambient, c.block_sat, c.tile_dot, c.tile_sub,
                 c.us_per_candidate);
    std::fclose(f);
}

struct Buffers {
    void *V = nullptr, *H = nullptr, *C = nullptr;
    __bf16 *Vp = nullptr, *Vt = nullptr, *Hp = nullptr, *Cp = nullptr;  // split-BF16 planes
    PlaneGeom pg{};
    double *normpart = nullptr;
    DevState *st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Buffers()
    {
        for (void *p : {V, H, C, (void *)normpart, (void *)st, (void *)Vp, (void *)Vt, (void *)Hp, (void *)Cp})
            if (p)
                (void)hipFree(p);
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
    }
};

// One timed configuration: milliseconds of (coefficients + residual) for `b` candidates.
hipError_t time_step(const Buffers &B, int precision, int64_t D, int64_t n, int64_t ldc, int b, int td, int ts,
                     hipStream_t s, float *ms_out)
{
    auto launch = [&]() -> hipError_t {
        hipError_t e;
        if (precision == 0) {
            e = launch_gemm_dot_f64((const double *)B.V, B.st, (const double *)B.H, nullptr, nullptr, b, D, n, ldc,
                                    (double *)B.C, s);
            if (e == hipSuccess)
                e = launch_gemm_sub_f64((const double *)B.V, B.st, (double *)B.H, nullptr, nullptr,
                                        (const double *)B.C, n, ldc, b, D, B.normpart, s);
        } else if (precision == 1) {
            e = launch_gemm_dot_f32((const float *)B.V, B.st, (const float *)B.H, b, D, n, ldc, (float *)B.C, td, s);
            if (e == hipSuccess)
                e = launch_gemm_sub_f32((const float *)B.V, B.st, (const float *)B.H, (const float *)B.C, n, ldc, b, D,
                                        B.normpart, ts, s);
        } else {
            // split BF16: the plane GEMMs of single problems
            e = launch_bfp_dot(B.Hp, B.Vp, B.st, b, n, B.Cp, B.pg, s);
            if (e == hipSuccess)
                e = launch_bfp_sub(B.Cp, B.Vt, B.Hp, B.st, b, D, B.normpart, B.pg, s);
        }
        return e;
    };
    hipError_t e = launch();  // warm-up (code load, caches)
    if (e != hipSuccess)
        return e;
    float best = 1e30f;
    for (int r = 0; r < kTuneReps; ++r) {
        if ((e = hipEventRecord(B.e0, s)) != hipSuccess || (e = launch()) != hipSuccess ||
            (e = hipEventRecord(B.e1, s)) != hipSuccess || (e = hipEventSynchronize(B.e1)) != hipSuccess)
            return e;
        float ms = 0;
        if ((e = hipEventElapsedTime(&ms, B.e0, B.e1)) != hipSuccess)
            return e;
        best = std::min(best, ms);
    }
    *ms_out = best;
    return hipSuccess;
}

}  // namespace

hipError_t autotune_block_step(int device, int precision, int d, int64_t ambient, int max_block, const char *cache_path,
                               hipStream_t s, TuneChoice *out, bool *from_cache)
{
    *from_cache = false;
    const Key key{device_arch(device), precision, d, ambient};
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const auto &kv : g_mem)
            if (kv.first == key && kv.second.block_sat <= max_block) {
                *out = kv.second;
                *from_cache = true;
                return hipSuccess;
            }
        if (cache_path && file_lookup(cache_path, key, out) && out->block_sat <= max_block) {
            g_mem.emplace_back(key, *out);
            *from_cache = true;
            return hipSuccess;
        }
    }
    const int64_t D = (int64_t)d * d;
    const int64_t n = std::max<int64_t>(ambient, 1);
    const int64_t ldc = coef_ld(n);
    std::vector<int> blocks;
    for (int b : {1024, 2048, 4096, 8192, 16384})
        if (b <= max_block)
            blocks.push_back(b);
    if (blocks.empty())
        blocks.push_back(std::max(1, max_block));
    const int bmax = *std::max_element(blocks.begin(), blocks.end());
    const size_t w = precision == 0 ? sizeof(double) : sizeof(float);
    const int ntile = precision == 0 ? gemm_sub_tiles_f64(D)
                                     : std::max(precision == 1 ? gemm_sub_tiles_f32(D, 1) : gemm_sub_tiles_bf16(D, 1),
                                                precision == 1 ? gemm_sub_tiles_f32(D, 2) : gemm_sub_tiles_bf16(D, 2));
    Buffers B;
    hipError_t e;
    if ((e = hipMalloc(&B.V, (size_t)n * D * w)) != hipSuccess || (e = hipMalloc(&B.H, (size_t)bmax * D * w)) != hipSuccess ||
        (e = hipMalloc(&B.C, (size_t)bmax * ldc * w)) != hipSuccess ||
        (e = hipMalloc((void **)&B.normpart, (size_t)bmax * ntile * 2 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void **)&B.st, sizeof(DevState))) != hipSuccess ||
        (e = hipEventCreate(&B.e0)) != hipSuccess || (e = hipEventCreate(&B.e1)) != hipSuccess)
        return e;
    DevState hs{};
    hs.N = n;
    hs.min_acc = INFINITY;
    if ((e = hipMemcpyAsync(B.st, &hs, sizeof hs, hipMemcpyHostToDevice, s)) != hipSuccess)
        return e;
    // synthetic operands of unit scale (the timing does not depend on the values)
    if (precision == 0) {
        hipLaunchKernelGGL(k_fill64, dim3(1024), dim3(256), 0, s, (double *)B.V, n * D, 1.0 / std::sqrt((double)D));
        hipLaunchKernelGGL(k_fill64, dim3(1024), dim3(256), 0, s, (double *)B.H, (int64_t)bmax * D, 1.0);
    } else {
        hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, (float *)B.V, n * D, 1.0f / std::sqrt((float)D));
        hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, (float *)B.H, (int64_t)bmax * D, 1.0f);
    }
    if (precision == 2) {
        // planes of unit-scale synthetic values (the timing does not depend on them)
        B.pg = plane_geom(D, n, bmax);
        const PlaneGeom &g = B.pg;
        if ((e = hipMalloc((void **)&B.Vp, (size_t)(g.cap_rows * g.ld) * 2)) != hipSuccess ||
            (e = hipMalloc((void **)&B.Vt, (size_t)(g.d_rows * g.ldt) * 2)) != hipSuccess ||
            (e = hipMalloc((void **)&B.Hp, (size_t)(g.b_rows * g.ld) * 2)) != hipSuccess ||
            (e = hipMalloc((void **)&B.Cp, (size_t)(g.b_rows * g.ldt) * 2)) != hipSuccess)
            return e;
        for (auto pz : {std::make_pair((void *)B.Vp, (size_t)(g.cap_rows * g.ld)),
                        std::make_pair((void *)B.Vt, (size_t)(g.d_rows * g.ldt)),
                        std::make_pair((void *)B.Hp, (size_t)(g.b_rows * g.ld)),
                        std::make_pair((void *)B.Cp, (size_t)(g.b_rows * g.ldt))})
            hipLaunchKernelGGL(k_fill_bf16, dim3(1024), dim3(256), 0, s, (__bf16 *)pz.first, (int64_t)pz.second,
                               1.0f / std::sqrt((float)D));
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    TuneChoice best{blocks.front(), 0, 0, 1e30};
    // the plane GEMMs have one tile shape (reported as 2: 128 x 128)
    const std::vector<int> tiles = precision == 0 ? std::vector<int>{0}
                                   : precision == 2 ? std::vector<int>{2} : std::vector<int>{1, 2};
    for (int b : blocks)
        for (int td : tiles)
            for (int ts : tiles) {
                float ms = 0;
                if ((e = time_step(B, precision, D, n, ldc, b, td, ts, s, &ms)) != hipSuccess)
                    return e;
                const double us = 1e3 * ms / b;
                if (us < best.us_per_candidate)
                    best = TuneChoice{b, td, ts, us};
            }
    *out = best;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_mem.emplace_back(key, best);
        if (cache_path)
            file_append(cache_path, key, best);
    }
    return hipSuccess;
}

}  // namespace lie
