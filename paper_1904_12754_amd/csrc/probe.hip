// Measurement probes (include/mlmc_probe.h): the rate (or the serial latency) of uniformly
// random 16-byte gathers from a table of a given size, in device memory or staged in LDS,
// and the issue rate of plain 32-bit integer VALU work. They calibrate the rooflines the
// walk kernels are measured against; no walk uses them.
#include "../../include/mlmc_expv.h"
#include "../../include/mlmc_probe.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "common.h"

namespace mlmc {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kChains = 8;   // independent gathers (or integer chains) in flight per lane

// xorshift32 (Marsaglia 2003): three shifts and three xors, no multiply, so the index
// arithmetic stays far below the memory rate being measured.
__device__ __forceinline__ uint32_t xorshift32(uint32_t x)
{
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

// kLds: the workgroup first copies the table (at most 4096 records, 64 KB) into LDS and
// gathers from there. kDep: a stream's next index takes in the first word of the record it
// just read, so one stream's gathers are serial and the launch measures their latency.
template <bool kLds, bool kDep, int kC>
__global__ __launch_bounds__(kProbeBlock) void gather_probe_kernel(const uint4 *__restrict__ table,
                                                                   uint32_t mask, uint32_t iters,
                                                                   uint32_t seed, uint32_t *sink)
{
    extern __shared__ uint4 lds_table[];
    if constexpr (kLds) {
        for (uint32_t i = threadIdx.x; i <= mask; i += kProbeBlock) lds_table[i] = table[i];
        __syncthreads();
    }
    const uint32_t tid = blockIdx.x * kProbeBlock + threadIdx.x;
    uint32_t x[kC];
#pragma unroll
    for (int j = 0; j < kC; ++j) x[j] = (tid * 0x9E3779B9u) ^ (seed + 0x85EBCA6Bu * (j + 1)) ^ 0x2545F491u;
    uint32_t acc = 0;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kC; ++j) {
            x[j] = xorshift32(x[j]);
            uint4 v;
            if constexpr (kLds) v = lds_table[x[j] & mask];
            else v = table[x[j] & mask];
            if constexpr (kDep) x[j] ^= v.x;
            acc ^= v.x ^ v.y ^ v.z ^ v.w;
        }
    }
    if (acc == 0x6A09E667u) sink[tid & 255u] = acc;   // keeps the loads; practically never taken
}

__global__ __launch_bounds__(kProbeBlock) void valu_probe_kernel(uint32_t iters, uint32_t seed,
                                                                 uint32_t *sink)
{
    const uint32_t tid = blockIdx.x * kProbeBlock + threadIdx.x;
    uint32_t a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = tid + seed * (j + 1);
#pragma unroll 4
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = xor3(a[j], a[(j + 1) % kChains], i);   // one v_bitop3_b32
    }
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc ^= a[j];
    if (acc == 0x6A09E667u) sink[tid & 255u] = acc;
}

int probe_fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

// Time one launch of `launch` with a pair of events on stream s (after one untimed launch).
template <class F>
int time_launch(F &&launch, hipStream_t s, double *ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MLMC_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return probe_fail(MLMC_ERR_HIP, "hipEventCreate");
    }
    launch();
    (void)hipEventRecord(e0, s);
    launch();
    (void)hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return probe_fail(MLMC_ERR_HIP, std::string("probe launch: ") + hipGetErrorString(e));
    *ms = t;
    return MLMC_OK;
}

uint32_t *g_sink = nullptr;   // 256 words, allocated on the first probe call

int sink_buffer(uint32_t **out)
{
    if (!g_sink) MLMC_HIP_TRY(hipMalloc(reinterpret_cast<void **>(&g_sink), 256 * sizeof(uint32_t)));
    *out = g_sink;
    return MLMC_OK;
}

int grid_for(int32_t waves_per_cu, uint32_t *blocks)
{
    int dev = 0, cus = 0;
    MLMC_HIP_TRY(hipGetDevice(&dev));
    MLMC_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    *blocks = static_cast<uint32_t>(std::max(1, cus) * waves_per_cu / (kProbeBlock / 64));
    return MLMC_OK;
}

}  // namespace
}  // namespace mlmc

using namespace mlmc;

extern "C" {

int mlmc_probe_gather_mode(const void *table, int32_t log2_records, int32_t waves_per_cu, int32_t iters,
                           int32_t mode, uint64_t *gathers, double *ms, void *stream)
{
    if (!table || !gathers || !ms) return probe_fail(MLMC_ERR_INVALID_ARG, "null argument");
    if (mode & ~(MLMC_PROBE_LDS | MLMC_PROBE_DEPENDENT)) return probe_fail(MLMC_ERR_INVALID_ARG, "unknown mode bits");
    const bool lds = (mode & MLMC_PROBE_LDS) != 0, dep = (mode & MLMC_PROBE_DEPENDENT) != 0;
    if (log2_records < 0 || log2_records > (lds ? 12 : 32))
        return probe_fail(MLMC_ERR_INVALID_ARG, lds ? "log2_records must be in [0, 12] with MLMC_PROBE_LDS"
                                                    : "log2_records must be in [0, 32]");
    if (waves_per_cu < 4 || waves_per_cu > 32 || waves_per_cu % 4)
        return probe_fail(MLMC_ERR_INVALID_ARG, "waves_per_cu must be 4, 8, ..., 32");
    if (iters < 1) return probe_fail(MLMC_ERR_INVALID_ARG, "iters must be >= 1");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t blocks = 0, *sink = nullptr;
    int rc = grid_for(waves_per_cu, &blocks);
    if (!rc) rc = sink_buffer(&sink);
    if (rc) return rc;
    const uint32_t mask = log2_records >= 32 ? 0xFFFFFFFFu : (1u << log2_records) - 1u;
    const size_t shmem = lds ? (static_cast<size_t>(16) << log2_records) : 0;
    const uint4 *t = static_cast<const uint4 *>(table);
    const uint32_t it = static_cast<uint32_t>(iters);
    uint32_t seed = 1;
    rc = time_launch([&] {
        if (lds && dep)
            hipLaunchKernelGGL((gather_probe_kernel<true, true, 1>), dim3(blocks), dim3(kProbeBlock), shmem, s, t, mask,
                               it, seed++, sink);
        else if (lds)
            hipLaunchKernelGGL((gather_probe_kernel<true, false, kChains>), dim3(blocks), dim3(kProbeBlock), shmem, s, t,
                               mask, it, seed++, sink);
        else if (dep)
            hipLaunchKernelGGL((gather_probe_kernel<false, true, 1>), dim3(blocks), dim3(kProbeBlock), 0, s, t, mask, it,
                               seed++, sink);
        else
            hipLaunchKernelGGL((gather_probe_kernel<false, false, kChains>), dim3(blocks), dim3(kProbeBlock), 0, s, t,
                               mask, it, seed++, sink);
    }, s, ms);
    if (rc) return rc;
    *gathers = static_cast<uint64_t>(blocks) * kProbeBlock * static_cast<uint64_t>(iters) * (dep ? 1 : kChains);
    return MLMC_OK;
}

int mlmc_probe_gather(const void *table, int32_t log2_records, int32_t waves_per_cu, int32_t iters,
                      uint64_t *gathers, double *ms, void *stream)
{
    return mlmc_probe_gather_mode(table, log2_records, waves_per_cu, iters, 0, gathers, ms, stream);
}

int mlmc_probe_valu(int32_t waves_per_cu, int32_t iters, uint64_t *lane_ops, double *ms, void *stream)
{
    if (!lane_ops || !ms) return probe_fail(MLMC_ERR_INVALID_ARG, "null argument");
    if (waves_per_cu < 4 || waves_per_cu > 32 || waves_per_cu % 4)
        return probe_fail(MLMC_ERR_INVALID_ARG, "waves_per_cu must be 4, 8, ..., 32");
    if (iters < 1) return probe_fail(MLMC_ERR_INVALID_ARG, "iters must be >= 1");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t blocks = 0, *sink = nullptr;
    int rc = grid_for(waves_per_cu, &blocks);
    if (!rc) rc = sink_buffer(&sink);
    if (rc) return rc;
    uint32_t seed = 1;
    rc = time_launch([&] {
        hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(kProbeBlock), 0, s,
                           static_cast<uint32_t>(iters), seed++, sink);
    }, s, ms);
    if (rc) return rc;
    *lane_ops = static_cast<uint64_t>(blocks) * kProbeBlock * static_cast<uint64_t>(iters) * kChains;
    return MLMC_OK;
}

}  // extern "C"
