// Scalar functional (w, exp(beta A) u) by walks from random start rows: the full-vector
// representation of section 2.1 (a walk started at row l with probability |u_l| / U, U the
// sum of |u|, evolving with the transposed generator) summed against w. The walks run on the
// plan of A^T, whose rows are the columns of A: walk m draws its start row from an alias
// table over rows and its sample is U sign(u_l) w_j (eta_fine - eta_coarse) above l0 and
// U sign(u_l) w_j eta_fine at l0, j the final state. Levels combine by the estimator of
// section 2.2, sample sizes by Algorithm 1 on the scalar's variance. For a symmetric A (a
// network's adjacency matrix) the plan of A serves, and u = w = 1 gives the total
// communicability.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mlmc_expv.h"
#include "common.h"
#include "driver.h"
#include "kernels.h"
#include "plan.h"
#include "walk_engine.h"

namespace mlmc {
namespace {

constexpr uint32_t kFuncChunk = 2048;   // walks per item (one wave)

template <typename R, typename U, bool kHash>
__global__ __launch_bounds__(kBlock, (sizeof(R) == 4 ? 4 : 2)) void functional_walks(LevelArgs L, AliasStart st, const U *__restrict__ w,
                                                           uint32_t walk0, uint32_t M, uint32_t items,
                                                           double *partial, unsigned long long *counters,
                                                           unsigned long long *hash_sum)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t item = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (item >= items) return;
    const uint64_t wb = static_cast<uint64_t>(item) * kFuncChunk;
    const uint64_t we = (wb + kFuncChunk < M) ? wb + kFuncChunk : static_cast<uint64_t>(M);
    SinkR1<R, U> sink{w, nullptr};
    walk_range_from<R, kHash, false, false>(L, st, walk0, wb, we, sink);
    const double a = wave_sum(sink.mom.first());
    const double b = wave_sum(sink.mom.second());
    const unsigned long long jumps = wave_sum_u(sink.jumps);
    const unsigned long long nonfinite = wave_sum_u(sink.nonfinite);
    const unsigned long long hsum = wave_sum_u(sink.hash);
    if (lane == 0) {
        partial[static_cast<size_t>(item) * 2 + 0] = a;
        partial[static_cast<size_t>(item) * 2 + 1] = b;
        unsigned long long *c = counter_slot(counters, item);
        if (jumps) atomicAdd(&c[0], jumps);
        if (nonfinite) atomicAdd(&c[1], nonfinite);
        if (kHash) atomicAdd(hash_sum, hsum);
    }
}

// The forward representation of the full vector: the same walks deposit their samples at
// their final states.
template <typename R, bool kHash>
__global__ __launch_bounds__(kBlock, (sizeof(R) == 4 ? 6 : 2)) void forward_walks(LevelArgs L, AliasStart st, uint32_t walk0, uint32_t M,
                                                        uint32_t items, double *sum1, double *sum2,
                                                        unsigned long long *counters,
                                                        unsigned long long *hash_sum)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t item = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (item >= items) return;
    const uint64_t wb = static_cast<uint64_t>(item) * kFuncChunk;
    const uint64_t we = (wb + kFuncChunk < M) ? wb + kFuncChunk : static_cast<uint64_t>(M);
    SinkDeposit<R> sink{sum1, sum2};
    walk_range_from<R, kHash, false, false>(L, st, walk0, wb, we, sink);
    const unsigned long long jumps = wave_sum_u(sink.jumps);
    const unsigned long long nonfinite = wave_sum_u(sink.nonfinite);
    const unsigned long long hsum = wave_sum_u(sink.hash);
    if (lane == 0) {
        unsigned long long *c = counter_slot(counters, item);
        if (jumps) atomicAdd(&c[0], jumps);
        if (nonfinite) atomicAdd(&c[1], nonfinite);
        if (kHash) atomicAdd(hash_sum, hsum);
    }
}

// x += scale sum1 and, with var, var += scale^2 (sum2 / M - (sum1 / M)^2) / (M - 1) (a level's
// term of the forward estimate and of its per-entry variance, the per-walk variance made
// unbiased; M = 1 divides by M).
__global__ void forward_combine(const double *__restrict__ sum1, const double *__restrict__ sum2, int64_t n,
                                double U, double M, double *x, double *var)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double m = sum1[j] / M;
    x[j] += U * m;
    if (var) var[j] += U * U * fmax(sum2[j] / M - m * m, 0.0) / (M > 1.0 ? M - 1.0 : M);
}

// Per-level moments over the entries: sum of (U m_j)^2 and of U^2 (sum2_j / M - m_j^2), in a
// fixed order: each workgroup reduces a contiguous range of entries into part[2 b], part[2 b
// + 1], then one workgroup adds the partial sums in order.
__device__ __forceinline__ void block_sum2(double &a, double &b)
{
    __shared__ double s1[256], s2[256];
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    a = s1[0];
    b = s2[0];
}

__global__ __launch_bounds__(256) void forward_moments_partial(const double *__restrict__ sum1,
                                                               const double *__restrict__ sum2, int64_t n,
                                                               double U, double M, int64_t per_block,
                                                               double *part)
{
    const int64_t begin = static_cast<int64_t>(blockIdx.x) * per_block;
    const int64_t end = min(begin + per_block, n);
    double a = 0.0, b = 0.0;
    for (int64_t j = begin + threadIdx.x; j < end; j += 256) {
        const double m = sum1[j] / M;
        a += (U * m) * (U * m);
        b += U * U * fmax(sum2[j] / M - m * m, 0.0);
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

__global__ __launch_bounds__(256) void forward_moments_final(const double *__restrict__ part, int blocks,
                                                             double *out)
{
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < blocks; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

// out[0..1] as above; out[2 .. 2 + 2 kMomentBlocks) holds the partial sums.
hipError_t launch_forward_moments(const double *sum1, const double *sum2, int64_t n, double U, double M,
                                  double *out, hipStream_t s)
{
    const int64_t per_block = std::max<int64_t>((n + kMomentBlocks - 1) / kMomentBlocks, 4096);
    const int blocks = static_cast<int>(std::max<int64_t>(1, (n + per_block - 1) / per_block));
    hipLaunchKernelGGL(forward_moments_partial, dim3(blocks), dim3(256), 0, s, sum1, sum2, n, U, M, per_block,
                       out + 2);
    hipLaunchKernelGGL(forward_moments_final, dim3(1), dim3(256), 0, s, out + 2, blocks, out);
    return hipGetLastError();
}

// Sums of the items' partial sums in a fixed order.
__global__ void functional_total(const double *partial, uint32_t items, double *out)
{
    __shared__ double s1[256], s2[256];
    double a = 0.0, b = 0.0;
    for (uint32_t i = threadIdx.x; i < items; i += 256) {
        a += partial[static_cast<size_t>(i) * 2];
        b += partial[static_cast<size_t>(i) * 2 + 1];
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s1[0];
        out[1] = s2[0];
    }
}

// Device buffers of one functional call: the start tables and the scratch.
struct FuncCall {
    uint32_t *thr = nullptr;
    int32_t *alias = nullptr;
    uint8_t *neg = nullptr;
    double *partial = nullptr;
    size_t partial_items = 0;
    double *total = nullptr;           // 2 doubles
    unsigned long long *ctr = nullptr; // a counter set, then its two sums and the hash sum
    double U = 0.0;
    ~FuncCall()
    {
        (void)hipFree(thr);
        (void)hipFree(alias);
        (void)hipFree(neg);
        (void)hipFree(partial);
        (void)hipFree(total);
        (void)hipFree(ctr);
    }
};

// A pair of timing events, destroyed when it goes out of scope.
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~EventPair()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

template <typename T>
int dalloc(T **p, size_t count)
{
    const hipError_t e = hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? MLMC_ERR_OUT_OF_MEMORY : MLMC_ERR_HIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return MLMC_OK;
}

// Start law |u_l| / U: U is the sum of |u_l| in row order; the alias table is the slot
// construction of the plan (scaled probabilities (|u_l| / U) n, two LIFO lists filled in
// row order).
int prepare(FuncCall &fc, const mlmc_plan *p, const void *u, int u_f64, hipStream_t s)
{
    const int64_t n = p->n;
    std::vector<double> h(static_cast<size_t>(n));
    if (u_f64) {
        MLMC_HIP_TRY(hipMemcpyAsync(h.data(), u, n * sizeof(double), hipMemcpyDeviceToHost, s));
        MLMC_HIP_TRY(hipStreamSynchronize(s));
    } else {
        std::vector<float> f(static_cast<size_t>(n));
        MLMC_HIP_TRY(hipMemcpyAsync(f.data(), u, n * sizeof(float), hipMemcpyDeviceToHost, s));
        MLMC_HIP_TRY(hipStreamSynchronize(s));
        for (int64_t i = 0; i < n; ++i) h[i] = static_cast<double>(f[i]);
    }
    double U = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(h[i])) return fail(MLMC_ERR_INVALID_ARG, "u has a non-finite entry");
        U += std::fabs(h[i]);
    }
    fc.U = U;
    std::vector<uint32_t> thr(static_cast<size_t>(n), 0xFFFFFFFFu);
    std::vector<int32_t> alias(static_cast<size_t>(n));
    std::vector<uint8_t> neg(static_cast<size_t>(n));
    std::vector<double> q(static_cast<size_t>(n));
    std::vector<int64_t> small, large;
    for (int64_t i = 0; i < n; ++i) {
        alias[i] = static_cast<int32_t>(i);
        neg[i] = h[i] < 0.0 ? 1 : 0;
        q[i] = U > 0.0 ? (std::fabs(h[i]) / U) * static_cast<double>(n) : 1.0;
        (q[i] < 1.0 ? small : large).push_back(i);
    }
    while (!small.empty() && !large.empty()) {
        const int64_t lo = small.back();
        small.pop_back();
        const int64_t hi = large.back();
        large.pop_back();
        thr[lo] = static_cast<uint32_t>(std::floor(q[lo] * 4294967296.0));
        alias[lo] = static_cast<int32_t>(hi);
        q[hi] = (q[hi] + q[lo]) - 1.0;
        (q[hi] < 1.0 ? small : large).push_back(hi);
    }
    int rc;
    if ((rc = dalloc(&fc.thr, n)) || (rc = dalloc(&fc.alias, n)) || (rc = dalloc(&fc.neg, n)) ||
        (rc = dalloc(&fc.total, 2)) || (rc = dalloc(&fc.ctr, kCounterSetU64 + 3)))
        return rc;
    MLMC_HIP_TRY(hipMemcpyAsync(fc.thr, thr.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    MLMC_HIP_TRY(hipMemcpyAsync(fc.alias, alias.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    MLMC_HIP_TRY(hipMemcpyAsync(fc.neg, neg.data(), n * sizeof(uint8_t), hipMemcpyHostToDevice, s));
    MLMC_HIP_TRY(hipStreamSynchronize(s));   // the host vectors go out of scope
    return MLMC_OK;
}

struct LevelOut {
    double s1 = 0.0, s2 = 0.0;   // sums of the samples (without the factor U) and squares
    unsigned long long jumps = 0, nonfinite = 0, hash = 0;
    float ms = 0.0f;
};

// Walks [walk0, walk0 + M) of one level: sums of the samples, counters, hash sum. Waits.
int run_level(FuncCall &fc, mlmc_plan *p, const void *w, int u_f64, uint64_t seed, int instance, int lev,
          uint32_t walk0, uint64_t M, bool hash, LevelOut &out, hipStream_t s)
{
    out = LevelOut{};
    if (M == 0 || p->n == 0 || fc.U == 0.0) return MLMC_OK;
    if (static_cast<uint64_t>(walk0) + M > 0x100000000ull)
        return fail(MLMC_ERR_RNG_OVERFLOW, "walk indices must stay below 2^32 (the walk word of the Philox counter)");
    int rc = upload_level(p, lev, s);
    if (rc) return rc;
    LevelArgs L = level_args(p, lev, seed, instance);
    L.is_slots = nullptr;
    L.src = nullptr;
    AliasStart st{fc.thr, fc.alias, fc.neg, static_cast<uint32_t>(p->n), stream_word(lev, instance, 2)};
    const uint32_t items = static_cast<uint32_t>((M + kFuncChunk - 1) / kFuncChunk);
    if (items > fc.partial_items) {
        (void)hipFree(fc.partial);
        fc.partial = nullptr;
        if ((rc = dalloc(&fc.partial, 2 * static_cast<size_t>(items)))) return rc;
        fc.partial_items = items;
    }
    MLMC_HIP_TRY(hipMemsetAsync(fc.ctr, 0, (kCounterSetU64 + 3) * sizeof(unsigned long long), s));
    EventPair ev;   // destroyed on every return path
    hipEvent_t &e0 = ev.e0, &e1 = ev.e1;
    MLMC_HIP_TRY(hipEventCreate(&e0));
    MLMC_HIP_TRY(hipEventCreate(&e1));
    MLMC_HIP_TRY(hipEventRecord(e0, s));
    const dim3 grid((items + kWavesPerBlock - 1) / kWavesPerBlock), block(kBlock);
    const uint32_t Mu = static_cast<uint32_t>(M);
#define MLMC_FUNC(R, U, H)                                                                      \
    hipLaunchKernelGGL((functional_walks<R, U, H>), grid, block, 0, s, L, st,                  \
                       static_cast<const U *>(w), walk0, Mu, items, fc.partial, fc.ctr,                 \
                       fc.ctr + kCounterSetU64 + 2)
    if (p->precision == MLMC_PRECISION_FP64) {
        if (u_f64) { if (hash) MLMC_FUNC(double, double, true); else MLMC_FUNC(double, double, false); }
        else { if (hash) MLMC_FUNC(double, float, true); else MLMC_FUNC(double, float, false); }
    } else {
        if (u_f64) { if (hash) MLMC_FUNC(float, double, true); else MLMC_FUNC(float, double, false); }
        else { if (hash) MLMC_FUNC(float, float, true); else MLMC_FUNC(float, float, false); }
    }
#undef MLMC_FUNC
    MLMC_HIP_TRY(hipGetLastError());
    MLMC_HIP_TRY(hipEventRecord(e1, s));
    hipLaunchKernelGGL(functional_total, dim3(1), dim3(256), 0, s, fc.partial, items, fc.total);
    MLMC_HIP_TRY(hipGetLastError());
    MLMC_HIP_TRY(launch_counter_sum(fc.ctr, 1, fc.ctr + kCounterSetU64, s));
    double tot[2];
    unsigned long long c[3];
    void *pin = nullptr;
    if ((rc = plan_pinned(p, sizeof tot + sizeof c, &pin))) return rc;
    MLMC_HIP_TRY(hipMemcpyAsync(pin, fc.total, sizeof tot, hipMemcpyDeviceToHost, s));
    MLMC_HIP_TRY(hipMemcpyAsync(static_cast<char *>(pin) + sizeof tot, fc.ctr + kCounterSetU64, sizeof c,
                                hipMemcpyDeviceToHost, s));
    MLMC_HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(tot, pin, sizeof tot);
    std::memcpy(c, static_cast<char *>(pin) + sizeof tot, sizeof c);
    (void)hipEventElapsedTime(&out.ms, e0, e1);
    out.s1 = tot[0];
    out.s2 = tot[1];
    out.jumps = c[0];
    out.nonfinite = c[1];
    out.hash = c[2];
    return MLMC_OK;
}

// Walks [walk0, walk0 + M) of one level of the forward representation: the deposits into
// sum1, sum2 (zeroed first), counters and hash sum. Waits.
int run_forward_level(FuncCall &fc, mlmc_plan *p, uint64_t seed, int instance, int lev, uint32_t walk0,
                      uint64_t M, bool hash, double *sum1, double *sum2, LevelOut &out, hipStream_t s,
                      bool accumulate = false)
{
    out = LevelOut{};
    if (p->n == 0) return MLMC_OK;
    if (!accumulate) {
        MLMC_HIP_TRY(hipMemsetAsync(sum1, 0, p->n * sizeof(double), s));
        MLMC_HIP_TRY(hipMemsetAsync(sum2, 0, p->n * sizeof(double), s));
    }
    if (M == 0 || fc.U == 0.0) return MLMC_OK;
    if (static_cast<uint64_t>(walk0) + M > 0x100000000ull)
        return fail(MLMC_ERR_RNG_OVERFLOW, "walk indices must stay below 2^32 (the walk word of the Philox counter)");
    int rc = upload_level(p, lev, s);
    if (rc) return rc;
    LevelArgs L = level_args(p, lev, seed, instance);
    L.is_slots = nullptr;
    L.src = nullptr;
    AliasStart st{fc.thr, fc.alias, fc.neg, static_cast<uint32_t>(p->n), stream_word(lev, instance, 2)};
    const uint32_t items = static_cast<uint32_t>((M + kFuncChunk - 1) / kFuncChunk);
    MLMC_HIP_TRY(hipMemsetAsync(fc.ctr, 0, (kCounterSetU64 + 3) * sizeof(unsigned long long), s));
    EventPair ev;   // destroyed on every return path
    hipEvent_t &e0 = ev.e0, &e1 = ev.e1;
    MLMC_HIP_TRY(hipEventCreate(&e0));
    MLMC_HIP_TRY(hipEventCreate(&e1));
    MLMC_HIP_TRY(hipEventRecord(e0, s));
    const dim3 grid((items + kWavesPerBlock - 1) / kWavesPerBlock), block(kBlock);
    const uint32_t Mu = static_cast<uint32_t>(M);
    unsigned long long *hs = fc.ctr + kCounterSetU64 + 2;
    if (p->precision == MLMC_PRECISION_FP64) {
        if (hash) hipLaunchKernelGGL((forward_walks<double, true>), grid, block, 0, s, L, st, walk0, Mu, items, sum1, sum2, fc.ctr, hs);
        else hipLaunchKernelGGL((forward_walks<double, false>), grid, block, 0, s, L, st, walk0, Mu, items, sum1, sum2, fc.ctr, hs);
    } else {
        if (hash) hipLaunchKernelGGL((forward_walks<float, true>), grid, block, 0, s, L, st, walk0, Mu, items, sum1, sum2, fc.ctr, hs);
        else hipLaunchKernelGGL((forward_walks<float, false>), grid, block, 0, s, L, st, walk0, Mu, items, sum1, sum2, fc.ctr, hs);
    }
    MLMC_HIP_TRY(hipGetLastError());
    MLMC_HIP_TRY(hipEventRecord(e1, s));
    MLMC_HIP_TRY(launch_counter_sum(fc.ctr, 1, fc.ctr + kCounterSetU64, s));
    unsigned long long c[3];
    void *pin = nullptr;
    if ((rc = plan_pinned(p, sizeof c, &pin))) return rc;
    MLMC_HIP_TRY(hipMemcpyAsync(pin, fc.ctr + kCounterSetU64, sizeof c, hipMemcpyDeviceToHost, s));
    MLMC_HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(c, pin, sizeof c);
    (void)hipEventElapsedTime(&out.ms, e0, e1);
    out.jumps = c[0];
    out.nonfinite = c[1];
    out.hash = c[2];
    return MLMC_OK;
}

int check_args(const mlmc_plan *p, const void *u, const void *w, int32_t dtype)
{
    if (!p) return fail(MLMC_ERR_INVALID_ARG, "null plan");
    if (p->n > 0 && (!u || !w)) return fail(MLMC_ERR_INVALID_ARG, "u or w is null");
    if (dtype != MLMC_DTYPE_F32 && dtype != MLMC_DTYPE_F64)
        return fail(MLMC_ERR_INVALID_ARG, "dtype must be MLMC_DTYPE_F32 or MLMC_DTYPE_F64");
    if (p->n >= (int64_t(1) << 32)) return fail(MLMC_ERR_UNSUPPORTED, "n must be below 2^32");
    return MLMC_OK;
}

}  // namespace
}  // namespace mlmc

using namespace mlmc;

extern "C" {

int mlmc_expv_functional_level_sums(mlmc_plan_t *p, const void *u, const void *w, int32_t dtype, uint64_t seed,
                                    int32_t instance, int32_t level, uint32_t walk0, uint32_t walks,
                                    double *sum1, double *sum2, int64_t *jumps, uint64_t *hash_sum,
                                    double *U, void *stream)
{
    int rc = check_args(p, u, w, dtype);
    if (rc) return rc;
    if (!sum1 || !sum2) return fail(MLMC_ERR_INVALID_ARG, "sum1 or sum2 is null");
    if (instance < 0 || instance > 4095) return fail(MLMC_ERR_INVALID_ARG, "instance must be in [0, 4095]");
    if (level < 0 || level > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "level out of range [0, 28]");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    FuncCall fc;
    const int f64 = dtype == MLMC_DTYPE_F64;
    if ((rc = prepare(fc, p, u, f64, s))) return rc;
    LevelOut o;
    if ((rc = run_level(fc, p, w, f64, seed, instance, level, walk0, walks, hash_sum != nullptr, o, s))) return rc;
    *sum1 = o.s1;
    *sum2 = o.s2;
    if (jumps) *jumps = static_cast<int64_t>(o.jumps);
    if (hash_sum) *hash_sum = o.hash;
    if (U) *U = fc.U;
    if (o.nonfinite) return fail(MLMC_ERR_NONFINITE, std::to_string(o.nonfinite) + " non-finite samples");
    return MLMC_OK;
}

int mlmc_expv_functional(mlmc_plan_t *p, const void *u, const void *w, int32_t dtype, const mlmc_run_opts_t *o,
                         double *result, double *variance, mlmc_stats_t *stats, void *stream)
{
    int rc = check_args(p, u, w, dtype);
    if (rc) return rc;
    if (!o || !result) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    if (o->instance < 0 || o->instance > 4095) return fail(MLMC_ERR_INVALID_ARG, "instance must be in [0, 4095]");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const bool adaptive = o->eps > 0.0;
    int max_levels;
    const int64_t pilot = o->pilot_walks == 0 ? default_pilot(1) : o->pilot_walks;
    if (adaptive) {
        if (pilot < 2 || pilot >= (int64_t(1) << 32))
            return fail(MLMC_ERR_INVALID_ARG, "pilot_walks must be 0 or in [2, 2^32)");
        max_levels = o->max_levels > 0 ? o->max_levels : 20;
        max_levels = std::min(max_levels, std::min(MLMC_MAX_LEVELS, kMaxLevel - p->l0 + 1));
        if (max_levels < 2) return fail(MLMC_ERR_INVALID_ARG, "max_levels must allow at least two levels");
    } else {
        if (o->num_levels < 1 || o->num_levels > MLMC_MAX_LEVELS || p->l0 + o->num_levels - 1 > kMaxLevel)
            return fail(MLMC_ERR_INVALID_ARG, "num_levels out of range");
        if (!o->walks) return fail(MLMC_ERR_INVALID_ARG, "walks is null");
        for (int q = 0; q < o->num_levels; ++q)
            if (o->walks[q] < 1 || o->walks[q] >= (int64_t(1) << 32))
                return fail(MLMC_ERR_INVALID_ARG, "walks per level must be in [1, 2^32)");
        max_levels = o->num_levels;
    }
    const int f64 = dtype == MLMC_DTYPE_F64;
    FuncCall fc;
    if ((rc = prepare(fc, p, u, f64, s))) return rc;
    const double UU = fc.U;
    std::vector<int64_t> M(static_cast<size_t>(max_levels), 0);
    std::vector<double> S1(max_levels, 0.0), S2(max_levels, 0.0);
    std::vector<unsigned long long> J(max_levels, 0);
    unsigned long long nonfinite = 0;
    double wk_ms = 0.0;
    int64_t launches = 0;
    auto add = [&](int q, int64_t extra) -> int {
        LevelOut lo;
        const int r2 = run_level(fc, p, w, f64, o->seed, o->instance, p->l0 + q, static_cast<uint32_t>(M[q]),
                             static_cast<uint64_t>(extra), false, lo, s);
        if (r2) return r2;
        S1[q] += lo.s1;
        S2[q] += lo.s2;
        J[q] += lo.jumps;
        nonfinite += lo.nonfinite;
        wk_ms += lo.ms;
        ++launches;
        M[q] += extra;
        return MLMC_OK;
    };
    // per-walk variance of U * sample, and the cost per walk N_l + 4 jumps
    auto var_of = [&](int q) {
        const double m = S1[q] / static_cast<double>(M[q]);
        return unbiased_var(std::max(S2[q] / static_cast<double>(M[q]) - m * m, 0.0) * UU * UU, M[q]);
    };
    auto cost_of = [&](int q) {
        return std::ldexp(1.0, p->l0 + q) + 4.0 * static_cast<double>(J[q]) / static_cast<double>(M[q]);
    };
    auto mean_of = [&](int q) { return UU * S1[q] / static_cast<double>(M[q]); };
    int levels = 0, iterations = 0;
    bool converged = false;
    double bias = 0.0;
    EventPair ev;   // destroyed on every return path
    hipEvent_t &e0 = ev.e0, &e1 = ev.e1;
    MLMC_HIP_TRY(hipEventCreate(&e0));
    MLMC_HIP_TRY(hipEventCreate(&e1));
    MLMC_HIP_TRY(hipEventRecord(e0, s));
    if (!adaptive) {
        levels = o->num_levels;
        for (int q = 0; q < levels; ++q)
            if ((rc = add(q, o->walks[q]))) return rc;
        converged = true;
    } else {
        // Algorithm 1 on the scalar's variance
        DriverOpts d;
        d.eps = o->eps;
        d.pilot = pilot;
        d.max_levels = max_levels;
        d.cap = o->max_walks > 0 ? std::min<int64_t>(o->max_walks, 0xFFFFFFFFll) : 0xFFFFFFFFll;
        auto measure = [&](int lv, std::vector<LevelEstimate> &est) -> int {
            for (int q = 0; q < lv; ++q)
                est[q] = LevelEstimate{var_of(q), cost_of(q), debiased_rms(mean_of(q) * mean_of(q), var_of(q), M[q])};
            return MLMC_OK;
        };
        DriverOut out;
        if ((rc = algorithm1(d, M, add, measure, out))) return rc;
        levels = out.levels;
        converged = out.converged;
        iterations = out.iterations;
        bias = out.bias;
    }
    MLMC_HIP_TRY(hipEventRecord(e1, s));
    MLMC_HIP_TRY(hipEventSynchronize(e1));
    double x = 0.0, var = 0.0;
    for (int q = 0; q < levels; ++q) {
        x += mean_of(q);
        var += var_of(q) / static_cast<double>(M[q]);
    }
    *result = x;
    if (variance) *variance = var;
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->l0 = p->l0;
        stats->num_levels = levels;
        stats->converged = converged ? 1 : 0;
        stats->driver_iterations = iterations;
        for (int q = 0; q < levels; ++q) {
            stats->walks[q] = M[q];
            stats->jumps[q] = static_cast<int64_t>(J[q]);
            stats->level_mean_rms[q] = debiased_rms(mean_of(q) * mean_of(q), var_of(q), M[q]);
            stats->level_var[q] = var_of(q);
            stats->level_cost[q] = cost_of(q);
            stats->steps += M[q] * (int64_t(1) << (p->l0 + q));
            stats->total_jumps += static_cast<int64_t>(J[q]);
        }
        stats->nonfinite = static_cast<int64_t>(nonfinite);
        stats->est_variance = var;
        stats->est_bias = adaptive ? bias : 0.0;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        stats->kernel_ms = ms;
        stats->walk_kernel_ms = wk_ms;
        stats->walk_launches = launches;
    }
    if (nonfinite) return fail(MLMC_ERR_NONFINITE, std::to_string(nonfinite) + " non-finite samples");
    if (adaptive && !converged) return fail(MLMC_ERR_NOT_CONVERGED, "level or walk cap reached before eps");
    return MLMC_OK;
}

int mlmc_expv_forward_level_sums(mlmc_plan_t *p, const void *u, int32_t dtype, uint64_t seed, int32_t instance,
                                 int32_t level, uint32_t walk0, uint32_t walks, double *sum1, double *sum2,
                                 int64_t *jumps, uint64_t *hash_sum, double *U, void *stream)
{
    int rc = check_args(p, u, u, dtype);
    if (rc) return rc;
    if (p->n > 0 && (!sum1 || !sum2)) return fail(MLMC_ERR_INVALID_ARG, "sum1 or sum2 is null");
    if (instance < 0 || instance > 4095) return fail(MLMC_ERR_INVALID_ARG, "instance must be in [0, 4095]");
    if (level < 0 || level > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "level out of range [0, 28]");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    FuncCall fc;
    if ((rc = prepare(fc, p, u, dtype == MLMC_DTYPE_F64, s))) return rc;
    LevelOut o;
    if ((rc = run_forward_level(fc, p, seed, instance, level, walk0, walks, hash_sum != nullptr, sum1, sum2, o, s)))
        return rc;
    if (jumps) *jumps = static_cast<int64_t>(o.jumps);
    if (hash_sum) *hash_sum = o.hash;
    if (U) *U = fc.U;
    if (o.nonfinite) return fail(MLMC_ERR_NONFINITE, std::to_string(o.nonfinite) + " non-finite samples");
    return MLMC_OK;
}

int mlmc_expv_forward(mlmc_plan_t *p, const void *u, int32_t dtype, const mlmc_run_opts_t *o, double *x,
                      double *variance, mlmc_stats_t *stats, void *stream)
{
    int rc = check_args(p, u, u, dtype);
    if (rc) return rc;
    if (!o) return fail(MLMC_ERR_INVALID_ARG, "null options");
    if (p->n > 0 && !x) return fail(MLMC_ERR_INVALID_ARG, "x is null");
    if (o->instance < 0 || o->instance > 4095) return fail(MLMC_ERR_INVALID_ARG, "instance must be in [0, 4095]");
    const bool adaptive = o->eps > 0.0;
    int max_levels;
    const int64_t pilot = o->pilot_walks == 0 ? default_pilot(1) : o->pilot_walks;
    if (adaptive) {
        if (pilot < 2 || pilot >= (int64_t(1) << 32))
            return fail(MLMC_ERR_INVALID_ARG, "pilot_walks must be 0 or in [2, 2^32)");
        max_levels = o->max_levels > 0 ? o->max_levels : 20;
        max_levels = std::min(max_levels, std::min(MLMC_MAX_LEVELS, kMaxLevel - p->l0 + 1));
        if (max_levels < 2) return fail(MLMC_ERR_INVALID_ARG, "max_levels must allow at least two levels");
    } else {
        if (o->num_levels < 1 || o->num_levels > MLMC_MAX_LEVELS || p->l0 + o->num_levels - 1 > kMaxLevel)
            return fail(MLMC_ERR_INVALID_ARG, "num_levels out of range");
        if (!o->walks) return fail(MLMC_ERR_INVALID_ARG, "walks is null");
        for (int q = 0; q < o->num_levels; ++q)
            if (o->walks[q] < 1 || o->walks[q] >= (int64_t(1) << 32))
                return fail(MLMC_ERR_INVALID_ARG, "walks per level must be in [1, 2^32)");
        max_levels = o->num_levels;
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = p->n;
    FuncCall fc;
    if ((rc = prepare(fc, p, u, dtype == MLMC_DTYPE_F64, s))) return rc;
    const double UU = fc.U;
    // per level: the deposit sums (2n doubles, kept while walks are added), then two moments
    struct Sums {
        std::vector<double *> v;
        ~Sums()
        {
            for (double *q : v) (void)hipFree(q);
        }
    } lv;
    double *mom = nullptr;
    if ((rc = dalloc(&mom, 2 + 2 * static_cast<size_t>(kMomentBlocks)))) return rc;
    lv.v.push_back(mom);
    std::vector<double *> sums(static_cast<size_t>(max_levels), nullptr);
    std::vector<int64_t> M(static_cast<size_t>(max_levels), 0);
    std::vector<double> rms(max_levels, 0.0), V(max_levels, 0.0);
    std::vector<unsigned long long> J(max_levels, 0);
    unsigned long long nonfinite = 0;
    double wk_ms = 0.0;
    int64_t launches = 0;
    const double nn = static_cast<double>(std::max<int64_t>(n, 1));
    // walks [M[q], M[q] + extra) of level l0 + q added to its sums; then the level's moments
    auto add = [&](int q, int64_t extra) -> int {
        if (!sums[q]) {
            int r2 = dalloc(&sums[q], 2 * static_cast<size_t>(n));
            if (r2) return r2;
            lv.v.push_back(sums[q]);
            if (n > 0) MLMC_HIP_TRY(hipMemsetAsync(sums[q], 0, 2 * n * sizeof(double), s));
        }
        LevelOut lo;
        int r2 = run_forward_level(fc, p, o->seed, o->instance, p->l0 + q, static_cast<uint32_t>(M[q]),
                                   static_cast<uint64_t>(extra), false, sums[q], sums[q] + n, lo, s, true);
        if (r2) return r2;
        M[q] += extra;
        J[q] += lo.jumps;
        nonfinite += lo.nonfinite;
        wk_ms += lo.ms;
        ++launches;
        double h[2] = {0.0, 0.0};
        if (n > 0) {
            MLMC_HIP_TRY(launch_forward_moments(sums[q], sums[q] + n, n, UU, static_cast<double>(M[q]), mom, s));
            void *pin = nullptr;
            if ((r2 = plan_pinned(p, sizeof h, &pin))) return r2;
            MLMC_HIP_TRY(hipMemcpyAsync(pin, mom, sizeof h, hipMemcpyDeviceToHost, s));
            MLMC_HIP_TRY(hipStreamSynchronize(s));
            std::memcpy(h, pin, sizeof h);
        }
        V[q] = unbiased_var(h[1] / nn, M[q]);        // mean over the entries of the per-walk variance
        rms[q] = debiased_rms(h[0] / nn, V[q], M[q]);  // root mean square of the level term
        return MLMC_OK;
    };
    auto cost_of = [&](int q) {
        return std::ldexp(1.0, p->l0 + q) + 4.0 * static_cast<double>(J[q]) / static_cast<double>(M[q]);
    };
    int levels = 0, iterations = 0;
    bool converged = false;
    double bias = 0.0;
    EventPair ev;   // destroyed on every return path
    hipEvent_t &e0 = ev.e0, &e1 = ev.e1;
    MLMC_HIP_TRY(hipEventCreate(&e0));
    MLMC_HIP_TRY(hipEventCreate(&e1));
    MLMC_HIP_TRY(hipEventRecord(e0, s));
    if (!adaptive) {
        levels = o->num_levels;
        for (int q = 0; q < levels; ++q)
            if ((rc = add(q, o->walks[q]))) return rc;
        converged = true;
    } else {
        // Algorithm 1 on the mean over the entries of the per-entry variance and the
        // root-mean-square level terms, as for the backward full vector
        DriverOpts d;
        d.eps = o->eps;
        d.pilot = pilot;
        d.max_levels = max_levels;
        d.cap = o->max_walks > 0 ? std::min<int64_t>(o->max_walks, 0xFFFFFFFFll) : 0xFFFFFFFFll;
        auto measure = [&](int lv, std::vector<LevelEstimate> &est) -> int {
            for (int q = 0; q < lv; ++q) est[q] = LevelEstimate{V[q], cost_of(q), rms[q]};
            return MLMC_OK;
        };
        DriverOut out;
        if ((rc = algorithm1(d, M, add, measure, out))) return rc;
        levels = out.levels;
        converged = out.converged;
        iterations = out.iterations;
        bias = out.bias;
    }
    // x = sum over levels of U sum1 / M, and its per-entry variance
    double est_var = 0.0;
    if (n > 0) {
        MLMC_HIP_TRY(hipMemsetAsync(x, 0, n * sizeof(double), s));
        if (variance) MLMC_HIP_TRY(hipMemsetAsync(variance, 0, n * sizeof(double), s));
    }
    for (int q = 0; q < levels; ++q) {
        est_var += V[q] / static_cast<double>(M[q]);
        if (n > 0) {
            hipLaunchKernelGGL(forward_combine, dim3(static_cast<uint32_t>((n + 255) / 256)), dim3(256), 0, s,
                               sums[q], sums[q] + n, n, UU, static_cast<double>(M[q]), x, variance);
            MLMC_HIP_TRY(hipGetLastError());
        }
    }
    MLMC_HIP_TRY(hipEventRecord(e1, s));
    MLMC_HIP_TRY(hipEventSynchronize(e1));
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->l0 = p->l0;
        stats->num_levels = levels;
        stats->converged = converged ? 1 : 0;
        stats->driver_iterations = iterations;
        for (int q = 0; q < levels; ++q) {
            stats->walks[q] = M[q];
            stats->jumps[q] = static_cast<int64_t>(J[q]);
            stats->level_mean_rms[q] = rms[q];
            stats->level_var[q] = V[q];
            stats->level_cost[q] = cost_of(q);
            stats->steps += M[q] * (int64_t(1) << (p->l0 + q));
            stats->total_jumps += static_cast<int64_t>(J[q]);
        }
        stats->nonfinite = static_cast<int64_t>(nonfinite);
        stats->est_variance = est_var;
        stats->est_bias = adaptive ? bias : 0.0;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        stats->kernel_ms = ms;
        stats->walk_kernel_ms = wk_ms;
        stats->walk_launches = launches;
    }
    if (nonfinite) return fail(MLMC_ERR_NONFINITE, std::to_string(nonfinite) + " non-finite samples");
    if (adaptive && !converged) return fail(MLMC_ERR_NOT_CONVERGED, "level or walk cap reached before eps");
    return MLMC_OK;
}

}  // extern "C"
