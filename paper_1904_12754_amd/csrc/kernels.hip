// Kernels of the single-level path for gfx950: per-row level sums of the walks of one level
// (the sampling of Algorithm 2, see walk_engine.h), step thresholds, moments, the FP64
// level combine and path traces.
#include "common.h"
#include "kernels.h"
#include "walk_engine.h"

#include <algorithm>
#include <cmath>

namespace mlmc {
namespace {

// Sums of item-and-right-hand-side index i (with one chunk per row, i is also the output's
// (row, rhs) index).
__device__ __forceinline__ void store_sums(const SumsOut &o, uint64_t i, double a, double b)
{
    if (o.direct == 0) {
        o.partial[i * 2 + 0] = a;
        o.partial[i * 2 + 1] = b;
    } else if (o.direct == 1) {
        o.out1[i] = a;
        o.out2[i] = b;
    } else {
        o.out1[i] += a;
        o.out2[i] += b;
    }
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Waves per SIMD the single-level kernel is compiled for. The loop waits on dependent
// gathers and long-latency instructions more than it issues, so more resident waves run it
// faster even at the price of spilled registers: with FP32 weights seven on the coarsest
// level (72 VGPRs, 26 spilled) and six above it (80, 21 spilled), five under a proposal or
// with a source term (96, 4 and 10 spilled; under a proposal at the coarsest level 94, none
// spilled, where six waves spill 9 and ran slower). With FP64 weights three run faster than
// two.
template <typename R, bool kIS, bool kSrc, bool kBase>
constexpr int walk_min_waves()
{
    return sizeof(R) == 4 ? (kIS ? 5 : kSrc ? 5 : kBase ? 7 : 6) : 3;
}

// Items are (requested row, walk chunk) pairs; a wave takes 64 / lpr consecutive items, one
// per group of lpr lanes (lpr a power of two, 1..64).
template <typename R, typename U, bool kHash, bool kIS, bool kSrc, bool kBase>
__global__ __launch_bounds__(kBlock, (walk_min_waves<R, kIS, kSrc, kBase>())) void level_walks_r1(LevelArgs L, const U *__restrict__ u,
                                                         const int64_t *__restrict__ rows,
                                                         uint32_t n_rows, uint32_t walk0,
                                                         uint32_t M, uint32_t chunk,
                                                         uint32_t chunks, uint32_t lpr,
                                                         SumsOut out,
                                                         unsigned long long *counters,
                                                         unsigned long long *hash_sums)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t per_wave = kWave / lpr;
    const uint64_t total = static_cast<uint64_t>(n_rows) * chunks;
    const uint64_t wave = static_cast<uint64_t>(blockIdx.x) * kWavesPerBlock + (threadIdx.x / kWave);
    if (wave * per_wave >= total) return;
    const uint64_t item = wave * per_wave + lane / lpr;
    const bool has = item < total;
    const uint32_t q = has ? static_cast<uint32_t>(item / chunks) : 0u;
    const uint32_t c = has ? static_cast<uint32_t>(item % chunks) : 0u;
    const uint32_t row = rows ? static_cast<uint32_t>(rows[q]) : q;
    const uint64_t wb = has ? static_cast<uint64_t>(c) * chunk : 0ull;
    const uint64_t we = has ? min(wb + chunk, static_cast<uint64_t>(M)) : 0ull;
    SinkR1<R, U, kSrc> sink{u, static_cast<const U *>(L.src)};
    bool done = false;
    if constexpr (!kIS && !kSrc) {
        // one item per wave: its row and walk range are wave-uniform, so the engine's group
        // bookkeeping and the start row's record stay in scalar registers (the walks under
        // a proposal or with a source term keep the general path: a second copy of the
        // engine would cost them a wave per SIMD)
        if (lpr == kWave) {
            const uint32_t urow = __builtin_amdgcn_readfirstlane(row);
            const uint64_t uwb = uniform64(wb), uwe = uniform64(we);
            walk_range<R, kHash, kIS, kSrc, kBase>(L, urow, walk0, uwb, uwe, sink);
            done = true;
        }
    }
    if (!done) walk_range<R, kHash, kIS, kSrc, kBase>(L, row, walk0, wb, we, sink, lpr);
    const double a = group_sum(sink.mom.first(), lpr);
    const double b = group_sum(sink.mom.second(), lpr);
    const unsigned long long jumps = wave_sum_u(sink.jumps);
    const unsigned long long nonfinite = wave_sum_u(sink.nonfinite);
    const unsigned long long hsum = group_sum_u(sink.hash, lpr);
    if (has && (lane & (lpr - 1)) == 0) {
        store_sums(out, item, a, b);
        if (kHash) atomicAdd(&hash_sums[q], hsum);
    }
    if (lane == 0) {
        unsigned long long *c = counter_slot(counters, wave);
        if (jumps) atomicAdd(&c[0], jumps);
        if (nonfinite) atomicAdd(&c[1], nonfinite);
    }
}

template <typename R, typename U, bool kHash, bool kIS>
__global__ __launch_bounds__(kRhsBlock, (sizeof(R) == 4 ? 4 : 2)) void level_walks_rhs(LevelArgs L, const U *__restrict__ u,
                                                          int32_t nrhs,
                                                          const int64_t *__restrict__ rows,
                                                          uint32_t n_rows, uint32_t walk0,
                                                          uint32_t M, uint32_t chunk,
                                                          uint32_t chunks, SumsOut out,
                                                          unsigned long long *counters,
                                                          unsigned long long *hash_sums)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t item = blockIdx.x;                  // one wave per workgroup
    if (item >= static_cast<uint64_t>(n_rows) * chunks) return;
    const uint32_t q = static_cast<uint32_t>(item / chunks);
    const uint32_t c = static_cast<uint32_t>(item % chunks);
    const uint32_t row = rows ? static_cast<uint32_t>(rows[q]) : q;
    const uint64_t wb = static_cast<uint64_t>(c) * chunk;
    const uint64_t we = min(wb + chunk, static_cast<uint64_t>(M));
    SinkRhs<R, U> sink{u, nrhs, (nrhs + kWave - 1) / kWave};
    walk_range<R, kHash, kIS, false, false, !kHash>(L, row, walk0, wb, we, sink);
    const unsigned long long jumps = wave_sum_u(sink.jumps);
    const unsigned long long nojump = wave_sum_u(sink.nojump);
    const unsigned long long nonfinite = wave_sum_u(sink.nonfinite);
    const unsigned long long hsum = wave_sum_u(sink.hash);
    // walks without a jump: Y = u_row e^{d_row beta} at the base level, 0 above it
    const R hd = static_cast<R>(L.half_dt);
    R y0 = 0;
    if (nojump && L.base) {
        const RowRec rr = L.rec[row];
        y0 = expR(d_of<R>(rr) * static_cast<R>(2 * L.N) * hd);
    }
#pragma unroll
    for (int g = 0; g < kMaxRhsGroups; ++g) {
        const int r = static_cast<int>(lane) + g * kWave;
        if (g < sink.groups && r < nrhs) {
            double a = sink.mom[g].first(), b = sink.mom[g].second();
            if (y0 != static_cast<R>(0)) {
                const double yr = static_cast<double>(
                    y0 * static_cast<R>(u[static_cast<uint64_t>(row) * nrhs + r]));
                a += static_cast<double>(nojump) * yr;
                b += static_cast<double>(nojump) * yr * yr;
            }
            store_sums(out, item * nrhs + r, a, b);
        }
    }
    if (lane == 0) {
        unsigned long long *c = counter_slot(counters, item);
        if (jumps) atomicAdd(&c[0], jumps);   // most items of a screened level have none
        if (nonfinite) atomicAdd(&c[1], nonfinite);
        if (kHash) atomicAdd(&hash_sums[q], hsum);
    }
}

__global__ void thresholds_kernel(RowRec *rec, int64_t n, double dt, unsigned int *bad)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double inv_r = rec[i].inv_r;
    uint32_t thr;
    if (!(inv_r < INFINITY)) {
        thr = 0xFFFFFFFFu;                                    // absorbing: never jumps
    } else if (neg_log_uniform(0xFFFFFFFFu) * inv_r >= dt) {
        thr = 0xFFFFFFFFu;                                    // no word is small enough
    } else if (neg_log_uniform(0u) * inv_r < dt) {
        atomicOr(bad, 1u);                                    // every word jumps
        thr = 0u;
    } else {
        // largest w with -ln U(w) / r >= dt: invariant tau(lo) >= dt > tau(hi)
        uint32_t lo = 0u, hi = 0xFFFFFFFFu;
        while (hi - lo > 1u) {
            const uint32_t mid = lo + (hi - lo) / 2u;
            if (neg_log_uniform(mid) * inv_r >= dt) lo = mid;
            else hi = mid;
        }
        thr = lo;
    }
    rec[i].thr = thr;
}

__global__ void finalize_kernel(const double *__restrict__ partial, int64_t n_rows,
                                uint32_t chunks, int32_t nrhs, double *out1, double *out2,
                                int accumulate)
{
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n_rows * nrhs) return;
    const int64_t q = idx / nrhs;
    const int64_t r = idx % nrhs;
    double a = 0.0, b = 0.0;
    for (uint32_t c = 0; c < chunks; ++c) {
        const int64_t p = ((q * chunks + c) * nrhs + r) * 2;
        a += partial[p];
        b += partial[p + 1];
    }
    if (accumulate) {
        out1[idx] += a;
        out2[idx] += b;
    } else {
        out1[idx] = a;
        out2[idx] = b;
    }
}

constexpr int kMomentThreads = 256;

// Block sums of (m, m^2, V) over a contiguous range of (row, rhs) pairs per block, then a
// fixed-order tree: deterministic for a given count.
__device__ __forceinline__ void block_reduce3(double &a, double &b, double &v)
{
    __shared__ double sh[3][kMomentThreads];
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    sh[2][threadIdx.x] = v;
    __syncthreads();
    for (int o = kMomentThreads / 2; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + o];
        }
        __syncthreads();
    }
    a = sh[0][0];
    b = sh[1][0];
    v = sh[2][0];
}

__global__ __launch_bounds__(kMomentThreads) void moments_partial(const double *__restrict__ s1,
                                                                  const double *__restrict__ s2,
                                                                  int64_t count, double M,
                                                                  int64_t per_block, double *part)
{
    const int64_t begin = static_cast<int64_t>(blockIdx.x) * per_block;
    const int64_t end = min(begin + per_block, count);
    double a = 0.0, b = 0.0, v = 0.0;
    for (int64_t i = begin + threadIdx.x; i < end; i += kMomentThreads) {
        const double m = s1[i] / M;
        a += m;
        b += m * m;
        v += fmax(s2[i] / M - m * m, 0.0);
    }
    block_reduce3(a, b, v);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = a;
        part[3 * blockIdx.x + 1] = b;
        part[3 * blockIdx.x + 2] = v;
    }
}

__global__ __launch_bounds__(kMomentThreads) void moments_final(const double *__restrict__ part,
                                                                int32_t blocks, double *out)
{
    double a = 0.0, b = 0.0, v = 0.0;
    for (int i = threadIdx.x; i < blocks; i += kMomentThreads) {
        a += part[3 * i + 0];
        b += part[3 * i + 1];
        v += part[3 * i + 2];
    }
    block_reduce3(a, b, v);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
        out[2] = v;
    }
}

__global__ void combine_kernel(CombineArgs a, int64_t count, double *x)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double v = 0.0;
    for (int q = 0; q < a.levels; ++q) v += a.s1[q][i] * a.inv_M[q];
    x[i] = v;
}

template <typename R, bool kIS>
__global__ void trace_kernel(LevelArgs L, int64_t count, const int64_t *__restrict__ rows,
                             const uint32_t *__restrict__ walks, int64_t *final_state,
                             int32_t *sign, int64_t *jumps, uint64_t *hash, double *log_fine,
                             double *log_coarse)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t row = rows[i];
    if (row < 0 || row >= L.n) {       // not a row of A: no walk
        final_state[i] = -1;
        sign[i] = 0;
        jumps[i] = 0;
        hash[i] = 0;
        log_fine[i] = 0.0;
        log_coarse[i] = 0.0;
        return;
    }
    const WalkOut<R> o = run_walk<R, true, kIS>(L, static_cast<uint32_t>(row), walks[i]);
    const R hd = static_cast<R>(L.half_dt);
    const double lw = kIS ? log(static_cast<double>(o.wr)) : 0.0;
    final_state[i] = o.k;
    sign[i] = o.neg ? -1 : 1;
    jumps[i] = o.jumps;
    hash[i] = o.hash;
    log_fine[i] = static_cast<double>(o.ef2 * hd) + lw;
    log_coarse[i] = static_cast<double>(o.ec2 * hd) + lw;
}

uint32_t blocks_for(int64_t n, int threads)
{
    return static_cast<uint32_t>((n + threads - 1) / threads);
}

__global__ void zero_u64_kernel(unsigned long long *dst, int64_t count)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = 0ull;
}

__global__ void counter_sum_kernel(const unsigned long long *sets, int slots, unsigned long long *out)
{
    // one block per set, thread t adds the slots t, t + 256, ... of both counters
    __shared__ unsigned long long sh[2][256];
    const unsigned long long *set = sets + static_cast<size_t>(blockIdx.x) * slots * kCounterStride;
    unsigned long long a = 0, b = 0;
    for (int slot = threadIdx.x; slot < slots; slot += 256) {
        a += set[slot * kCounterStride + 0];
        b += set[slot * kCounterStride + 1];
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x + 0] = sh[0][0];
        out[2 * blockIdx.x + 1] = sh[1][0];
    }
}

}  // namespace

hipError_t launch_counter_sum(const unsigned long long *sets, int nsets, unsigned long long *out,
                              hipStream_t s, int slots)
{
    if (nsets <= 0) return hipSuccess;
    hipLaunchKernelGGL(counter_sum_kernel, dim3(nsets), dim3(256), 0, s, sets, slots, out);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *dst, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, dst, count);
    return hipGetLastError();
}

hipError_t launch_thresholds(RowRec *rec, int64_t n, double dt, unsigned int *bad, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(thresholds_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, rec, n, dt, bad);
    return hipGetLastError();
}

hipError_t launch_level_walks(const LevelArgs &L, Prec prec, const void *u, int u_f64,
                              int32_t nrhs, const int64_t *rows, int64_t n_rows, uint32_t walk0,
                              uint32_t M, uint32_t chunk, uint32_t chunks, const SumsOut &out,
                              unsigned long long *counters, unsigned long long *hash_sums,
                              hipStream_t s)
{
    const uint64_t items = static_cast<uint64_t>(n_rows) * chunks;
    if (items == 0) return hipSuccess;
    if (out.direct != 0 && chunks != 1) return hipErrorInvalidValue;
    // single right-hand side: groups of lpr lanes (the power of two >= the walks of an item,
    // at most 64) so that items of few walks still fill the wave
    uint32_t lpr = kWave;
    if (nrhs == 1)
        while (lpr > 1 && lpr / 2 >= chunk) lpr /= 2;
    const uint64_t waves = nrhs == 1 ? (items + kWave / lpr - 1) / (kWave / lpr) : items;
    const dim3 grid(static_cast<uint32_t>(nrhs == 1 ? (waves + kWavesPerBlock - 1) / kWavesPerBlock : waves));
    const dim3 block(nrhs == 1 ? kBlock : kRhsBlock);
    const uint32_t nr = static_cast<uint32_t>(n_rows);
#define MLMC_LAUNCH_WALKS(R, U, H, IS)                                                        \
    do {                                                                                      \
        if (nrhs == 1 && L.src)                                                               \
            hipLaunchKernelGGL((level_walks_r1<R, U, H, IS, true, false>), grid, block, 0, s, \
                               L, static_cast<const U *>(u), rows, nr, walk0, M, chunk,       \
                               chunks, lpr, out, counters, hash_sums);                        \
        else if (nrhs == 1 && L.base)   /* the base level, compiled as such */               \
            hipLaunchKernelGGL((level_walks_r1<R, U, H, IS, false, true>), grid, block, 0,    \
                               s, L, static_cast<const U *>(u), rows, nr, walk0, M, chunk,    \
                               chunks, lpr, out, counters, hash_sums);                        \
        else if (nrhs == 1)                                                                   \
            hipLaunchKernelGGL((level_walks_r1<R, U, H, IS, false, false>), grid, block, 0, s, L, \
                               static_cast<const U *>(u), rows, nr, walk0, M, chunk, chunks,  \
                               lpr, out, counters, hash_sums);                                \
        else                                                                                  \
            hipLaunchKernelGGL((level_walks_rhs<R, U, H, IS>), grid, block, 0, s, L,          \
                               static_cast<const U *>(u), nrhs, rows, nr, walk0, M, chunk,    \
                               chunks, out, counters, hash_sums);                             \
    } while (0)
#define MLMC_LAUNCH_WALKS_H(R, U)                                                             \
    do {                                                                                      \
        if (L.is_slots) {                                                                     \
            if (hash_sums) MLMC_LAUNCH_WALKS(R, U, true, true);                               \
            else MLMC_LAUNCH_WALKS(R, U, false, true);                                        \
        } else {                                                                              \
            if (hash_sums) MLMC_LAUNCH_WALKS(R, U, true, false);                              \
            else MLMC_LAUNCH_WALKS(R, U, false, false);                                       \
        }                                                                                     \
    } while (0)
    if (prec == Prec::FP64) {
        if (u_f64) MLMC_LAUNCH_WALKS_H(double, double);
        else MLMC_LAUNCH_WALKS_H(double, float);
    } else {
        if (u_f64) MLMC_LAUNCH_WALKS_H(float, double);
        else MLMC_LAUNCH_WALKS_H(float, float);
    }
#undef MLMC_LAUNCH_WALKS_H
#undef MLMC_LAUNCH_WALKS
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partial, int64_t n_rows, uint32_t chunks, int32_t nrhs,
                           double *out1, double *out2, int accumulate, hipStream_t s)
{
    const int64_t count = n_rows * nrhs;
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, partial,
                       n_rows, chunks, nrhs, out1, out2, accumulate);
    return hipGetLastError();
}

hipError_t launch_level_moments(const double *s1, const double *s2, int64_t count, double M,
                                double *out, double *scratch, hipStream_t s)
{
    const int64_t target = (count + kMomentBlocks - 1) / kMomentBlocks;
    const int64_t per_block = std::max<int64_t>(target, 4096);
    const int32_t blocks = static_cast<int32_t>(std::max<int64_t>(1, (count + per_block - 1) / per_block));
    hipLaunchKernelGGL(moments_partial, dim3(blocks), dim3(kMomentThreads), 0, s, s1, s2, count, M,
                       per_block, scratch);
    hipLaunchKernelGGL(moments_final, dim3(1), dim3(kMomentThreads), 0, s, scratch, blocks, out);
    return hipGetLastError();
}

hipError_t launch_combine(const CombineArgs &a, int64_t count, double *x, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(combine_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, a, count, x);
    return hipGetLastError();
}

hipError_t launch_trace(const LevelArgs &L, Prec prec, int64_t count, const int64_t *rows,
                        const uint32_t *walks, int64_t *final_state, int32_t *sign,
                        int64_t *jumps, uint64_t *hash, double *log_fine, double *log_coarse,
                        hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const dim3 grid(blocks_for(count, 256));
#define MLMC_LAUNCH_TRACE(R, IS)                                                              \
    hipLaunchKernelGGL((trace_kernel<R, IS>), grid, dim3(256), 0, s, L, count, rows, walks,   \
                       final_state, sign, jumps, hash, log_fine, log_coarse)
    if (prec == Prec::FP64) {
        if (L.is_slots) MLMC_LAUNCH_TRACE(double, true); else MLMC_LAUNCH_TRACE(double, false);
    } else {
        if (L.is_slots) MLMC_LAUNCH_TRACE(float, true); else MLMC_LAUNCH_TRACE(float, false);
    }
#undef MLMC_LAUNCH_TRACE
    return hipGetLastError();
}

}  // namespace mlmc
