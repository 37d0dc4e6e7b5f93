// Batched runs: many plans (matrices, right-hand sides, times) with fixed level schedules in
// a few launches, captured once in a hipGraph and replayed.
//
// The batch is a list of segments, one per (instance, level). A segment's work is split into
// items of `chunk` walks of one requested row, so instances of very different sizes and
// levels of very different walk lengths share the chip without a launch per segment. The
// items are run either by a grid of one wave per item (two launches: the coarsest levels,
// then the rest) or by a resident grid whose waves deal the items of a phase round robin.
// The graph is: reset the counters -> walks -> per-row chunk sums -> per-instance FP64
// combine of the levels (the estimator of section 2.2). The launch shape (walks per item,
// grid) comes from a small autotuner that times candidates on a subset of the batch's
// instances at full sample sizes and caches the winner per class of batch; without it, the
// walks per item follow from the batch's total walk count and the grid has one wave per item.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mlmc_expv.h"
#include "common.h"
#include "driver.h"
#include "kernels.h"
#include "plan.h"
#include "walk_engine.h"

namespace mlmc {
namespace {

constexpr int kCUs = 256;
constexpr uint32_t kXcds = 8;
// Items per wave in one phase of the walk launches of a resident grid.
constexpr uint64_t kItemsPerWavePhase = 64;
// Items per launch of a grid of one wave per item (grid.x stays far below 2^32 workgroups).
constexpr uint64_t kItemsPerGridLaunch = uint64_t(1) << 28;
// Consecutive workgroups an XCD takes in a grid of one wave per item.
constexpr uint32_t kXcdRun = 16;
// Items per launch the walks-per-item rule aims for: about 128 per wave of a 32-waves-per-CU
// grid, so that the end of the launch is short against its length.
constexpr double kBatchTargetItems = 1 << 20;

struct Segment {
    LevelArgs L;                      // tables of the instance at this level (key set per launch)
    const void *u;
    const int64_t *rows;              // requested rows of the plan, nullptr = all
    double *partial;                  // items x nrhs x 2
    double *acc;                      // [sum Y: n_rows x nrhs][sum Y^2: n_rows x nrhs]
    unsigned long long *counters;     // a counter set of kSegSlots slots (jumps, non-finite)
    uint64_t item_begin;              // first global item of the segment
    uint64_t pair_begin;              // first global (row, rhs) pair of the segment
    double inv_M;
    uint32_t n_rows, M, chunk, chunks;
    int32_t nrhs;
    int32_t direct;                   // 1: one chunk per row, the walks write acc themselves
};

// Each segment's counters are spread over kSegSlots 64-byte slots (the wave's index picks the
// slot), so that the items of a segment do not all add to one address.
constexpr int kSegSlots = 32;
constexpr size_t kSegSetU64 = static_cast<size_t>(kSegSlots) * kCounterStride;

struct InstanceOut {
    double *x;
    uint64_t pair_begin;              // first global (row, rhs) pair of the instance
    int32_t seg0, levels;             // its coarsest level's segment, and its levels
    int32_t seg_stride;               // segments between two of its levels
    int32_t pad;
};

struct BatchParams {
    unsigned long long unused;
    uint32_t k0, k1;                  // Philox key of the current launch
};

// Items [item_lo, item_hi) of the batch (one phase of the launch sequence). kBase: every item
// of the range is at its instance's coarsest level (the segments are ordered level by level),
// so the walks are compiled for it (fine functional only, each sample taken as its walk ends).
// Workgroup b runs on XCD b mod 8 (the dispatcher deals them to the XCDs in turn). Renumber
// them so that within each window of 8 * run workgroups, XCD x takes the run consecutive
// numbers x * run .. x * run + run - 1: neighbouring items then share one XCD's L2. A last
// partial window keeps its order. A bijection of [0, G).
__device__ __forceinline__ uint32_t xcd_renumber(uint32_t b, uint32_t G, uint32_t run)
{
    const uint32_t win = kXcds * run;
    if (b >= G / win * win) return b;
    const uint32_t p = b % win;
    return b - p + (p % kXcds) * run + p / kXcds;
}

// Waves per SIMD as for the single-level kernels: with FP32 weights and one right-hand side,
// seven on the coarsest levels and six above; four with several right-hand sides (their
// per-lane sums of up to 256 right-hand sides take registers), two with FP64 weights.
template <typename R, typename U, bool kMulti, bool kBase>
__global__ __launch_bounds__((kMulti ? kRhsBlock : kBlock), (sizeof(R) == 4 ? (kMulti ? 4 : (kBase ? 7 : 6)) : 2)) void batch_walks(const Segment *__restrict__ segs, int32_t nseg,
                                                      uint64_t item_lo, uint64_t item_hi,
                                                      uint32_t xcd_run, BatchParams *prm)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t k0 = prm->k0, k1 = prm->k1;
    // Items are dealt to the waves round robin (wave v takes v, v + W, v + 2W, ...; with a
    // grid of one wave per item, just v): consecutive items belong to the same (instance,
    // level), so a resident wave gets a mix of all segments. The workgroups are renumbered
    // so that each XCD takes runs of neighbouring items (a resident grid passes run = G / 8:
    // a contiguous eighth of every round of W items; a grid of one wave per item a short
    // run, so that the XCDs sweep the range together and none is left with a costlier
    // stretch of it). The index is read with readfirstlane so the loop is wave-uniform in the
    // compiled control flow. (A shared atomic work counter was measured to serialise at about
    // one returning atomic per microsecond across the XCDs.)
    constexpr int kWpb = kMulti ? kRhsBlock / kWave : kWavesPerBlock;   // waves per workgroup
    const uint64_t waves = static_cast<uint64_t>(gridDim.x) * kWpb;
    const uint32_t xcd_block = xcd_renumber(blockIdx.x, gridDim.x, xcd_run);
    const uint64_t wave_id = __builtin_amdgcn_readfirstlane(
        static_cast<uint64_t>(xcd_block) * kWpb + threadIdx.x / kWave);
    for (uint64_t item = item_lo + wave_id; item < item_hi; item += waves) {
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segs[mid].item_begin <= item) lo = mid;
            else hi = mid - 1;
        }
        const Segment &sg = segs[lo];
        LevelArgs L = sg.L;
        L.k0 = k0;
        L.k1 = k1;
        const uint64_t local = item - sg.item_begin;
        const uint32_t q = static_cast<uint32_t>(local / sg.chunks);
        const uint32_t c = static_cast<uint32_t>(local % sg.chunks);
        const uint32_t row = __builtin_amdgcn_readfirstlane(sg.rows ? static_cast<uint32_t>(sg.rows[q]) : q);
        const uint64_t wb = static_cast<uint64_t>(c) * sg.chunk;
        const uint64_t we = min(wb + sg.chunk, static_cast<uint64_t>(sg.M));
        const U *u = static_cast<const U *>(sg.u);
        unsigned long long jumps, nonfinite;
        if (!kMulti) {
            SinkR1<R, U> sink{u};
            walk_range<R, false, false, false, kBase>(L, row, 0u, wb, we, sink);
            const double a = wave_sum(sink.mom.first());
            const double b = wave_sum(sink.mom.second());
            jumps = wave_sum_u(sink.jumps);
            nonfinite = wave_sum_u(sink.nonfinite);
            if (lane == 0) {
                if (sg.direct) {   // one chunk per row: local is the row
                    sg.acc[local] = a;
                    sg.acc[sg.n_rows + local] = b;
                } else {
                    sg.partial[local * 2 + 0] = a;
                    sg.partial[local * 2 + 1] = b;
                }
            }
        } else {
            const int32_t nrhs = sg.nrhs;
            SinkRhs<R, U> sink{u, nrhs, (nrhs + kWave - 1) / kWave};
            walk_range<R, false, false, false, false, true>(L, row, 0u, wb, we, sink);
            jumps = wave_sum_u(sink.jumps);
            nonfinite = wave_sum_u(sink.nonfinite);
            const unsigned long long nojump = wave_sum_u(sink.nojump);
            R y0 = 0;
            if (nojump && L.base) {
                const RowRec rr = L.rec[row];
                y0 = expR(d_of<R>(rr) * static_cast<R>(2 * L.N) * static_cast<R>(L.half_dt));
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
                    if (sg.direct) {
                        const uint64_t count = static_cast<uint64_t>(sg.n_rows) * nrhs;
                        sg.acc[local * nrhs + r] = a;
                        sg.acc[count + local * nrhs + r] = b;
                    } else {
                        sg.partial[(local * nrhs + r) * 2 + 0] = a;
                        sg.partial[(local * nrhs + r) * 2 + 1] = b;
                    }
                }
            }
        }
        if (lane == 0) {
            unsigned long long *c = sg.counters + (wave_id % kSegSlots) * kCounterStride;
            if (jumps) atomicAdd(&c[0], jumps);   // most items of a screened level have none
            if (nonfinite) atomicAdd(&c[1], nonfinite);
        }
    }
}

__global__ void batch_reset(BatchParams *prm, unsigned long long *counters, int32_t n)
{
    const int i = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    (void)prm;
    if (i < n) counters[i] = 0ull;
}

__global__ void batch_set_key(BatchParams *prm, uint32_t k0, uint32_t k1)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        prm->k0 = k0;
        prm->k1 = k1;
    }
}

// acc of every segment from its chunk partials (fixed order); segments of one chunk per row
// were written by the walks.
__global__ void batch_finalize(const Segment *__restrict__ segs, int32_t nseg, uint64_t total_pairs)
{
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= total_pairs) return;
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].pair_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    const Segment &sg = segs[lo];
    if (sg.direct) return;
    const uint64_t local = t - sg.pair_begin;
    const uint64_t q = local / sg.nrhs, r = local % sg.nrhs;
    double a = 0.0, b = 0.0;
    for (uint32_t c = 0; c < sg.chunks; ++c) {
        const uint64_t p = ((q * sg.chunks + c) * sg.nrhs + r) * 2;
        a += sg.partial[p];
        b += sg.partial[p + 1];
    }
    const uint64_t count = static_cast<uint64_t>(sg.n_rows) * sg.nrhs;
    sg.acc[local] = a;
    sg.acc[count + local] = b;
}

// x of every instance: the FP64 sum over its levels of sum Y / M_l.
__global__ void batch_combine(const Segment *__restrict__ segs, const InstanceOut *__restrict__ outs,
                              int32_t count, uint64_t total_pairs)
{
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= total_pairs) return;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (outs[mid].pair_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    const InstanceOut &o = outs[lo];
    const uint64_t local = t - o.pair_begin;
    double v = 0.0;
    for (int q = 0; q < o.levels; ++q) {
        const Segment &sg = segs[o.seg0 + q * o.seg_stride];
        v += sg.acc[local] * sg.inv_M;
    }
    o.x[local] = v;
}

uint32_t blocks_of(uint64_t n, uint32_t threads)
{
    return static_cast<uint32_t>((n + threads - 1) / threads);
}

// A launch shape: walks per item, and resident waves per CU of a grid that loops over the
// items of a phase (0: one wave per item).
struct Shape {
    uint32_t chunk;
    int32_t waves_per_cu;
};

std::mutex g_tune_mutex;
std::map<std::string, Shape> g_tune_cache;   // the chosen shape per class of batch

}  // namespace
}  // namespace mlmc

using namespace mlmc;

struct mlmc_batch {
    int32_t count = 0, levels = 0, multi = 0, u_f64 = 0, precision = 0;
    std::vector<mlmc_plan *> plans;
    std::vector<int32_t> nrhs;
    std::vector<const void *> u;      // count device pointers
    std::vector<int64_t> walks;       // count x levels
    Shape shape{4096, 0};
    std::vector<Segment> h_segs;
    std::vector<InstanceOut> h_outs;
    Segment *d_segs = nullptr;
    InstanceOut *d_outs = nullptr;
    BatchParams *d_prm = nullptr;
    unsigned long long *d_counters = nullptr;
    unsigned long long *d_counter_sums = nullptr;
    double *d_partial = nullptr;
    double *d_acc = nullptr;
    double *d_moments = nullptr;
    double *d_moment_scratch = nullptr;
    uint64_t total_items = 0, total_pairs = 0, total_out_pairs = 0;
    uint64_t base_items = 0;          // items of the coarsest levels: [0, base_items)
    int32_t phases = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t graph_nodes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool launched = false;
    int32_t tune_n = 0;                // candidates timed by the autotuner
    double tune_ms[MLMC_BATCH_TUNE_MAX] = {};
    int32_t tune_chunk[MLMC_BATCH_TUNE_MAX] = {}, tune_waves[MLMC_BATCH_TUNE_MAX] = {};
    int64_t bytes = 0;
};

namespace {

void free_batch(mlmc_batch *b)
{
    if (!b) return;
    // teardown: a failure here leaves nothing to recover, so the statuses are not kept
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    (void)hipFree(b->d_segs);
    (void)hipFree(b->d_outs);
    (void)hipFree(b->d_prm);
    (void)hipFree(b->d_counters);
    (void)hipFree(b->d_counter_sums);
    (void)hipFree(b->d_partial);
    (void)hipFree(b->d_acc);
    (void)hipFree(b->d_moments);
    (void)hipFree(b->d_moment_scratch);
    delete b;
}

template <typename T>
int balloc(mlmc_batch *b, T **ptr, size_t count)
{
    *ptr = nullptr;
    if (count == 0) count = 1;
    const hipError_t e = hipMalloc(reinterpret_cast<void **>(ptr), count * sizeof(T));
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(e == hipErrorOutOfMemory ? MLMC_ERR_OUT_OF_MEMORY : MLMC_ERR_HIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    b->bytes += static_cast<int64_t>(count * sizeof(T));
    return MLMC_OK;
}

// Segment tables for a shape and sample sizes (walks[b * levels + q]) of every instance, or of
// every stride-th one; device buffers are laid out by the caller through the offsets returned
// in the segments. The segments are ordered level by level (every instance's coarsest level
// first, then every instance's next level, ...), so the items of the coarsest levels form the
// range [0, base_items) and run in a kernel compiled for them.
void layout(const mlmc_batch *b, const Shape &sh, const std::vector<int64_t> &walks,
            std::vector<Segment> &segs, std::vector<InstanceOut> &outs, uint64_t &items,
            uint64_t &pairs, uint64_t &out_pairs, uint64_t &partial_doubles, uint64_t &base_items,
            int stride = 1)
{
    segs.clear();
    outs.clear();
    items = pairs = out_pairs = partial_doubles = base_items = 0;
    std::vector<int> inst;
    for (int i = 0; i < b->count; i += stride) inst.push_back(i);
    const int32_t n_inst = static_cast<int32_t>(inst.size());
    for (int32_t k = 0; k < n_inst; ++k) {
        const int i = inst[static_cast<size_t>(k)];
        InstanceOut o{};
        o.pair_begin = out_pairs;
        o.seg0 = k;
        o.levels = b->levels;
        o.seg_stride = n_inst;
        out_pairs += static_cast<uint64_t>(b->plans[i]->n_rows) * b->nrhs[i];
        outs.push_back(o);
    }
    for (int q = 0; q < b->levels; ++q) {
        if (q == 1) base_items = items;
        for (int i : inst) {
            mlmc_plan *p = b->plans[i];
            Segment sg{};
            const int level = p->l0 + q;
            sg.L = level_args(p, level, 0, i);
            sg.u = b->u[i];
            sg.rows = p->req_rows;
            sg.n_rows = static_cast<uint32_t>(p->n_rows);
            sg.M = static_cast<uint32_t>(walks[static_cast<size_t>(i) * b->levels + q]);
            sg.chunk = std::min<uint32_t>(sh.chunk, (sg.M + 63) / 64 * 64);
            sg.chunks = (sg.M + sg.chunk - 1) / sg.chunk;
            sg.nrhs = b->nrhs[i];
            sg.inv_M = 1.0 / static_cast<double>(sg.M);
            sg.item_begin = items;
            sg.pair_begin = pairs;
            const uint64_t seg_items = static_cast<uint64_t>(sg.n_rows) * sg.chunks;
            items += seg_items;
            pairs += static_cast<uint64_t>(sg.n_rows) * sg.nrhs;
            // partial offset (in doubles) kept in the pointer field until buffers exist
            sg.partial = reinterpret_cast<double *>(partial_doubles);
            partial_doubles += seg_items * sg.nrhs * 2;
            segs.push_back(sg);
        }
    }
    if (b->levels == 1) base_items = items;
}

hipError_t launch_walks(const mlmc_batch *b, const Shape &sh, const Segment *d_segs, int32_t nseg,
                        uint64_t item_lo, uint64_t item_hi, bool base, hipStream_t s)
{
    // a resident grid of waves_per_cu waves per CU, or one wave per item; a multiple of kXcds
    // workgroups either way (the kernel's renumbering of the waves needs it)
    const uint64_t waves = sh.waves_per_cu > 0 ? static_cast<uint64_t>(kCUs) * sh.waves_per_cu
                                               : item_hi - item_lo;
    const uint64_t wpb = b->multi ? kRhsBlock / kWave : kWavesPerBlock;   // waves per workgroup
    const uint64_t blocks = (waves + wpb * kXcds - 1) / (wpb * kXcds) * kXcds;
    if (blocks == 0 || blocks > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
    const dim3 grid(static_cast<uint32_t>(blocks));
    const uint32_t xcd_run = sh.waves_per_cu > 0 ? grid.x / kXcds : kXcdRun;
    const dim3 block(b->multi ? kRhsBlock : kBlock);
#define MLMC_BATCH(R, U, MULTI)                                                                        \
    do {                                                                                               \
        if (!(MULTI) && base)                                                                          \
            hipLaunchKernelGGL((batch_walks<R, U, MULTI, true>), grid, block, 0, s, d_segs, nseg,      \
                               item_lo, item_hi, xcd_run, b->d_prm);                                   \
        else                                                                                           \
            hipLaunchKernelGGL((batch_walks<R, U, MULTI, false>), grid, block, 0, s, d_segs, nseg,     \
                               item_lo, item_hi, xcd_run, b->d_prm);                                   \
    } while (0)
    if (b->precision == MLMC_PRECISION_FP64) {
        if (b->u_f64) {
            if (b->multi) MLMC_BATCH(double, double, true); else MLMC_BATCH(double, double, false);
        } else {
            if (b->multi) MLMC_BATCH(double, float, true); else MLMC_BATCH(double, float, false);
        }
    } else {
        if (b->u_f64) {
            if (b->multi) MLMC_BATCH(float, double, true); else MLMC_BATCH(float, double, false);
        } else {
            if (b->multi) MLMC_BATCH(float, float, true); else MLMC_BATCH(float, float, false);
        }
    }
#undef MLMC_BATCH
    return hipGetLastError();
}

// The walks of items [0, total_items) as a sequence of launches (phases) of consecutive
// items. With a resident grid, the waves of a launch drift apart (their items differ in
// cost) and the chip ends up working on many instances at once, whose tables then compete
// for the L2; the end of each launch brings the waves back together (on the 512-instance
// batch this halves the L2 misses of one long launch), at the price of the waves that idle
// while the launch drains. A grid of one wave per item has neither problem: the dispatcher
// hands out the items in order as waves end, so the waves in flight hold a window of
// neighbouring rows and no slot idles before the end of the range. The phases of the
// coarsest levels' items [0, base_items) use the kernel compiled for the coarsest level.
hipError_t launch_phases(const mlmc_batch *b, const Shape &sh, const Segment *d_segs, int32_t nseg,
                         uint64_t total_items, uint64_t base_items, hipStream_t s, int32_t *phases)
{
    const uint64_t per_phase = sh.waves_per_cu > 0
                                   ? static_cast<uint64_t>(kCUs) * sh.waves_per_cu * kItemsPerWavePhase
                                   : kItemsPerGridLaunch;
    *phases = 0;
    for (int part = 0; part < 2; ++part) {
        const uint64_t begin = part == 0 ? 0 : base_items, end = part == 0 ? base_items : total_items;
        for (uint64_t lo = begin; lo < end; lo += per_phase) {
            const hipError_t e = launch_walks(b, sh, d_segs, nseg, lo, std::min(end, lo + per_phase),
                                              part == 0, s);
            if (e != hipSuccess) return e;
            ++*phases;
        }
    }
    return hipSuccess;
}

// Device buffers and segment table for the final shape.
int build_tables(mlmc_batch *b, hipStream_t s)
{
    uint64_t partial_doubles = 0;
    layout(b, b->shape, b->walks, b->h_segs, b->h_outs, b->total_items, b->total_pairs,
           b->total_out_pairs, partial_doubles, b->base_items);
    int rc;
    if ((rc = balloc(b, &b->d_partial, partial_doubles))) return rc;
    if ((rc = balloc(b, &b->d_acc, 2 * b->total_pairs))) return rc;
    if ((rc = balloc(b, &b->d_counters, kSegSetU64 * b->h_segs.size()))) return rc;
    if ((rc = balloc(b, &b->d_counter_sums, 2 * b->h_segs.size()))) return rc;
    if ((rc = balloc(b, &b->d_moments, 3 * b->h_segs.size()))) return rc;
    if ((rc = balloc(b, &b->d_moment_scratch, 3 * kMomentBlocks))) return rc;
    uint64_t acc_off = 0;
    for (size_t g = 0; g < b->h_segs.size(); ++g) {
        Segment &sg = b->h_segs[g];
        sg.partial = b->d_partial + reinterpret_cast<uintptr_t>(sg.partial);
        sg.acc = b->d_acc + acc_off;
        sg.direct = sg.chunks == 1 ? 1 : 0;
        acc_off += 2ull * sg.n_rows * sg.nrhs;
        sg.counters = b->d_counters + kSegSetU64 * g;
    }
    for (int i = 0; i < b->count; ++i) b->h_outs[i].x = nullptr;   // filled by create
    if ((rc = balloc(b, &b->d_segs, b->h_segs.size()))) return rc;
    MLMC_HIP_TRY(hipMemcpyAsync(b->d_segs, b->h_segs.data(), sizeof(Segment) * b->h_segs.size(),
                                hipMemcpyHostToDevice, s));
    return MLMC_OK;
}

// Walks per item: the total walk count over kBatchTargetItems, rounded up to a multiple of
// 64, within [64, 4096]. Long items keep the lanes busy (a lane that ends a walk takes the
// item's next one; only the last walks of an item leave lanes idle), so items are only cut
// shorter when the batch would otherwise give the waves too few of them.
uint32_t items_chunk(const mlmc_batch *b)
{
    double total = 0.0;
    for (int i = 0; i < b->count; ++i)
        for (int q = 0; q < b->levels; ++q)
            total += static_cast<double>(b->walks[static_cast<size_t>(i) * b->levels + q]) *
                     static_cast<double>(b->plans[i]->n_rows);
    const double c = std::ceil(total / kBatchTargetItems / 64.0) * 64.0;
    return static_cast<uint32_t>(std::min(4096.0, std::max(64.0, c)));
}

// Time candidate shapes (walks per item: 1024, 4096 and the size rule's choice; a grid of one
// wave per item, or resident grids of 16, 20 or 32 waves per CU, where 20 fills the 5 waves
// per SIMD of the FP32 one-right-hand-side kernel in one round) on every kTuneStride-th
// instance of the batch at its full sample sizes, with the phases of the real launch, and
// keep the fastest. The choice is cached per class of batch for the process.
constexpr int kTuneStride = 8;

int autotune(mlmc_batch *b, hipStream_t s)
{
    std::string key = std::to_string(b->precision) + "/" + std::to_string(b->multi) + "/" +
                      std::to_string(b->u_f64);
    {
        double steps = 0.0, rows = 0.0, slots = 0.0;
        for (int i = 0; i < b->count; ++i) {
            rows += static_cast<double>(b->plans[i]->n_rows);
            slots += static_cast<double>(b->plans[i]->n_slots) /
                     std::max<double>(1.0, static_cast<double>(b->plans[i]->n));
            for (int q = 0; q < b->levels; ++q)
                steps += static_cast<double>(b->walks[static_cast<size_t>(i) * b->levels + q]) *
                         std::ldexp(1.0, b->plans[i]->l0 + q) * b->plans[i]->n_rows;
        }
        key += "/" + std::to_string(static_cast<int>(std::log2(std::max(steps, 1.0)))) + "/" +
               std::to_string(static_cast<int>(std::log2(std::max(rows, 1.0)))) + "/" +
               std::to_string(static_cast<int>(slots / std::max(1, b->count) + 0.5));
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            b->shape = it->second;
            return MLMC_OK;
        }
    }
    std::vector<Shape> cands;
    {
        std::vector<uint32_t> chunks = {1024, 4096};
        if (std::find(chunks.begin(), chunks.end(), b->shape.chunk) == chunks.end())
            chunks.push_back(b->shape.chunk);
        for (uint32_t c : chunks)
            for (int w : {0, 16, 20, 32}) cands.push_back(Shape{c, w});
    }
    const int stride = b->count >= kTuneStride ? kTuneStride : b->count;
    double best = 1e300;
    Shape pick = b->shape;
    hipEvent_t e0, e1;
    MLMC_HIP_TRY(hipEventCreate(&e0));
    MLMC_HIP_TRY(hipEventCreate(&e1));
    int rc = MLMC_OK;
    b->tune_n = 0;
    for (size_t ci = 0; ci < cands.size() && rc == MLMC_OK; ++ci) {
        std::vector<Segment> segs;
        std::vector<InstanceOut> outs;
        uint64_t items, pairs, opairs, pdoubles, base;
        layout(b, cands[ci], b->walks, segs, outs, items, pairs, opairs, pdoubles, base, stride);
        double *part = nullptr;
        unsigned long long *ctr = nullptr;
        Segment *dseg = nullptr;
        if (hipMalloc(&part, std::max<uint64_t>(pdoubles, 1) * sizeof(double)) != hipSuccess ||
            hipMalloc(&ctr, kSegSetU64 * std::max<size_t>(segs.size(), 1) * sizeof(unsigned long long)) !=
                hipSuccess ||
            hipMalloc(&dseg, std::max<size_t>(segs.size(), 1) * sizeof(Segment)) != hipSuccess) {
            rc = fail(MLMC_ERR_OUT_OF_MEMORY, "autotune scratch");
        } else {
            for (size_t g = 0; g < segs.size(); ++g) {
                segs[g].partial = part + reinterpret_cast<uintptr_t>(segs[g].partial);
                segs[g].acc = nullptr;
                segs[g].counters = ctr + kSegSetU64 * g;
            }
            if (hipMemcpyAsync(dseg, segs.data(), sizeof(Segment) * segs.size(), hipMemcpyHostToDevice, s) !=
                hipSuccess)
                rc = fail(MLMC_ERR_HIP, "autotune upload");
            // the first candidate runs twice (the first run warms the tables up), the others once
            float ms = 0.0f;
            for (int rep = 0; rep < (ci == 0 ? 2 : 1) && rc == MLMC_OK; ++rep) {
                hipLaunchKernelGGL(batch_reset, dim3(blocks_of(kSegSetU64 * segs.size(), 256)), dim3(256), 0, s,
                                   b->d_prm, ctr, static_cast<int32_t>(kSegSetU64 * segs.size()));
                hipLaunchKernelGGL(batch_set_key, dim3(1), dim3(64), 0, s, b->d_prm, 0x5EEDu, rep + 1u);
                if (hipEventRecord(e0, s) != hipSuccess) rc = fail(MLMC_ERR_HIP, "autotune event");
                int32_t phases = 0;
                if (rc == MLMC_OK &&
                    launch_phases(b, cands[ci], dseg, static_cast<int32_t>(segs.size()), items, base, s,
                                  &phases) != hipSuccess)
                    rc = fail(MLMC_ERR_HIP, "autotune launch");
                if (rc == MLMC_OK && hipEventRecord(e1, s) != hipSuccess) rc = fail(MLMC_ERR_HIP, "autotune event");
                if (rc == MLMC_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(MLMC_ERR_HIP, "autotune sync");
                if (rc == MLMC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                    rc = fail(MLMC_ERR_HIP, "autotune timing");
            }
            if (rc == MLMC_OK && b->tune_n < MLMC_BATCH_TUNE_MAX) {
                b->tune_ms[b->tune_n] = ms;
                b->tune_chunk[b->tune_n] = static_cast<int32_t>(cands[ci].chunk);
                b->tune_waves[b->tune_n] = cands[ci].waves_per_cu;
                ++b->tune_n;
            }
            if (rc == MLMC_OK && ms < best) {
                best = ms;
                pick = cands[ci];
            }
        }
        (void)hipFree(part);
        (void)hipFree(ctr);
        (void)hipFree(dseg);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    b->shape = pick;
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    g_tune_cache[key] = pick;
    return MLMC_OK;
}

}  // namespace

extern "C" {

int mlmc_expv_batch_create(mlmc_batch_t **out, const mlmc_batch_desc_t *d, void *stream)
{
    if (!out || !d) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (d->count < 1 || d->count > 4096) return fail(MLMC_ERR_INVALID_ARG, "count must be in [1, 4096]");
    if (!d->plans || !d->u || !d->nrhs || !d->x || !d->walks)
        return fail(MLMC_ERR_INVALID_ARG, "null array in the batch description");
    if (d->u_dtype != MLMC_DTYPE_F32 && d->u_dtype != MLMC_DTYPE_F64)
        return fail(MLMC_ERR_INVALID_ARG, "u_dtype must be MLMC_DTYPE_F32 or MLMC_DTYPE_F64");
    if (d->num_levels < 1 || d->num_levels > MLMC_MAX_LEVELS)
        return fail(MLMC_ERR_INVALID_ARG, "num_levels out of range");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    auto *b = new (std::nothrow) mlmc_batch;
    if (!b) return fail(MLMC_ERR_OUT_OF_MEMORY, "host allocation");
    std::unique_ptr<mlmc_batch, void (*)(mlmc_batch *)> guard(b, free_batch);
    b->count = d->count;
    b->levels = d->num_levels;
    b->u_f64 = d->u_dtype == MLMC_DTYPE_F64;
    b->plans.assign(d->plans, d->plans + d->count);
    b->nrhs.assign(d->nrhs, d->nrhs + d->count);
    b->u.assign(d->u, d->u + d->count);
    b->walks.assign(d->walks, d->walks + static_cast<size_t>(d->count) * d->num_levels);
    for (int i = 0; i < d->count; ++i) {
        mlmc_plan *p = b->plans[i];
        if (!p) return fail(MLMC_ERR_INVALID_ARG, "null plan in the batch");
        if (p->proposal_on) return fail(MLMC_ERR_UNSUPPORTED, "batched runs walk with the plain jump law; disable the proposal");
        if (i == 0) b->precision = p->precision;
        if (p->precision != b->precision)
            return fail(MLMC_ERR_UNSUPPORTED, "all plans of a batch must share one precision");
        if (b->nrhs[i] < 1 || b->nrhs[i] > 256) return fail(MLMC_ERR_INVALID_ARG, "nrhs must be in [1, 256]");
        if (b->nrhs[i] > 1) b->multi = 1;
        if (!d->u[i]) return fail(MLMC_ERR_INVALID_ARG, "null u in the batch");
        if (!d->x[i] && p->n_rows > 0) return fail(MLMC_ERR_INVALID_ARG, "null x in the batch");
        if (p->l0 + d->num_levels - 1 > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "levels exceed 28");
        for (int q = 0; q < d->num_levels; ++q) {
            const int64_t w = b->walks[static_cast<size_t>(i) * d->num_levels + q];
            if (w < 1 || w >= (int64_t(1) << 32))
                return fail(MLMC_ERR_INVALID_ARG, "walks per level must be in [1, 2^32)");
            int rc = upload_level(p, p->l0 + q, s);
            if (rc) return rc;
        }
    }
    int rc;
    if ((rc = balloc(b, &b->d_prm, 1))) return rc;
    MLMC_HIP_TRY(hipEventCreate(&b->ev0));
    MLMC_HIP_TRY(hipEventCreate(&b->ev1));
    if (!d->autotune && (d->waves_per_cu < 0 || d->waves_per_cu > 64))
        return fail(MLMC_ERR_INVALID_ARG, "waves_per_cu must be in [0, 64]");
    b->shape.chunk = items_chunk(b);
    b->shape.waves_per_cu = d->autotune ? 0 : d->waves_per_cu;
    if (d->autotune && (rc = autotune(b, s))) return rc;
    if ((rc = build_tables(b, s))) return rc;
    for (int i = 0; i < b->count; ++i) b->h_outs[i].x = d->x[i];
    if ((rc = balloc(b, &b->d_outs, b->h_outs.size()))) return rc;
    MLMC_HIP_TRY(hipMemcpyAsync(b->d_outs, b->h_outs.data(), sizeof(InstanceOut) * b->h_outs.size(),
                                hipMemcpyHostToDevice, s));
    MLMC_HIP_TRY(hipStreamSynchronize(s));
    // capture the launch sequence once
    MLMC_HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    MLMC_HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    const int32_t nseg = static_cast<int32_t>(b->h_segs.size());
    hipLaunchKernelGGL(batch_reset, dim3(blocks_of(kSegSetU64 * nseg, 256)), dim3(256), 0, b->cap_stream,
                       b->d_prm, b->d_counters, static_cast<int32_t>(kSegSetU64 * nseg));
    hipError_t le = launch_phases(b, b->shape, b->d_segs, nseg, b->total_items, b->base_items,
                                  b->cap_stream, &b->phases);
    if (b->total_pairs)
        hipLaunchKernelGGL(batch_finalize, dim3(blocks_of(b->total_pairs, 256)), dim3(256), 0,
                           b->cap_stream, b->d_segs, nseg, b->total_pairs);
    if (b->total_out_pairs)
        hipLaunchKernelGGL(batch_combine, dim3(blocks_of(b->total_out_pairs, 256)), dim3(256), 0,
                           b->cap_stream, b->d_segs, b->d_outs, b->count, b->total_out_pairs);
    const hipError_t ce = hipStreamEndCapture(b->cap_stream, &b->graph);
    if (le != hipSuccess) return fail(MLMC_ERR_HIP, std::string("capture launch: ") + hipGetErrorString(le));
    MLMC_HIP_TRY(ce);
    MLMC_HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    MLMC_HIP_TRY(hipGraphGetNodes(b->graph, nullptr, &b->graph_nodes));
    *out = guard.release();
    return MLMC_OK;
}

int mlmc_expv_batch_launch(mlmc_batch_t *b, uint64_t seed, void *stream)
{
    if (!b) return fail(MLMC_ERR_INVALID_ARG, "null batch");
    for (const mlmc_plan *p : b->plans)
        if (p->proposal_on) return fail(MLMC_ERR_UNSUPPORTED, "a plan of the batch has an active proposal");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(batch_set_key, dim3(1), dim3(64), 0, s, b->d_prm, static_cast<uint32_t>(seed),
                       static_cast<uint32_t>(seed >> 32));
    MLMC_HIP_TRY(hipGetLastError());
    MLMC_HIP_TRY(hipEventRecord(b->ev0, s));
    MLMC_HIP_TRY(hipGraphLaunch(b->exec, s));
    MLMC_HIP_TRY(hipEventRecord(b->ev1, s));
    b->launched = true;
    return MLMC_OK;
}

int mlmc_expv_batch_stats(mlmc_batch_t *b, mlmc_stats_t *per_instance, void *stream)
{
    if (!b || !per_instance) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    if (!b->launched) return fail(MLMC_ERR_INVALID_ARG, "the batch has not been launched");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nseg = b->h_segs.size();
    for (size_t g = 0; g < nseg; ++g) {
        const Segment &sg = b->h_segs[g];
        const int64_t cnt = static_cast<int64_t>(sg.n_rows) * sg.nrhs;
        MLMC_HIP_TRY(launch_level_moments(sg.acc, sg.acc + cnt, cnt, static_cast<double>(sg.M),
                                          b->d_moments + 3 * g, b->d_moment_scratch, s));
    }
    std::vector<double> mom(3 * nseg);
    std::vector<unsigned long long> ctr(2 * nseg);
    MLMC_HIP_TRY(launch_counter_sum(b->d_counters, static_cast<int>(nseg), b->d_counter_sums, s, kSegSlots));
    MLMC_HIP_TRY(hipMemcpyAsync(mom.data(), b->d_moments, sizeof(double) * mom.size(), hipMemcpyDeviceToHost, s));
    MLMC_HIP_TRY(hipMemcpyAsync(ctr.data(), b->d_counter_sums, sizeof(unsigned long long) * ctr.size(),
                                hipMemcpyDeviceToHost, s));
    MLMC_HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.0f;
    MLMC_HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    int64_t nonfinite = 0;
    for (int i = 0; i < b->count; ++i) {
        mlmc_stats_t &st = per_instance[i];
        std::memset(&st, 0, sizeof st);
        const mlmc_plan *p = b->plans[i];
        st.l0 = p->l0;
        st.num_levels = b->levels;
        st.converged = 1;
        double var = 0.0;
        for (int q = 0; q < b->levels; ++q) {
            const size_t g = static_cast<size_t>(q) * b->count + i;   // segments level by level
            const Segment &sg = b->h_segs[g];
            const double cnt = std::max<double>(1.0, static_cast<double>(sg.n_rows) * sg.nrhs);
            st.walks[q] = sg.M;
            st.jumps[q] = static_cast<int64_t>(ctr[2 * g]);
            st.level_var[q] = unbiased_var(mom[3 * g + 2] / cnt, sg.M);
            st.level_mean_rms[q] = debiased_rms(mom[3 * g + 1] / cnt, st.level_var[q], sg.M);
            const double walks_total = static_cast<double>(sg.M) * std::max<uint32_t>(sg.n_rows, 1);
            st.level_cost[q] = std::ldexp(1.0, p->l0 + q) + 4.0 * static_cast<double>(ctr[2 * g]) / walks_total;
            st.steps += static_cast<int64_t>(sg.M) * sg.n_rows * (int64_t(1) << (p->l0 + q));
            st.total_jumps += static_cast<int64_t>(ctr[2 * g]);
            st.nonfinite += static_cast<int64_t>(ctr[2 * g + 1]);
            var += st.level_var[q] / static_cast<double>(sg.M);
        }
        st.est_variance = var;
        st.kernel_ms = ms;
        st.walk_kernel_ms = ms;   // the graph's time: the walk phases plus the short sums
        st.walk_launches = b->phases;
        nonfinite += st.nonfinite;
    }
    if (nonfinite) return fail(MLMC_ERR_NONFINITE, std::to_string(nonfinite) + " non-finite samples");
    return MLMC_OK;
}

int mlmc_expv_batch_info(const mlmc_batch_t *b, mlmc_batch_info_t *info)
{
    if (!b || !info) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    std::memset(info, 0, sizeof *info);
    info->count = b->count;
    info->segments = static_cast<int32_t>(b->h_segs.size());
    info->items = static_cast<int64_t>(b->total_items);
    info->walks_per_item = static_cast<int32_t>(b->shape.chunk);
    info->waves_per_cu = b->shape.waves_per_cu;
    info->graph_nodes = static_cast<int32_t>(b->graph_nodes);
    info->phases = b->phases;
    info->device_bytes = b->bytes;
    info->tune_count = b->tune_n;
    for (int i = 0; i < b->tune_n; ++i) {
        info->tune_ms[i] = b->tune_ms[i];
        info->tune_walks_per_item[i] = b->tune_chunk[i];
        info->tune_waves_per_cu[i] = b->tune_waves[i];
    }
    return MLMC_OK;
}

void mlmc_expv_batch_destroy(mlmc_batch_t *b) { free_batch(b); }

}  // extern "C"
