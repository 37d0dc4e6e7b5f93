// Host-side launchers of the walk, threshold and reduction kernels (kernels.hip).
#pragma once

#include "common.h"

namespace mlmc {

// Everything a walk at one level reads.
struct LevelArgs {
    const RowRec *rec;       // the level's row records
    const SlotRec *slots;    // alias tables of all rows
    const SlotRecIS *is_slots;  // the level's proposal tables (used by the proposal kernels)
    const void *src;         // source vector F of Algorithm 3 (element type of u), or null
    int64_t n;               // rows of A
    uint32_t N;              // steps, 2^level
    int32_t level;
    int32_t base;            // 1 at the coarsest level l0 (sample u eta_fine only)
    double dt;               // beta / 2^level
    double half_dt;
    float dt_below, dt_above;  // FP32 bounds around dt for the certified holding-time test
    uint32_t k0, k1;         // Philox key (seed)
    uint32_t c3_step, c3_jump;
    uint32_t screen;         // 1: most walks never jump, so kernels that can screen them
                             // first test every step of each walk at its start row
};

enum class Prec { FP64, FP32 };

// A counter set: kCounterSlots slots of kCounterStride u64 (one 64-byte line each), [0] the
// jumps and [1] the non-finite samples. Wave w adds its totals to slot w mod kCounterSlots,
// so that no single address takes an atomic from every wave (atomics on one address
// serialise across the XCDs); launch_counter_sum adds the slots up (integer sums, so the
// order does not matter).
constexpr int kCounterSlots = 256;
constexpr int kCounterStride = 8;
constexpr size_t kCounterSetU64 = static_cast<size_t>(kCounterSlots) * kCounterStride;

__device__ __forceinline__ unsigned long long *counter_slot(unsigned long long *set, uint64_t wave)
{
    return set + (wave % kCounterSlots) * kCounterStride;
}

// out[2 i + j] = sum over the slots of counter j of set i, for sets 0 .. nsets - 1 of
// `slots` slots each (kCounterSlots for the single-level path).
hipError_t launch_counter_sum(const unsigned long long *sets, int nsets, unsigned long long *out,
                              hipStream_t s, int slots = kCounterSlots);

// Fill rec[i].thr for one level: the largest word w with -ln U(w) / r_i >= dt (no jump).
// Sets *bad if some row jumps at every word (r_i dt too large for 32-bit words).
hipError_t launch_thresholds(RowRec *rec, int64_t n, double dt, unsigned int *bad,
                             hipStream_t s);

// Where the walk kernels put their sums of Y and Y^2: per-(row, chunk) partials
// (partial[((q * chunks + c) * nrhs + r) * 2 + {0, 1}], reduced by launch_finalize), or,
// when a row's walks form one chunk, straight into out1/out2[q * nrhs + r] (written, or
// added to).
struct SumsOut {
    double *partial;
    double *out1, *out2;
    int32_t direct;          // 0: partials; 1: write out1/out2; 2: add to out1/out2
};

// Sums of Y and Y^2 for walks [walk0, walk0 + M) of each requested row, into `out`.
// counters: a counter set (jumps, non-finite samples); hash_sums (nullable) [q] += the path
// hashes of row q's walks (mod 2^64).
hipError_t launch_level_walks(const LevelArgs &L, Prec prec, const void *u, int u_f64,
                              int32_t nrhs, const int64_t *rows, int64_t n_rows,
                              uint32_t walk0, uint32_t M, uint32_t chunk, uint32_t chunks,
                              const SumsOut &out, unsigned long long *counters,
                              unsigned long long *hash_sums, hipStream_t s);

// out1/out2[q * nrhs + r] (=, or += when accumulate) the chunk sums of the partials.
hipError_t launch_finalize(const double *partial, int64_t n_rows, uint32_t chunks,
                           int32_t nrhs, double *out1, double *out2, int accumulate,
                           hipStream_t s);

// One level's moments over all (row, rhs): out[0] = sum m, out[1] = sum m^2,
// out[2] = sum V, with m = s1 / M and V = max(s2 / M - m^2, 0). Deterministic order.
// scratch: kMomentBlocks * 3 doubles, reusable once the call's work has run.
constexpr int kMomentBlocks = 1024;
hipError_t launch_level_moments(const double *s1, const double *s2, int64_t count, double M,
                                double *out, double *scratch, hipStream_t s);

// x[idx] = sum_q s1[q][idx] / M[q] over `levels` accumulators.
struct CombineArgs {
    const double *s1[64];
    double inv_M[64];
    int32_t levels;
};
hipError_t launch_combine(const CombineArgs &a, int64_t count, double *x, hipStream_t s);

// dst[0 .. count) = 0 by a kernel (no memset node, so the call may sit in a captured graph).
hipError_t launch_zero_u64(unsigned long long *dst, int64_t count, hipStream_t s);

hipError_t launch_trace(const LevelArgs &L, Prec prec, int64_t count, const int64_t *rows,
                        const uint32_t *walks, int64_t *final_state, int32_t *sign,
                        int64_t *jumps, uint64_t *hash, double *log_fine, double *log_coarse,
                        hipStream_t s);

}  // namespace mlmc
