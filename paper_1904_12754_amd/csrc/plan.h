// Internal layout of a plan (the object behind mlmc_plan_t) and the helpers the C-ABI
// translation units share. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mlmc_expv.h"
#include "common.h"
#include "kernels.h"

namespace mlmc {

constexpr int kMaxLevel = 28;   // N = 2^28 steps per walk at most

int fail(int code, const std::string &msg);

}  // namespace mlmc

struct mlmc_plan {
    using RowRec = mlmc::RowRec;
    using SlotRec = mlmc::SlotRec;
    using SlotRecIS = mlmc::SlotRecIS;
    static constexpr int kMaxLevel = mlmc::kMaxLevel;
    int64_t n = 0, n_rows = 0, n_slots = 0;
    int32_t l0 = 0, precision = 0;
    double beta = 0, r_max = 0, d_min = 0, d_max = 0;
    double jump_probability = 0;             // mean over the requested rows of 1 - e^{-beta r_i}
    int32_t screen = 0;                      // walks are screened (jump_probability < 1/4)
    SlotRec *slots = nullptr;
    RowRec *rows_base = nullptr;
    RowRec *level_rec[kMaxLevel + 1] = {};
    int64_t *req_rows = nullptr;             // device; null = all rows
    double *partial = nullptr;
    size_t partial_bytes = 0;
    unsigned long long *counters = nullptr;  // one counter set per level
    unsigned long long *counter_sums = nullptr;  // 2 per level: jumps, non-finite samples
    unsigned int *bad = nullptr;
    double *moments = nullptr;               // 3 per level
    double *moment_scratch = nullptr;        // 3 * kMomentBlocks
    double *acc = nullptr;                   // 2 * n_rows * nrhs per level
    size_t acc_doubles = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // per-launch timing of the walk kernel (pairs of events around each launch)
    bool timing = false;
    std::vector<hipEvent_t> tev;
    size_t tev_used = 0;
    // learned proposal: per-level importance-sampling slot tables (empty until set) and
    // whether walks use them
    std::vector<SlotRecIS *> is_slots;
    bool proposal_on = false;
    std::vector<float> p_slot_host;          // plain jump law per slot, |a_kj| / r_k
    float *p_slot = nullptr;                 // device copy, uploaded with the first proposal
    float *prop_P = nullptr;                 // proposal parameters (FP32)
    short *prop_frag = nullptr;              // their BF16 MFMA fragments
    double *prop_xhat = nullptr;             // pilot estimate the features read
    double *prop_xmax = nullptr;             // max |xhat| (1 when zero)
    float *prop_logp = nullptr;              // max(log p, -20) per slot (a feature)
    double *prop_logx = nullptr;             // log(|xhat| + 1e-6 max |xhat|) per row
    int32_t prop_levels = 0;                 // levels l0 .. l0 + prop_levels - 1 carry tables
    int32_t prop_identity = 0;               // 1: the tables are the plain ones (ratio 1)
    // scratch buffers kept between proposal training calls and between gradient calls
    std::vector<std::pair<void *, size_t>> train_pool, grad_pool;
    // pinned host memory for the small reads of a training call (grown on demand)
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    // source vector of the current Algorithm 3 call (device, element type of u), else null
    const void *cur_src = nullptr;
    int64_t bytes = 0;
};

namespace mlmc {

// Upload the row records of `level` (thresholds included) if not done yet.
int upload_level(mlmc_plan *p, int level, hipStream_t s);
// Everything a walk of `level` of this plan reads.
LevelArgs level_args(const mlmc_plan *p, int level, uint64_t seed, int instance);
// Train the proposal on the pilot estimate xhat = sum_q s1_q inv_M_q (the level sums of a
// run's pilot) and set it: capture, Adam, tables, as mlmc_expv_proposal_train without its
// own pilot and judge (their options are not read). Waits for the stream.
int train_from_levels(mlmc_plan *p, const void *u, const mlmc_train_opts_t *o, const CombineArgs &xhat,
                      float *params_out, mlmc_train_stats_t *st, hipStream_t s);
// At least `bytes` of the plan's pinned host memory, for the small reads that wait for the
// device (direct copies instead of staged ones); grown on demand, freed with the plan. A
// pointer from an earlier call is invalid after a call that grows it.
int plan_pinned(mlmc_plan *p, size_t bytes, void **out);
// The options train_from_levels reads, checked before a run starts.
int check_learned_opts(const mlmc_plan *p, const mlmc_train_opts_t *o);

}  // namespace mlmc
