// Algorithm 1 (the multilevel driver), shared by the full-vector, scalar and forward runs.
//
// Start with L = l0 + 4 and M0 walks on every level; then repeat: compute Giles' optimal
// sample sizes M_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k)) (variance budget
// eps^2 / 2, section 2.2) and run the missing walks. The error of Algorithm 1 is read as two
// parts:
//   - the estimator's variance sum_l V_l / M_l against eps^2 / 2: after new walks the
//     variances are re-estimated and the sizes recomputed, until they ask for no more walks;
//   - the extrapolated bias of the finest level, max(|m_L|, |m_{L-1}| / 2^a) / (2^a - 1)
//     with the weak order a = 2 of the Strang splitting (section 4), against eps / sqrt(2):
//     when it fails, the level L + 1 is added with M0 walks.
// Host code only; the caller supplies the two operations that touch the device.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/mlmc_expv.h"

namespace mlmc {

// What the driver reads of level index q (level l0 + q) after its walks so far.
struct LevelEstimate {
    double var = 0.0;    // unbiased per-walk variance V_l (averaged over the estimated entries)
    double cost = 0.0;   // cost per walk C_l: N_l + 4 jumps per walk
    double rms = 0.0;    // the level term m_l (root mean square over the entries, debiased)
};

struct DriverOpts {
    double eps = 0.0;
    int64_t pilot = 0;          // M0
    int max_levels = 0;         // cap on L - l0 + 1
    int64_t cap = 0;            // cap on M_l
    int max_iterations = 100;   // cap on the loop (each iteration waits for the device once)
};

struct DriverOut {
    int levels = 0, iterations = 0;
    bool converged = false;
    double var = 0.0, bias = 0.0;   // the last error test's two parts
};

constexpr double kWeakOrder = 2.0;

// M0 when the caller leaves it to the driver (pilot_walks = 0): enough walks per row that a
// pilot level holds at least 2^18 samples over its rows and right-hand sides, and at least 2.
constexpr int64_t kPilotSamples = int64_t(1) << 18;
inline int64_t default_pilot(int64_t rows_times_rhs)
{
    const int64_t r = std::max<int64_t>(1, rows_times_rhs);
    return std::max<int64_t>(2, (kPilotSamples + r - 1) / r);
}

// The per-walk variance from M samples' mean square minus squared mean (Algorithm 2's m_l
// and m2l, each divided by M once), made unbiased by the factor M / (M - 1).
inline double unbiased_var(double raw, int64_t M)
{
    return M > 1 ? raw * (static_cast<double>(M) / static_cast<double>(M - 1)) : raw;
}

// The root mean square of a level term over its entries from M-walk means: the mean of the
// squared means overstates the mean square of the terms by the sampling noise var / M
// (var the unbiased per-walk variance averaged over the entries), which is taken off.
inline double debiased_rms(double mean_sq, double var, int64_t M)
{
    return std::sqrt(std::max(mean_sq - var / static_cast<double>(std::max<int64_t>(M, 1)), 0.0));
}

// The extrapolated bias of the finest level from the two finest level terms.
inline double extrapolated_bias(double mL, double mLm1)
{
    const double a = std::exp2(kWeakOrder);
    return std::max(std::fabs(mL), std::fabs(mLm1) / a) / (a - 1.0);
}

// add(q, extra) -> status: run `extra` more walks at level index q and count them in M[q].
// measure(levels, est) -> status: fill est[q], q < levels, from the walks so far.
// after_pilot(levels, est, again) -> status: called once, after the pilot's measurement and
// before any sample size is computed; it may replace walks (and M), and sets `again` when
// the levels must be measured anew.
template <class Add, class Measure, class AfterPilot>
int algorithm1(const DriverOpts &o, std::vector<int64_t> &M, Add &&add, Measure &&measure,
               AfterPilot &&after_pilot, DriverOut &out)
{
    const double eps2 = o.eps * o.eps;
    const double budget = eps2 / 2.0 * 1.0000001;
    int levels = std::min(5, o.max_levels);
    int rc;
    for (int q = 0; q < levels; ++q)
        if ((rc = add(q, o.pilot))) return rc;
    std::vector<LevelEstimate> est(static_cast<size_t>(o.max_levels));
    out = DriverOut{};
    while (out.iterations < o.max_iterations) {
        ++out.iterations;
        if ((rc = measure(levels, est))) return rc;
        if (out.iterations == 1) {
            bool again = false;
            if ((rc = after_pilot(levels, est, again))) return rc;
            if (again && (rc = measure(levels, est))) return rc;
        }
        double tot = 0.0;
        for (int q = 0; q < levels; ++q) tot += std::sqrt(std::max(est[q].var, 1e-300) * est[q].cost);
        bool topped = false, nan_size = false;
        for (int q = 0; q < levels; ++q) {
            const double Mopt = std::ceil(2.0 / eps2 * std::sqrt(std::max(est[q].var, 1e-300) / est[q].cost) * tot);
            if (std::isnan(Mopt)) {   // non-finite samples: stop and write what there is
                nan_size = true;
                break;
            }
            const int64_t target = Mopt >= static_cast<double>(o.cap) ? o.cap : static_cast<int64_t>(Mopt);
            if (target > M[q]) {
                if ((rc = add(q, target - M[q]))) return rc;
                topped = true;
            }
        }
        if (nan_size) break;
        if (topped) continue;   // the variance part: re-estimate, resize
        out.var = 0.0;
        for (int q = 0; q < levels; ++q) out.var += est[q].var / static_cast<double>(M[q]);
        out.bias = extrapolated_bias(est[levels - 1].rms, est[levels - 2].rms);
        if (out.var <= budget && out.bias <= o.eps / std::sqrt(2.0)) {
            out.converged = true;
            break;
        }
        if (out.var > budget || levels >= o.max_levels) break;   // walk cap, or no level left
        ++levels;
        if ((rc = add(levels - 1, o.pilot))) return rc;
    }
    out.levels = levels;
    return MLMC_OK;
}

template <class Add, class Measure>
int algorithm1(const DriverOpts &o, std::vector<int64_t> &M, Add &&add, Measure &&measure,
               DriverOut &out)
{
    return algorithm1(o, M, add, measure, [](int, std::vector<LevelEstimate> &, bool &) { return 0; }, out);
}

}  // namespace mlmc
