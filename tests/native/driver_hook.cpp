// Host-only checks of Algorithm 1's driver (paper_1904_12754_amd/csrc/driver.h) on a mock of
// the device side: levels with fixed per-walk variances, costs and level terms.
//   1. With the hook that does nothing, the driver's walks, levels and verdict are those of
//      the overload without a hook.
//   2. A hook that replaces the coarsest level's pilot walks by walks of a tenfold lower
//      variance (as the learned run does) is called exactly once, after the pilot's first
//      measurement; the levels are measured again before any sample size is computed, and
//      the coarsest level's final sample size is Giles' optimum for the lower variance.
// Prints "driver hook ok" and returns 0 when every check holds.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../paper_1904_12754_amd/csrc/driver.h"

using namespace mlmc;

namespace {

int failures = 0;

void check(bool ok, const char *what)
{
    if (!ok) {
        std::printf("FAILED: %s\n", what);
        ++failures;
    }
}

struct Mock {
    // level q: per-walk variance 0.9 4^-q, cost 2^(q + 2) + 8, level term 0.04 4^-q
    double var0_factor = 1.0;   // the coarsest level's variance is scaled by this
    int measures = 0;
    std::vector<std::pair<int, int64_t>> adds;
    double var(int q) const { return 0.9 * std::pow(4.0, -q) * (q == 0 ? var0_factor : 1.0); }
    double cost(int q) const { return std::ldexp(1.0, q + 2) + 8.0; }
    double rms(int q) const { return 0.04 * std::pow(4.0, -q); }
};

struct Result {
    std::vector<int64_t> M;
    DriverOut out;
    Mock mock;
    int hook_calls = 0;
    int measures_at_hook = -1;
};

DriverOpts options()
{
    DriverOpts o;
    o.eps = 2e-3;
    o.pilot = 4;
    o.max_levels = 10;
    o.cap = int64_t(1) << 40;
    return o;
}

// hook: 0 = the overload without a hook, 1 = a hook that does nothing, 2 = the replacement
Result run(int hook)
{
    Result r;
    const DriverOpts o = options();
    r.M.assign(static_cast<size_t>(o.max_levels), 0);
    auto add = [&](int q, int64_t extra) -> int {
        r.mock.adds.emplace_back(q, extra);
        r.M[q] += extra;
        return MLMC_OK;
    };
    auto measure = [&](int lv, std::vector<LevelEstimate> &est) -> int {
        ++r.mock.measures;
        for (int q = 0; q < lv; ++q) est[q] = LevelEstimate{r.mock.var(q), r.mock.cost(q), r.mock.rms(q)};
        return MLMC_OK;
    };
    int rc = MLMC_OK;
    if (hook == 0) {
        rc = algorithm1(o, r.M, add, measure, r.out);
    } else {
        auto after = [&](int lv, std::vector<LevelEstimate> &est, bool &again) -> int {
            ++r.hook_calls;
            r.measures_at_hook = r.mock.measures;
            if (hook == 1) return MLMC_OK;
            // the pilot's level-l0 walks are replaced by as many walks of a lower variance
            check(lv == 5, "the hook sees the pilot's five levels");
            check(est[0].var == 0.9, "the hook sees the pilot's measured variance");
            const int64_t m = r.M[0];
            r.M[0] = 0;
            r.mock.var0_factor = 0.1;
            const int rc2 = add(0, m);
            again = true;
            return rc2;
        };
        rc = algorithm1(o, r.M, add, measure, after, r.out);
    }
    check(rc == MLMC_OK, "the driver returns MLMC_OK");
    return r;
}

// Giles' optimum for level q under the mock's variances over `levels` levels
int64_t optimum(const Mock &m, int q, int levels, double eps)
{
    double tot = 0.0;
    for (int k = 0; k < levels; ++k) tot += std::sqrt(m.var(k) * m.cost(k));
    return static_cast<int64_t>(std::ceil(2.0 / (eps * eps) * std::sqrt(m.var(q) / m.cost(q)) * tot));
}

}  // namespace

int main()
{
    const Result a = run(0), b = run(1), c = run(2);
    // 1. the no-op hook changes nothing
    check(a.M == b.M, "no-op hook: the same sample sizes");
    check(a.mock.adds == b.mock.adds, "no-op hook: the same walks added, in the same order");
    check(a.out.levels == b.out.levels && a.out.converged == b.out.converged &&
              a.out.iterations == b.out.iterations,
          "no-op hook: the same levels, verdict and iterations");
    check(b.hook_calls == 1 && b.measures_at_hook == 1, "no-op hook: called once, after the first measurement");
    check(a.out.converged, "the plain driver converges");
    // 2. the replacement
    check(c.hook_calls == 1, "replacement: the hook is called once");
    check(c.measures_at_hook == 1, "replacement: after the pilot's first measurement");
    check(c.out.converged, "replacement: the driver converges");
    const double eps = options().eps;
    const int64_t want0 = std::max<int64_t>(options().pilot, optimum(c.mock, 0, c.out.levels, eps));
    check(c.M[0] == want0, "replacement: level l0 ends at the optimum for the lower variance");
    check(c.M[0] < a.M[0], "replacement: fewer walks at l0 than the plain driver");
    for (int q = 1; q < c.out.levels; ++q)
        check(c.M[q] == std::max<int64_t>(options().pilot, optimum(c.mock, q, c.out.levels, eps)),
              "replacement: the other levels at their optimum");
    // the walks the hook added at l0 follow the pilot's, and sizing comes after
    bool seen_pilot_replay = false;
    for (size_t i = 0; i < c.mock.adds.size(); ++i)
        if (i == 5 && c.mock.adds[i].first == 0 && c.mock.adds[i].second == options().pilot) seen_pilot_replay = true;
    check(seen_pilot_replay, "replacement: the hook's walks come right after the five pilot levels");
    std::printf("plain M0 %lld, replaced M0 %lld (optimum %lld), levels %d / %d\n",
                static_cast<long long>(a.M[0]), static_cast<long long>(c.M[0]), static_cast<long long>(want0),
                a.out.levels, c.out.levels);
    if (failures == 0) std::printf("driver hook ok\n");
    return failures == 0 ? 0 : 1;
}
