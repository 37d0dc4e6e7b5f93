// Runs the library's host-side plan construction on valid and malformed matrices, for a build
// of the host code with AddressSanitizer and UndefinedBehaviorSanitizer (test
// infrastructure): CSR validation, the decomposition A = D - T, the alias tables of the jump
// law and the coarsest-level rule run on the host before any device call. Without a GPU the
// first device allocation fails and the plan call returns MLMC_ERR_HIP; with one it succeeds
// and the plan is destroyed. Any sanitizer report ends the program with a nonzero status.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/mlmc_expv.h"

namespace {

struct Csr {
    int64_t n = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
};

// A random sparse signed matrix with rows of 0..deg off-diagonal entries (some rows absorbing,
// some without a diagonal entry) and, when `hub`, one row linked to every other.
Csr random_matrix(int64_t n, int deg, uint32_t seed, bool hub)
{
    Csr a;
    a.n = n;
    a.row_ptr.push_back(0);
    uint32_t x = seed;
    auto next = [&] {
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        return x;
    };
    for (int64_t i = 0; i < n; ++i) {
        std::vector<char> used(static_cast<size_t>(n), 0);
        const int k = (hub && i == 0) ? static_cast<int>(n) : static_cast<int>(next() % (deg + 1));
        if (next() % 3 != 0) {
            a.col.push_back(static_cast<int32_t>(i));
            a.val.push_back(-1.0 - static_cast<int>(next() % 100) / 50.0);
            used[static_cast<size_t>(i)] = 1;
        }
        for (int t = 0; t < k; ++t) {
            const int64_t j = (hub && i == 0) ? t : static_cast<int64_t>(next() % n);
            if (used[static_cast<size_t>(j)]) continue;
            used[static_cast<size_t>(j)] = 1;
            a.col.push_back(static_cast<int32_t>(j));
            a.val.push_back((static_cast<int>(next() % 200) - 100) / 37.0);
        }
        a.row_ptr.push_back(static_cast<int64_t>(a.col.size()));
    }
    return a;
}

int plan_status(const Csr &a, double beta, int32_t precision, int32_t l0, const int64_t *rows,
                int64_t n_rows)
{
    mlmc_csr_t m{a.n, a.row_ptr.data(), a.col.data(), a.val.data(), MLMC_DTYPE_F64};
    mlmc_plan_opts_t o{beta, precision, l0, rows, n_rows};
    mlmc_plan_t *p = nullptr;
    const int rc = mlmc_expv_plan(&p, &m, &o, nullptr);
    if (rc == MLMC_OK) {
        mlmc_plan_info_t info;
        if (mlmc_expv_plan_info(p, &info) != MLMC_OK) return -1;
        mlmc_expv_destroy(p);
    }
    return rc;
}

}  // namespace

int main()
{
    int bad = 0;
    auto expect = [&](bool ok, const char *what) {
        if (!ok) {
            std::printf("unexpected status: %s (%s)\n", what, mlmc_last_error());
            ++bad;
        }
    };
    auto valid = [](int rc) { return rc == MLMC_OK || rc == MLMC_ERR_HIP || rc == MLMC_ERR_OUT_OF_MEMORY; };
    for (uint32_t seed = 1; seed <= 6; ++seed) {
        const Csr a = random_matrix(40 + 13 * seed, 1 + static_cast<int>(seed % 5), seed, seed % 2 == 0);
        expect(valid(plan_status(a, 0.5, MLMC_PRECISION_FP32, -1, nullptr, 0)), "valid matrix, fp32");
        expect(valid(plan_status(a, 2.0, MLMC_PRECISION_FP64, 3, nullptr, 0)), "valid matrix, fp64");
        const int64_t rows[3] = {0, a.n - 1, a.n / 2};
        expect(valid(plan_status(a, 1.0, MLMC_PRECISION_FP32, -1, rows, 3)), "requested rows");
        const int64_t out_of_range[1] = {a.n};
        expect(plan_status(a, 1.0, MLMC_PRECISION_FP32, -1, out_of_range, 1) == MLMC_ERR_INVALID_ARG,
               "row out of range");
        expect(plan_status(a, 0.0, MLMC_PRECISION_FP32, -1, nullptr, 0) == MLMC_ERR_INVALID_ARG, "beta 0");
        expect(plan_status(a, 1e308, MLMC_PRECISION_FP32, -1, nullptr, 0) == MLMC_ERR_INVALID_ARG,
               "coarsest level beyond 28");
        Csr c = a;
        if (!c.col.empty()) {
            c.col[c.col.size() / 2] = static_cast<int32_t>(c.n);
            expect(plan_status(c, 1.0, MLMC_PRECISION_FP32, -1, nullptr, 0) == MLMC_ERR_INVALID_MATRIX,
                   "column out of range");
        }
        c = a;
        if (!c.val.empty()) {
            c.val.back() = NAN;
            expect(plan_status(c, 1.0, MLMC_PRECISION_FP32, -1, nullptr, 0) == MLMC_ERR_INVALID_MATRIX,
                   "non-finite value");
        }
        c = a;
        if (c.n > 3) {
            std::swap(c.row_ptr[2], c.row_ptr[3]);
            if (c.row_ptr[2] != c.row_ptr[3])
                expect(plan_status(c, 1.0, MLMC_PRECISION_FP32, -1, nullptr, 0) == MLMC_ERR_INVALID_MATRIX,
                       "row_ptr not monotone");
        }
    }
    Csr empty;
    empty.row_ptr.push_back(0);
    expect(valid(plan_status(empty, 1.0, MLMC_PRECISION_FP32, -1, nullptr, 0)), "empty matrix");
    expect(mlmc_expv_plan(nullptr, nullptr, nullptr, nullptr) == MLMC_ERR_INVALID_ARG, "null arguments");
    for (int code = 0; code < 9; ++code)
        if (!mlmc_status_string(code)) ++bad;
    std::printf("plan sanitize %s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
