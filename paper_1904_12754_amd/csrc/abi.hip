// C-ABI of the library (include/mlmc_expv.h): plan construction (the decomposition
// A = D - T of section 2.1 and the alias tables of the jump law), fixed-schedule and
// adaptive runs (the estimator of section 2.2 and Algorithm 1), level sums and traces.
#include "../../include/mlmc_expv.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "driver.h"
#include "kernels.h"
#include "plan.h"

namespace mlmc {

thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

}  // namespace mlmc

using namespace mlmc;

namespace mlmc {

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

}  // namespace mlmc

namespace {

constexpr size_t kPartialCapBytes = 256u << 20;  // per sub-launch scratch
constexpr int64_t kTargetItems = 16384;          // (row, chunk) items per launch, to fill 256 CUs

}  // namespace



namespace {

template <typename T>
int dev_alloc(mlmc_plan *p, T **ptr, size_t count)
{
    *ptr = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(ptr), count * sizeof(T));
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(e == hipErrorOutOfMemory ? MLMC_ERR_OUT_OF_MEMORY : MLMC_ERR_HIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    p->bytes += static_cast<int64_t>(count * sizeof(T));
    return MLMC_OK;
}

void free_plan(mlmc_plan *p)
{
    if (!p) return;
    (void)hipFree(p->slots);
    (void)hipFree(p->rows_base);
    for (auto &r : p->level_rec) (void)hipFree(r);
    for (auto *t : p->is_slots) (void)hipFree(t);
    (void)hipFree(p->p_slot);
    (void)hipFree(p->prop_P);
    (void)hipFree(p->prop_frag);
    (void)hipFree(p->prop_xhat);
    (void)hipFree(p->prop_xmax);
    (void)hipFree(p->prop_logp);
    (void)hipFree(p->prop_logx);
    if (p->pinned) (void)hipHostFree(p->pinned);
    for (auto &b : p->train_pool) (void)hipFree(b.first);
    for (auto &b : p->grad_pool) (void)hipFree(b.first);
    (void)hipFree(p->req_rows);
    (void)hipFree(p->partial);
    (void)hipFree(p->counters);
    (void)hipFree(p->counter_sums);
    (void)hipFree(p->bad);
    (void)hipFree(p->moments);
    (void)hipFree(p->moment_scratch);
    (void)hipFree(p->acc);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    for (hipEvent_t e : p->tev) (void)hipEventDestroy(e);
    delete p;
}

double value_at(const mlmc_csr_t *A, int64_t e)
{
    return A->values_dtype == MLMC_DTYPE_F64 ? static_cast<const double *>(A->values)[e]
                                              : static_cast<double>(static_cast<const float *>(A->values)[e]);
}

// Walker/Vose alias table of one row. q holds the scaled probabilities deg * p_k and is
// consumed. Entries are processed with two LIFO work lists filled in slot order, so the
// table is a deterministic function of the row.
void build_alias(std::vector<double> &q, std::vector<uint32_t> &thr, std::vector<uint32_t> &alias,
                 std::vector<uint32_t> &small, std::vector<uint32_t> &large)
{
    const uint32_t k = static_cast<uint32_t>(q.size());
    thr.assign(k, 0xFFFFFFFFu);
    alias.resize(k);
    small.clear();
    large.clear();
    for (uint32_t s = 0; s < k; ++s) {
        alias[s] = s;
        (q[s] < 1.0 ? small : large).push_back(s);
    }
    while (!small.empty() && !large.empty()) {
        const uint32_t lo = small.back();
        small.pop_back();
        const uint32_t hi = large.back();
        large.pop_back();
        thr[lo] = static_cast<uint32_t>(std::floor(q[lo] * 4294967296.0));
        alias[lo] = hi;
        q[hi] = (q[hi] + q[lo]) - 1.0;
        (q[hi] < 1.0 ? small : large).push_back(hi);
    }
    // whatever remains has probability one of keeping its own column (thr, alias preset)
}

}  // namespace

namespace mlmc {

int plan_pinned(mlmc_plan *p, size_t bytes, void **out)
{
    if (p->pinned_bytes < bytes) {
        if (p->pinned) (void)hipHostFree(p->pinned);
        p->pinned = nullptr;
        p->pinned_bytes = 0;
        const size_t want = std::max<size_t>(bytes, size_t(64) << 10);   // one allocation for most calls
        MLMC_HIP_TRY(hipHostMalloc(&p->pinned, want, hipHostMallocDefault));
        p->pinned_bytes = want;
    }
    *out = p->pinned;
    return MLMC_OK;
}

int upload_level(mlmc_plan *p, int level, hipStream_t s)
{
    if (level < 0 || level > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "level out of range [0, 28]");
    if (p->level_rec[level]) return MLMC_OK;
    RowRec *rec = nullptr;
    int rc = dev_alloc(p, &rec, static_cast<size_t>(p->n));
    if (rc) return rc;
    p->level_rec[level] = rec;
    if (p->n) {
        MLMC_HIP_TRY(hipMemcpyAsync(rec, p->rows_base, sizeof(RowRec) * p->n, hipMemcpyDeviceToDevice, s));
        MLMC_HIP_TRY(launch_thresholds(rec, p->n, std::ldexp(p->beta, -level), p->bad, s));
    }
    return MLMC_OK;
}

LevelArgs level_args(const mlmc_plan *p, int level, uint64_t seed, int instance)
{
    LevelArgs L;
    L.rec = p->level_rec[level];
    L.slots = p->slots;
    L.src = p->cur_src;
    L.is_slots = (p->proposal_on && level < static_cast<int>(p->is_slots.size())) ? p->is_slots[level]
                                                                                   : nullptr;
    L.n = p->n;
    L.N = 1u << level;
    L.level = level;
    L.base = (level == p->l0);
    L.dt = std::ldexp(p->beta, -level);
    L.half_dt = L.dt * 0.5;
    // FP32 bounds for the walk kernels' certified comparison of a chain's holding time with
    // dt. A float rounds its value by at most 2^-24 relative, so a bracket whose upper end
    // sums in FP32 below dt_below (<= dt (1 - 2^-21)(1 + 2^-24)) lies below dt, and one whose
    // lower end is at or above dt_above lies at or above dt. Outside [2^-100, 2^100] every
    // decision takes the exact FP64 path.
    if (L.dt > 0x1p-100 && L.dt < 0x1p+100) {
        L.dt_below = static_cast<float>(L.dt * (1.0 - 0x1p-21));
        L.dt_above = static_cast<float>(L.dt * (1.0 + 0x1p-21));
    } else {
        L.dt_below = -INFINITY;
        L.dt_above = INFINITY;
    }
    L.k0 = static_cast<uint32_t>(seed);
    L.k1 = static_cast<uint32_t>(seed >> 32);
    L.c3_step = stream_word(level, instance, 0);
    L.c3_jump = stream_word(level, instance, 1);
    L.screen = static_cast<uint32_t>(p->screen);
    return L;
}

}  // namespace mlmc

namespace {

int ensure_partial(mlmc_plan *p, size_t bytes)
{
    if (bytes <= p->partial_bytes) return MLMC_OK;
    (void)hipFree(p->partial);
    p->bytes -= static_cast<int64_t>(p->partial_bytes);
    p->partial = nullptr;
    p->partial_bytes = 0;
    int rc = dev_alloc(p, reinterpret_cast<char **>(&p->partial), bytes);
    if (rc) return rc;
    p->partial_bytes = bytes;
    return MLMC_OK;
}

// Where level_sums keeps the per-(row, chunk) partial sums of a sub-launch: the plan's own
// buffer (grown with hipMalloc as needed), or a fixed caller-provided buffer, in which case
// nothing is allocated, the level's tables must exist already and no timing events are
// recorded.
struct PartialBuf {
    double *fixed = nullptr;
    size_t fixed_bytes = 0;
};

// Walks [walk0, walk0 + M) of every requested row at `level`: per-(row, rhs) sums of Y and
// Y^2 into out1/out2 (overwritten, or added to when accumulate). Jump and non-finite
// counts are added to the counter set `counters`.
int level_sums(mlmc_plan *p, int level, uint64_t seed, int instance, const void *u, int u_f64,
               int32_t nrhs, uint32_t walk0, uint64_t M, double *out1, double *out2, int accumulate,
               unsigned long long *counters, unsigned long long *hash_sums, hipStream_t s,
               const PartialBuf &buf = PartialBuf{})
{
    const bool fixed = buf.fixed != nullptr;
    if (M == 0 || p->n_rows == 0) {
        if (!accumulate && p->n_rows) {
            const int64_t cnt = p->n_rows * nrhs;   // doubles are zero as u64 zero words
            MLMC_HIP_TRY(launch_zero_u64(reinterpret_cast<unsigned long long *>(out1), cnt, s));
            MLMC_HIP_TRY(launch_zero_u64(reinterpret_cast<unsigned long long *>(out2), cnt, s));
        }
        return MLMC_OK;
    }
    if (static_cast<uint64_t>(walk0) + M > 0x100000000ull)
        return fail(MLMC_ERR_RNG_OVERFLOW, "walk indices must stay below 2^32 (the walk word of the Philox counter)");
    int rc;
    if (fixed) {
        if (!p->level_rec[level])
            return fail(MLMC_ERR_INVALID_ARG, "the tables of level " + std::to_string(level) +
                        " are not built yet (a plan builds l0 at creation; any earlier call at a "
                        "level builds it)");
    } else if ((rc = upload_level(p, level, s))) {
        return rc;
    }
    const bool timing = p->timing && !fixed;
    const LevelArgs L = level_args(p, level, seed, instance);
    const Prec prec = p->precision == MLMC_PRECISION_FP64 ? Prec::FP64 : Prec::FP32;
    // walks per item: enough items to fill the chip, at most 64 walks per lane
    const int64_t per_row_items = std::max<int64_t>(1, (kTargetItems + p->n_rows - 1) / p->n_rows);
    uint64_t chunk = (M + per_row_items - 1) / per_row_items;
    chunk = std::min<uint64_t>(std::max<uint64_t>((chunk + 63) / 64 * 64, 64), 64 * 64);
    if (M < 64) chunk = M;   // one item per row; the kernel packs several rows into a wave
    // bound the scratch: sub-launches over walk ranges
    // (one chunk per launch writes the row sums directly and needs no partials)
    const uint64_t bytes_per_item = static_cast<uint64_t>(nrhs) * 2 * sizeof(double);
    const uint64_t cap = fixed ? buf.fixed_bytes : kPartialCapBytes;
    uint64_t max_items = std::max<uint64_t>(1, cap / bytes_per_item);
    uint64_t chunks_per_launch = std::max<uint64_t>(1, max_items / static_cast<uint64_t>(p->n_rows));
    const uint64_t total_chunks = (M + chunk - 1) / chunk;
    chunks_per_launch = std::min(chunks_per_launch, total_chunks);
    double *partial = buf.fixed;
    if (!fixed) {
        rc = ensure_partial(p, chunks_per_launch * p->n_rows * bytes_per_item);
        if (rc) return rc;
        partial = p->partial;
    } else if (chunks_per_launch > 1 && chunks_per_launch * p->n_rows * bytes_per_item > buf.fixed_bytes) {
        return fail(MLMC_ERR_INVALID_ARG, "partial sums exceed the fixed scratch");   // not reached
    }
    bool first = true;
    for (uint64_t c0 = 0; c0 < total_chunks; c0 += chunks_per_launch) {
        const uint64_t nch = std::min(chunks_per_launch, total_chunks - c0);
        const uint64_t wb = c0 * chunk;
        const uint64_t Msub = std::min<uint64_t>(M - wb, nch * chunk);
        if (timing) {
            while (p->tev.size() < p->tev_used + 2) {
                hipEvent_t e;
                MLMC_HIP_TRY(hipEventCreate(&e));
                p->tev.push_back(e);
            }
            MLMC_HIP_TRY(hipEventRecord(p->tev[p->tev_used], s));
        }
        // one chunk per row: the kernel writes (or adds) the row sums itself
        const bool direct = nch == 1;
        const SumsOut lo{partial, out1, out2, direct ? ((first && !accumulate) ? 1 : 2) : 0};
        MLMC_HIP_TRY(launch_level_walks(L, prec, u, u_f64, nrhs, p->req_rows, p->n_rows,
                                        walk0 + static_cast<uint32_t>(wb), static_cast<uint32_t>(Msub),
                                        static_cast<uint32_t>(chunk), static_cast<uint32_t>(nch),
                                        lo, counters, hash_sums, s));
        if (timing) {
            MLMC_HIP_TRY(hipEventRecord(p->tev[p->tev_used + 1], s));
            p->tev_used += 2;
        }
        if (!direct)
            MLMC_HIP_TRY(launch_finalize(partial, p->n_rows, static_cast<uint32_t>(nch), nrhs, out1,
                                         out2, (first && !accumulate) ? 0 : 1, s));
        first = false;
    }
    return MLMC_OK;
}

int check_u(const void *u, int32_t nrhs, int32_t u_dtype)
{
    if (!u) return fail(MLMC_ERR_INVALID_ARG, "u is null");
    if (nrhs < 1 || nrhs > 256) return fail(MLMC_ERR_INVALID_ARG, "nrhs must be in [1, 256]");
    if (u_dtype != MLMC_DTYPE_F32 && u_dtype != MLMC_DTYPE_F64)
        return fail(MLMC_ERR_INVALID_ARG, "u_dtype must be MLMC_DTYPE_F32 or MLMC_DTYPE_F64");
    return MLMC_OK;
}

int ensure_acc(mlmc_plan *p, int levels, int32_t nrhs)
{
    const size_t need = static_cast<size_t>(levels) * 2 * p->n_rows * nrhs;
    if (need <= p->acc_doubles) return MLMC_OK;
    (void)hipFree(p->acc);
    p->bytes -= static_cast<int64_t>(p->acc_doubles * sizeof(double));
    p->acc = nullptr;
    p->acc_doubles = 0;
    int rc = dev_alloc(p, &p->acc, need);
    if (rc) return rc;
    p->acc_doubles = need;
    return MLMC_OK;
}

}  // namespace

extern "C" {

const char *mlmc_status_string(int status)
{
    switch (status) {
    case MLMC_OK: return "ok";
    case MLMC_ERR_INVALID_ARG: return "invalid argument";
    case MLMC_ERR_INVALID_MATRIX: return "invalid matrix";
    case MLMC_ERR_OUT_OF_MEMORY: return "out of memory";
    case MLMC_ERR_HIP: return "HIP runtime error";
    case MLMC_ERR_NONFINITE: return "non-finite samples";
    case MLMC_ERR_NOT_CONVERGED: return "not converged";
    case MLMC_ERR_UNSUPPORTED: return "unsupported";
    case MLMC_ERR_RNG_OVERFLOW: return "random-number counter overflow";
    default: return "unknown status";
    }
}

const char *mlmc_last_error(void) { return g_last_error.c_str(); }

// A matrix whose arrays are in device memory, copied to the host (the plan is built there).
struct HostCopy {
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col_idx;
    std::vector<double> values;     // FP64 values
    std::vector<float> values32;    // FP32 values (value_at widens them)
    mlmc_csr_t csr{};
};

int copy_to_host(const mlmc_csr_t *A, HostCopy &h, hipStream_t s)
{
    const int64_t n = A->n;
    try {
        h.row_ptr.resize(static_cast<size_t>(n) + 1);
        MLMC_HIP_TRY(hipMemcpyAsync(h.row_ptr.data(), A->row_ptr, sizeof(int64_t) * (n + 1),
                                    hipMemcpyDeviceToHost, s));
        MLMC_HIP_TRY(hipStreamSynchronize(s));
        const int64_t nnz = h.row_ptr[n];
        if (h.row_ptr[0] != 0) return fail(MLMC_ERR_INVALID_MATRIX, "row_ptr[0] != 0");
        if (nnz < 0 || nnz >= (int64_t(1) << 40)) return fail(MLMC_ERR_INVALID_MATRIX, "row_ptr[n] out of range");
        h.col_idx.resize(static_cast<size_t>(nnz));
        if (A->values_dtype == MLMC_DTYPE_F64) h.values.resize(static_cast<size_t>(nnz));
        else h.values32.resize(static_cast<size_t>(nnz));
    } catch (const std::bad_alloc &) {
        return fail(MLMC_ERR_OUT_OF_MEMORY, "host copy of the matrix");
    }
    const size_t nnz = h.col_idx.size();
    if (nnz) {
        if (!A->values) return fail(MLMC_ERR_INVALID_ARG, "null values");
        MLMC_HIP_TRY(hipMemcpyAsync(h.col_idx.data(), A->col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
        if (A->values_dtype == MLMC_DTYPE_F64)
            MLMC_HIP_TRY(hipMemcpyAsync(h.values.data(), A->values, sizeof(double) * nnz, hipMemcpyDeviceToHost, s));
        else
            MLMC_HIP_TRY(hipMemcpyAsync(h.values32.data(), A->values, sizeof(float) * nnz, hipMemcpyDeviceToHost, s));
        MLMC_HIP_TRY(hipStreamSynchronize(s));
    }
    h.csr.n = n;
    h.csr.row_ptr = h.row_ptr.data();
    h.csr.col_idx = h.col_idx.data();
    h.csr.values = A->values_dtype == MLMC_DTYPE_F64 ? static_cast<const void *>(h.values.data())
                                                     : static_cast<const void *>(h.values32.data());
    h.csr.values_dtype = A->values_dtype;
    h.csr.memory = MLMC_MEMORY_HOST;
    return MLMC_OK;
}

int mlmc_expv_plan(mlmc_plan_t **out, const mlmc_csr_t *A, const mlmc_plan_opts_t *o, void *stream)
{
    if (!out || !A || !o) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = A->n;
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(MLMC_ERR_INVALID_ARG, "n out of range");
    if (n > 0 && (!A->row_ptr || !A->col_idx)) return fail(MLMC_ERR_INVALID_ARG, "null CSR array");
    if (A->values_dtype != MLMC_DTYPE_F32 && A->values_dtype != MLMC_DTYPE_F64)
        return fail(MLMC_ERR_INVALID_ARG, "values_dtype must be MLMC_DTYPE_F32 or MLMC_DTYPE_F64");
    if (A->memory != MLMC_MEMORY_HOST && A->memory != MLMC_MEMORY_DEVICE)
        return fail(MLMC_ERR_INVALID_ARG, "memory must be MLMC_MEMORY_HOST or MLMC_MEMORY_DEVICE");
    HostCopy host;
    if (A->memory == MLMC_MEMORY_DEVICE && n > 0) {
        const int rc = copy_to_host(A, host, s);
        if (rc) return rc;
        A = &host.csr;
    }
    if (!(o->beta > 0.0) || !std::isfinite(o->beta)) return fail(MLMC_ERR_INVALID_ARG, "beta must be finite and > 0");
    if (o->precision != MLMC_PRECISION_FP64 && o->precision != MLMC_PRECISION_FP32)
        return fail(MLMC_ERR_INVALID_ARG, "precision must be MLMC_PRECISION_FP64 or MLMC_PRECISION_FP32");
    if (o->l0 > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "l0 out of range");
    // ---- validate the CSR structure
    if (n > 0 && A->row_ptr[0] != 0) return fail(MLMC_ERR_INVALID_MATRIX, "row_ptr[0] != 0");
    const int64_t nnz = n > 0 ? A->row_ptr[n] : 0;
    if (nnz > 0 && !A->values) return fail(MLMC_ERR_INVALID_ARG, "null values");
    std::vector<int64_t> stamp(static_cast<size_t>(n), -1);
    int64_t n_slots = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t b = A->row_ptr[i], e = A->row_ptr[i + 1];
        if (e < b || e > nnz) return fail(MLMC_ERR_INVALID_MATRIX, "row_ptr not monotone at row " + std::to_string(i));
        for (int64_t t = b; t < e; ++t) {
            const int32_t c = A->col_idx[t];
            if (c < 0 || c >= n) return fail(MLMC_ERR_INVALID_MATRIX, "column out of range in row " + std::to_string(i));
            if (stamp[c] == i) return fail(MLMC_ERR_INVALID_MATRIX, "repeated column in row " + std::to_string(i));
            stamp[c] = i;
            const double v = value_at(A, t);
            if (!std::isfinite(v)) return fail(MLMC_ERR_INVALID_MATRIX, "non-finite value in row " + std::to_string(i));
            if (c != i && v != 0.0) ++n_slots;
        }
    }
    if (n_slots >= (int64_t(1) << 32)) return fail(MLMC_ERR_UNSUPPORTED, "more than 2^32 - 1 off-diagonal nonzeros");
    // ---- requested rows
    std::vector<int64_t> req;
    if (o->rows) {
        if (o->n_rows < 0) return fail(MLMC_ERR_INVALID_ARG, "n_rows < 0");
        req.assign(o->rows, o->rows + o->n_rows);
        for (int64_t r : req)
            if (r < 0 || r >= n) return fail(MLMC_ERR_INVALID_ARG, "requested row out of range");
    }
    // ---- decomposition A = D - T and alias tables (section 2.1; jump law of section 3)
    std::vector<SlotRec> slots(static_cast<size_t>(std::max<int64_t>(n_slots, 1)));
    std::vector<RowRec> rows(static_cast<size_t>(n));
    std::vector<float> p_slot(static_cast<size_t>(std::max<int64_t>(n_slots, 1)), 0.0f);
    std::vector<double> q;
    std::vector<uint32_t> cols, signs, thr, alias, small, large;
    double r_max = 0.0, d_min = INFINITY, d_max = -INFINITY;
    uint32_t sb = 0;
    for (int64_t i = 0; i < n; ++i) {
        double diag = 0.0, r = 0.0;
        cols.clear();
        signs.clear();
        for (int64_t t = A->row_ptr[i]; t < A->row_ptr[i + 1]; ++t) {
            const double v = value_at(A, t);
            if (A->col_idx[t] == i) {
                diag += v;
            } else if (v != 0.0) {
                r += std::fabs(v);
                cols.push_back(static_cast<uint32_t>(A->col_idx[t]));
                signs.push_back(v < 0.0 ? 1u : 0u);
            }
        }
        const uint32_t deg = static_cast<uint32_t>(cols.size());
        q.clear();
        for (int64_t t = A->row_ptr[i]; t < A->row_ptr[i + 1]; ++t) {
            const double v = value_at(A, t);
            if (A->col_idx[t] != i && v != 0.0) {
                p_slot[sb + q.size()] = static_cast<float>(std::fabs(v) / r);
                q.push_back((std::fabs(v) * static_cast<double>(deg)) / r);
            }
        }
        build_alias(q, thr, alias, small, large);
        for (uint32_t k = 0; k < deg; ++k) {
            SlotRec &sr = slots[sb + k];
            sr.own = cols[k] | (signs[k] << 31);
            sr.alias = cols[alias[k]] | (signs[alias[k]] << 31);
            sr.thr = thr[k];
            sr.pad = 0;
        }
        RowRec &rr = rows[static_cast<size_t>(i)];
        const double d = diag + r;
        rr.slot_begin = sb;
        rr.deg = deg;
        rr.thr = 0xFFFFFFFFu;
        rr.d32 = static_cast<float>(d);
        rr.inv_r = r > 0.0 ? 1.0 / r : INFINITY;
        rr.d64 = d;
        r_max = std::max(r_max, r);
        d_min = std::min(d_min, d);
        d_max = std::max(d_max, d);
        sb += deg;
    }
    int l0 = o->l0;
    if (l0 < 0) {
        l0 = 0;
        if (r_max > 0.0) {
            // clamp before the conversion: 2 beta r_max may overflow to infinity
            const double e = std::ceil(std::log2(2.0 * o->beta * r_max));
            l0 = e > static_cast<double>(kMaxLevel) ? kMaxLevel + 1 : std::max(0, static_cast<int>(e));
        }
    }
    if (l0 > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "coarsest level from the l0 rule exceeds 28");
    // a walk takes beta r jumps on average, the j-th reading Philox block j of its jump stream
    if (o->beta * r_max >= 2147483648.0)
        return fail(MLMC_ERR_RNG_OVERFLOW, "beta * max_i r_i >= 2^31: a walk's jump index (a 32-bit counter "
                                           "word) could wrap");
    // ---- upload
    auto *p = new (std::nothrow) mlmc_plan;
    if (!p) return fail(MLMC_ERR_OUT_OF_MEMORY, "host allocation");
    std::unique_ptr<mlmc_plan, void (*)(mlmc_plan *)> guard(p, free_plan);
    p->n = n;
    p->n_rows = o->rows ? o->n_rows : n;
    p->n_slots = n_slots;
    p->l0 = l0;
    p->precision = o->precision;
    p->beta = o->beta;
    p->r_max = r_max;
    p->d_min = n ? d_min : 0.0;
    p->d_max = n ? d_max : 0.0;
    // the share of walks that jump at all: a walk from row i holds there for the whole time
    // beta with probability e^{-beta r_i}
    {
        double sum = 0.0;
        const int64_t cnt = o->rows ? o->n_rows : n;
        for (int64_t t = 0; t < cnt; ++t) {
            const RowRec &rr = rows[static_cast<size_t>(o->rows ? req[static_cast<size_t>(t)] : t)];
            const double r = rr.deg ? 1.0 / rr.inv_r : 0.0;
            sum += -std::expm1(-o->beta * r);
        }
        p->jump_probability = cnt ? sum / static_cast<double>(cnt) : 0.0;
        p->screen = p->jump_probability < 0.25 ? 1 : 0;
    }
    p->p_slot_host.swap(p_slot);
    int rc;
    if ((rc = dev_alloc(p, &p->slots, slots.size()))) return rc;
    if ((rc = dev_alloc(p, &p->rows_base, rows.size()))) return rc;
    if ((rc = dev_alloc(p, &p->counters, kCounterSetU64 * (kMaxLevel + 1)))) return rc;
    if ((rc = dev_alloc(p, &p->counter_sums, 2 * (kMaxLevel + 1)))) return rc;
    if ((rc = dev_alloc(p, &p->bad, 1))) return rc;
    if ((rc = dev_alloc(p, &p->moments, 3 * (kMaxLevel + 1)))) return rc;
    if ((rc = dev_alloc(p, &p->moment_scratch, 3 * kMomentBlocks))) return rc;
    MLMC_HIP_TRY(hipEventCreate(&p->ev0));
    MLMC_HIP_TRY(hipEventCreate(&p->ev1));
    MLMC_HIP_TRY(hipMemcpyAsync(p->slots, slots.data(), sizeof(SlotRec) * slots.size(), hipMemcpyHostToDevice, s));
    if (n) MLMC_HIP_TRY(hipMemcpyAsync(p->rows_base, rows.data(), sizeof(RowRec) * rows.size(), hipMemcpyHostToDevice, s));
    if (o->rows && o->n_rows > 0) {
        if ((rc = dev_alloc(p, &p->req_rows, req.size()))) return rc;
        MLMC_HIP_TRY(hipMemcpyAsync(p->req_rows, req.data(), sizeof(int64_t) * req.size(), hipMemcpyHostToDevice, s));
    }
    MLMC_HIP_TRY(hipMemsetAsync(p->bad, 0, sizeof(unsigned int), s));
    if ((rc = upload_level(p, l0, s))) return rc;
    unsigned int bad = 0;
    MLMC_HIP_TRY(hipMemcpyAsync(&bad, p->bad, sizeof bad, hipMemcpyDeviceToHost, s));
    MLMC_HIP_TRY(hipStreamSynchronize(s));
    if (bad) return fail(MLMC_ERR_INVALID_ARG, "coarsest level too coarse: some row jumps in every step (r dt > 22)");
    *out = guard.release();
    return MLMC_OK;
}

int mlmc_expv_plan_info(const mlmc_plan_t *p, mlmc_plan_info_t *info)
{
    if (!p || !info) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    info->n = p->n;
    info->n_rows = p->n_rows;
    info->n_slots = p->n_slots;
    info->l0 = p->l0;
    info->precision = p->precision;
    info->beta = p->beta;
    info->r_max = p->r_max;
    info->d_min = p->d_min;
    info->d_max = p->d_max;
    info->device_bytes = p->bytes;
    info->jump_probability = p->jump_probability;
    info->screened = p->screen;
    info->pad = 0;
    return MLMC_OK;
}

void mlmc_expv_destroy(mlmc_plan_t *p) { free_plan(p); }

int mlmc_expv_level_sums(mlmc_plan_t *p, const void *u, int32_t nrhs, int32_t u_dtype, uint64_t seed,
                         int32_t instance, int32_t level, uint32_t walk0, uint32_t walks, double *sum1,
                         double *sum2, int64_t *jumps, uint64_t *hash_sums, void *stream)
{
    if (!p) return fail(MLMC_ERR_INVALID_ARG, "null plan");
    if (p->n_rows > 0 && (!sum1 || !sum2)) return fail(MLMC_ERR_INVALID_ARG, "null output");
    int rc = check_u(u, nrhs, u_dtype);
    if (rc) return rc;
    if (instance < 0 || instance > 4095) return fail(MLMC_ERR_INVALID_ARG, "instance must be in [0, 4095]");
    if (level < p->l0 || level > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "level must be in [l0, 28]");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    MLMC_HIP_TRY(hipMemsetAsync(p->counters, 0, kCounterSetU64 * sizeof(unsigned long long), s));
    if (hash_sums && p->n_rows > 0)
        MLMC_HIP_TRY(hipMemsetAsync(hash_sums, 0, sizeof(uint64_t) * p->n_rows, s));
    rc = level_sums(p, level, seed, instance, u, u_dtype == MLMC_DTYPE_F64, nrhs, walk0, walks, sum1,
                    sum2, 0, p->counters, reinterpret_cast<unsigned long long *>(hash_sums), s);
    if (rc) return rc;
    if (jumps) {
        unsigned long long c[2];
        MLMC_HIP_TRY(launch_counter_sum(p->counters, 1, p->counter_sums, s));
        MLMC_HIP_TRY(hipMemcpyAsync(c, p->counter_sums, sizeof c, hipMemcpyDeviceToHost, s));
        MLMC_HIP_TRY(hipStreamSynchronize(s));
        *jumps = static_cast<int64_t>(c[0]);
        if (c[1]) return fail(MLMC_ERR_NONFINITE, std::to_string(c[1]) + " non-finite samples");
    }
    return MLMC_OK;
}

}  // extern "C"

// ---- allocation-free level sums ---------------------------------------------------------
// The per-(row, chunk) partial sums of mlmc_expv_level_sums_noalloc live in this fixed device
// array (one copy per device, loaded with the code object and held until the process ends)
// instead of the plan's hipMalloc-grown buffer. Host code never passes the array's name to a
// kernel: its device address is looked up once per device with hipGetSymbolAddress.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device (looked up on first use).
int scratch_on_current_device(double **out)
{
    int dev = -1;
    MLMC_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MLMC_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MLMC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return MLMC_OK;
}

}  // namespace

extern "C" {

int mlmc_expv_level_sums_noalloc(mlmc_plan_t *p, const void *u, int32_t nrhs, int32_t u_dtype,
                                 uint64_t seed, int32_t instance, int32_t level, uint32_t walk0,
                                 uint32_t walks, double *sum1, double *sum2, int64_t *jumps,
                                 uint64_t *hash_sums, void *stream)
{
    if (!p) return fail(MLMC_ERR_INVALID_ARG, "null plan");
    if (p->n_rows > 0 && (!sum1 || !sum2)) return fail(MLMC_ERR_INVALID_ARG, "null output");
    int rc = check_u(u, nrhs, u_dtype);
    if (rc) return rc;
    if (instance < 0 || instance > 4095) return fail(MLMC_ERR_INVALID_ARG, "instance must be in [0, 4095]");
    if (level < p->l0 || level > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "level must be in [l0, 28]");
    double *scr = nullptr;
    if ((rc = scratch_on_current_device(&scr))) return rc;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    MLMC_HIP_TRY(launch_zero_u64(p->counters, static_cast<int64_t>(kCounterSetU64), s));
    if (hash_sums && p->n_rows > 0)
        MLMC_HIP_TRY(launch_zero_u64(reinterpret_cast<unsigned long long *>(hash_sums), p->n_rows, s));
    PartialBuf buf;
    buf.fixed = scr;
    buf.fixed_bytes = kNoAllocScratchBytes;
    rc = level_sums(p, level, seed, instance, u, u_dtype == MLMC_DTYPE_F64, nrhs, walk0, walks, sum1,
                    sum2, 0, p->counters, reinterpret_cast<unsigned long long *>(hash_sums), s, buf);
    if (rc) return rc;
    if (jumps) {
        unsigned long long c[2];
        MLMC_HIP_TRY(launch_counter_sum(p->counters, 1, p->counter_sums, s));
        MLMC_HIP_TRY(hipMemcpyAsync(c, p->counter_sums, sizeof c, hipMemcpyDeviceToHost, s));
        MLMC_HIP_TRY(hipStreamSynchronize(s));
        *jumps = static_cast<int64_t>(c[0]);
        if (c[1]) return fail(MLMC_ERR_NONFINITE, std::to_string(c[1]) + " non-finite samples");
    }
    return MLMC_OK;
}

int mlmc_expv_trace(mlmc_plan_t *p, uint64_t seed, int32_t instance, int32_t level, int64_t count,
                    const int64_t *rows, const uint32_t *walks, int64_t *final_state, int32_t *sign,
                    int64_t *jumps, uint64_t *hash, double *log_fine, double *log_coarse, void *stream)
{
    if (!p) return fail(MLMC_ERR_INVALID_ARG, "null plan");
    if (count < 0) return fail(MLMC_ERR_INVALID_ARG, "count < 0");
    if (count > 0 && (!rows || !walks || !final_state || !sign || !jumps || !hash || !log_fine || !log_coarse))
        return fail(MLMC_ERR_INVALID_ARG, "null array");
    if (instance < 0 || instance > 4095) return fail(MLMC_ERR_INVALID_ARG, "instance must be in [0, 4095]");
    if (level < p->l0 || level > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "level must be in [l0, 28]");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = upload_level(p, level, s);
    if (rc) return rc;
    const LevelArgs L = level_args(p, level, seed, instance);
    MLMC_HIP_TRY(launch_trace(L, p->precision == MLMC_PRECISION_FP64 ? Prec::FP64 : Prec::FP32, count, rows,
                              walks, final_state, sign, jumps, hash, log_fine, log_coarse, s));
    return MLMC_OK;
}

namespace {

// The full-vector run (fixed schedule or Algorithm 1). With `learn`, the adaptive run
// trains the proposal of level l0 after its plain pilot (see mlmc_expv_run_learned).
int run_impl(mlmc_plan *p, const void *u, int32_t nrhs, int32_t u_dtype, const mlmc_run_opts_t *o, double *x,
             mlmc_stats_t *stats, const mlmc_train_opts_t *learn, float *params_out, mlmc_train_stats_t *tst,
             void *stream)
{
    if (!p || !o) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    if (!x && p->n_rows > 0) return fail(MLMC_ERR_INVALID_ARG, "x is null");
    int rc = check_u(u, nrhs, u_dtype);
    if (rc) return rc;
    if (o->instance < 0 || o->instance > 4095) return fail(MLMC_ERR_INVALID_ARG, "instance must be in [0, 4095]");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int u_f64 = u_dtype == MLMC_DTYPE_F64;
    const int64_t count = p->n_rows * nrhs;
    const bool adaptive = o->eps > 0.0;
    int max_levels;
    int64_t pilot = o->pilot_walks;
    if (adaptive) {
        if (pilot == 0) pilot = default_pilot(count);
        if (pilot < 2 || pilot >= (int64_t(1) << 32))
            return fail(MLMC_ERR_INVALID_ARG, "pilot_walks must be 0 or in [2, 2^32)");
        max_levels = o->max_levels > 0 ? o->max_levels : 20;
        max_levels = std::min(max_levels, std::min(MLMC_MAX_LEVELS, kMaxLevel - p->l0 + 1));
        if (max_levels < 2) return fail(MLMC_ERR_INVALID_ARG, "max_levels must allow at least two levels");
    } else {
        if (o->num_levels < 1 || o->num_levels > MLMC_MAX_LEVELS || p->l0 + o->num_levels - 1 > kMaxLevel)
            return fail(MLMC_ERR_INVALID_ARG, "num_levels out of range");
        if (!o->walks) return fail(MLMC_ERR_INVALID_ARG, "walks is null");
        for (int qq = 0; qq < o->num_levels; ++qq)
            if (o->walks[qq] < 1 || o->walks[qq] >= (int64_t(1) << 32))
                return fail(MLMC_ERR_INVALID_ARG, "walks per level must be in [1, 2^32)");
        max_levels = o->num_levels;
    }
    // a learned run keeps one more pair of accumulators: level l0 under the proposal
    if ((rc = ensure_acc(p, max_levels + (learn ? 1 : 0), nrhs))) return rc;
    const size_t stride = static_cast<size_t>(2) * count;
    bool alt0 = false;   // level l0 sits in the spare pair
    auto base_of = [&](int qq) { return p->acc + (qq == 0 && alt0 ? max_levels : qq) * stride; };
    auto s1_of = [&](int qq) { return base_of(qq); };
    auto s2_of = [&](int qq) { return base_of(qq) + count; };
    std::vector<int64_t> M(static_cast<size_t>(max_levels), 0);
    int64_t extra0 = 0;  // walks of level l0 run but left out of the estimate
    if (learn) p->proposal_on = false;   // the pilot walks with the plain law
    p->timing = stats != nullptr;
    p->tev_used = 0;
    struct TimingOff {   // the events time this run's launches only
        mlmc_plan *p;
        ~TimingOff() { p->timing = false; }
    } timing_off{p};
    MLMC_HIP_TRY(hipMemsetAsync(p->counters, 0, kCounterSetU64 * sizeof(unsigned long long) * max_levels, s));
    MLMC_HIP_TRY(hipEventRecord(p->ev0, s));
    // add `extra` walks at level index qq
    auto add_walks = [&](int qq, int64_t extra) -> int {
        const int level = p->l0 + qq;
        const int r2 = level_sums(p, level, o->seed, o->instance, u, u_f64, nrhs,
                                  static_cast<uint32_t>(M[qq]), static_cast<uint64_t>(extra), s1_of(qq),
                                  s2_of(qq), M[qq] > 0 ? 1 : 0, p->counters + kCounterSetU64 * qq, nullptr, s);
        if (r2) return r2;
        M[qq] += extra;
        return MLMC_OK;
    };
    struct Mom { double sum_m, sum_m2, sum_v; };
    std::vector<Mom> mom(static_cast<size_t>(max_levels));
    std::vector<unsigned long long> ctr(2 * static_cast<size_t>(kMaxLevel + 1));
    auto read_moments = [&](int levels) -> int {
        for (int qq = 0; qq < levels; ++qq)
            MLMC_HIP_TRY(launch_level_moments(s1_of(qq), s2_of(qq), count, static_cast<double>(M[qq]),
                                              p->moments + 3 * qq, p->moment_scratch, s));
        std::vector<double> h(3 * static_cast<size_t>(levels));
        const size_t hb = sizeof(double) * h.size(), cb = sizeof(unsigned long long) * 2 * levels;
        void *pin = nullptr;
        const int r2 = plan_pinned(p, hb + cb, &pin);
        if (r2) return r2;
        MLMC_HIP_TRY(hipMemcpyAsync(pin, p->moments, hb, hipMemcpyDeviceToHost, s));
        MLMC_HIP_TRY(launch_counter_sum(p->counters, levels, p->counter_sums, s));
        MLMC_HIP_TRY(hipMemcpyAsync(static_cast<char *>(pin) + hb, p->counter_sums, cb, hipMemcpyDeviceToHost, s));
        MLMC_HIP_TRY(hipStreamSynchronize(s));
        std::memcpy(h.data(), pin, hb);
        std::memcpy(ctr.data(), static_cast<char *>(pin) + hb, cb);
        for (int qq = 0; qq < levels; ++qq) mom[qq] = Mom{h[3 * qq], h[3 * qq + 1], h[3 * qq + 2]};
        return MLMC_OK;
    };
    const double cnt = static_cast<double>(std::max<int64_t>(count, 1));
    auto level_var = [&](int qq) { return unbiased_var(mom[qq].sum_v / cnt, M[qq]); };
    auto level_rms = [&](int qq) { return debiased_rms(mom[qq].sum_m2 / cnt, level_var(qq), M[qq]); };
    auto level_cost = [&](int qq) {
        const double walks_total =
            static_cast<double>(M[qq] + (qq == 0 ? extra0 : 0)) * std::max<int64_t>(p->n_rows, 1);
        return std::ldexp(1.0, p->l0 + qq) + 4.0 * static_cast<double>(ctr[2 * qq]) / walks_total;
    };
    int levels = 0;
    bool converged = false;
    int iterations = 0;
    double bias = 0.0;
    if (!adaptive) {
        levels = o->num_levels;
        for (int qq = 0; qq < levels; ++qq)
            if ((rc = add_walks(qq, o->walks[qq]))) return rc;
        MLMC_HIP_TRY(hipEventRecord(p->ev1, s));
        converged = true;
    } else {
        // Algorithm 1 on the row means: V_l = mean_i V_{l,i}, m_l = RMS_i m_{l,i}
        DriverOpts d;
        d.eps = o->eps;
        d.pilot = pilot;
        d.max_levels = max_levels;
        d.cap = o->max_walks > 0 ? std::min<int64_t>(o->max_walks, 0xFFFFFFFFll) : 0xFFFFFFFFll;
        auto measure = [&](int lv, std::vector<LevelEstimate> &est) -> int {
            const int r2 = read_moments(lv);
            if (r2) return r2;
            for (int qq = 0; qq < lv; ++qq) est[qq] = LevelEstimate{level_var(qq), level_cost(qq), level_rms(qq)};
            return MLMC_OK;
        };
        // learned run: after the pilot, train on its estimate; the variance judge runs as many
        // level-l0 walks under the proposal (the same walk indices) into the spare pair and
        // keeps them, in place of the plain ones, if their variance is lower
        auto after_pilot = [&](int lv, std::vector<LevelEstimate> &est, bool &again) -> int {
            if (!learn) return MLMC_OK;
            hipEvent_t te[2] = {nullptr, nullptr};
            struct Ev {
                hipEvent_t *e;
                ~Ev()
                {
                    for (int i = 0; i < 2; ++i)
                        if (e[i]) (void)hipEventDestroy(e[i]);
                }
            } ev_guard{te};
            MLMC_HIP_TRY(hipEventCreate(&te[0]));
            MLMC_HIP_TRY(hipEventCreate(&te[1]));
            MLMC_HIP_TRY(hipEventRecord(te[0], s));
            CombineArgs xa{};
            xa.levels = lv;
            for (int qq = 0; qq < lv; ++qq) {
                xa.s1[qq] = s1_of(qq);
                xa.inv_M[qq] = 1.0 / static_cast<double>(M[qq]);
            }
            int r2 = train_from_levels(p, u, learn, xa, params_out, tst, s);
            if (r2) return r2;
            const double var_plain = est[0].var;
            const int64_t m_plain = M[0];
            p->proposal_on = true;
            alt0 = true;
            M[0] = 0;
            if ((r2 = add_walks(0, m_plain))) return r2;
            MLMC_HIP_TRY(launch_level_moments(s1_of(0), s2_of(0), count, static_cast<double>(M[0]), p->moments,
                                              p->moment_scratch, s));
            double h[3];
            void *pin = nullptr;
            if ((r2 = plan_pinned(p, sizeof h, &pin))) return r2;
            MLMC_HIP_TRY(hipMemcpyAsync(pin, p->moments, sizeof h, hipMemcpyDeviceToHost, s));
            MLMC_HIP_TRY(hipEventRecord(te[1], s));
            MLMC_HIP_TRY(hipStreamSynchronize(s));
            std::memcpy(h, pin, sizeof h);
            const double var_learned = unbiased_var(h[2] / cnt, M[0]);
            const bool accepted = var_learned < var_plain;
            if (!accepted) {
                alt0 = false;
                M[0] = m_plain;
                p->proposal_on = false;
            }
            extra0 = m_plain;
            if (tst) {
                float ms = 0.0f;
                MLMC_HIP_TRY(hipEventElapsedTime(&ms, te[0], te[1]));
                tst->train_ms = ms;
                tst->judge_var_plain = var_plain;
                tst->judge_var_learned = var_learned;
                tst->accepted = accepted ? 1 : 0;
            }
            again = true;
            return MLMC_OK;
        };
        DriverOut out;
        if ((rc = algorithm1(d, M, add_walks, measure, after_pilot, out))) return rc;
        levels = out.levels;
        converged = out.converged;
        iterations = out.iterations;
        bias = out.bias;
        MLMC_HIP_TRY(hipEventRecord(p->ev1, s));
    }
    // x = sum_l m_l (FP64 combine)
    CombineArgs ca{};
    ca.levels = levels;
    for (int qq = 0; qq < levels; ++qq) {
        ca.s1[qq] = s1_of(qq);
        ca.inv_M[qq] = 1.0 / static_cast<double>(M[qq]);
    }
    MLMC_HIP_TRY(launch_combine(ca, count, x, s));
    if (stats || adaptive) {
        if ((rc = read_moments(levels))) return rc;
    }
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->l0 = p->l0;
        stats->num_levels = levels;
        stats->converged = converged ? 1 : 0;
        stats->driver_iterations = iterations;
        double var = 0.0;
        for (int qq = 0; qq < levels; ++qq) {
            stats->walks[qq] = M[qq];
            stats->jumps[qq] = static_cast<int64_t>(ctr[2 * qq]);
            stats->level_mean_rms[qq] = level_rms(qq);
            stats->level_var[qq] = level_var(qq);
            stats->level_cost[qq] = level_cost(qq);
            stats->steps += (M[qq] + (qq == 0 ? extra0 : 0)) * p->n_rows * (int64_t(1) << (p->l0 + qq));
            stats->total_jumps += static_cast<int64_t>(ctr[2 * qq]);
            stats->nonfinite += static_cast<int64_t>(ctr[2 * qq + 1]);
            var += level_var(qq) / static_cast<double>(M[qq]);
        }
        stats->est_variance = var;
        stats->est_bias = adaptive ? bias : 0.0;
        float ms = 0.0f;
        MLMC_HIP_TRY(hipEventElapsedTime(&ms, p->ev0, p->ev1));
        stats->kernel_ms = ms;
        double wk = 0.0;
        for (size_t e = 0; e + 1 < p->tev_used; e += 2) {
            float t = 0.0f;
            MLMC_HIP_TRY(hipEventElapsedTime(&t, p->tev[e], p->tev[e + 1]));
            wk += t;
        }
        stats->walk_kernel_ms = wk;
        stats->walk_launches = static_cast<int64_t>(p->tev_used / 2);
        if (stats->nonfinite) return fail(MLMC_ERR_NONFINITE, std::to_string(stats->nonfinite) + " non-finite samples");
    }
    if (adaptive && !converged) return fail(MLMC_ERR_NOT_CONVERGED, "level or walk cap reached before eps");
    return MLMC_OK;
}

}  // namespace

int mlmc_expv_run(mlmc_plan_t *p, const void *u, int32_t nrhs, int32_t u_dtype, const mlmc_run_opts_t *o,
                  double *x, mlmc_stats_t *stats, void *stream)
{
    return run_impl(p, u, nrhs, u_dtype, o, x, stats, nullptr, nullptr, nullptr, stream);
}

int mlmc_expv_run_learned(mlmc_plan_t *p, const void *u, int32_t u_dtype, const mlmc_run_opts_t *o,
                          const mlmc_train_opts_t *t, float *params_out, double *x, mlmc_stats_t *stats,
                          mlmc_train_stats_t *train_stats, void *stream)
{
    if (!p || !o || !t) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    if (!(o->eps > 0.0)) return fail(MLMC_ERR_INVALID_ARG, "the learned run is adaptive: eps must be > 0");
    if (u_dtype != MLMC_DTYPE_F32) return fail(MLMC_ERR_UNSUPPORTED, "training reads an FP32 right-hand side");
    if (t->num_levels != 1) return fail(MLMC_ERR_INVALID_ARG, "the learned run sets tables for level l0 only");
    int rc;
    if ((rc = check_learned_opts(p, t))) return rc;
    if (train_stats) std::memset(train_stats, 0, sizeof *train_stats);
    return run_impl(p, u, 1, u_dtype, o, x, stats, t, params_out, train_stats, stream);
}


// Algorithm 3: the same calls with a source vector F (x' = A x + F, F constant in time).
namespace {

struct SourceScope {
    mlmc_plan *p;
    SourceScope(mlmc_plan *q, const void *F) : p(q) { p->cur_src = F; }
    ~SourceScope() { p->cur_src = nullptr; }
};

int check_source(const mlmc_plan *p, const void *F)
{
    if (!F && p->n > 0) return fail(MLMC_ERR_INVALID_ARG, "F is null");
    if (p->l0 < 1)
        return fail(MLMC_ERR_INVALID_ARG, "a source term needs l0 >= 1 (Simpson's rule needs two intervals on every grid)");
    return MLMC_OK;
}

}  // namespace

int mlmc_expv_run_source(mlmc_plan_t *p, const void *u, const void *F, int32_t u_dtype,
                         const mlmc_run_opts_t *opts, double *x, mlmc_stats_t *stats, void *stream)
{
    if (!p) return fail(MLMC_ERR_INVALID_ARG, "null plan");
    int rc = check_source(p, F);
    if (rc) return rc;
    SourceScope scope(p, F);
    return mlmc_expv_run(p, u, 1, u_dtype, opts, x, stats, stream);
}

int mlmc_expv_level_sums_source(mlmc_plan_t *p, const void *u, const void *F, int32_t u_dtype,
                                uint64_t seed, int32_t instance, int32_t level, uint32_t walk0,
                                uint32_t walks, double *sum1, double *sum2, int64_t *jumps,
                                uint64_t *hash_sums, void *stream)
{
    if (!p) return fail(MLMC_ERR_INVALID_ARG, "null plan");
    int rc = check_source(p, F);
    if (rc) return rc;
    SourceScope scope(p, F);
    return mlmc_expv_level_sums(p, u, 1, u_dtype, seed, instance, level, walk0, walks, sum1, sum2, jumps,
                                hash_sums, stream);
}

}  // extern "C"
