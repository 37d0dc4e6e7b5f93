// Learned proposal for the jump law (importance sampling).
//
// The walks jump from row k with the law p_s = |a_ks| / r_k over the row's off-diagonal
// slots (section 3). Drawing the jump from another law q with the same support and
// multiplying the path's functional by p/q of the slot taken keeps every level's
// expectation, so the estimator stays unbiased. q comes from a small MLP of row features:
//
//   features (16): max(log p_s, -20) and clip(log((|xhat(col_s)| + delta) / (|xhat_k| +
//                  delta)), -8, 8) for six slots, r_k dt, d_k dt, |xhat_k| / max|xhat|,
//                  (l - l0) / 8   (xhat: a pilot estimate of x, delta = 1e-6 max|xhat|)
//   The log features make the variance-optimal law q_s ~ p_s |x(col_s)| linear in the
//   inputs.
//   16 -> 64 (ReLU) -> 64 (ReLU) -> 7;  q_s = alpha softmax_s(z) + (1 - alpha) p_s over the
//   valid slots, z_s = feature s + feature 6 + s + output s (the log-ratio prior, whose
//   softmax is p_s (|xhat(col_s)| + delta) normalised, plus the network's correction),
//   alpha = 0.9 sigmoid(output 6)
//
// Rows with more than six slots keep q = p. Inference runs on the matrix cores: every wave
// evaluates 16 rows with v_mfma_f32_16x16x16_bf16 in the transposed form H^T = W^T X^T, so
// the output fragment of one layer is the input fragment of the next, and the lanes that
// hold a row's outputs build its alias table and likelihood ratios. Training (the
// cross-entropy method: minimise the |Y|-weighted negative log-likelihood of the jumps the
// plain walks took, whose minimiser over all laws is q ~ |Y| p) runs in FP32 with plain
// per-thread kernels; the parameters are updated by Adam.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mlmc_expv.h"
#include "common.h"
#include "kernels.h"
#include "plan.h"
#include "walk_engine.h"

namespace mlmc {
namespace {

constexpr int NF = 16, NH = 64, NO = 7, NS = 6;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NF * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NO, NPARAM = OFF_B3 + NO;
constexpr float kAlphaMax = 0.9f;
constexpr double kLogPMin = -20.0;        // floor of the log p_s features
constexpr double kLogRatioMax = 8.0;      // clip of the log value-ratio features
constexpr int kCaptureJumps = 8;   // transitions recorded per captured walk
constexpr int kMaxHeldOut = 1 << 16;  // held-out transitions of a training call
constexpr int kEvalEvery = 16;        // Adam steps between held-out evaluations

static_assert(NPARAM == MLMC_PROPOSAL_PARAMS, "parameter layout");

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

uint32_t nblk(uint64_t n, uint32_t t) { return static_cast<uint32_t>((n + t - 1) / t); }

__device__ __forceinline__ short bf16_bits(float x)
{
    // round to nearest even (finite inputs)
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return static_cast<short>(b >> 16);
}

struct FeatureArgs {
    const RowRec *rec;        // the level's row records (d, 1/r, slot range)
    const SlotRec *slots;     // plain slots (own column)
    const float *p_slot;      // plain law per slot
    const float *logp;        // max(log p_s, -20) per slot (formed in FP64, rounded once)
    const double *xhat;       // pilot estimate (nullable: zeros)
    const double *logx;       // log(|xhat_i| + delta) per row, delta = 1e-6 max |xhat|
    const double *xmax;       // device scalar: max |xhat| (1 when xhat is null or zero)
    int64_t n;
    float dt, lvl;            // dt of the level, (l - l0) / 8
};

// The logarithms the features take, formed once: per slot of the plan, and per row for each
// pilot estimate (the log value ratio of a slot is then a difference, in FP64).
__global__ void logp_kernel(const float *p, int64_t n, float *out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = static_cast<float>(fmax(log(static_cast<double>(p[i])), kLogPMin));
}

__global__ void logx_kernel(const double *x, const double *xmax, int64_t n, double *out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = log((x ? fabs(x[i]) : 0.0) + 1e-6 * *xmax);
}

// The 16 features of row `row`, each formed in FP64 and rounded once to FP32. Slot
// features are 0 past the row's slots and for rows with more than NS slots. Every load of
// the row (its slots' log probabilities and the log estimates at their columns) is issued
// before the first use.
__device__ __forceinline__ void row_features(const FeatureArgs &a, const RowRec &rr, uint32_t row, double xmax,
                                             float f[NF])
{
    const uint32_t deg = rr.deg;
    const bool elig = deg >= 1 && deg <= NS;
    const double xr = a.xhat ? fabs(a.xhat[row]) : 0.0;
#pragma unroll
    for (int s = 0; s < 2 * NS; ++s) f[s] = 0.0f;
    if (elig) {
        float lp[NS];
        double lx[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            // slots past the row's last repeat its last slot (in range, results unused)
            const uint32_t si = rr.slot_begin + min(static_cast<uint32_t>(s), deg - 1);
            lp[s] = a.logp[si];
            lx[s] = a.logx[a.slots[si].own & kColMask];
        }
        const double lxr = a.logx[row];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (static_cast<uint32_t>(s) < deg) {
                f[s] = lp[s];
                f[NS + s] = static_cast<float>(fmin(fmax(lx[s] - lxr, -kLogRatioMax), kLogRatioMax));
            }
        }
    }
    f[12] = (rr.inv_r < INFINITY) ? static_cast<float>(1.0 / rr.inv_r) * a.dt : 0.0f;
    f[13] = rr.d32 * a.dt;
    f[14] = static_cast<float>(xr / xmax);
    f[15] = a.lvl;
}

// Features of rows[i] (of row i when rows is null) into F[i], i < count; one record per
// thread, stored as four 16-byte vectors.
__global__ __launch_bounds__(256) void features_kernel(FeatureArgs a, const uint32_t *rows, int64_t count, float *F)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t row = rows ? rows[i] : static_cast<uint32_t>(i);
    const RowRec rr = a.rec[row];
    float f[NF];
    row_features(a, rr, row, *a.xmax, f);
    float4_t *out = reinterpret_cast<float4_t *>(F + i * NF);
#pragma unroll
    for (int v = 0; v < NF / 4; ++v) out[v] = float4_t{f[4 * v], f[4 * v + 1], f[4 * v + 2], f[4 * v + 3]};
}

// max |x| in two stages: kAbsmaxBlocks partial maxima, then the final one (1 when x is
// null or zero). Maxima do not depend on the order of evaluation.
constexpr int kAbsmaxBlocks = 256;

__global__ void absmax_partial(const double *x, int64_t n, double *part)
{
    __shared__ double sh[256];
    double m = 0.0;
    if (x)
        for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += kAbsmaxBlocks * 256)
            m = fmax(m, fabs(x[i]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void absmax_final(const double *part, double *out)
{
    __shared__ double sh[kAbsmaxBlocks];
    sh[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int o = kAbsmaxBlocks / 2; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0] > 0.0 ? sh[0] : 1.0;
}

// out[0] = max |x| (1 when zero); out[1 .. kAbsmaxBlocks] is scratch.
void absmax(const double *x, int64_t n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(absmax_partial, dim3(kAbsmaxBlocks), dim3(256), 0, s, x, n, out + 1);
    hipLaunchKernelGGL(absmax_final, dim3(1), dim3(kAbsmaxBlocks), 0, s, out + 1, out);
}

// What the features read of a pilot estimate: xmax[0] = max |x| (1 when zero) and
// logx[i] = log(|x_i| + 1e-6 xmax[0]).
void prepare_xhat(const double *x, int64_t n, double *xmax, double *logx, hipStream_t s)
{
    absmax(x, n, xmax, s);
    if (n > 0) hipLaunchKernelGGL(logx_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, x, xmax, n, logx);
}

// ------------------------------------------------------------------------------------
// Weight fragments for v_mfma_f32_16x16x16_bf16 in the transposed form. For the A operand
// of a 16x16x16 MFMA lane l holds A[l % 16][4 (l / 16) + i], i = 0..3; A = W^T, so lane l
// of the fragment (layer, out tile c, k step kk) holds W[16 kk + 4 (l / 16) + i][16 c + l % 16].
// ------------------------------------------------------------------------------------
constexpr int FR1 = 0;                      // [c 0..3][lane][4]
constexpr int FR2 = FR1 + 4 * 64 * 4;       // [c 0..3][kk 0..3][lane][4]
constexpr int FR3 = FR2 + 16 * 64 * 4;      // [kk 0..3][lane][4]
constexpr int NFRAG = FR3 + 4 * 64 * 4;

__global__ void fragments_kernel(const float *P, short *frag)
{
    const int t = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= NFRAG) return;
    int idx, lane, i, c = 0, kk = 0, layer;
    if (t < FR2) { layer = 1; idx = t - FR1; c = idx / 256; }
    else if (t < FR3) { layer = 2; idx = t - FR2; c = idx / 1024; kk = (idx / 256) % 4; }
    else { layer = 3; idx = t - FR3; kk = idx / 256; }
    lane = (idx / 4) % 64;
    i = idx % 4;
    const int krow = 16 * kk + 4 * (lane / 16) + i;   // input feature
    const int ocol = 16 * c + lane % 16;              // output feature
    float w = 0.0f;
    if (layer == 1) w = P[OFF_W1 + krow * NH + ocol];
    else if (layer == 2) w = P[OFF_W2 + krow * NH + ocol];
    else w = (lane % 16) < NO ? P[OFF_W3 + krow * NO + (lane % 16)] : 0.0f;
    frag[t] = bf16_bits(w);
}

struct TableArgs {
    FeatureArgs fa;
    const short *frag;
    const float *P;           // FP32 parameters (biases)
    SlotRecIS *out;           // the level's proposal slot table
    // optional per-slot export for inspection: threshold, alias slot, ratio p/q, q
    uint32_t *x_thr;
    int32_t *x_alias;
    float *x_ratio;
    float *x_q;
    int identity;             // 1: q = p (copy of the plain tables, ratio 1)
};

__device__ __forceinline__ float4_t mfma16(short4_t a, short4_t b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ short4_t pack4(float4_t v)
{
    short4_t r;
    r.x = bf16_bits(v.x);
    r.y = bf16_bits(v.y);
    r.z = bf16_bits(v.z);
    r.w = bf16_bits(v.w);
    return r;
}

// Alias table of row `row` for the law q (FP64 scaled probabilities, the construction of
// the plain plan) with likelihood ratios p/q; copies the plain row when identity.
__device__ void build_row(const TableArgs &a, const RowRec &rr, const float *q)
{
    const uint32_t k = rr.deg, sb = rr.slot_begin;
    if (k == 0) return;
    const bool use_q = !a.identity && k <= NS;
    if (!use_q) {
        for (uint32_t s = 0; s < k; ++s) {
            const SlotRec pr = a.fa.slots[sb + s];
            SlotRecIS o;
            o.own = pr.own;
            o.alias = pr.alias;
            o.thr = pr.thr;
            o.pad = 0;
            o.ratio_own = 1.0f;
            o.ratio_alias = 1.0f;
            o.pad2[0] = o.pad2[1] = 0;
            a.out[sb + s] = o;
            if (a.x_thr) {
                a.x_thr[sb + s] = pr.thr;
                // alias slot: the slot of the row whose column is the alias column
                int32_t al = static_cast<int32_t>(s);
                for (uint32_t t = 0; t < k; ++t)
                    if ((a.fa.slots[sb + t].own & kColMask) == (pr.alias & kColMask)) al = static_cast<int32_t>(t);
                a.x_alias[sb + s] = al;
                a.x_ratio[sb + s] = 1.0f;
                a.x_q[sb + s] = a.fa.p_slot[sb + s];
            }
        }
        return;
    }
    double qs[NS];
    uint32_t thr[NS];
    uint32_t alias[NS];
    int small[NS], large[NS];
    int ns = 0, nl = 0;
    for (uint32_t s = 0; s < k; ++s) {
        qs[s] = static_cast<double>(q[s]) * static_cast<double>(k);
        thr[s] = 0xFFFFFFFFu;
        alias[s] = s;
        if (qs[s] < 1.0) small[ns++] = static_cast<int>(s); else large[nl++] = static_cast<int>(s);
    }
    while (ns > 0 && nl > 0) {
        const int lo = small[--ns];
        const int hi = large[--nl];
        thr[lo] = static_cast<uint32_t>(floor(qs[lo] * 4294967296.0));
        alias[lo] = static_cast<uint32_t>(hi);
        qs[hi] = (qs[hi] + qs[lo]) - 1.0;
        if (qs[hi] < 1.0) small[ns++] = hi; else large[nl++] = hi;
    }
    for (uint32_t s = 0; s < k; ++s) {
        const float ratio_s = a.fa.p_slot[sb + s] / q[s];
        const float ratio_a = a.fa.p_slot[sb + alias[s]] / q[alias[s]];
        SlotRecIS o;
        o.own = a.fa.slots[sb + s].own;
        o.alias = a.fa.slots[sb + alias[s]].own;
        o.thr = thr[s];
        o.pad = 0;
        o.ratio_own = ratio_s;
        o.ratio_alias = ratio_a;
        o.pad2[0] = o.pad2[1] = 0;
        a.out[sb + s] = o;
        if (a.x_thr) {
            a.x_thr[sb + s] = thr[s];
            a.x_alias[sb + s] = static_cast<int32_t>(alias[s]);
            a.x_ratio[sb + s] = ratio_s;
            a.x_q[sb + s] = q[s];
        }
    }
}

// The alias table of one row's law q over its k <= NS slots, and the ratios p/q: the
// construction of the plain plan (scaled probabilities k q_s in FP64; slots below 1 and at
// or above 1 on two stacks; each step pairs the top small slot with the top large one).
// The stacks and the alias slots are packed 4 bits per slot, and the arrays are read and
// written by selects, so that the row stays in registers.
__device__ __forceinline__ void build_row_q(const TableArgs &a, uint32_t sb, uint32_t k, const float p[NS],
                                            const float q[NS])
{
    uint32_t own[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) own[s] = a.fa.slots[sb + min(static_cast<uint32_t>(s), k - 1)].own;
    double qs[NS];
    uint32_t thr[NS];
    uint32_t alias = 0, small = 0, large = 0;
    int ns = 0, nl = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        qs[s] = static_cast<double>(q[s]) * static_cast<double>(k);
        thr[s] = 0xFFFFFFFFu;
        alias |= static_cast<uint32_t>(s) << (4 * s);
        if (static_cast<uint32_t>(s) < k) {
            if (qs[s] < 1.0) {
                small |= static_cast<uint32_t>(s) << (4 * ns);
                ++ns;
            } else {
                large |= static_cast<uint32_t>(s) << (4 * nl);
                ++nl;
            }
        }
    }
    while (ns > 0 && nl > 0) {
        --ns;
        --nl;
        const int lo = static_cast<int>((small >> (4 * ns)) & 15u);
        const int hi = static_cast<int>((large >> (4 * nl)) & 15u);
        double qlo = 0.0, qhi = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            qlo = s == lo ? qs[s] : qlo;
            qhi = s == hi ? qs[s] : qhi;
        }
        const uint32_t t = static_cast<uint32_t>(floor(qlo * 4294967296.0));
        const double nh = (qhi + qlo) - 1.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            thr[s] = s == lo ? t : thr[s];
            qs[s] = s == hi ? nh : qs[s];
        }
        alias = (alias & ~(15u << (4 * lo))) | (static_cast<uint32_t>(hi) << (4 * lo));
        if (nh < 1.0) {
            small = (small & ~(15u << (4 * ns))) | (static_cast<uint32_t>(hi) << (4 * ns));
            ++ns;
        } else {
            large = (large & ~(15u << (4 * nl))) | (static_cast<uint32_t>(hi) << (4 * nl));
            ++nl;
        }
    }
    float ratio[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) ratio[s] = p[s] / q[s];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (static_cast<uint32_t>(s) >= k) break;
        const int al = static_cast<int>((alias >> (4 * s)) & 15u);
        uint32_t own_a = own[0];
        float ratio_a = ratio[0];
#pragma unroll
        for (int j = 1; j < NS; ++j) {
            own_a = j == al ? own[j] : own_a;
            ratio_a = j == al ? ratio[j] : ratio_a;
        }
        SlotRecIS o;
        o.own = own[s];
        o.alias = own_a;
        o.thr = thr[s];
        o.pad = 0;
        o.ratio_own = ratio[s];
        o.ratio_alias = ratio_a;
        o.pad2[0] = o.pad2[1] = 0;
        a.out[sb + s] = o;
        if (a.x_thr) {
            a.x_thr[sb + s] = thr[s];
            a.x_alias[sb + s] = al;
            a.x_ratio[sb + s] = ratio[s];
            a.x_q[sb + s] = q[s];
        }
    }
}

// Rows per workgroup and iteration of the tables kernel: four waves of 64 rows, one row
// per lane. Each wave evaluates its 64 rows as four 16-row MFMA tiles.
constexpr int kTabRows = 256;
constexpr int kTabWaves = kTabRows / 64;
constexpr int kTabGridMax = 256 * 7;   // seven workgroups (28 waves) for each of the 256 CUs

// Features -> MFMA MLP -> q -> alias tables and ratios. A workgroup stages the weight
// fragments and biases in LDS once, then takes 256 rows per iteration (grid stride): every
// lane forms its row's features, the wave's 64 rows pass through LDS into the B-operand
// layout of the MFMA tiles, the tiles' outputs pass back through LDS to the row's lane, and
// that lane builds the row's alias table.
__global__ __launch_bounds__(kTabRows, 6) void tables_kernel(TableArgs a)
{
    __shared__ short4_t s_frag[NFRAG / 4];
    __shared__ float4_t s_b1[NH / 4], s_b2[NH / 4], s_b3[2];
    // 32 bytes per row: its BF16 features, then (written after the row's tile has read
    // them) its outputs 0..6 and one unused
    __shared__ float4_t s_row[kTabWaves][64][2];
    const int tid = static_cast<int>(threadIdx.x);
    const int w = tid / 64, lane = tid & 63, r = lane % 16, g = lane / 16;
    short4_t *const s_x = reinterpret_cast<short4_t *>(&s_row[w][0][0]);
    const int64_t n = a.fa.n;
    const int64_t nit = (n + kTabRows - 1) / kTabRows;
    if (a.identity) {           // uniform over the launch
        for (int64_t it = blockIdx.x; it < nit; it += gridDim.x) {
            const int64_t row = it * kTabRows + tid;
            if (row < n) build_row(a, a.fa.rec[row], nullptr);
        }
        return;
    }
    {
        const short4_t *fr = reinterpret_cast<const short4_t *>(a.frag);
        for (int i = tid; i < NFRAG / 4; i += kTabRows) s_frag[i] = fr[i];
        const float4_t *P4 = reinterpret_cast<const float4_t *>(a.P);
        if (tid < NH / 4) s_b1[tid] = P4[OFF_B1 / 4 + tid];
        else if (tid < NH / 2) s_b2[tid - NH / 4] = P4[OFF_B2 / 4 + tid - NH / 4];
        else if (tid < NH / 2 + 2) {
            const int j = tid - NH / 2;
            float4_t b;
            b.x = a.P[OFF_B3 + 4 * j + 0];
            b.y = a.P[OFF_B3 + 4 * j + 1];
            b.z = a.P[OFF_B3 + 4 * j + 2];
            b.w = 4 * j + 3 < NO ? a.P[OFF_B3 + 4 * j + 3] : 0.0f;
            s_b3[j] = b;
        }
    }
    const double xmax = *a.fa.xmax;
    for (int64_t it = blockIdx.x; it < nit; it += gridDim.x) {
        const int64_t row64 = it * kTabRows + tid;
        const bool inrow = row64 < n;
        const uint32_t row = inrow ? static_cast<uint32_t>(row64) : 0u;
        const RowRec rr = a.fa.rec[row];
        // the log-ratio prior of the logits: features s and NS + s, summed in FP32
        float prior[NS];
        {
            float f[NF];
            row_features(a.fa, rr, row, xmax, f);
#pragma unroll
            for (int v = 0; v < NF / 4; ++v) {
                float4_t fv = {f[4 * v], f[4 * v + 1], f[4 * v + 2], f[4 * v + 3]};
                if (!inrow) fv = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
                s_x[lane * (NF / 4) + v] = pack4(fv);
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) prior[s] = f[s] + f[NS + s];
        }
        __syncthreads();
        // four tiles of 16 rows: lane r + 16 g holds inputs 4g..4g+3 of tile row r, and
        // the layer outputs 16 c + 4g + i of tile row r
#pragma unroll 1
        for (int t = 0; t < 4; ++t) {
            // an opaque zero keeps the weight and bias reads from LDS inside the loop
            // (hoisted out of it they would hold 84 registers for the whole kernel)
            int z0 = 0;
            asm volatile("" : "+v"(z0));
            const short4_t *fr = s_frag + z0;
            const float4_t *b1 = s_b1 + z0, *b2 = s_b2 + z0, *b3 = s_b3 + z0;
            const short4_t x = s_x[(16 * t + r) * (NF / 4) + g];
            short4_t h1[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                float4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
                acc = mfma16(fr[(FR1 / 4) + c * 64 + lane], x, acc);
                const float4_t b = b1[4 * c + g];
                float4_t v;
                v.x = fmaxf(acc.x + b.x, 0.0f);
                v.y = fmaxf(acc.y + b.y, 0.0f);
                v.z = fmaxf(acc.z + b.z, 0.0f);
                v.w = fmaxf(acc.w + b.w, 0.0f);
                h1[c] = pack4(v);
            }
            short4_t h2[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                float4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) acc = mfma16(fr[(FR2 / 4) + (c * 4 + kk) * 64 + lane], h1[kk], acc);
                const float4_t b = b2[4 * c + g];
                float4_t v;
                v.x = fmaxf(acc.x + b.x, 0.0f);
                v.y = fmaxf(acc.y + b.y, 0.0f);
                v.z = fmaxf(acc.z + b.z, 0.0f);
                v.w = fmaxf(acc.w + b.w, 0.0f);
                h2[c] = pack4(v);
            }
            float4_t o = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) o = mfma16(fr[(FR3 / 4) + kk * 64 + lane], h2[kk], o);
            if (g < 2) {
                const float4_t b = b3[g];
                float4_t ob;
                ob.x = o.x + b.x;
                ob.y = o.y + b.y;
                ob.z = o.z + b.z;
                ob.w = o.w + b.w;
                s_row[w][16 * t + r][g] = ob;
            }
        }
        __syncthreads();
        if (!inrow) continue;
        const uint32_t k = rr.deg;
        if (k < 1 || k > NS) {      // q = p: the plain row
            build_row(a, rr, nullptr);
            continue;
        }
        float pl[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) pl[s] = a.fa.p_slot[rr.slot_begin + min(static_cast<uint32_t>(s), k - 1)];
        const float4_t o0 = s_row[w][lane][0], o1 = s_row[w][lane][1];
        const float out[NO] = {o0.x, o0.y, o0.z, o0.w, o1.x, o1.y, o1.z};
        // logits: the log-ratio prior (features s and NS + s, FP32) plus the correction
        float z[NS];
        float zmax = -INFINITY;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            z[s] = out[s] + prior[s];
            if (static_cast<uint32_t>(s) < k) zmax = fmaxf(zmax, z[s]);
        }
        float den = 0.0f, e[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            e[s] = expf(z[s] - zmax);
            if (static_cast<uint32_t>(s) < k) den += e[s];
        }
        const float alpha = kAlphaMax / (1.0f + expf(-out[NS]));
        float q[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) q[s] = alpha * (e[s] / den) + (1.0f - alpha) * pl[s];
        build_row_q(a, rr.slot_begin, k, pl, q);
    }
}

// ------------------------------------------------------------------------------------
// Transition capture: plain walks at one level record, for each of their first jumps out
// of an eligible row, the row and the slot taken, and the walk's |Y| as the weight.
// ------------------------------------------------------------------------------------
// Records the first kCaptureJumps jumps out of eligible rows: the row and the slot taken.
struct CaptureObs {
    const SlotRec *slots;
    uint32_t count = 0;
    uint32_t rows[kCaptureJumps];
    int32_t taken[kCaptureJumps];
    __device__ __forceinline__ void jump(uint32_t from, const RowRec &rr, uint32_t cs)
    {
        if (count >= kCaptureJumps || rr.deg > NS) return;
        int32_t t = -1;
        for (uint32_t s = 0; s < rr.deg; ++s)
            if (((slots[rr.slot_begin + s].own ^ cs) & kColMask) == 0) t = static_cast<int32_t>(s);
        rows[count] = from;
        taken[count] = t;
        ++count;
    }
};

__global__ void capture_kernel(LevelArgs L, const float *__restrict__ u, uint32_t stride_rows,
                               uint32_t n_sample, uint32_t walks, uint32_t *t_row, int32_t *t_slot,
                               float *t_w)
{
    const uint64_t id = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= static_cast<uint64_t>(n_sample) * walks) return;
    const uint64_t row64 = (id / walks) * stride_rows;
    const uint32_t walk = static_cast<uint32_t>(id % walks);
    CaptureObs obs;
    obs.slots = L.slots;
    float wy = 0.0f;
    if (row64 < static_cast<uint64_t>(L.n)) {
        const WalkOut<float> o = run_walk<float, false, false, CaptureObs>(L, static_cast<uint32_t>(row64), walk, &obs);
        wy = fabsf(weight_of<float>(o, L.base, static_cast<float>(L.half_dt)) * u[o.k]);
    }
    for (uint32_t j = 0; j < kCaptureJumps; ++j) {
        const uint64_t o = id * kCaptureJumps + j;
        const bool has = j < obs.count;
        t_row[o] = has ? obs.rows[j] : 0u;
        t_slot[o] = has ? obs.taken[j] : -1;
        t_w[o] = has ? wy : 0.0f;
    }
}

// ------------------------------------------------------------------------------------
// The recorded transitions that carry a sample (weight > 0 and finite, a slot taken) are kept
// in their recorded order. Kept transition r (its rank in that order) is held out when
// r mod 8 = 7 and r / 8 < kMaxHeldOut (as held-out transition r / 8); the others train, as
// training transition r - min(r / 8, kMaxHeldOut). Three passes: per-block counts, one
// workgroup scans the counts, and every block scatters its kept transitions.
// ------------------------------------------------------------------------------------
constexpr int kKeepPer = 4;                    // transitions per thread
constexpr int kKeepBlock = 256 * kKeepPer;     // transitions per block

__device__ __forceinline__ bool kept_transition(float w, int32_t slot)
{
    return w > 0.0f && isfinite(w) && slot >= 0;
}

// Exclusive scan of v over the 256 threads of the block (sh: 256 entries); returns the
// thread's offset, and the block total in *total.
__device__ __forceinline__ uint32_t block_scan_256(uint32_t v, uint32_t *sh, uint32_t *total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t add = t >= o ? sh[t - o] : 0u;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const uint32_t incl = sh[t];
    *total = sh[255];
    __syncthreads();
    return incl - v;
}

__global__ void keep_count_kernel(const int32_t *__restrict__ slot, const float *__restrict__ w,
                                  uint64_t T, uint32_t *counts)
{
    __shared__ uint32_t sh[256];
    const uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * kKeepBlock + threadIdx.x * kKeepPer;
    uint32_t c = 0;
    for (int k = 0; k < kKeepPer; ++k)
        if (i0 + k < T && kept_transition(w[i0 + k], slot[i0 + k])) ++c;
    uint32_t total;
    block_scan_256(c, sh, &total);
    if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// counts[0..nb) -> exclusive offsets in place; offsets[nb] = the total. One workgroup.
__global__ void keep_scan_kernel(uint32_t *counts, uint32_t nb)
{
    __shared__ uint32_t sh[256];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += 256) {
        const uint32_t b = b0 + threadIdx.x;
        const uint32_t v = b < nb ? counts[b] : 0u;
        uint32_t total;
        const uint32_t off = block_scan_256(v, sh, &total);
        if (b < nb) counts[b] = carry + off;
        carry += total;
    }
    if (threadIdx.x == 0) counts[nb] = carry;
}

__global__ void keep_scatter_kernel(const uint32_t *__restrict__ row, const int32_t *__restrict__ slot,
                                    const float *__restrict__ w, uint64_t T,
                                    const uint32_t *__restrict__ offsets, uint32_t *tr_row,
                                    int32_t *tr_slot, float *tr_w, uint32_t *va_row, int32_t *va_slot,
                                    float *va_w)
{
    __shared__ uint32_t sh[256];
    const uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * kKeepBlock + threadIdx.x * kKeepPer;
    bool keep[kKeepPer];
    uint32_t c = 0;
    for (int k = 0; k < kKeepPer; ++k) {
        keep[k] = i0 + k < T && kept_transition(w[i0 + k], slot[i0 + k]);
        c += keep[k] ? 1u : 0u;
    }
    uint32_t total;
    uint64_t r = offsets[blockIdx.x] + block_scan_256(c, sh, &total);
    for (int k = 0; k < kKeepPer; ++k) {
        if (!keep[k]) continue;
        const uint64_t i = i0 + k;
        const uint64_t q = r / 8;
        if ((r & 7u) == 7u && q < static_cast<uint64_t>(kMaxHeldOut)) {
            va_row[q] = row[i];
            va_slot[q] = slot[i];
            va_w[q] = w[i];
        } else {
            const uint64_t t = r - min(q, static_cast<uint64_t>(kMaxHeldOut));
            tr_row[t] = row[i];
            tr_slot[t] = slot[i];
            tr_w[t] = w[i];
        }
        ++r;
    }
}

// ------------------------------------------------------------------------------------
// Training: FP32 forward / backward, one workgroup per chunk of kTC transitions of the batch,
// activations in LDS; every workgroup writes its own partial gradient and the partials are
// added in a fixed order (deterministic).
// ------------------------------------------------------------------------------------
constexpr int kTC = 16;               // transitions per chunk
constexpr int kMaxTrainBlocks = 1024; // workgroups of a training pass (they loop over chunks)

// The transitions of a batch: element b is transition ((begin + b) * mult) % T of the arrays.
struct BatchSrc {
    const uint32_t *row;
    const int32_t *slot;
    const float *w;
    uint64_t T, begin, mult;
    __device__ __forceinline__ uint64_t at(int b) const
    {
        return ((begin + static_cast<uint64_t>(b)) * mult) % T;
    }
};

__device__ __forceinline__ float block_sum_256(float v, float *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const float r = sh[0];
    __syncthreads();
    return r;
}

// Loss terms of the batch (lossb[b]) and, with kBackward, the workgroup's partial gradient
// partial[blockIdx.x][NPARAM] summed over the chunks it takes. Thread t works on hidden unit
// j = t % 64 for the rows (or inputs) of group g = t / 64, with independent accumulators;
// W2 sits in LDS with a padded row stride so that reads along either index are free of bank
// conflicts.
constexpr int kRG = kTC / 4;          // rows per thread group
constexpr int kW2S = NH + 1;          // padded LDS row stride of W2

template <bool kBackward>
__global__ __launch_bounds__(256) void train_kernel(const float *__restrict__ P, const float *__restrict__ F,
                                                    const float *__restrict__ p_slot,
                                                    const RowRec *__restrict__ rec, BatchSrc src, int B,
                                                    float shrink, float *__restrict__ partial,
                                                    float *__restrict__ lossb)
{
    __shared__ float sW1[NF * NH], sW2[NH * kW2S], sW3[NH * NO], sB1[NH], sB2[NH], sB3[8];
    __shared__ float sX[kTC * NF], sH1[kTC * NH], sH2[kTC * NH], sD2[kTC * NH];
    __shared__ float sdO[kTC * 8], sP6[kTC * NS], sW[kTC];
    __shared__ int sSlot[kTC];
    __shared__ int sValid[kTC];           // bit s: slot s is one of the row's entries
    __shared__ uint32_t sRow[kTC];
    __shared__ uint32_t sT[kTC];          // index of the transition (its record in F)
    __shared__ float sRed[256];
    const int tid = static_cast<int>(threadIdx.x);
    const int j = tid & (NH - 1), g = tid >> 6;
    for (int e = tid; e < NF * NH; e += 256) sW1[e] = P[OFF_W1 + e];
    for (int e = tid; e < NH * NH; e += 256) sW2[(e / NH) * kW2S + (e % NH)] = P[OFF_W2 + e];
    for (int e = tid; e < NH * NO; e += 256) sW3[e] = P[OFF_W3 + e];
    if (tid < NH) {
        sB1[tid] = P[OFF_B1 + tid];
        sB2[tid] = P[OFF_B2 + tid];
    }
    if (tid < NO) sB3[tid] = P[OFF_B3 + tid];
    // total weight of the batch, in the same order in every workgroup; element b + 256 of
    // the batch is 256 mult (mod T) past element b
    float acc = 0.0f;
    if (tid < B) {
        uint64_t idx = src.at(tid);
        const uint64_t stride = (256ull * (src.mult % src.T)) % src.T;
        for (int b = tid; b < B; b += 256) {
            acc += src.w[idx];
            idx += stride;
            if (idx >= src.T) idx -= src.T;
        }
    }
    const float Wsum = block_sum_256(acc, sRed);
    float *G = partial + static_cast<size_t>(blockIdx.x) * NPARAM;
    const int chunks = (B + kTC - 1) / kTC;
    bool first = true;
    for (int c = static_cast<int>(blockIdx.x); c < chunks; c += static_cast<int>(gridDim.x)) {
        const int b0 = c * kTC;
        const int nb = min(kTC, B - b0);
        __syncthreads();
        if (tid < kTC) {
            int slot = -1, valid = 0;
            float w = 0.0f;
            uint32_t row = 0, tix = 0;
            if (tid < nb) {
                const uint64_t t = src.at(b0 + tid);
                tix = static_cast<uint32_t>(t);
                row = src.row[t];
                const RowRec rr = rec[row];
                slot = src.slot[t];
                w = src.w[t];
                const bool elig = rr.deg >= 1 && rr.deg <= NS;
                for (int q = 0; q < NS; ++q) {
                    const bool ok = elig && q < static_cast<int>(rr.deg);
                    sP6[tid * NS + q] = ok ? p_slot[rr.slot_begin + q] : 0.0f;
                    valid |= ok ? (1 << q) : 0;
                }
            } else {
                for (int q = 0; q < NS; ++q) sP6[tid * NS + q] = 0.0f;
            }
            sSlot[tid] = slot;
            sValid[tid] = valid;
            sW[tid] = w;
            sRow[tid] = row;
            sT[tid] = tix;
        }
        __syncthreads();
        for (int e = tid; e < kTC * NF; e += 256) {
            const int b = e / NF;
            sX[e] = b < nb ? F[static_cast<size_t>(sT[b]) * NF + (e % NF)] : 0.0f;
        }
        __syncthreads();
        // forward: unit j of rows g kRG .. g kRG + kRG - 1
        {
            float a[kRG];
#pragma unroll
            for (int r = 0; r < kRG; ++r) a[r] = sB1[j];
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                const float w = sW1[i * NH + j];
#pragma unroll
                for (int r = 0; r < kRG; ++r) a[r] += sX[(g * kRG + r) * NF + i] * w;
            }
#pragma unroll
            for (int r = 0; r < kRG; ++r) sH1[(g * kRG + r) * NH + j] = fmaxf(a[r], 0.0f);
        }
        __syncthreads();
        {
            float a[kRG];
#pragma unroll
            for (int r = 0; r < kRG; ++r) a[r] = sB2[j];
#pragma unroll 8
            for (int i = 0; i < NH; ++i) {
                const float w = sW2[i * kW2S + j];
#pragma unroll
                for (int r = 0; r < kRG; ++r) a[r] += sH1[(g * kRG + r) * NH + i] * w;
            }
#pragma unroll
            for (int r = 0; r < kRG; ++r) sH2[(g * kRG + r) * NH + j] = fmaxf(a[r], 0.0f);
        }
        __syncthreads();
        // outputs: one thread per (row, output)
        if (tid < kTC * NO) {
            const int b = tid / NO, q = tid % NO;
            float a = sB3[q];
#pragma unroll 8
            for (int i = 0; i < NH; ++i) a += sH2[b * NH + i] * sW3[i * NO + q];
            sdO[b * 8 + q] = a;
        }
        __syncthreads();
        // loss and output gradient: one thread per transition (sdO holds the outputs on entry)
        if (tid < kTC) {
            const int b = tid;
            float o[NO];
            for (int q = 0; q < NO; ++q) o[q] = sdO[b * 8 + q];
            const int sl = sSlot[b];
            const int valid = sValid[b];
            float dO[NO] = {0, 0, 0, 0, 0, 0, 0};
            float lb = 0.0f;
            if (b < nb && sl >= 0 && sl < NS && Wsum > 0.0f && ((valid >> sl) & 1)) {
                float z[NS];
                float zmax = -INFINITY;
                for (int t = 0; t < NS; ++t) {
                    z[t] = o[t] + (sX[b * NF + t] + sX[b * NF + NS + t]);
                    if ((valid >> t) & 1) zmax = fmaxf(zmax, z[t]);
                }
                float e[NS], den = 0.0f;
                for (int t = 0; t < NS; ++t) {
                    e[t] = ((valid >> t) & 1) ? expf(z[t] - zmax) : 0.0f;
                    den += e[t];
                }
                float soft[NS];
                for (int t = 0; t < NS; ++t) soft[t] = e[t] / den;
                const float sg = 1.0f / (1.0f + expf(-o[NS]));
                const float alpha = kAlphaMax * sg;
                const float ps = sP6[b * NS + sl];
                const float qs = alpha * soft[sl] + (1.0f - alpha) * ps;
                const float wb = sW[b];
                float pen = 0.0f;
                for (int t = 0; t < NS; ++t)
                    if ((valid >> t) & 1) pen += o[t] * o[t];
                lb = (-wb * logf(qs) + shrink * wb * pen) / Wsum;
                const float coef = -(wb / Wsum) / qs;
                for (int t = 0; t < NS; ++t)
                    dO[t] = ((valid >> t) & 1) ? coef * alpha * soft[sl] * ((t == sl ? 1.0f : 0.0f) - soft[t]) +
                                                     2.0f * shrink * (wb / Wsum) * o[t]
                                               : 0.0f;
                dO[NS] = coef * (soft[sl] - ps) * kAlphaMax * sg * (1.0f - sg);
            }
            for (int q = 0; q < NO; ++q) sdO[b * 8 + q] = dO[q];
            if (b < nb) lossb[b0 + b] = lb;
        }
        __syncthreads();
        if (!kBackward) continue;
        // dH2 = (dO W3^T) [H2 > 0]: unit j of the group's rows
#pragma unroll
        for (int r = 0; r < kRG; ++r) {
            const int b = g * kRG + r;
            float a = 0.0f;
#pragma unroll
            for (int q = 0; q < NO; ++q) a += sdO[b * 8 + q] * sW3[j * NO + q];
            sD2[b * NH + j] = sH2[b * NH + j] > 0.0f ? a : 0.0f;
        }
        __syncthreads();
        // output layer gradients: one thread per weight
        for (int t = tid; t < NH * NO + NO; t += 256) {
            float a = 0.0f;
            if (t < NH * NO) {
                const int i = t / NO, q = t % NO;
                for (int b = 0; b < nb; ++b) a += sH2[b * NH + i] * sdO[b * 8 + q];
                G[OFF_W3 + t] = (first ? 0.0f : G[OFF_W3 + t]) + a;
            } else {
                const int q = t - NH * NO;
                for (int b = 0; b < nb; ++b) a += sdO[b * 8 + q];
                G[OFF_B3 + q] = (first ? 0.0f : G[OFF_B3 + q]) + a;
            }
        }
        // second layer: dW2[i][j] for i = 16 g .. 16 g + 15
        {
            float a[16];
#pragma unroll
            for (int ii = 0; ii < 16; ++ii) a[ii] = 0.0f;
            float bsum = 0.0f;
            for (int b = 0; b < nb; ++b) {
                const float d = sD2[b * NH + j];
                bsum += d;
#pragma unroll
                for (int ii = 0; ii < 16; ++ii) a[ii] += sH1[b * NH + g * 16 + ii] * d;
            }
#pragma unroll
            for (int ii = 0; ii < 16; ++ii) {
                const int t = (g * 16 + ii) * NH + j;
                G[OFF_W2 + t] = (first ? 0.0f : G[OFF_W2 + t]) + a[ii];
            }
            if (g == 0) G[OFF_B2 + j] = (first ? 0.0f : G[OFF_B2 + j]) + bsum;
        }
        __syncthreads();
        // dH1 = (dH2 W2^T) [H1 > 0] into sH2 (no longer needed): unit j of the group's rows
        {
            float a[kRG];
#pragma unroll
            for (int r = 0; r < kRG; ++r) a[r] = 0.0f;
#pragma unroll 8
            for (int q = 0; q < NH; ++q) {
                const float w = sW2[j * kW2S + q];
#pragma unroll
                for (int r = 0; r < kRG; ++r) a[r] += sD2[(g * kRG + r) * NH + q] * w;
            }
#pragma unroll
            for (int r = 0; r < kRG; ++r) {
                const int e = (g * kRG + r) * NH + j;
                sH2[e] = sH1[e] > 0.0f ? a[r] : 0.0f;
            }
        }
        __syncthreads();
        // first layer: dW1[i][j] for i = 4 g .. 4 g + 3
        {
            float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            float bsum = 0.0f;
            for (int b = 0; b < nb; ++b) {
                const float d = sH2[b * NH + j];
                bsum += d;
#pragma unroll
                for (int ii = 0; ii < 4; ++ii) a[ii] += sX[b * NF + g * 4 + ii] * d;
            }
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) {
                const int t = (g * 4 + ii) * NH + j;
                G[OFF_W1 + t] = (first ? 0.0f : G[OFF_W1 + t]) + a[ii];
            }
            if (g == 0) G[OFF_B1 + j] = (first ? 0.0f : G[OFF_B1 + j]) + bsum;
        }
        first = false;
    }
}

// G = sum of the partial gradients in a fixed order; with kAdam, one Adam step on P instead.
// A workgroup serves kGradParams parameters with kGradGroups threads each: thread group g
// adds the partials g, g + kGradGroups, ... in turn, and the group sums are added in the
// order g = 0, 1, ... (deterministic).
constexpr int kGradParams = 32;
constexpr int kGradGroups = 8;

template <bool kAdam>
__global__ __launch_bounds__(kGradParams * kGradGroups) void grad_sum_kernel(
    const float *__restrict__ partial, int blocks, float *out, float *P, float *m, float *v, float lr,
    float b1, float b2, float eps, float c1, float c2)
{
    __shared__ float sh[kGradGroups][kGradParams];
    const int jj = static_cast<int>(threadIdx.x) % kGradParams;
    const int g = static_cast<int>(threadIdx.x) / kGradParams;
    const int t = static_cast<int>(blockIdx.x) * kGradParams + jj;
    float acc = 0.0f;
    if (t < NPARAM)
        for (int q = g; q < blocks; q += kGradGroups) acc += partial[static_cast<size_t>(q) * NPARAM + t];
    sh[g][jj] = acc;
    __syncthreads();
    if (g != 0 || t >= NPARAM) return;
    float gs = sh[0][jj];
    for (int k = 1; k < kGradGroups; ++k) gs += sh[k][jj];
    if (!kAdam) {
        out[t] = gs;
        return;
    }
    m[t] = b1 * m[t] + (1.0f - b1) * gs;
    v[t] = b2 * v[t] + (1.0f - b2) * gs * gs;
    P[t] -= lr * (m[t] / c1) / (sqrtf(v[t] / c2) + eps);
}

// Sum of n floats in FP64 in a fixed order (thread t adds t, t + 1024, ...; the 1024 partial
// sums meet in a fixed tree): the loss of a minibatch or of the held-out set, kept on the
// device so that the training loop does not wait for the host.
constexpr int kLossThreads = 1024;

__global__ __launch_bounds__(kLossThreads) void loss_sum_kernel(const float *__restrict__ x, int n, double *out)
{
    __shared__ double sh[kLossThreads];
    const int t = static_cast<int>(threadIdx.x);
    double acc = 0.0;
    for (int i = t; i < n; i += kLossThreads) acc += static_cast<double>(x[i]);
    sh[t] = acc;
    __syncthreads();
    for (int o = kLossThreads / 2; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    if (t == 0) *out = sh[0];
}

// The parameters of the lowest held-out loss so far: when *val < *best_val, P is copied to
// best and the step recorded. One workgroup: every thread reads best_val before the barrier,
// thread 0 writes it after.
__global__ __launch_bounds__(256) void keep_best_kernel(const double *__restrict__ val, int step,
                                                        double *best_val, int *best_step,
                                                        const float *__restrict__ P, float *best)
{
    const bool better = *val < *best_val;
    __syncthreads();
    if (!better) return;
    for (int i = static_cast<int>(threadIdx.x); i < NPARAM; i += 256) best[i] = P[i];
    if (threadIdx.x == 0) {
        *best_val = *val;
        *best_step = step;
    }
}


int train_blocks(int B) { return std::min(kMaxTrainBlocks, (B + kTC - 1) / kTC); }

// Loss terms (and, with backward, the partial gradients) of a batch.
hipError_t train_pass(bool backward, const float *P, const float *F, const mlmc_plan *p, int level,
                      const BatchSrc &src, int B, float shrink, float *partial, float *lossb, hipStream_t s)
{
    const int blocks = train_blocks(B);
    if (backward)
        hipLaunchKernelGGL(train_kernel<true>, dim3(blocks), dim3(256), 0, s, P, F, p->p_slot, p->level_rec[level],
                           src, B, shrink, partial, lossb);
    else
        hipLaunchKernelGGL(train_kernel<false>, dim3(blocks), dim3(256), 0, s, P, F, p->p_slot, p->level_rec[level],
                           src, B, shrink, partial, lossb);
    return hipGetLastError();
}

// Scratch of a training call, kept by the plan between calls: the k-th buffer a call asks
// for is the plan's k-th pooled buffer, reallocated only when it is too small (the calls ask
// in the same order every time). The call's stream is synchronised when the session ends, so
// that no kernel of this call still uses the buffers when the next call (on any stream)
// takes them.
struct Session {
    mlmc_plan *plan;
    std::vector<std::pair<void *, size_t>> &pool;
    hipStream_t stream;
    size_t next = 0;
    Session(mlmc_plan *p, std::vector<std::pair<void *, size_t>> &pl, hipStream_t s) : plan(p), pool(pl), stream(s) {}
    ~Session() { (void)hipStreamSynchronize(stream); }
    template <typename T>
    int alloc(T **p, size_t count)
    {
        *p = nullptr;
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (next == pool.size()) pool.emplace_back(nullptr, 0);
        auto &b = pool[next++];
        if (b.second < bytes) {
            (void)hipStreamSynchronize(stream);
            if (b.first) (void)hipFree(b.first);
            plan->bytes -= static_cast<int64_t>(b.second);
            b = {nullptr, 0};
            void *q = nullptr;
            const hipError_t e = hipMalloc(&q, bytes);
            if (e != hipSuccess)
                return fail(e == hipErrorOutOfMemory ? MLMC_ERR_OUT_OF_MEMORY : MLMC_ERR_HIP,
                            std::string("hipMalloc: ") + hipGetErrorString(e));
            b = {q, bytes};
            plan->bytes += static_cast<int64_t>(bytes);
        }
        *p = static_cast<T *>(b.first);
        return MLMC_OK;
    }
};

FeatureArgs feature_args(const mlmc_plan *p, int level, const double *xhat, const double *logx, const double *xmax)
{
    FeatureArgs fa;
    fa.rec = p->level_rec[level];
    fa.slots = p->slots;
    fa.p_slot = p->p_slot;
    fa.logp = p->prop_logp;
    fa.xhat = xhat;
    fa.logx = logx;
    fa.xmax = xmax;
    fa.n = p->n;
    fa.dt = static_cast<float>(std::ldexp(p->beta, -level));
    fa.lvl = static_cast<float>(level - p->l0) / 8.0f;
    return fa;
}

int check_level(const mlmc_plan *p, int level)
{
    if (level < p->l0 || level > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "level must be in [l0, 28]");
    return MLMC_OK;
}

template <typename T>
int plan_alloc(mlmc_plan *p, T **ptr, size_t count)
{
    if (*ptr) return MLMC_OK;
    const hipError_t e = hipMalloc(reinterpret_cast<void **>(ptr), std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(e == hipErrorOutOfMemory ? MLMC_ERR_OUT_OF_MEMORY : MLMC_ERR_HIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    p->bytes += static_cast<int64_t>(std::max<size_t>(count, 1) * sizeof(T));
    return MLMC_OK;
}

// Device buffers every proposal call reads: the plain law per slot and the parameters.
int ensure_proposal_buffers(mlmc_plan *p, hipStream_t s)
{
    const bool fresh = p->p_slot == nullptr;
    int rc;
    if ((rc = plan_alloc(p, &p->p_slot, p->p_slot_host.size())) || (rc = plan_alloc(p, &p->prop_P, NPARAM)) ||
        (rc = plan_alloc(p, &p->prop_frag, NFRAG)) || (rc = plan_alloc(p, &p->prop_xhat, static_cast<size_t>(p->n))) ||
        (rc = plan_alloc(p, &p->prop_xmax, 1 + kAbsmaxBlocks)) ||
        (rc = plan_alloc(p, &p->prop_logp, p->p_slot_host.size())) ||
        (rc = plan_alloc(p, &p->prop_logx, static_cast<size_t>(p->n))))
        return rc;
    if (fresh) {
        MLMC_HIP_TRY(hipMemcpyAsync(p->p_slot, p->p_slot_host.data(), p->p_slot_host.size() * sizeof(float),
                                    hipMemcpyHostToDevice, s));
        const uint64_t ns = p->p_slot_host.size();
        if (ns > 0) hipLaunchKernelGGL(logp_kernel, dim3(nblk(ns, 256)), dim3(256), 0, s, p->p_slot, static_cast<int64_t>(ns),
                                       p->prop_logp);
        MLMC_HIP_TRY(hipGetLastError());
    }
    return MLMC_OK;
}

// Build (and optionally export) the proposal tables of one level.
int build_tables(mlmc_plan *p, int level, SlotRecIS *out, uint32_t *x_thr, int32_t *x_alias, float *x_ratio,
                 float *x_q, hipStream_t s)
{
    TableArgs ta;
    ta.fa = feature_args(p, level, p->prop_xhat, p->prop_logx, p->prop_xmax);
    ta.frag = p->prop_frag;
    ta.P = p->prop_P;
    ta.out = out;
    ta.x_thr = x_thr;
    ta.x_alias = x_alias;
    ta.x_ratio = x_ratio;
    ta.x_q = x_q;
    ta.identity = p->prop_identity;
    const uint64_t iters = (static_cast<uint64_t>(p->n) + kTabRows - 1) / kTabRows;
    if (iters == 0) return MLMC_OK;
    const uint32_t grid = static_cast<uint32_t>(std::min<uint64_t>(iters, kTabGridMax));
    hipLaunchKernelGGL(tables_kernel, dim3(grid), dim3(kTabRows), 0, s, ta);
    MLMC_HIP_TRY(hipGetLastError());
    return MLMC_OK;
}

// Copy the parameters and the pilot estimate in, and build the tables of the levels.
// params: host, or the device when params_on_device (p->prop_P itself is not copied).
// xhat_prepared: xhat is p->prop_xhat and p->prop_xmax, p->prop_logx already hold its
// maximum and logarithms.
int set_proposal(mlmc_plan *p, const float *params, const double *xhat, int num_levels, hipStream_t s,
                 bool params_on_device = false, bool xhat_prepared = false)
{
    int rc;
    if ((rc = ensure_proposal_buffers(p, s))) return rc;
    p->prop_identity = params == nullptr;
    if (params) {
        if (params != p->prop_P)
            MLMC_HIP_TRY(hipMemcpyAsync(p->prop_P, params, NPARAM * sizeof(float),
                                        params_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(fragments_kernel, dim3(nblk(NFRAG, 256)), dim3(256), 0, s, p->prop_P, p->prop_frag);
        MLMC_HIP_TRY(hipGetLastError());
    }
    if (!(xhat_prepared && xhat == p->prop_xhat)) {
        if (p->n > 0) {
            if (xhat) {
                if (xhat != p->prop_xhat)
                    MLMC_HIP_TRY(hipMemcpyAsync(p->prop_xhat, xhat, p->n * sizeof(double), hipMemcpyDeviceToDevice, s));
            } else {
                MLMC_HIP_TRY(hipMemsetAsync(p->prop_xhat, 0, p->n * sizeof(double), s));
            }
        }
        prepare_xhat(p->prop_xhat, p->n, p->prop_xmax, p->prop_logx, s);
        MLMC_HIP_TRY(hipGetLastError());
    }
    if (p->is_slots.size() < static_cast<size_t>(kMaxLevel + 1)) p->is_slots.resize(kMaxLevel + 1, nullptr);
    for (int q = 0; q < num_levels; ++q) {
        const int level = p->l0 + q;
        if ((rc = upload_level(p, level, s))) return rc;
        if ((rc = plan_alloc(p, &p->is_slots[level], static_cast<size_t>(p->n_slots)))) return rc;
        if ((rc = build_tables(p, level, p->is_slots[level], nullptr, nullptr, nullptr, nullptr, s))) return rc;
    }
    // levels past the new range walk with the plain tables
    for (int level = p->l0 + num_levels; level <= kMaxLevel; ++level)
        if (p->is_slots[level]) {
            (void)hipFree(p->is_slots[level]);
            p->bytes -= static_cast<int64_t>(std::max<int64_t>(p->n_slots, 1) * sizeof(SlotRecIS));
            p->is_slots[level] = nullptr;
        }
    p->prop_levels = num_levels;
    p->proposal_on = true;
    return MLMC_OK;
}

}  // namespace
}  // namespace mlmc

using namespace mlmc;

extern "C" {

int mlmc_expv_proposal_set(mlmc_plan_t *p, const float *params, const double *xhat, int32_t num_levels,
                           void *stream)
{
    if (!p) return fail(MLMC_ERR_INVALID_ARG, "null plan");
    if (num_levels < 1 || p->l0 + num_levels - 1 > kMaxLevel) return fail(MLMC_ERR_INVALID_ARG, "num_levels out of range");
    return set_proposal(p, params, xhat, num_levels, static_cast<hipStream_t>(stream));
}

int mlmc_expv_proposal_enable(mlmc_plan_t *p, int32_t on)
{
    if (!p) return fail(MLMC_ERR_INVALID_ARG, "null plan");
    if (on && p->prop_levels == 0) return fail(MLMC_ERR_INVALID_ARG, "no proposal has been set");
    p->proposal_on = on != 0;
    return MLMC_OK;
}

int mlmc_expv_proposal_tables(mlmc_plan_t *p, int32_t level, uint32_t *thr, int32_t *alias_slot, float *ratio,
                              float *q, void *stream)
{
    if (!p || !thr || !alias_slot || !ratio || !q) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    if (p->prop_levels == 0) return fail(MLMC_ERR_INVALID_ARG, "no proposal has been set");
    int rc = check_level(p, level);
    if (rc) return rc;
    if (level >= p->l0 + p->prop_levels) return fail(MLMC_ERR_INVALID_ARG, "level has no proposal table");
    return build_tables(p, level, p->is_slots[level], thr, alias_slot, ratio, q, static_cast<hipStream_t>(stream));
}

int mlmc_expv_proposal_loss_grad(mlmc_plan_t *p, const float *params, const double *xhat, int32_t level,
                                 int32_t count, const int64_t *rows, const int32_t *slots, const float *weights,
                                 double shrink, float *grad, double *loss, void *stream)
{
    if (!(shrink >= 0.0) || !std::isfinite(shrink)) return fail(MLMC_ERR_INVALID_ARG, "shrink must be finite and >= 0");
    if (!p || !params || !rows || !slots || !weights || !grad || !loss) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    if (count < 1 || count > (1 << 20)) return fail(MLMC_ERR_INVALID_ARG, "count must be in [1, 2^20]");
    int rc = check_level(p, level);
    if (rc) return rc;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = upload_level(p, level, s)) || (rc = ensure_proposal_buffers(p, s))) return rc;
    for (int32_t b = 0; b < count; ++b) {
        if (rows[b] < 0 || rows[b] >= p->n) return fail(MLMC_ERR_INVALID_ARG, "transition row out of range");
        if (slots[b] < -1 || slots[b] >= NS) return fail(MLMC_ERR_INVALID_ARG, "transition slot out of range [-1, 6)");
        if (!(weights[b] >= 0.0f) || !std::isfinite(weights[b])) return fail(MLMC_ERR_INVALID_ARG, "weights must be finite and >= 0");
    }
    std::vector<uint32_t> rows32(count);
    for (int32_t b = 0; b < count; ++b) rows32[b] = static_cast<uint32_t>(rows[b]);
    Session ss(p, p->grad_pool, s);
    float *dP = nullptr, *F = nullptr, *d_w = nullptr, *part = nullptr, *G = nullptr, *lossb = nullptr;
    uint32_t *d_rows = nullptr;
    int32_t *d_slots = nullptr;
    double *xmax = nullptr, *logx = nullptr;
    const int blocks = train_blocks(count);
    if ((rc = ss.alloc(&dP, NPARAM)) || (rc = ss.alloc(&F, static_cast<size_t>(count) * NF)) ||
        (rc = ss.alloc(&xmax, 1 + kAbsmaxBlocks)) || (rc = ss.alloc(&d_rows, count)) || (rc = ss.alloc(&d_slots, count)) ||
        (rc = ss.alloc(&d_w, count)) || (rc = ss.alloc(&part, static_cast<size_t>(blocks) * NPARAM)) ||
        (rc = ss.alloc(&G, NPARAM)) || (rc = ss.alloc(&lossb, count)) || (rc = ss.alloc(&logx, p->n)))
        return rc;
    MLMC_HIP_TRY(hipMemcpyAsync(dP, params, NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
    MLMC_HIP_TRY(hipMemcpyAsync(d_rows, rows32.data(), count * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    MLMC_HIP_TRY(hipMemcpyAsync(d_slots, slots, count * sizeof(int32_t), hipMemcpyHostToDevice, s));
    MLMC_HIP_TRY(hipMemcpyAsync(d_w, weights, count * sizeof(float), hipMemcpyHostToDevice, s));
    prepare_xhat(xhat, p->n, xmax, logx, s);
    const FeatureArgs fa = feature_args(p, level, xhat, logx, xmax);
    hipLaunchKernelGGL(features_kernel, dim3(nblk(count, 256)), dim3(256), 0, s, fa, d_rows,
                       static_cast<int64_t>(count), F);
    const BatchSrc src{d_rows, d_slots, d_w, static_cast<uint64_t>(count), 0, 1};
    MLMC_HIP_TRY(train_pass(true, dP, F, p, level, src, count, static_cast<float>(shrink), part, lossb, s));
    hipLaunchKernelGGL(grad_sum_kernel<false>, dim3(nblk(NPARAM, kGradParams)), dim3(kGradParams * kGradGroups), 0,
                       s, part, blocks, G, nullptr, nullptr, nullptr, 0.0f, 0.0f, 0.0f, 0.0f, 1.0f, 1.0f);
    MLMC_HIP_TRY(hipGetLastError());
    std::vector<float> lb(count);
    MLMC_HIP_TRY(hipMemcpyAsync(grad, G, NPARAM * sizeof(float), hipMemcpyDeviceToHost, s));
    MLMC_HIP_TRY(hipMemcpyAsync(lb.data(), lossb, count * sizeof(float), hipMemcpyDeviceToHost, s));
    MLMC_HIP_TRY(hipStreamSynchronize(s));
    double L = 0.0;
    for (float v : lb) L += v;
    *loss = L;
    return MLMC_OK;
}

}  // extern "C"

namespace mlmc {
namespace {

// The state of a training before its first step: the kept parameters are the initial ones,
// Adam's moments and the records are zero.
__global__ void train_init_kernel(const float *P, float *best, float *m, float *v, double *recs, int n_recs)
{
    const int i = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < NPARAM) {
        best[i] = P[i];
        m[i] = 0.0f;
        v[i] = 0.0f;
    }
    if (i < n_recs) recs[i] = 0.0;
}

// What the training steps after the pilot leave: the kept parameters and the records.
struct CoreOut {
    std::vector<float> P;
    uint64_t kept = 0, n_val = 0;
    int best_step = 0;
    double first_val = 0.0, best_val = 0.0;
    std::vector<double> losses;
};

int check_train_opts(const mlmc_plan *p, const mlmc_train_opts_t *o, bool own_pilot)
{
    if (!o->init_params) return fail(MLMC_ERR_INVALID_ARG, "init_params is null");
    if (o->capture_walks < 1 || o->steps < 0 || o->batch < 1 || o->batch > (1 << 20) || o->num_levels < 1 ||
        p->l0 + o->num_levels - 1 > kMaxLevel || o->sample_stride < 1 || !(o->lr > 0.0) || !(o->shrink >= 0.0) ||
        !std::isfinite(o->shrink))
        return fail(MLMC_ERR_INVALID_ARG, "training options out of range");
    if (own_pilot && (o->pilot_walks < 1 || o->pilot_walks > 0xFFFFFFFFll || o->judge_walks < 0 ||
                      o->judge_walks == 1 || o->judge_walks > 65536))
        return fail(MLMC_ERR_INVALID_ARG, "training options out of range");
    if (p->n_rows != p->n) return fail(MLMC_ERR_UNSUPPORTED, "training needs a plan over all rows");
    return MLMC_OK;
}

// The training steps after the pilot estimate (in p->prop_xhat, max |xhat| in xmax):
// capture of plain walks' jumps, minibatch Adam with early stopping, and the tables of the
// kept parameters. Waits for the stream once, to read the records.
int train_core(mlmc_plan *p, Session &ss, const void *u, const mlmc_train_opts_t *o, double *xmax, CoreOut &co,
               hipStream_t s)
{
    int rc;
    const int level = p->l0;
    // 2. transitions of plain walks from every sample_stride-th row
    const uint32_t n_sample = static_cast<uint32_t>((p->n + o->sample_stride - 1) / o->sample_stride);
    const uint64_t walks_cap = static_cast<uint64_t>(n_sample) * static_cast<uint64_t>(o->capture_walks);
    const uint64_t T = walks_cap * kCaptureJumps;
    if (T > (uint64_t(1) << 31)) return fail(MLMC_ERR_INVALID_ARG, "capture too large (rows x walks x 8 > 2^31)");
    const uint64_t nb_keep = (T + kKeepBlock - 1) / kKeepBlock;
    if (nb_keep > 0xFFFFFFFFull) return fail(MLMC_ERR_INVALID_ARG, "capture too large");
    const uint64_t val_cap = std::min<uint64_t>(T / 8, static_cast<uint64_t>(kMaxHeldOut));
    // the steps after which the minibatch loss is recorded (and, after the first, the
    // held-out loss evaluated): the first, every kEvalEvery-th and the last
    auto eval_after = [&](int step) { return step == 0 || step == o->steps - 1 || (step + 1) % kEvalEvery == 0; };
    int n_eval = 0;
    for (int step = 0; step < o->steps; ++step) n_eval += eval_after(step) ? 1 : 0;
    // buffers (in the same order on every call) and the parameters' initial state, all
    // before the one wait for the count of kept transitions
    uint32_t *t_row = nullptr, *keep_off = nullptr, *tr_row = nullptr, *v_row = nullptr;
    int32_t *t_slot = nullptr, *tr_slot = nullptr, *v_slot = nullptr;
    float *t_w = nullptr, *tr_w = nullptr, *v_w = nullptr;
    float *m = nullptr, *v = nullptr, *best = nullptr, *part = nullptr, *lossb = nullptr, *lossv = nullptr;
    // device records: the best held-out loss, its step (an int in the next slot), the
    // minibatch losses [n_eval] and the held-out losses [1 + n_eval] (the initial first)
    double *recs = nullptr;
    const size_t n_recs = 2 + 2 * static_cast<size_t>(n_eval) + 1;
    if ((rc = ss.alloc(&t_row, T)) || (rc = ss.alloc(&t_slot, T)) || (rc = ss.alloc(&t_w, T)) ||
        (rc = ss.alloc(&keep_off, nb_keep + 1)) || (rc = ss.alloc(&tr_row, T)) || (rc = ss.alloc(&tr_slot, T)) ||
        (rc = ss.alloc(&tr_w, T)) || (rc = ss.alloc(&v_row, val_cap)) || (rc = ss.alloc(&v_slot, val_cap)) ||
        (rc = ss.alloc(&v_w, val_cap)) || (rc = ss.alloc(&m, NPARAM)) || (rc = ss.alloc(&v, NPARAM)) ||
        (rc = ss.alloc(&best, NPARAM)) ||
        (rc = ss.alloc(&part, static_cast<size_t>(train_blocks(o->batch)) * NPARAM)) ||
        (rc = ss.alloc(&lossb, static_cast<size_t>(o->batch))) || (rc = ss.alloc(&lossv, std::max<uint64_t>(val_cap, 1))) ||
        (rc = ss.alloc(&recs, n_recs)))
        return rc;
    double *d_best_val = recs;
    int *d_best_step = reinterpret_cast<int *>(recs + 1);
    double *d_loss = recs + 2, *d_val = recs + 2 + n_eval;
    co.P.assign(o->init_params, o->init_params + NPARAM);
    MLMC_HIP_TRY(hipMemcpyAsync(p->prop_P, co.P.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(train_init_kernel, dim3(nblk(std::max<size_t>(NPARAM, n_recs), 256)), dim3(256), 0, s,
                       p->prop_P, best, m, v, recs, static_cast<int>(n_recs));
    MLMC_HIP_TRY(hipGetLastError());
    LevelArgs L = level_args(p, level, o->seed, 4094);
    L.is_slots = nullptr;
    if (walks_cap > 0) {
        hipLaunchKernelGGL(capture_kernel, dim3(nblk(walks_cap, 256)), dim3(256), 0, s, L,
                           static_cast<const float *>(u), static_cast<uint32_t>(o->sample_stride), n_sample,
                           static_cast<uint32_t>(o->capture_walks), t_row, t_slot, t_w);
        MLMC_HIP_TRY(hipGetLastError());
    }
    // 3. the transitions that carry a sample, in their recorded order: every 8th is held out
    //    (at most kMaxHeldOut of them), the rest train (compacted on the device). Adam on
    //    minibatches of the training transitions, taken by a fixed stride (coprime with the
    //    count) so that each batch spreads over all sampled rows; the parameters with the
    //    lowest held-out loss (the initial ones included) are kept
    uint32_t kept32 = 0;
    if (T > 0) {
        hipLaunchKernelGGL(keep_count_kernel, dim3(static_cast<uint32_t>(nb_keep)), dim3(256), 0, s, t_slot, t_w, T,
                           keep_off);
        hipLaunchKernelGGL(keep_scan_kernel, dim3(1), dim3(256), 0, s, keep_off, static_cast<uint32_t>(nb_keep));
        hipLaunchKernelGGL(keep_scatter_kernel, dim3(static_cast<uint32_t>(nb_keep)), dim3(256), 0, s, t_row, t_slot,
                           t_w, T, keep_off, tr_row, tr_slot, tr_w, v_row, v_slot, v_w);
        MLMC_HIP_TRY(hipGetLastError());
        void *hk = nullptr;
        if ((rc = plan_pinned(p, sizeof kept32, &hk))) return rc;
        MLMC_HIP_TRY(hipMemcpyAsync(hk, keep_off + nb_keep, sizeof kept32, hipMemcpyDeviceToHost, s));
        MLMC_HIP_TRY(hipStreamSynchronize(s));
        std::memcpy(&kept32, hk, sizeof kept32);
    }
    const uint64_t kept = kept32;
    const uint64_t n_val = std::min<uint64_t>(kept / 8, static_cast<uint64_t>(kMaxHeldOut));
    const uint64_t n_train = kept - n_val;
    const int B = static_cast<int>(std::min<uint64_t>(static_cast<uint64_t>(o->batch), std::max<uint64_t>(n_train, 1)));
    const bool training = n_train > 0 && o->steps > 0;
    // the network inputs of the kept transitions' rows, one record per transition
    float *F_tr = nullptr, *F_v = nullptr;
    if ((rc = ss.alloc(&F_tr, std::max<uint64_t>(n_train, 1) * NF)) || (rc = ss.alloc(&F_v, std::max<uint64_t>(n_val, 1) * NF)))
        return rc;
    const FeatureArgs fa = feature_args(p, level, p->prop_xhat, p->prop_logx, xmax);
    if (n_train > 0)
        hipLaunchKernelGGL(features_kernel, dim3(nblk(n_train, 256)), dim3(256), 0, s, fa, tr_row,
                           static_cast<int64_t>(n_train), F_tr);
    if (n_val > 0)
        hipLaunchKernelGGL(features_kernel, dim3(nblk(n_val, 256)), dim3(256), 0, s, fa, v_row,
                           static_cast<int64_t>(n_val), F_v);
    MLMC_HIP_TRY(hipGetLastError());
    const BatchSrc vsrc{v_row, v_slot, v_w, std::max<uint64_t>(n_val, 1), 0, 1};
    const float shrink = static_cast<float>(o->shrink);
    // held-out loss of the current parameters into *out (on the device)
    auto val_loss = [&](double *out) -> int {
        MLMC_HIP_TRY(train_pass(false, p->prop_P, F_v, p, level, vsrc, static_cast<int>(n_val), shrink, part, lossv, s));
        hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(kLossThreads), 0, s, lossv, static_cast<int>(n_val), out);
        MLMC_HIP_TRY(hipGetLastError());
        return MLMC_OK;
    };
    if (n_val > 0) {
        if ((rc = val_loss(d_val))) return rc;
        MLMC_HIP_TRY(hipMemcpyAsync(d_best_val, d_val, sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    int n_val_evals = 0, e = 0;
    if (training) {
        auto gcd = [](uint64_t a, uint64_t b) {
            while (b) {
                const uint64_t t = a % b;
                a = b;
                b = t;
            }
            return a;
        };
        uint64_t mult = n_train == 1 ? 1 : 2654435761ull % n_train;
        while (n_train > 1 && (mult == 0 || gcd(mult, n_train) != 1)) mult = (mult + 1) % n_train;
        const float b1 = 0.9f, b2 = 0.999f;
        const int blocks = train_blocks(B);
        for (int step = 0; step < o->steps; ++step) {
            const BatchSrc src{tr_row, tr_slot, tr_w, n_train, static_cast<uint64_t>(step) * B, mult};
            MLMC_HIP_TRY(train_pass(true, p->prop_P, F_tr, p, level, src, B, shrink, part, lossb, s));
            const float c1 = 1.0f - std::pow(b1, static_cast<float>(step + 1));
            const float c2 = 1.0f - std::pow(b2, static_cast<float>(step + 1));
            hipLaunchKernelGGL(grad_sum_kernel<true>, dim3(nblk(NPARAM, kGradParams)), dim3(kGradParams * kGradGroups),
                               0, s, part, blocks, nullptr, p->prop_P, m, v, static_cast<float>(o->lr), b1, b2,
                               1e-8f, c1, c2);
            MLMC_HIP_TRY(hipGetLastError());
            if (eval_after(step)) {
                hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(kLossThreads), 0, s, lossb, B, d_loss + e);
                MLMC_HIP_TRY(hipGetLastError());
                ++e;
                if (n_val > 0 && step > 0) {
                    ++n_val_evals;
                    if ((rc = val_loss(d_val + n_val_evals))) return rc;
                    hipLaunchKernelGGL(keep_best_kernel, dim3(1), dim3(256), 0, s, d_val + n_val_evals, step + 1,
                                       d_best_val, d_best_step, p->prop_P, best);
                    MLMC_HIP_TRY(hipGetLastError());
                }
            }
        }
        if (n_val > 0) MLMC_HIP_TRY(hipMemcpyAsync(p->prop_P, best, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    // 4. the levels' tables from the kept parameters (on the device) and the pilot estimate
    if ((rc = set_proposal(p, p->prop_P, p->prop_xhat, o->num_levels, s, true, true))) return rc;
    // the parameters and the records, read once (through the plan's pinned memory)
    std::vector<double> h(n_recs);
    void *hp = nullptr;
    const size_t p_bytes = (NPARAM * sizeof(float) + 7) / 8 * 8;
    if ((rc = plan_pinned(p, p_bytes + n_recs * sizeof(double), &hp))) return rc;
    MLMC_HIP_TRY(hipMemcpyAsync(hp, p->prop_P, NPARAM * sizeof(float), hipMemcpyDeviceToHost, s));
    MLMC_HIP_TRY(hipMemcpyAsync(static_cast<char *>(hp) + p_bytes, recs, n_recs * sizeof(double),
                                hipMemcpyDeviceToHost, s));
    MLMC_HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(co.P.data(), hp, NPARAM * sizeof(float));
    std::memcpy(h.data(), static_cast<char *>(hp) + p_bytes, n_recs * sizeof(double));
    co.kept = kept;
    co.n_val = n_val;
    co.losses.assign(h.begin() + 2, h.begin() + 2 + e);
    if (n_val > 0) {
        co.best_val = h[0];
        std::memcpy(&co.best_step, &h[1], sizeof(int));
        co.first_val = h[2 + n_eval];
    }
    return MLMC_OK;
}

void fill_train_stats(mlmc_train_stats_t *st, const mlmc_train_opts_t *o, const CoreOut &co)
{
    std::memset(st, 0, sizeof *st);
    st->transitions = static_cast<int64_t>(co.kept);
    st->held_out = static_cast<int64_t>(co.n_val);
    st->steps = o->steps;
    st->best_step = co.best_step;
    st->first_val_loss = co.first_val;
    st->best_val_loss = co.best_val;
    const int nl = static_cast<int>(std::min<size_t>(co.losses.size(), 64));
    st->n_losses = nl;
    for (int i = 0; i < nl; ++i) st->losses[i] = co.losses[co.losses.size() - nl + i];
    st->first_loss = co.losses.empty() ? 0.0 : co.losses.front();
    st->last_loss = co.losses.empty() ? 0.0 : co.losses.back();
    st->accepted = 1;
}

}  // namespace

int check_learned_opts(const mlmc_plan *p, const mlmc_train_opts_t *o) { return check_train_opts(p, o, false); }

int train_from_levels(mlmc_plan *p, const void *u, const mlmc_train_opts_t *o, const CombineArgs &xhat,
                      float *params_out, mlmc_train_stats_t *st, hipStream_t s)
{
    int rc;
    if ((rc = check_train_opts(p, o, false))) return rc;
    if ((rc = upload_level(p, p->l0, s)) || (rc = ensure_proposal_buffers(p, s))) return rc;
    Session ss(p, p->train_pool, s);
    // the same first buffers as a training call with its own pilot, so that both calls
    // reuse the pooled buffers in the same order
    double *s1 = nullptr, *s2 = nullptr;
    if ((rc = ss.alloc(&s1, p->n)) || (rc = ss.alloc(&s2, p->n))) return rc;
    MLMC_HIP_TRY(launch_combine(xhat, p->n, p->prop_xhat, s));
    prepare_xhat(p->prop_xhat, p->n, p->prop_xmax, p->prop_logx, s);
    CoreOut co;
    if ((rc = train_core(p, ss, u, o, p->prop_xmax, co, s))) return rc;
    if (st) fill_train_stats(st, o, co);
    if (params_out) std::memcpy(params_out, co.P.data(), NPARAM * sizeof(float));
    return MLMC_OK;
}

}  // namespace mlmc

extern "C" {

int mlmc_expv_proposal_train(mlmc_plan_t *p, const void *u, int32_t u_dtype, const mlmc_train_opts_t *o,
                             float *params_out, mlmc_train_stats_t *st, void *stream)
{
    if (!p || !u || !o) return fail(MLMC_ERR_INVALID_ARG, "null argument");
    if (u_dtype != MLMC_DTYPE_F32) return fail(MLMC_ERR_UNSUPPORTED, "training reads an FP32 right-hand side");
    int rc;
    if ((rc = check_train_opts(p, o, true))) return rc;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int level = p->l0;
    if ((rc = upload_level(p, level, s)) || (rc = ensure_proposal_buffers(p, s))) return rc;
    hipEvent_t e0, e1;
    MLMC_HIP_TRY(hipEventCreate(&e0));
    MLMC_HIP_TRY(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev()
        {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    MLMC_HIP_TRY(hipEventRecord(e0, s));
    Session ss(p, p->train_pool, s);
    // 1. pilot estimate xhat: the level-l0 mean of plain walks (an independent stream family)
    const bool was_on = p->proposal_on;
    p->proposal_on = false;
    double *s1 = nullptr, *s2 = nullptr;
    if ((rc = ss.alloc(&s1, p->n)) || (rc = ss.alloc(&s2, p->n))) return rc;
    rc = mlmc_expv_level_sums(p, u, 1, MLMC_DTYPE_F32, o->seed ^ 0x9E3779B97F4A7C15ull, 4095, level, 0,
                              static_cast<uint32_t>(o->pilot_walks), s1, s2, nullptr, nullptr, stream);
    p->proposal_on = was_on;
    if (rc) return rc;
    CombineArgs ca{};
    ca.levels = 1;
    ca.s1[0] = s1;
    ca.inv_M[0] = 1.0 / static_cast<double>(o->pilot_walks);
    MLMC_HIP_TRY(launch_combine(ca, p->n, p->prop_xhat, s));
    prepare_xhat(p->prop_xhat, p->n, p->prop_xmax, p->prop_logx, s);
    CoreOut co;
    if ((rc = train_core(p, ss, u, o, p->prop_xmax, co, s))) return rc;
    // 5. the plain law judges: the per-walk variance at l0 (mean over rows) of fresh walks
    //    under the plain law and under the proposal; the proposal stays enabled only if it
    //    is lower
    double judge_plain = 0.0, judge_learned = 0.0;
    bool accepted = true;
    if (o->judge_walks > 0) {
        auto level_var = [&](bool on, double &out) -> int {
            p->proposal_on = on;
            int r2 = mlmc_expv_level_sums(p, u, 1, MLMC_DTYPE_F32, o->seed ^ 0xD1B54A32D192ED03ull, 4093, level,
                                          0, static_cast<uint32_t>(o->judge_walks), s1, s2, nullptr, nullptr,
                                          stream);
            if (r2) return r2;
            MLMC_HIP_TRY(launch_level_moments(s1, s2, p->n, static_cast<double>(o->judge_walks), p->moments,
                                              p->moment_scratch, s));
            double h[3];
            MLMC_HIP_TRY(hipMemcpyAsync(h, p->moments, sizeof h, hipMemcpyDeviceToHost, s));
            MLMC_HIP_TRY(hipStreamSynchronize(s));
            out = h[2] / static_cast<double>(std::max<int64_t>(p->n, 1));
            return MLMC_OK;
        };
        if ((rc = level_var(false, judge_plain)) || (rc = level_var(true, judge_learned))) return rc;
        accepted = judge_learned < judge_plain;
        p->proposal_on = accepted;
    }
    MLMC_HIP_TRY(hipEventRecord(e1, s));
    MLMC_HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    MLMC_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (params_out) std::memcpy(params_out, co.P.data(), NPARAM * sizeof(float));
    if (st) {
        fill_train_stats(st, o, co);
        st->judge_var_plain = judge_plain;
        st->judge_var_learned = judge_learned;
        st->accepted = accepted ? 1 : 0;
        st->train_ms = ms;
    }
    return MLMC_OK;
}

}  // extern "C"
