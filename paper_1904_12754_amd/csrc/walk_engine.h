// Device-side walk engine shared by the single-level and the batched kernels.
//
// Walk (section 2.1, section 3, Algorithm 2). A walk at level l starts at row i and takes
// N = 2^l steps of length dt = beta / N. In each step the chain holds at its state k for
// an exponential time of rate r_k and, while the accumulated time stays below dt, jumps
// to j with probability |a_kj| / r_k, flipping its sign when a_kj < 0; the holding time
// after a jump has the rate of the state jumped to. Only the states at the grid points
// 0..N enter the weights:
//   fine   (level l):    E_f = dt * sum_n (d_{s_{n-1}} + d_{s_n}) / 2
//   coarse (level l-1):  E_c = dt * sum_m (d_{s_{2m-2}} + d_{s_{2m}})
// i.e. the Strang factors of section 2.1 multiplied out (the products of Algorithm 2's
// eta_2 and eta_1). A run of grid points [a, b] held at one state k adds d_k times an
// integer count to 2 E_f / dt, 2 E_c / dt and 2 (E_f - E_c) / dt, so the work on
// weights is O(jumps), and steps without a jump touch no memory. The sample is
//   Y = phi u_{s_N} e^{E_f}                       at l = l0,
//   Y = phi u_{s_N} (e^{E_f} - e^{E_c})
//     = phi u_{s_N} e^{E_c} expm1(E_f - E_c)      at l > l0,
// and a walk with no jump has E_f = E_c exactly, so Y = 0 (the "no transition" case of
// the paper's Fig. 1).
//
// Step test. A step of state k jumps iff the holding time -ln U(w) / r_k drawn from the
// step's word w is below dt. Because -ln U(w) decreases in w, this is the integer test
// w > thr_k(l) with thr from launch_thresholds, evaluated with the very same logarithm;
// so a step without a jump costs only its share of one Philox block (four steps per
// block) and a compare.
#pragma once

#include "common.h"
#include "kernels.h"

#include <cmath>

namespace mlmc {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
// The kernels with several right-hand sides run in workgroups of one wave: their waves are
// short (an item of a screened level is its walks' step draws and the per-row sums), and a
// slot of one wave is refilled as soon as that wave ends, where a slot of four waits for the
// slowest of them.
constexpr int kRhsBlock = kWave;

template <typename R>
__device__ __forceinline__ R d_of(const RowRec &r);
template <>
__device__ __forceinline__ float d_of<float>(const RowRec &r) { return r.d32; }
template <>
__device__ __forceinline__ double d_of<double>(const RowRec &r) { return r.d64; }

__device__ __forceinline__ float expR(float x) { return expf(x); }
__device__ __forceinline__ double expR(double x) { return exp(x); }

// e^{a h} for an exponent sum a and its scale h: in FP32 one v_exp_f32 of a * (h log2 e) (the
// rounding of the scaled exponent is of the order of that of a h itself), in FP64 exp(a h).
__device__ __forceinline__ float exp_scaled(float a, float h)
{
    return __builtin_amdgcn_exp2f(a * (h * 0x1.715476p+0f));
}
__device__ __forceinline__ double exp_scaled(double a, double h) { return exp(a * h); }
__device__ __forceinline__ float expm1R(float x) { return expm1f(x); }
__device__ __forceinline__ double expm1R(double x) { return expm1(x); }

template <typename R>
struct WalkOut {
    uint32_t k;       // final state
    uint32_t neg;     // 1 if the product of jump signs is -1
    uint32_t jumps;
    uint64_t hash;
    R ef2, ec2, ed2;  // 2/dt times E_f, E_c, E_f - E_c
    R wr;             // product of the likelihood ratios p/q (1 without a proposal)
};

// The jump from the alias table of the current row: returns the packed column | sign, and
// under a proposal multiplies wr by the likelihood ratio of the slot taken.
template <typename R, bool kIS>
__device__ __forceinline__ uint32_t jump_pick(const LevelArgs &L, uint32_t slot_index,
                                              uint32_t coin, R &wr)
{
    if (kIS) {
        const SlotRecIS sr = L.is_slots[slot_index];
        const bool own = coin < sr.thr;
        wr *= static_cast<R>(own ? sr.ratio_own : sr.ratio_alias);
        return own ? sr.own : sr.alias;
    }
    const SlotRec sr = L.slots[slot_index];
    return (coin < sr.thr) ? sr.own : sr.alias;
}

// Add the grid points a..b (held at one state with weight d) to the three sums; at the
// coarsest level (fine_only) the sample needs the fine sum alone.
template <typename R>
__device__ __forceinline__ void add_run(R d, uint32_t a, uint32_t b, uint32_t N, R &ef2, R &ec2,
                                        R &ed2, bool fine_only = false)
{
    const int a0 = (a == 0), bN = (b == N);
    const int f2 = 2 * static_cast<int>(b - a + 1) - a0 - bN;                 // 2 sum w_f
    ef2 += d * static_cast<R>(f2);
    if (fine_only) return;
    const int even = static_cast<int>(b >> 1) - static_cast<int>((a + 1) >> 1) + 1;
    const int c2 = 4 * even - 2 * a0 - 2 * bN;                                 // 2 sum w_c
    ec2 += d * static_cast<R>(c2);
    ed2 += d * static_cast<R>(f2 - c2);
}

// Observer of the jumps of run_walk: called with the state left, its record and the packed
// column | sign jumped to. NoObs compiles away.
struct NoObs {
    __device__ __forceinline__ void jump(uint32_t, const RowRec &, uint32_t) {}
};

template <typename R, bool kHash, bool kIS, typename Obs = NoObs>
__device__ __forceinline__ WalkOut<R> run_walk(const LevelArgs &L, uint32_t row, uint32_t walk,
                                               Obs *obs = nullptr)
{
    RowRec cur = L.rec[row];
    uint32_t k = row, neg = 0, J = 0, run_start = 0;
    uint64_t h = kFnvOffset;
    R ef2 = 0, ec2 = 0, ed2 = 0, wr = 1;
    const uint32_t nblk = (L.N + 3) >> 2;
    for (uint32_t q = 0; q < nblk; ++q) {
        Word4 w = philox10(Word4{q, walk, row, L.c3_step}, L.k0, L.k1);
        if (L.N < 4) {          // levels 0 and 1: words past step N never jump
            w.w = 0;
            w.z = 0;
            if (L.N < 2) w.y = 0;
        }
        const uint32_t mx = max(max(w.x, w.y), max(w.z, w.w));
        if (mx <= cur.thr) continue;
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (ws[m] <= cur.thr) continue;
            const uint32_t n = 4 * q + m;   // 0-based step: the jump falls between grid n and n+1
            add_run<R>(d_of<R>(cur), run_start, n, L.N, ef2, ec2, ed2);
            double tau = neg_log_uniform(ws[m]) * cur.inv_r;
            do {
                const Word4 jw = philox10(Word4{J, walk, row, L.c3_jump}, L.k0, L.k1);
                const uint32_t slot = mulhi32(jw.x, cur.deg);
                const uint32_t cs = jump_pick<R, kIS>(L, cur.slot_begin + slot, jw.y, wr);
                if (obs) obs->jump(k, cur, cs);
                k = cs & kColMask;
                neg ^= cs >> 31;
                cur = L.rec[k];
                ++J;
                if (kHash) {
                    h = (h ^ static_cast<uint64_t>(k)) * kFnvPrime;
                    h = (h ^ static_cast<uint64_t>(n + 1)) * kFnvPrime;
                }
                tau = tau + neg_log_uniform(jw.z) * cur.inv_r;
            } while (tau < L.dt);
            run_start = n + 1;
        }
    }
    add_run<R>(d_of<R>(cur), run_start, L.N, L.N, ef2, ec2, ed2);
    WalkOut<R> o;
    o.k = k;
    o.neg = neg;
    o.jumps = J;
    o.hash = h;
    o.ef2 = ef2;
    o.ec2 = ec2;
    o.ed2 = ed2;
    o.wr = wr;
    return o;
}

// The sample without its u factor: +-e^{E_f} at the base level, +-e^{E_c} expm1(E_f - E_c)
// above it.
template <typename R>
__device__ __forceinline__ R weight_of(const WalkOut<R> &o, int base, R hd)
{
    R v = (base ? expR(o.ef2 * hd) : expR(o.ec2 * hd) * expm1R(o.ed2 * hd)) * o.wr;
    return o.neg ? -v : v;
}

template <typename R>
struct Kahan {
    R s = 0, c = 0;
    __device__ __forceinline__ void add(R x)
    {
        const R y = x - c;
        const R t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const
    {
        return static_cast<double>(s) - static_cast<double>(c);
    }
};

// Per-lane running sums of the samples and of their squares, compensated in the precision
// of the weights (Kahan sums).
template <typename R>
struct LaneMoments {
    Kahan<R> k1, k2;
    __device__ __forceinline__ void add(R y)
    {
        k1.add(y);
        k2.add(y * y);
    }
    __device__ __forceinline__ double first() const { return k1.value(); }
    __device__ __forceinline__ double second() const { return k2.value(); }
};

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u(unsigned long long v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over each aligned group of lpr lanes (lpr a power of two <= 64), in a fixed order.
__device__ __forceinline__ double group_sum(double v, uint32_t lpr)
{
    for (uint32_t o = lpr / 2; o > 0; o >>= 1) v += __shfl_xor(v, static_cast<int>(o), kWave);
    return v;
}

__device__ __forceinline__ unsigned long long group_sum_u(unsigned long long v, uint32_t lpr)
{
    for (uint32_t o = lpr / 2; o > 0; o >>= 1) v += __shfl_xor(v, static_cast<int>(o), kWave);
    return v;
}

template <typename U>
__device__ __forceinline__ double load_u(const U *u, uint64_t idx)
{
    return static_cast<double>(u[idx]);
}

// ------------------------------------------------------------------------------------
// Lane-refilling walk engine. A wave (or a group of its lanes) owns the walks [wb, we) of
// one row (or, with a random start, walks of many rows); each lane runs one walk at a time
// and takes the next unassigned walk as soon as its walk ends. In an iteration a busy lane
// draws at most one Philox block: the next step block when it has scanned past its cached
// one, or the jump block (slot, alias coin, next holding time) while it jumps. A chain of
// jumps that ends inside the cached step block is followed by the scan in the same
// iteration, on the same code path as the other scanning lanes. The end of a walk only
// stores its exponents; the expensive evaluation (exp, expm1, the sink) runs for many
// lanes at once. The divergent work between the blocks is therefore short, and the wave
// stays busy on the generator instead of waiting on its slowest lane.
// ------------------------------------------------------------------------------------
struct ScanOut {
    bool jump;       // a step of the block jumps
    uint32_t word;   // that step's word
};

// First step n' >= n of the cached block (b0..b3, block q = n >> 2) whose word exceeds
// thr. On a jump, n is set to that step; otherwise n moves to the end of the block (or N).
__device__ __forceinline__ ScanOut scan_block(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3,
                                              uint32_t thr, uint32_t &n, uint32_t N)
{
    const uint32_t m0 = n & 3u;
    const uint32_t base = n - m0;
    // words past step N were zeroed when the block was loaded and never exceed thr
    const bool j0 = m0 == 0 && b0 > thr;
    const bool j1 = m0 <= 1 && b1 > thr;
    const bool j2 = m0 <= 2 && b2 > thr;
    const bool j3 = b3 > thr;
    ScanOut o;
    o.jump = j0 || j1 || j2 || j3;
    const uint32_t m = j0 ? 0u : j1 ? 1u : j2 ? 2u : 3u;
    o.word = j0 ? b0 : j1 ? b1 : j2 ? b2 : b3;
    n = o.jump ? base + m : min(base + 4u, N);
    return o;
}

// What a lane does: scans the step words of its walk, follows a chain of jumps of step n,
// waits (its walk has ended while its slot for finished walks was full), or has no walk.
constexpr uint32_t kScan = 0, kJump = 1, kWait = 2, kIdle = 3;
static_assert(kScan == 0 && kJump == 1, "the stream word of a lane's block is c3_step + state");

template <typename R, bool kHash>
struct Walker {
    // per-lane state of the current walk
    uint32_t st = kIdle;
    uint32_t w = 0, k = 0, neg = 0, J = 0, run_start = 0, n = 0;
    uint32_t row0 = 0;                    // the walk's start row (its counters' row), when
                                          // it differs between walks
    uint32_t bq = 0xFFFFFFFFu;            // index of the cached step block
    uint32_t b0 = 0, b1 = 0, b2 = 0, b3 = 0;
    RowRec cur;
    // the holding time accumulated in step n: bracket [tau_h - tau_e, tau_h + tau_e] around
    // the exact FP64 value, and what is needed to replay it exactly (state and jump count
    // at the start of the chain; the step's word is in the cached block)
    float tau_h = 0.0f, tau_e = 0.0f;
    uint32_t chain_k = 0, chain_J = 0;
    R ef2 = 0, ec2 = 0, ed2 = 0;
    R wr = 1;                             // likelihood ratio of the path under a proposal
    R jf = 0, jc = 0;                     // source term: fine and coarse Simpson sums
    uint64_t hash = kFnvOffset;
};

// Result of a finished walk, handed to the sink.
template <typename R>
struct Finished {
    uint32_t k;        // final state
    uint32_t jumps;
    R W;               // the sample without its u factor (sign included)
    uint64_t hash;
    R src;             // the source term's part of the sample (0 without a source)
};

// A finished walk waiting for its evaluation: the final state, the sign, the exponents of
// the sample (2 E_f / dt at the base level, 2 E_c / dt and 2 (E_f - E_c) / dt above), the
// likelihood ratio, and what the counters need.
constexpr int kFlushAt = 40;
constexpr int kMaxWaiting = 4;

template <typename R, bool kSrc>
struct Pending {
    bool valid = false;
    uint32_t k = 0, neg = 0, jumps = 0;
    R e1 = 0, e2 = 0, wr = 1;
    R src = 0;                            // the source term's part (Algorithm 3)
    uint64_t hash = 0;
    template <typename W>
    __device__ __forceinline__ void hold(const W &s, int base, R hd)
    {
        valid = true;
        k = s.k;
        neg = s.neg;
        jumps = s.J;
        wr = s.wr;
        hash = s.hash;
        e1 = base ? s.ef2 : s.ec2;
        e2 = s.ed2;
        if constexpr (kSrc) {
            // dt/3 times the fine sum, minus 2 dt/3 times the coarse sum above l0
            const R third = (hd + hd) / static_cast<R>(3);
            src = base ? third * s.jf : third * s.jf - (third + third) * s.jc;
        }
    }
    __device__ __forceinline__ Finished<R> finished(int base, R hd) const
    {
        Finished<R> f{k, jumps, static_cast<R>(0), hash, static_cast<R>(0)};
        const R v = (base ? exp_scaled(e1, hd) : exp_scaled(e1, hd) * expm1R(e2 * hd)) * wr;
        f.W = neg ? -v : v;
        if constexpr (kSrc) f.src = src;
        return f;
    }
};

// ------------------------------------------------------------------------------------
// Source term (Algorithm 3): int_0^beta exp(sA) F ds by the composite Simpson rule over
// the walk's grid times, the fine functional on the N intervals of the level and the coarse
// one on the N/2 intervals of the even points. Within a holding run of grid points a..b at
// state k the functionals grow by q = e^{d_k dt} per fine step, so a run adds
//   sign * F_k * eta(a) * sum_n w_n q^{n - a}
// with w_n = 2 + 2 [n odd] - [n = 0] - [n = N]: geometric series, O(1) per run.
// ------------------------------------------------------------------------------------
// sum_{j < L} e^{j x}
template <typename R>
__device__ __forceinline__ R geo_sum(uint32_t L, R x)
{
    if (L == 0) return static_cast<R>(0);
    if (x == static_cast<R>(0)) return static_cast<R>(L);
    return expm1R(static_cast<R>(L) * x) / expm1R(x);
}

// sum_{n = a}^{b} w_n e^{(n - a) x} for the Simpson weights of K intervals (a <= b <= K)
template <typename R>
__device__ __forceinline__ R simpson_run(uint32_t a, uint32_t b, uint32_t K, R x)
{
    R s = static_cast<R>(2) * geo_sum<R>(b - a + 1, x);
    const uint32_t o = a | 1u;                       // first odd point >= a
    if (o <= b) s += static_cast<R>(2) * ((a & 1u) ? static_cast<R>(1) : expR(x)) *
                     geo_sum<R>((b - o) / 2 + 1, static_cast<R>(2) * x);
    if (a == 0) s -= static_cast<R>(1);
    if (b == K) s -= expR(static_cast<R>(K - a) * x);
    return s;
}

// The run a..b at the walker's state: add its fine and coarse Simpson sums. Called before
// add_run, while ef2 and ec2 hold the exponents of the points before a.
template <typename R, typename W>
__device__ __forceinline__ void source_run(W &s, R d, R hd, uint32_t a, uint32_t b, uint32_t N,
                                           R Fk)
{
    const R x = d * (hd + hd);                        // d dt
    const R sgn = (s.neg ? -s.wr : s.wr) * Fk;
    const R ea = (a == 0) ? static_cast<R>(1) : expR(hd * (s.ef2 + d));
    s.jf += sgn * ea * simpson_run<R>(a, b, N, x);
    const uint32_t e0 = a + (a & 1u), e1 = b - (b & 1u);
    if (N >= 2 && e0 <= e1) {
        const R ec = (e0 == 0) ? static_cast<R>(1) : expR(hd * (s.ec2 + d + d));
        s.jc += sgn * ec * simpson_run<R>(e0 / 2, e1 / 2, N / 2, x + x);
    }
}

// Holding time of the current step's chain in the exact FP64 sequence: the step's word at
// the chain's first state, then the next-holding-time word of each jump J0 .. J1 - 1 at
// the state that jump reached (the jumps are replayed from their blocks).
template <bool kIS>
__device__ __forceinline__ double chain_tau_exact(const LevelArgs &L, uint32_t row, uint32_t walk,
                                                  uint32_t k0, uint32_t J0, uint32_t J1,
                                                  uint32_t word)
{
    RowRec rk = L.rec[k0];
    double tau = neg_log_uniform_rt(word) * rk.inv_r;
    for (uint32_t J = J0; J < J1; ++J) {
        const Word4 ph = philox10(Word4{J, walk, row, L.c3_jump}, L.k0, L.k1);
        const uint32_t slot = mulhi32(ph.x, rk.deg);
        float unused = 1.0f;
        const uint32_t cs = jump_pick<float, kIS>(L, rk.slot_begin + slot, ph.y, unused);
        rk = L.rec[cs & kColMask];
        tau = tau + neg_log_uniform_rt(ph.z) * rk.inv_r;
    }
    return tau;
}

// Start the bracket of a new chain with the holding time of its first state.
template <typename R, bool kHash>
__device__ __forceinline__ void chain_start(Walker<R, kHash> &s, uint32_t word)
{
    const float e = neg_log_uniform_fast(word);
    const float ir = static_cast<float>(s.cur.inv_r);      // this state jumps (r > 0)
    s.tau_h = e * ir;
    s.tau_e = (kFastLogAbs + kFastLogRel * e) * ir + s.tau_h * 0x1p-21f;
    s.chain_k = s.k;
    s.chain_J = s.J;
}

// The wave's lanes form groups of lpr lanes (lpr a power of two, 1..64); the lanes of a group
// run the walks [wb, we) of the group's row (row, wb and we are the same within a group).
// Groups of fewer than 64 lanes serve rows with few walks, so that a wave still has 64
// walks in flight.
// Start of a walk: every walk of the range starts at one row (the backward representation
// of a single entry) ...
struct FixedStart {
    static constexpr bool kPerLaneRow = false;   // the counters' row is `row` for every walk
    uint32_t row;
    RowRec rec;
    __device__ __forceinline__ void pick(const LevelArgs &, uint32_t, uint32_t &r, RowRec &rr,
                                         uint32_t &neg) const
    {
        r = row;
        rr = rec;
        neg = 0;
    }
    __device__ __forceinline__ uint32_t start_row() const { return row; }
};

// ... or walk m starts at row l with probability |u_l| / U, drawn from the alias table over
// rows with the words of the block (0, m, 0, stream 2); the walk then carries sign(u_l).
struct AliasStart {
    static constexpr bool kPerLaneRow = true;
    const uint32_t *thr;
    const int32_t *alias;
    const uint8_t *neg;
    uint32_t n;
    uint32_t c3;                         // stream word of the start draws
    __device__ __forceinline__ void pick(const LevelArgs &L, uint32_t walk, uint32_t &r,
                                         RowRec &rr, uint32_t &ng) const
    {
        const Word4 ph = philox10(Word4{0u, walk, 0u, c3}, L.k0, L.k1);
        const uint32_t slot = mulhi32(ph.x, n);
        r = (ph.y < thr[slot]) ? slot : static_cast<uint32_t>(alias[slot]);
        rr = L.rec[r];
        ng = neg[r];
    }
    __device__ __forceinline__ uint32_t start_row() const { return 0u; }   // per lane instead
};

// kBase: the level is the coarsest (l0) by construction, so the code for the coarse
// functional and for held walks is left out; otherwise L.base decides at run time.
// kScreen: when the level's walks mostly never jump (L.screen), each lane first draws the
// step blocks of its walks wb + lane + 64 j (j < 64) and tests every step at the start row.
// A walk none of whose steps jumps holds at its start row for the whole time: the sink
// counts it as such (sink.no_jumps(): its sample is the same for every such walk), at the
// cost of its step draws alone. The lane marks the others, and the loop runs them from
// their first step like any walk (their paths and samples are those of the unscreened
// loop). Only for one start row per range (the counters' row is the group's row), a
// range of at most 4096 walks and a whole wave per range.
template <typename R, bool kHash, bool kIS, bool kSrc, bool kBase = false, bool kScreen = false,
          typename Sink, typename Start>
__device__ __forceinline__ void walk_range_from(const LevelArgs &L, const Start &st, uint32_t walk0,
                                                uint64_t wb, uint64_t we, Sink &sink,
                                                uint32_t lpr = kWave);

template <typename R, bool kHash, bool kIS, bool kSrc = false, bool kBase = false,
          bool kScreen = false, typename Sink>
__device__ __forceinline__ void walk_range(const LevelArgs &L, uint32_t row, uint32_t walk0,
                                           uint64_t wb, uint64_t we, Sink &sink,
                                           uint32_t lpr = kWave)
{
    const FixedStart st{row, L.rec[row]};
    walk_range_from<R, kHash, kIS, kSrc, kBase, kScreen>(L, st, walk0, wb, we, sink, lpr);
}

constexpr uint64_t kScreenMaxWalks = static_cast<uint64_t>(kWave) * 64;

// The screening state of a lane: whether the range was screened, and its walks
// wb + lane + 64 j that jump (bit j). Empty where screening is compiled out.
template <bool kOn>
struct ScreenState {
    bool on = false;
    uint64_t marked = 0;
};
template <>
struct ScreenState<false> {};
__device__ __forceinline__ bool screening_on(const ScreenState<true> &s) { return s.on; }
__device__ __forceinline__ constexpr bool screening_on(const ScreenState<false> &) { return false; }

template <typename R, bool kHash, bool kIS, bool kSrc, bool kBase, bool kScreen, typename Sink,
          typename Start>
__device__ __forceinline__ void walk_range_from(const LevelArgs &L, const Start &st, uint32_t walk0,
                                                uint64_t wb, uint64_t we, Sink &sink, uint32_t lpr)
{
    static_assert(!kScreen || (!Start::kPerLaneRow && !kHash && !kSrc),
                  "screening needs one start row per range and no path hash or source term");
    const bool base = kBase || L.base != 0;
    const int ibase = base ? 1 : 0;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t group = lpr >= kWave ? ~0ull : ((1ull << lpr) - 1ull) << (lane & ~(lpr - 1u));
    const R hd = static_cast<R>(L.half_dt);
    Walker<R, kHash> s;
    Pending<R, kSrc> pend;
    uint64_t pool = wb;                    // next unassigned walk of the group
    [[maybe_unused]] ScreenState<kScreen> scr;
    if constexpr (kScreen) {
        scr.on = L.screen != 0 && lpr >= kWave && we - wb <= kScreenMaxWalks;
        if (scr.on) {
            const uint32_t thr = st.rec.thr;
            const uint32_t row0 = st.start_row();
            // the lane's (walk j, block q) pairs t = j * blocks + q, four independent Philox
            // blocks at a time (a block is a chain of dependent multiplies: four chains keep
            // the SIMD issuing while each waits)
            const uint32_t lb = L.N >= 4u ? static_cast<uint32_t>(__builtin_ctz(L.N)) - 2u : 0u;
            const uint32_t walks_lane = lane < we - wb ? static_cast<uint32_t>((we - wb - lane + kWave - 1) / kWave) : 0u;
            const uint32_t pairs = walks_lane << lb;
            const uint32_t pairs_max = static_cast<uint32_t>((we - wb + kWave - 1) / kWave) << lb;
            for (uint32_t t0 = 0; t0 < pairs_max; t0 += 4) {
                Word4 ph[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const uint32_t t = t0 + v;
                    const uint32_t w = walk0 + static_cast<uint32_t>(wb + static_cast<uint64_t>(t >> lb) * kWave + lane);
                    ph[v] = philox10(Word4{t & ((1u << lb) - 1u), w, row0, L.c3_step}, L.k0, L.k1);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const uint32_t t = t0 + v;
                    // words past step N (levels 0 and 1) are not steps
                    const bool jump = ph[v].x > thr || (L.N > 1u && ph[v].y > thr) ||
                                      (L.N > 2u && (ph[v].z > thr || ph[v].w > thr));
                    if (t < pairs && jump) scr.marked |= 1ull << (t >> lb);
                }
            }
            sink.no_jumps(walks_lane - static_cast<uint32_t>(__popcll(scr.marked)));
        }
    }
    for (;;) {
        if constexpr (kScreen) {
            if (scr.on) {
                // ---- the lane's next marked walk
                if (s.st == kIdle && scr.marked != 0) {
                    const uint32_t j = static_cast<uint32_t>(__builtin_ctzll(scr.marked));
                    scr.marked &= scr.marked - 1;
                    s.st = kScan;
                    s.w = walk0 + static_cast<uint32_t>(wb + static_cast<uint64_t>(j) * kWave + lane);
                    uint32_t r0 = 0, ng = 0;
                    st.pick(L, s.w, r0, s.cur, ng);
                    s.k = r0;
                    s.neg = ng;
                    s.J = 0;
                    s.run_start = 0;
                    s.n = 0;
                    s.bq = 0xFFFFFFFFu;
                    s.ef2 = s.ec2 = s.ed2 = 0;
                    s.wr = 1;
                    s.jf = s.jc = 0;
                }
            }
        }
        // ---- refill idle lanes with the next walks of the group's range (a screened range
        // runs its marked walks instead)
        const uint64_t idle = screening_on(scr) ? 0ull : __ballot(s.st == kIdle) & group;
        if (idle) {
            // the idle lanes of the group below this one (v_mbcnt)
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                static_cast<uint32_t>(idle >> 32),
                __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(idle), 0u));
            const uint64_t mine = pool + below;
            if (s.st == kIdle && mine < we) {
                s.st = kScan;
                s.w = walk0 + static_cast<uint32_t>(mine);
                uint32_t r0 = 0, ng = 0;
                st.pick(L, s.w, r0, s.cur, ng);
                if constexpr (Start::kPerLaneRow) s.row0 = r0;
                s.k = r0;
                s.neg = ng;
                s.J = 0;
                s.run_start = 0;
                s.n = 0;
                s.bq = 0xFFFFFFFFu;
                s.ef2 = s.ec2 = s.ed2 = 0;
                s.wr = 1;
                s.jf = s.jc = 0;
                if (kHash) s.hash = kFnvOffset;
            }
            pool += __popcll(idle);
        }
        if (__ballot(s.st != kIdle) == 0) break;

        // ---- at most one Philox block per busy lane: the block is evaluated for every lane
        // (the wave issues it whenever one lane needs it) and used by the lanes that jump
        // or that scanned past their cached block
        const bool jumping = s.st == kJump;
        const bool scanning = s.st == kScan;
        const uint32_t q = s.n >> 2;
        const uint32_t row0 = Start::kPerLaneRow ? s.row0 : st.start_row();
        // stream word: c3_step + 1 == c3_jump and kJump == 1, kScan == 0 (the sum is
        // meaningless for waiting and idle lanes, which do not use the block)
        const Word4 ph = philox10(Word4{jumping ? s.J : q, s.w, row0, L.c3_step + s.st},
                                  L.k0, L.k1);

        bool finish = false;
        if (jumping) {
            // jump from k by the alias table of row k: slot, coin, then the new state's record
            const uint32_t slot = mulhi32(ph.x, s.cur.deg);
            const uint32_t cs = jump_pick<R, kIS>(L, s.cur.slot_begin + slot, ph.y, s.wr);
            s.k = cs & kColMask;
            s.neg ^= cs >> 31;
            s.cur = L.rec[s.k];
            ++s.J;
            if (kHash) {
                s.hash = (s.hash ^ static_cast<uint64_t>(s.k)) * kFnvPrime;
                s.hash = (s.hash ^ static_cast<uint64_t>(s.n + 1)) * kFnvPrime;
            }
            // add the holding time at the new state; the chain goes on while the total is
            // below dt. An absorbing state (no off-diagonal entry: r = 0) holds forever; a
            // rate so small that 1/r is infinite in FP32 (or FP64) makes the bracket infinite
            // or NaN, and every comparison with one sends the decision to the exact path.
            const float ir = static_cast<float>(s.cur.inv_r);
            bool chain_over;
            if (s.cur.deg == 0u) {
                chain_over = true;
            } else {
                const float e = neg_log_uniform_fast(ph.z);
                s.tau_h = s.tau_h + e * ir;
                s.tau_e = s.tau_e + (kFastLogAbs + kFastLogRel * e) * ir + s.tau_h * 0x1p-21f;
                // the ends of the bracket in FP32; dt_below and dt_above absorb their rounding
                const float hi = s.tau_h + s.tau_e;
                const float lo = s.tau_h - s.tau_e;
                if (hi < L.dt_below) chain_over = false;
                else if (lo >= L.dt_above) chain_over = true;
                else {
                    // the chain's first word is that of step n in the cached block
                    const uint32_t m = s.n & 3u;
                    const uint32_t word = m == 0u ? s.b0 : m == 1u ? s.b1 : m == 2u ? s.b2 : s.b3;
                    chain_over = !(chain_tau_exact<kIS>(L, row0, s.w, s.chain_k, s.chain_J, s.J, word) <
                                   L.dt);
                }
            }
            if (chain_over) {
                // the chain of step n ends: the walk scans on from step n + 1 (below, in
                // this iteration when that step is in the cached block)
                s.st = kScan;
                s.n = s.n + 1;
                s.run_start = s.n;
                finish = s.n == L.N;
            }
        } else if (scanning && s.bq != q) {
            const bool short_walk = L.N < 4;   // levels 0, 1: words past step N never jump
            s.b0 = ph.x;
            s.b1 = (short_walk && L.N < 2) ? 0u : ph.y;
            s.b2 = short_walk ? 0u : ph.z;
            s.b3 = short_walk ? 0u : ph.w;
            s.bq = q;
        }
        // scan the cached block: the lanes that were scanning, and the lanes whose chain
        // just ended inside the cached block (one code path for both)
        bool chain = false;
        uint32_t chain_word = 0;
        if (s.st == kScan && !finish && (s.n >> 2) == s.bq) {
            const ScanOut so = scan_block(s.b0, s.b1, s.b2, s.b3, s.cur.thr, s.n, L.N);
            // the step's holding time at k is below dt: a chain of jumps starts
            chain = so.jump;
            chain_word = so.word;
            finish = !so.jump && s.n == L.N;
        }
        // the holding run at k ends: at the step that starts a chain, or at the end of the
        // walk (one code path for both)
        if (chain || finish) {
            const uint32_t run_end = chain ? s.n : L.N;
            if constexpr (kSrc) source_run<R>(s, d_of<R>(s.cur), hd, s.run_start, run_end, L.N, sink.source(s.k));
            add_run<R>(d_of<R>(s.cur), s.run_start, run_end, L.N, s.ef2, s.ec2, s.ed2, base);
        }
        if (chain) {
            chain_start(s, chain_word);
            s.st = kJump;
        }

        // ---- the end of a walk: its exponents wait in the lane's slot, and the slots are
        // evaluated together (exp, expm1, the sink) when kFlushAt lanes hold one, when
        // kMaxWaiting lanes have ended a walk while their slot was full (they wait, without
        // a new walk, for the evaluation), when no lane is still walking, or after the last
        // walk
        // At the coarsest level the sample is one exponential, so a sink that adds each
        // lane's samples on its own lane takes it at once (the lane's samples are added in
        // the order its walks end either way, so the sums are the same).
        const bool direct = Sink::kLaneLocal && base;
        if (finish) {
            if (direct) {
                Pending<R, kSrc> now;
                now.hold(s, 1, hd);
                sink.take(true, now.finished(1, hd));
                s.st = kIdle;
            } else if (!pend.valid) {
                pend.hold(s, ibase, hd);
                s.st = kIdle;
            } else {
                s.st = kWait;
            }
        }
        if (!direct) {
            const uint64_t waiting = __ballot(s.st == kWait);
            if (__popcll(__ballot(pend.valid)) >= kFlushAt ||
                (waiting != 0 && (__popcll(waiting) >= kMaxWaiting ||
                                  __ballot(s.st < kWait) == 0))) {
                sink.take(pend.valid, pend.finished(ibase, hd));
                pend.valid = false;
                if (s.st == kWait) {
                    pend.hold(s, ibase, hd);
                    s.st = kIdle;
                }
            }
        }
    }
    sink.take(pend.valid, pend.finished(ibase, hd));
}

// Single right-hand side: each lane adds its own samples to its running sums (kSrc: the
// samples carry a source-term part).
template <typename R, typename U, bool kSrc = false>
struct SinkR1 {
    static constexpr bool kLaneLocal = true;   // take() touches only the calling lane
    const U *u;
    const U *F;       // source vector (Algorithm 3), or null
    LaneMoments<R> mom;
    unsigned long long jumps = 0, hash = 0;
    uint32_t nonfinite = 0;   // a lane evaluates fewer than 2^32 samples in a launch
    __device__ __forceinline__ R source(uint32_t k) const { return static_cast<R>(F[k]); }
    __device__ __forceinline__ void take(bool done, const Finished<R> &f)
    {
        if (!done) return;
        R y = f.W * static_cast<R>(u[f.k]);
        if constexpr (kSrc) y += f.src;
        jumps += f.jumps;
        hash += f.hash;
        nonfinite += !isfinite(y);
        mom.add(y);
    }
};

// Forward representation of the full vector: each sample is deposited at the walk's final
// state (FP64 atomic adds of the sample and of its square; hipMalloc memory is coarse-grained,
// so these are the hardware's global_atomic_add_f64).
template <typename R>
struct SinkDeposit {
    static constexpr bool kLaneLocal = true;   // take() touches only the calling lane
    double *sum1, *sum2;
    unsigned long long jumps = 0, hash = 0;
    uint32_t nonfinite = 0;
    __device__ __forceinline__ void take(bool done, const Finished<R> &f)
    {
        if (!done) return;
        const double y = static_cast<double>(f.W);
        jumps += f.jumps;
        hash += f.hash;
        nonfinite += !isfinite(y);
        // a sample of exactly zero adds nothing, so it takes no atomics: above the coarsest
        // level, a walk that never leaves its start row has E_f = E_c exactly
        if (y == 0.0) return;
        unsafeAtomicAdd(&sum1[f.k], y);
        unsafeAtomicAdd(&sum2[f.k], y * y);
    }
};

// Several right-hand sides: the finished walks of an iteration are broadcast one by one
// and lane r adds right-hand side r (+64 g) from the contiguous row u[k, :]. Walks
// without a jump all end at the start row with the same weight; they are only counted.
constexpr int kMaxRhsGroups = 4;   // up to 256 right-hand sides

template <typename R, typename U>
struct SinkRhs {
    static constexpr bool kLaneLocal = false;  // take() is a wave-wide broadcast
    const U *u;
    int32_t nrhs;
    int groups;
    LaneMoments<R> mom[kMaxRhsGroups];
    unsigned long long jumps = 0, nojump = 0, nonfinite = 0, hash = 0;
    // a walk that never left its start row, screened before the loop (its path hash is not
    // kept: screening runs without hashes)
    __device__ __forceinline__ void no_jumps(uint32_t count) { nojump += count; }
    __device__ __forceinline__ void take(bool done, const Finished<R> &f)
    {
        const bool moved = done && f.jumps > 0;
        if (done) {
            jumps += f.jumps;
            hash += f.hash;
            nojump += f.jumps == 0;
        }
        uint64_t pending = __ballot(moved && f.W != static_cast<R>(0));
        const uint32_t lane = threadIdx.x & (kWave - 1);
        while (pending) {
            const int t = __ffsll(static_cast<unsigned long long>(pending)) - 1;
            pending &= pending - 1;
            const R Wt = __shfl(f.W, t, kWave);
            const uint32_t kt = __shfl(f.k, t, kWave);
#pragma unroll
            for (int g = 0; g < kMaxRhsGroups; ++g) {
                const int r = static_cast<int>(lane) + g * kWave;
                if (g < groups && r < nrhs) {
                    const R y = Wt * static_cast<R>(u[static_cast<uint64_t>(kt) * nrhs + r]);
                    nonfinite += !isfinite(y);
                    mom[g].add(y);
                }
            }
        }
    }
};

// One wave per (row, chunk) item.

}  // namespace mlmc
