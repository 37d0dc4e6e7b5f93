// Internal definitions shared by the library's translation units: table layouts in
// device memory, the counter-based generator, the logarithm behind the exponential
// holding times, and error plumbing. Not part of the public ABI (include/mlmc_expv.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

namespace mlmc {

// ------------------------------------------------------------------------------------
// Device tables
// ------------------------------------------------------------------------------------
// One off-diagonal slot of row k (a nonzero a_kj, j != k): the alias-table entry of the
// jump law |a_kj| / r_k. `own` and `alias` pack a column index with the sign bit
// sigma = [a < 0] in bit 31; a jump takes `own` when the coin word is below `thr`.
struct alignas(16) SlotRec {
    uint32_t own;
    uint32_t alias;
    uint32_t thr;
    uint32_t pad;
};

// One row at one level: where its slots start, how many there are, the integer step
// threshold of the level (no jump in a step iff the step's word is <= thr), the
// diagonal weight d = a_ii + r in both precisions and 1/r (inf for an absorbing row).
struct alignas(32) RowRec {
    uint32_t slot_begin;
    uint32_t deg;
    uint32_t thr;
    float d32;
    double inv_r;
    double d64;
};

// The same slot under a learned proposal q (importance sampling): the alias table of q,
// and the likelihood ratios p/q of the slot's own column and of its alias, one of which
// multiplies the path's functional when the jump takes it.
struct alignas(32) SlotRecIS {
    uint32_t own;
    uint32_t alias;
    uint32_t thr;
    uint32_t pad;
    float ratio_own;
    float ratio_alias;
    uint32_t pad2[2];
};

constexpr uint32_t kColMask = 0x7FFFFFFFu;
constexpr uint64_t kFnvOffset = 14695981039346656037ull;
constexpr uint64_t kFnvPrime = 1099511628211ull;

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, key bumped by the Weyl
// constants between rounds.
// ------------------------------------------------------------------------------------
struct Word4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umulhi(a, b);
#else
    return static_cast<uint32_t>((static_cast<uint64_t>(a) * b) >> 32);
#endif
}

// a ^ b ^ c: one v_bitop3_b32 on gfx950 (truth table 0x96), where the compiler would emit
// two v_xor_b32
__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

__host__ __device__ __forceinline__ Word4 philox10(Word4 c, uint32_t k0, uint32_t k1)
{
    // a round is two v_mad_u64_u32 (the 32x32->64 products) and two v_bitop3_b32
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c.x;
        const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
        c = Word4{xor3(static_cast<uint32_t>(pb >> 32), c.y, k0), static_cast<uint32_t>(pb),
                  xor3(static_cast<uint32_t>(pa >> 32), c.w, k1), static_cast<uint32_t>(pa)};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Stream selector word: level (6 bits), instance (12 bits), stream (0: step tests,
// 1: jumps).
__host__ __device__ __forceinline__ uint32_t stream_word(int level, int instance, int stream)
{
    return (static_cast<uint32_t>(level) << 26) |
           ((static_cast<uint32_t>(instance) & 0xFFFu) << 14) | static_cast<uint32_t>(stream);
}

// ------------------------------------------------------------------------------------
// -ln U for the uniform U = (w + 1/2) 2^-32 of a 32-bit word. The logarithm follows the
// series ln m = 2 atanh((m-1)/(m+1)) = 2 (s + s^3/3 + ... + s^23/23) (Abramowitz &
// Stegun 4.1.27) after reducing U = m 2^e with m in [sqrt(2)/2, sqrt(2)], and adds
// e ln 2 from a 29-bit head (exact product) and a tail. The operation sequence is part
// of the sampling definition: with contraction disabled, every step is a correctly
// rounded IEEE operation, so any conforming implementation of the same sequence
// returns the same bits.
// ------------------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t bits_of(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return static_cast<uint64_t>(__double_as_longlong(x));
#else
    uint64_t b;
    std::memcpy(&b, &x, sizeof b);
    return b;
#endif
}

__host__ __device__ __forceinline__ double double_of(uint64_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __longlong_as_double(static_cast<long long>(b));
#else
    double x;
    std::memcpy(&x, &b, sizeof x);
    return x;
#endif
}

__host__ __device__ __forceinline__ double uniform_of(uint32_t w)
{
    return (static_cast<double>(w) + 0.5) * 0x1p-32;
}

__host__ __device__ __forceinline__ double neg_log_uniform(uint32_t w)
{
    const double x = uniform_of(w);                 // normal, in [2^-33, 1)
    const uint64_t b = bits_of(x);
    int ex = static_cast<int>(b >> 52) - 1023;      // x = m 2^ex, m in [1, 2)
    double m = double_of((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > 0x1.6a09e667f3bcdp+0) {
        m = m * 0.5;
        ex = ex + 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, z, 1.0 / 21.0);
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    p = fma(p, z, 1.0);
    const double twice_atanh = 2.0 * (s * p);
    const double de = static_cast<double>(ex);
    const double ln_x = de * 0x1.62e42ffp-1 + (de * -0x1.718432a1b0e26p-35 + twice_atanh);
    return -ln_x;
}

// The same value for code inside a hot loop: the series coefficients 1/(2k+1) are divided
// out (correctly rounded, so equal to the constants above) in a loop that is not unrolled,
// instead of being held as eleven FP64 constants, which the compiler keeps live in 22
// VGPRs across the whole walk loop when the function is inlined there.
__device__ __forceinline__ double neg_log_uniform_rt(uint32_t w)
{
    const double x = uniform_of(w);
    const uint64_t b = bits_of(x);
    int ex = static_cast<int>(b >> 52) - 1023;
    double m = double_of((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > 0x1.6a09e667f3bcdp+0) {
        m = m * 0.5;
        ex = ex + 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 0.0;                                  // fma(0, z, 1/23) = 1/23 exactly
#pragma clang loop unroll(disable)
    for (int k = 11; k >= 0; --k) p = fma(p, z, 1.0 / static_cast<double>(2 * k + 1));
    const double twice_atanh = 2.0 * (s * p);
    const double de = static_cast<double>(ex);
    const double ln_x = de * 0x1.62e42ffp-1 + (de * -0x1.718432a1b0e26p-35 + twice_atanh);
    return -ln_x;
}

// ------------------------------------------------------------------------------------
// Fast bracket of -ln U(w) in FP32 from the hardware base-2 logarithm. For every 32-bit
// word w,
//     |neg_log_uniform_fast(w) - neg_log_uniform(w)| <= kFastLogAbs + kFastLogRel * E
// with E = neg_log_uniform_fast(w); the bound is checked exhaustively over all 2^32
// words by a GPU test. The walk kernel decides "accumulated holding time < dt" from
// these brackets and falls back to the exact FP64 sequence only when the bracket
// straddles dt, so its decisions equal the exact ones.
// ------------------------------------------------------------------------------------
constexpr float kFastLogAbs = 0x1p-20f;
constexpr float kFastLogRel = 0x1p-20f;

__device__ __forceinline__ float neg_log_uniform_fast(uint32_t w)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const float u = fmaf(static_cast<float>(w), 0x1p-32f, 0x1p-33f);
    return __builtin_amdgcn_logf(u) * -0x1.62e430p-1f;
#else
    (void)w;
    return 0.0f;   // device only
#endif
}

// ------------------------------------------------------------------------------------
// Errors
// ------------------------------------------------------------------------------------
void set_error(const std::string &msg);

}  // namespace mlmc

#define MLMC_HIP_TRY(expr)                                                             \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::mlmc::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));      \
            return (e_ == hipErrorOutOfMemory) ? MLMC_ERR_OUT_OF_MEMORY : MLMC_ERR_HIP; \
        }                                                                              \
    } while (0)
