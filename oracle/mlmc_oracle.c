/*
 * Oracle for the multilevel Monte Carlo (MLMC) estimator of x = exp(beta*A) u of
 * Acebron, Herrero & Monteiro, "A highly parallel algorithm for computing the action
 * of a matrix exponential on a vector based on a multilevel Monte Carlo method"
 * (arXiv:1904.12754).
 *
 * TEST INFRASTRUCTURE. This file is a plain, slow CPU implementation that the tests,
 * the smoke check and the CPU-baseline leg of the benchmark use to check the GPU
 * library. Nothing in the product path may link, load or call it. It shares no code
 * with the GPU library: the random-number generator, the logarithm, the
 * decomposition, the alias tables and the walk are all written here independently
 * from the paper and from the published definitions named below.
 *
 * Arithmetic: FP64 throughout, no contraction (build with -ffp-contract=off); the
 * fused multiply-adds in the logarithm are explicit calls to C99 fma(), which is
 * correctly rounded.
 *
 * What is computed, and where the paper defines it:
 *   - decomposition A = D - T (section 2.1, the definitions of L, d, sigma and T);
 *   - the jump law k_ij = |L_ij| / L_ii and exponential holding times of rate L_ii
 *     (section 3, the integral form of the backward equation);
 *   - the coupled fine/coarse path functional of one sample (Algorithm 2, with the
 *     level terms of the telescoping sum, section 2.2);
 *   - per-row level sums of Y and Y^2 that give m_l and V_l (Algorithm 2's
 *     accumulators; the variance read as mean(Y^2) - mean(Y)^2).
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   - the holding time S after a jump has the rate of the state jumped TO;
 *   - the final factor uses u at the final state of the path;
 *   - the base level l0 contributes u*eta_fine only (P_{l0-1} = 0);
 *   - N = 2^l steps of length dt = beta / 2^l at level l;
 *   - levels draw independent random streams; within a level the fine and the coarse
 *     functional share one path.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------ */
/* Philox4x32-10: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel    */
/* random numbers: as easy as 1, 2, 3", SC'11. Ten rounds of the 4x32 S-box with   */
/* multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 /        */
/* 0xBB67AE85 (the key is bumped between rounds).                                  */
/* ------------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Random stream layout. Key = the 64-bit seed (low word first). Counter =
 * (index, walk, row, level<<26 | instance<<14 | stream). Stream 0 holds the step
 * tests: step n (0-based) of a walk reads word n%4 of block n/4. Stream 1 holds the
 * jumps: the walk's j-th jump (0-based over the whole walk) reads block j, words
 * 0 (slot), 1 (alias coin) and 2 (the next holding time). */
static uint32_t c3_of(int level, uint32_t instance, uint32_t stream)
{
    return ((uint32_t)level << 26) | ((instance & 0xFFFu) << 14) | stream;
}

static uint32_t step_word(const uint32_t key[2], int level, uint32_t inst, uint32_t row,
                          uint32_t walk, uint32_t n)
{
    uint32_t ctr[4] = {n >> 2, walk, row, c3_of(level, inst, 0)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[n & 3u];
}

static void jump_words(const uint32_t key[2], int level, uint32_t inst, uint32_t row,
                       uint32_t walk, uint32_t j, uint32_t w[3])
{
    uint32_t ctr[4] = {j, walk, row, c3_of(level, inst, 1)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    w[0] = out[0]; w[1] = out[1]; w[2] = out[2];
}

/* A 32-bit word as a uniform variate on the open interval (0, 1): (w + 1/2) 2^-32.
 * It is exact in FP64 and never 0 or 1, so its logarithm is finite and negative. */
double orc_uniform(uint32_t w)
{
    return ((double)w + 0.5) * 0x1p-32;
}

/* ------------------------------------------------------------------------------ */
/* Natural logarithm on (0, 1), from the series                                    */
/*     ln m = 2 (s + s^3/3 + s^5/5 + ...),  s = (m - 1) / (m + 1)                  */
/* (Abramowitz & Stegun, Handbook of Mathematical Functions, 4.1.27), after the    */
/* reduction x = m 2^e with m in [sqrt(2)/2, sqrt(2)]. Twelve terms reach FP64     */
/* precision since s^2 <= 0.0295 there. ln 2 is split into a 29-bit head (so that  */
/* e * head is exact) and a tail.                                                  */
/* ------------------------------------------------------------------------------ */
double orc_log(double x)
{
    static const double ln2_head = 0x1.62e42ffp-1;
    static const double ln2_tail = -0x1.718432a1b0e26p-35;
    static const double sqrt2 = 0x1.6a09e667f3bcdp+0;
    int e;
    double m = frexp(x, &e);     /* x = m 2^e, m in [1/2, 1) */
    m = m * 2.0;                 /* m in [1, 2) */
    e = e - 1;
    if (m > sqrt2) {
        m = m * 0.5;
        e = e + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    /* coefficients 1/(2k+1), k = 0..11, Horner in z from the highest term */
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
    double b = 2.0 * (s * p);
    double de = (double)e;
    return de * ln2_head + (de * ln2_tail + b);
}

/* ------------------------------------------------------------------------------ */
/* Decomposition A = D - T (section 2.1).                                          */
/*   L_ij = -|a_ij| (j != i),  L_ii = r_i = sum_{j != i} |a_ij|,                   */
/*   d_i = a_ii + L_ii,        sigma_ij = [a_ij < 0].                              */
/* The off-diagonal nonzeros of row i, in CSR order, are its "slots"; the jump     */
/* law from i picks slot k with probability k_ij = |a_ij| / r_i. The law is        */
/* sampled with a Walker/Vose alias table (A. J. Walker 1977; M. D. Vose, IEEE     */
/* TSE 17(9), 1991), built as below and stored with 32-bit thresholds.             */
/* ------------------------------------------------------------------------------ */
int orc_decompose(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                  double *r, double *d, double *inv_r, int64_t *slot_begin, int32_t *deg,
                  int32_t *slot_col, uint8_t *slot_sign, uint32_t *slot_thr,
                  int32_t *slot_alias)
{
    int64_t s = 0;
    double *q = NULL;
    int32_t *small = NULL, *large = NULL;
    int64_t maxdeg = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t len = row_ptr[i + 1] - row_ptr[i];
        if (len > maxdeg) maxdeg = len;
    }
    q = (double *)malloc(sizeof(double) * (size_t)(maxdeg + 1));
    small = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
    large = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
    if (!q || !small || !large) {
        free(q); free(small); free(large);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) {
        double diag = 0.0, ri = 0.0;
        int32_t k = 0;
        slot_begin[i] = s;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (col[e] == i) {
                diag += val[e];
            } else if (val[e] != 0.0) {
                ri += fabs(val[e]);
                slot_col[s + k] = col[e];
                slot_sign[s + k] = (uint8_t)(val[e] < 0.0);
                ++k;
            }
        }
        deg[i] = k;
        r[i] = ri;
        d[i] = diag + ri;
        inv_r[i] = (ri > 0.0) ? 1.0 / ri : INFINITY;
        /* alias table: scaled probabilities q_k = |a_k| * deg / r */
        int32_t ns = 0, nl = 0;
        {
            int32_t kk = 0;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                if (col[e] == i || val[e] == 0.0) continue;
                q[kk] = (fabs(val[e]) * (double)k) / ri;
                if (q[kk] < 1.0) small[ns++] = kk; else large[nl++] = kk;
                ++kk;
            }
        }
        while (ns > 0 && nl > 0) {
            int32_t a = small[--ns];
            int32_t g = large[--nl];
            slot_thr[s + a] = (uint32_t)floor(q[a] * 4294967296.0);
            slot_alias[s + a] = g;
            q[g] = (q[g] + q[a]) - 1.0;
            if (q[g] < 1.0) small[ns++] = g; else large[nl++] = g;
        }
        while (nl > 0) {
            int32_t g = large[--nl];
            slot_thr[s + g] = 0xFFFFFFFFu;
            slot_alias[s + g] = g;
        }
        while (ns > 0) {
            int32_t a = small[--ns];
            slot_thr[s + a] = 0xFFFFFFFFu;
            slot_alias[s + a] = a;
        }
        s += k;
    }
    slot_begin[n] = s;
    free(q); free(small); free(large);
    return 0;
}

/* ------------------------------------------------------------------------------ */
/* One sample of Algorithm 2 at level `level` (N = 2^level steps of dt = beta/N).  */
/* ------------------------------------------------------------------------------ */
typedef struct {
    const double *d, *inv_r;
    const int64_t *slot_begin;
    const int32_t *deg, *slot_col, *slot_alias;
    const uint8_t *slot_sign;
    const uint32_t *slot_thr;
    /* importance sampling (NULL = the plain jump law): a proposal law q given by its own
     * alias tables, and per slot the likelihood ratio p/q multiplied into the functional
     * whenever that slot is taken */
    const uint32_t *q_thr;
    const int32_t *q_alias;
    const double *q_ratio;
} orc_tables;

typedef struct {
    int64_t final_state;
    int32_t sign;            /* +1 / -1: the product of the jump signs */
    int64_t jumps;
    uint64_t hash;           /* FNV-1a over (state, step) of every jump */
    double eta_fine, eta_coarse;
    /* with a source term F (Algorithm 3): the Simpson sums of the fine and coarse
     * functionals times F along the path, and their absolute magnitude */
    double integ_fine, integ_coarse, integ_mag;
} orc_walk_out;

/* Composite Simpson weight of grid point n of an even number K of intervals: 1 at both
 * ends, 4 at odd points, 2 at even interior points. */
static double simpson_weight(int64_t n, int64_t K)
{
    if (n == 0 || n == K) return 1.0;
    return (n % 2 != 0) ? 4.0 : 2.0;
}

#define ORC_FNV_OFFSET 14695981039346656037ull
#define ORC_FNV_PRIME 1099511628211ull

/* The source term's Simpson sums at one grid point (Algorithm 3): weight w of the point on
 * its grid, the path's weight eta there, F at the path's state. */
static void add_source_point(double w, double eta, double Fs, double *integ, double *imag)
{
    *integ += w * eta * Fs;
    *imag += w * fabs(eta * Fs);
}

/* One sample at `level`: the single-entry representation of section 2.1 with the Strang
 * splitting on the fine grid (step dt) and, on the same path, on the coarse grid (step 2 dt),
 * the coupling of the level terms (section 2.2, Algorithm 2); with a source vector F, also
 * the source integral int_0^beta exp(sA) F ds of Algorithm 3 by the composite Simpson rule on
 * both grids (F read at the path's state at each grid time).
 *
 * The path. Over each fine step the chain holds at its state for an exponential time of rate
 * r (section 3); while the time accumulated in the step stays below dt it jumps by the jump
 * law of the row it leaves and draws the next holding time at the state it reached. Only the
 * states at the grid points enter the weights.
 *
 * The weights. The Strang step e^{dt D/2} e^{-dt T} e^{dt D/2} contributes e^{dt d/2} at each
 * end of a fine step, so the fine weight multiplies, step by step, the factors at the step's
 * two ends; the coarse weight multiplies e^{dt d} at the two ends of each pair of fine steps.
 * Both carry the product of the jump signs (under a proposal also the likelihood ratios p/q
 * of the jumps taken). */
static void orc_one_walk(const orc_tables *t, double beta, int level, const uint32_t key[2],
                         uint32_t inst, int64_t row, uint32_t walk, const double *F,
                         orc_walk_out *o)
{
    const int64_t N = (int64_t)1 << level;
    const double dt = ldexp(beta, -level);
    int64_t s = row;                  /* the chain's state */
    int64_t pair_start = row;         /* its state at the start of the current pair of steps */
    int64_t jumps = 0;
    uint64_t h = ORC_FNV_OFFSET;
    double phi = 1.0;                 /* jump signs (and likelihood ratios) so far */
    double fine = 1.0, coarse = 1.0;  /* Strang factors on the two grids so far */
    double integ2 = 0.0, integ1 = 0.0, imag2 = 0.0, imag1 = 0.0;
    if (F) {
        /* grid point 0: no time elapsed, both weights are 1 */
        add_source_point(simpson_weight(0, N), 1.0, F[s], &integ2, &imag2);
        if (N >= 2) add_source_point(simpson_weight(0, N / 2), 1.0, F[s], &integ1, &imag1);
    }
    for (int64_t n = 1; n <= N; ++n) {
        const int64_t step_start = s;
        /* the step from grid point n - 1 to n */
        double tau = -orc_log(orc_uniform(step_word(key, level, inst, (uint32_t)row, walk,
                                                    (uint32_t)(n - 1)))) * t->inv_r[s];
        while (tau < dt) {
            const int64_t k = s;
            uint32_t w[3];
            jump_words(key, level, inst, (uint32_t)row, walk, (uint32_t)jumps, w);
            const uint32_t slot = (uint32_t)(((uint64_t)w[0] * (uint64_t)(uint32_t)t->deg[k]) >> 32);
            const int64_t sb = t->slot_begin[k];
            uint32_t pick;
            if (t->q_thr) {
                /* the proposal's alias table; its likelihood ratio keeps the estimator unbiased */
                pick = (w[1] < t->q_thr[sb + slot]) ? slot : (uint32_t)t->q_alias[sb + slot];
                phi = phi * t->q_ratio[sb + pick];
            } else {
                pick = (w[1] < t->slot_thr[sb + slot]) ? slot : (uint32_t)t->slot_alias[sb + slot];
            }
            if (t->slot_sign[sb + pick]) phi = -phi;
            s = t->slot_col[sb + pick];
            double S = -orc_log(orc_uniform(w[2])) * t->inv_r[s];
            tau = tau + S;
            ++jumps;
            h = (h ^ (uint64_t)(uint32_t)s) * ORC_FNV_PRIME;
            h = (h ^ (uint64_t)n) * ORC_FNV_PRIME;
        }
        /* the fine Strang factors at the two ends of step n */
        fine = fine * exp(t->d[step_start] * dt / 2.0);
        fine = fine * exp(t->d[s] * dt / 2.0);
        const int pair_ends = (n % 2 == 0);
        if (pair_ends) {
            /* the coarse factors at the two ends of the pair of steps n - 1, n */
            coarse = coarse * exp(t->d[pair_start] * dt);
            coarse = coarse * exp(t->d[s] * dt);
            pair_start = s;
        }
        if (F) {
            add_source_point(simpson_weight(n, N), phi * fine, F[s], &integ2, &imag2);
            if (pair_ends) add_source_point(simpson_weight(n / 2, N / 2), phi * coarse, F[s], &integ1, &imag1);
        }
    }
    o->final_state = s;
    o->sign = (phi < 0.0) ? -1 : 1;
    o->jumps = jumps;
    o->hash = h;
    o->eta_fine = phi * fine;
    o->eta_coarse = phi * coarse;
    o->integ_fine = dt / 3.0 * integ2;
    o->integ_coarse = 2.0 * dt / 3.0 * integ1;
    o->integ_mag = dt / 3.0 * imag2 + 2.0 * dt / 3.0 * imag1;
}

/* Trace of individual walks: for each (row[q], walk[q]) the final state, sign, jump
 * count, path hash and the two functionals. */
void orc_walk_trace(const double *d, const double *inv_r, const int64_t *slot_begin,
                    const int32_t *deg, const int32_t *slot_col, const uint8_t *slot_sign,
                    const uint32_t *slot_thr, const int32_t *slot_alias, const uint32_t *q_thr,
                    const int32_t *q_alias, const double *q_ratio, double beta,
                    int level, uint64_t seed, uint32_t instance, int64_t count,
                    const int64_t *rows, const uint32_t *walks, int64_t *final_state,
                    int32_t *sign, int64_t *jumps, uint64_t *hash, double *eta_fine,
                    double *eta_coarse)
{
    orc_tables t = {d, inv_r, slot_begin, deg, slot_col, slot_alias, slot_sign, slot_thr,
                    q_thr, q_alias, q_ratio};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < count; ++q) {
        orc_walk_out o;
        orc_one_walk(&t, beta, level, key, instance, rows[q], walks[q], NULL, &o);
        final_state[q] = o.final_state;
        sign[q] = o.sign;
        jumps[q] = o.jumps;
        hash[q] = o.hash;
        eta_fine[q] = o.eta_fine;
        eta_coarse[q] = o.eta_coarse;
    }
}

/* Neumaier's compensated summation (improved Kahan). */
typedef struct { double s, c; } orc_sum;
static void orc_add(orc_sum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/* ------------------------------------------------------------------------------ */
/* Per-row level sums (Algorithm 2's accumulators). For each requested row i and   */
/* walk w in [walk0, walk0 + M), the sample is                                     */
/*     Y = u_j (eta_fine - eta_coarse)   (level > l0)                              */
/*     Y = u_j  eta_fine                 (level = l0)                              */
/* with j the final state, for each of the R right-hand sides (u is n x R, row     */
/* major). Outputs per (row, rhs): sum Y, sum Y^2, the magnitude                  */
/* m = |u_j| (|eta_fine| + |eta_coarse|) (the scale of the rounding in Y) summed,  */
/* and sum m^2; per row: the total jump count and the sum (mod 2^64) of the path  */
/* hashes.                                                                         */
/* ------------------------------------------------------------------------------ */
void orc_level_sums(const double *d, const double *inv_r, const int64_t *slot_begin,
                    const int32_t *deg, const int32_t *slot_col, const uint8_t *slot_sign,
                    const uint32_t *slot_thr, const int32_t *slot_alias, const uint32_t *q_thr,
                    const int32_t *q_alias, const double *q_ratio, double beta,
                    int level, int l0, uint64_t seed, uint32_t instance, const double *u,
                    const double *F, int32_t R, int64_t n_rows, const int64_t *rows, uint32_t walk0,
                    uint32_t M, double *sum1, double *sum2, double *mass, double *mass2,
                    int64_t *jumps, uint64_t *hash_sum, int32_t nthreads)
{
    orc_tables t = {d, inv_r, slot_begin, deg, slot_col, slot_alias, slot_sign, slot_thr,
                    q_thr, q_alias, q_ratio};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        orc_sum *a1 = (orc_sum *)malloc(sizeof(orc_sum) * (size_t)R);
        orc_sum *a2 = (orc_sum *)malloc(sizeof(orc_sum) * (size_t)R);
        orc_sum *am = (orc_sum *)malloc(sizeof(orc_sum) * (size_t)R);
        orc_sum *am2 = (orc_sum *)malloc(sizeof(orc_sum) * (size_t)R);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n_rows; ++q) {
            int64_t i = rows[q];
            int64_t nj = 0;
            uint64_t hs = 0;
            memset(a1, 0, sizeof(orc_sum) * (size_t)R);
            memset(a2, 0, sizeof(orc_sum) * (size_t)R);
            memset(am, 0, sizeof(orc_sum) * (size_t)R);
            memset(am2, 0, sizeof(orc_sum) * (size_t)R);
            for (uint32_t w = 0; w < M; ++w) {
                orc_walk_out o;
                orc_one_walk(&t, beta, level, key, instance, i, walk0 + w, F, &o);
                nj += o.jumps;
                hs += o.hash;
                for (int32_t rr = 0; rr < R; ++rr) {
                    double uj = u[o.final_state * R + rr];
                    double y, m;
                    if (level > l0) {
                        y = uj * (o.eta_fine - o.eta_coarse);
                        m = fabs(uj) * (fabs(o.eta_fine) + fabs(o.eta_coarse));
                    } else {
                        y = uj * o.eta_fine;
                        m = fabs(uj) * fabs(o.eta_fine);
                    }
                    if (F) {
                        /* Algorithm 3: the source term's Simpson sums join the sample */
                        y += (level > l0) ? o.integ_fine - o.integ_coarse : o.integ_fine;
                        m += o.integ_mag;
                    }
                    orc_add(&a1[rr], y);
                    orc_add(&a2[rr], y * y);
                    orc_add(&am[rr], m);
                    orc_add(&am2[rr], m * m);
                }
            }
            for (int32_t rr = 0; rr < R; ++rr) {
                sum1[q * R + rr] = a1[rr].s + a1[rr].c;
                sum2[q * R + rr] = a2[rr].s + a2[rr].c;
                mass[q * R + rr] = am[rr].s + am[rr].c;
                mass2[q * R + rr] = am2[rr].s + am2[rr].c;
            }
            jumps[q] = nj;
            hash_sum[q] = hs;
        }
        free(a1); free(a2); free(am); free(am2);
    }
}

/* ------------------------------------------------------------------------------ */
/* Scalar functional (w, exp(beta A) u) by walks started at random rows (the        */
/* full-vector representation of section 2.1, summed against w): walk m draws its    */
/* start row l with probability |u_l| / U (U = sum |u_l|) from the alias table over   */
/* rows (start_thr, start_alias) with the words of the block (0, m, 0, stream 2),     */
/* then runs as the walk m of row l on the tables of A^T (jump law of column l of A); */
/* its sample is sign(u_l) w_j eta (eta_fine - eta_coarse above l0), times U outside. */
/* Outputs: the sums of the samples and of their squares (Neumaier), jumps, and the   */
/* sum (mod 2^64) of the path hashes.                                                */
/* ------------------------------------------------------------------------------ */
void orc_functional_sums(const double *d, const double *inv_r, const int64_t *slot_begin,
                         const int32_t *deg, const int32_t *slot_col, const uint8_t *slot_sign,
                         const uint32_t *slot_thr, const int32_t *slot_alias, double beta,
                         int level, int l0, uint64_t seed, uint32_t instance, int64_t n,
                         const uint32_t *start_thr, const int32_t *start_alias,
                         const uint8_t *start_neg, const double *w, uint32_t walk0, uint32_t M,
                         double *sum1, double *sum2, int64_t *jumps, uint64_t *hash_sum)
{
    orc_tables t = {d, inv_r, slot_begin, deg, slot_col, slot_alias, slot_sign, slot_thr,
                    NULL, NULL, NULL};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_sum a1 = {0, 0}, a2 = {0, 0};
    int64_t nj = 0;
    uint64_t hs = 0;
    for (uint32_t m = 0; m < M; ++m) {
        const uint32_t walk = walk0 + m;
        uint32_t ctr[4] = {0u, walk, 0u, c3_of(level, instance, 2)};
        uint32_t out[4];
        orc_philox4x32_10(ctr, key, out);
        uint32_t slot = (uint32_t)(((uint64_t)out[0] * (uint64_t)n) >> 32);
        uint32_t l = (out[1] < start_thr[slot]) ? slot : (uint32_t)start_alias[slot];
        orc_walk_out o;
        orc_one_walk(&t, beta, level, key, instance, (int64_t)l, walk, NULL, &o);
        double y = w[o.final_state] * ((level > l0) ? (o.eta_fine - o.eta_coarse) : o.eta_fine);
        if (start_neg[l]) y = -y;
        orc_add(&a1, y);
        orc_add(&a2, y * y);
        nj += o.jumps;
        hs += o.hash;
    }
    *sum1 = a1.s + a1.c;
    *sum2 = a2.s + a2.c;
    *jumps = nj;
    *hash_sum = hs;
}

/* ------------------------------------------------------------------------------ */
/* The full vector exp(beta A) u by the same walks (the forward representation of   */
/* section 2.1): walk m (start row l drawn as in orc_functional_sums, run on the     */
/* tables of A^T) deposits its sample sign(u_l) eta (eta_fine - eta_coarse above l0)  */
/* at its final state j: per state j the sums of the deposits and of their squares   */
/* (Neumaier, in walk order), the mass |eta_fine| (+ |eta_coarse| above l0) of the   */
/* deposits, and their count; the level term of x_j is U sum1[j] / M. Also the jumps */
/* and the sum (mod 2^64) of the path hashes. The arrays of n entries are            */
/* overwritten.                                                                      */
/* ------------------------------------------------------------------------------ */
int orc_forward_sums(const double *d, const double *inv_r, const int64_t *slot_begin,
                     const int32_t *deg, const int32_t *slot_col, const uint8_t *slot_sign,
                     const uint32_t *slot_thr, const int32_t *slot_alias, double beta,
                     int level, int l0, uint64_t seed, uint32_t instance, int64_t n,
                     const uint32_t *start_thr, const int32_t *start_alias,
                     const uint8_t *start_neg, uint32_t walk0, uint32_t M,
                     double *sum1, double *sum2, double *mass, int64_t *count,
                     int64_t *jumps, uint64_t *hash_sum)
{
    orc_tables t = {d, inv_r, slot_begin, deg, slot_col, slot_alias, slot_sign, slot_thr,
                    NULL, NULL, NULL};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_sum *a1 = (orc_sum *)calloc((size_t)(n > 0 ? n : 1), sizeof(orc_sum));
    orc_sum *a2 = (orc_sum *)calloc((size_t)(n > 0 ? n : 1), sizeof(orc_sum));
    if (!a1 || !a2) {
        free(a1); free(a2);
        return -1;
    }
    for (int64_t j = 0; j < n; ++j) {
        mass[j] = 0.0;
        count[j] = 0;
    }
    int64_t nj = 0;
    uint64_t hs = 0;
    for (uint32_t m = 0; m < M; ++m) {
        const uint32_t walk = walk0 + m;
        uint32_t ctr[4] = {0u, walk, 0u, c3_of(level, instance, 2)};
        uint32_t out[4];
        orc_philox4x32_10(ctr, key, out);
        uint32_t slot = (uint32_t)(((uint64_t)out[0] * (uint64_t)n) >> 32);
        uint32_t l = (out[1] < start_thr[slot]) ? slot : (uint32_t)start_alias[slot];
        orc_walk_out o;
        orc_one_walk(&t, beta, level, key, instance, (int64_t)l, walk, NULL, &o);
        const int64_t j = o.final_state;
        double y = (level > l0) ? (o.eta_fine - o.eta_coarse) : o.eta_fine;
        if (start_neg[l]) y = -y;
        orc_add(&a1[j], y);
        orc_add(&a2[j], y * y);
        mass[j] += fabs(o.eta_fine) + ((level > l0) ? fabs(o.eta_coarse) : 0.0);
        count[j] += 1;
        nj += o.jumps;
        hs += o.hash;
    }
    for (int64_t j = 0; j < n; ++j) {
        sum1[j] = a1[j].s + a1[j].c;
        sum2[j] = a2[j].s + a2[j].c;
    }
    free(a1);
    free(a2);
    *jumps = nj;
    *hash_sum = hs;
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Alias tables (the construction of orc_decompose) for an arbitrary law given per slot:
 * prob[s] for the slots of each row (summing to one per row). */
void orc_alias_tables(int64_t n, const int64_t *slot_begin, const int32_t *deg, const double *prob,
                      uint32_t *thr, int32_t *alias)
{
    int32_t maxdeg = 0;
    for (int64_t i = 0; i < n; ++i) if (deg[i] > maxdeg) maxdeg = deg[i];
    double *q = (double *)malloc(sizeof(double) * (size_t)(maxdeg + 1));
    int32_t *small = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
    int32_t *large = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
    for (int64_t i = 0; i < n; ++i) {
        const int64_t sb = slot_begin[i];
        const int32_t k = deg[i];
        int32_t ns = 0, nl = 0;
        for (int32_t s = 0; s < k; ++s) {
            q[s] = prob[sb + s] * (double)k;
            if (q[s] < 1.0) small[ns++] = s; else large[nl++] = s;
        }
        while (ns > 0 && nl > 0) {
            int32_t a = small[--ns];
            int32_t g = large[--nl];
            thr[sb + a] = (uint32_t)floor(q[a] * 4294967296.0);
            alias[sb + a] = g;
            q[g] = (q[g] + q[a]) - 1.0;
            if (q[g] < 1.0) small[ns++] = g; else large[nl++] = g;
        }
        while (nl > 0) { int32_t g = large[--nl]; thr[sb + g] = 0xFFFFFFFFu; alias[sb + g] = g; }
        while (ns > 0) { int32_t a = small[--ns]; thr[sb + a] = 0xFFFFFFFFu; alias[sb + a] = a; }
    }
    free(q); free(small); free(large);
}

/* Vectorised helpers for the tests: log of count values, and the uniform variate of
 * count words. */
void orc_log_array(int64_t count, const double *x, double *out)
{
    for (int64_t q = 0; q < count; ++q) out[q] = orc_log(x[q]);
}

void orc_philox_array(int64_t count, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t q = 0; q < count; ++q) orc_philox4x32_10(ctr + 4 * q, key + 2 * q, out + 4 * q);
}
