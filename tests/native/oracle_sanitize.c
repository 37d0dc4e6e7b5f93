/* Runs the oracle's C entry points on small matrices for an AddressSanitizer /
 * UndefinedBehaviorSanitizer build (test infrastructure): decomposition with an absorbing
 * row and signed entries, walk traces, level sums at the coarsest level and above (with
 * several right-hand sides, with a source term, under an importance-sampling table), the
 * scalar and forward functionals, and the alias tables of an arbitrary law. Prints a
 * checksum; any sanitizer report ends the program with a nonzero status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_decompose(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                  double *r, double *d, double *inv_r, int64_t *slot_begin, int32_t *deg,
                  int32_t *slot_col, uint8_t *slot_sign, uint32_t *slot_thr, int32_t *slot_alias);
void orc_walk_trace(const double *d, const double *inv_r, const int64_t *slot_begin,
                    const int32_t *deg, const int32_t *slot_col, const uint8_t *slot_sign,
                    const uint32_t *slot_thr, const int32_t *slot_alias, const uint32_t *q_thr,
                    const int32_t *q_alias, const double *q_ratio, double beta, int level,
                    uint64_t seed, uint32_t instance, int64_t count, const int64_t *rows,
                    const uint32_t *walks, int64_t *final_state, int32_t *sign, int64_t *jumps,
                    uint64_t *hash, double *eta_fine, double *eta_coarse);
void orc_level_sums(const double *d, const double *inv_r, const int64_t *slot_begin,
                    const int32_t *deg, const int32_t *slot_col, const uint8_t *slot_sign,
                    const uint32_t *slot_thr, const int32_t *slot_alias, const uint32_t *q_thr,
                    const int32_t *q_alias, const double *q_ratio, double beta, int level, int l0,
                    uint64_t seed, uint32_t instance, const double *u, const double *F, int32_t R,
                    int64_t n_rows, const int64_t *rows, uint32_t walk0, uint32_t M, double *sum1,
                    double *sum2, double *mass, double *mass2, int64_t *jumps, uint64_t *hash_sum,
                    int32_t nthreads);
void orc_functional_sums(const double *d, const double *inv_r, const int64_t *slot_begin,
                         const int32_t *deg, const int32_t *slot_col, const uint8_t *slot_sign,
                         const uint32_t *slot_thr, const int32_t *slot_alias, double beta,
                         int level, int l0, uint64_t seed, uint32_t instance, int64_t n,
                         const uint32_t *start_thr, const int32_t *start_alias,
                         const uint8_t *start_neg, const double *w, uint32_t walk0, uint32_t M,
                         double *sum1, double *sum2, int64_t *jumps, uint64_t *hash_sum);
int orc_forward_sums(const double *d, const double *inv_r, const int64_t *slot_begin,
                     const int32_t *deg, const int32_t *slot_col, const uint8_t *slot_sign,
                     const uint32_t *slot_thr, const int32_t *slot_alias, double beta, int level,
                     int l0, uint64_t seed, uint32_t instance, int64_t n, const uint32_t *start_thr,
                     const int32_t *start_alias, const uint8_t *start_neg, uint32_t walk0,
                     uint32_t M, double *sum1, double *sum2, double *mass, int64_t *count,
                     int64_t *jumps, uint64_t *hash_sum);
void orc_alias_tables(int64_t n, const int64_t *slot_begin, const int32_t *deg,
                      const double *prob, uint32_t *thr, int32_t *alias);

#define N 7
#define R 3

int main(void)
{
    /* a signed nonsymmetric 7 x 7 matrix; row 6 has no off-diagonal entry (absorbing) and row
     * 2 no diagonal entry */
    double a[N][N] = {{-2.0, 0.5, 0, -0.3, 0, 0, 0.1},  {0.4, -1.0, 0.2, 0, 0, -0.6, 0},
                      {0, 0.7, 0, 0.1, -0.2, 0, 0},     {0.3, 0, 0, -0.5, 0.9, 0, 0},
                      {0, 0, -0.8, 0.2, 0.3, 0.1, 0.4}, {1.1, 0, 0, 0, 0.5, -2.5, 0},
                      {0, 0, 0, 0, 0, 0, -0.7}};
    int64_t row_ptr[N + 1];
    int32_t col[N * N];
    double val[N * N];
    int64_t nnz = 0;
    for (int i = 0; i < N; ++i) {
        row_ptr[i] = nnz;
        for (int j = 0; j < N; ++j)
            if (a[i][j] != 0.0) {
                col[nnz] = j;
                val[nnz] = a[i][j];
                ++nnz;
            }
    }
    row_ptr[N] = nnz;
    double r[N], d[N], inv_r[N];
    int64_t slot_begin[N + 1];
    int32_t deg[N], slot_col[N * N], slot_alias[N * N];
    uint8_t slot_sign[N * N];
    uint32_t slot_thr[N * N];
    if (orc_decompose(N, row_ptr, col, val, r, d, inv_r, slot_begin, deg, slot_col, slot_sign,
                      slot_thr, slot_alias) != 0)
        return 2;
    int64_t n_slots = 0;
    for (int i = 0; i < N; ++i) n_slots += deg[i];
    const double beta = 1.5;
    const int l0 = 2;
    double checksum = 0.0;
    /* traces at levels 0..4 */
    {
        int64_t rows[2 * N], fs[2 * N], jumps[2 * N];
        uint32_t walks[2 * N];
        int32_t sign[2 * N];
        uint64_t hash[2 * N];
        double ef[2 * N], ec[2 * N];
        for (int q = 0; q < 2 * N; ++q) {
            rows[q] = q % N;
            walks[q] = 0xFFFFFF00u + (uint32_t)q;
        }
        for (int lev = 0; lev <= 4; ++lev) {
            orc_walk_trace(d, inv_r, slot_begin, deg, slot_col, slot_sign, slot_thr, slot_alias,
                           NULL, NULL, NULL, beta, lev, 12345u, 7u, 2 * N, rows, walks, fs, sign,
                           jumps, hash, ef, ec);
            for (int q = 0; q < 2 * N; ++q) checksum += ef[q] + (double)jumps[q];
        }
    }
    /* level sums, several right-hand sides, coarsest level and above, all rows and a subset */
    double u[N * R], F[N];
    for (int i = 0; i < N * R; ++i) u[i] = sin(1.0 + i);
    for (int i = 0; i < N; ++i) F[i] = cos(0.5 * i);
    {
        double s1[N * R], s2[N * R], m1[N * R], m2[N * R];
        int64_t jumps[N];
        uint64_t hs[N];
        int64_t sub[3] = {6, 0, 3};
        int64_t all[N];
        for (int i = 0; i < N; ++i) all[i] = i;
        for (int lev = l0; lev <= l0 + 3; ++lev) {
            orc_level_sums(d, inv_r, slot_begin, deg, slot_col, slot_sign, slot_thr, slot_alias,
                           NULL, NULL, NULL, beta, lev, l0, 99u, 0u, u, NULL, R, N, all, 0u, 500u,
                           s1, s2, m1, m2, jumps, hs, 2);
            for (int i = 0; i < N * R; ++i) checksum += s1[i];
            orc_level_sums(d, inv_r, slot_begin, deg, slot_col, slot_sign, slot_thr, slot_alias,
                           NULL, NULL, NULL, beta, lev, l0, 99u, 0u, u, NULL, R, 3, sub,
                           0xFFFFFE00u, 300u, s1, s2, m1, m2, jumps, hs, 1);
            /* Algorithm 3 with a source term, one right-hand side */
            orc_level_sums(d, inv_r, slot_begin, deg, slot_col, slot_sign, slot_thr, slot_alias,
                           NULL, NULL, NULL, beta, lev, l0, 5u, 1u, u, F, 1, N, all, 0u, 200u,
                           s1, s2, m1, m2, jumps, hs, 2);
            for (int i = 0; i < N; ++i) checksum += s1[i];
        }
    }
    /* an importance-sampling table: the law (|a| + 1/deg) / (r + 1) per slot, with ratios */
    {
        double *prob = malloc(sizeof(double) * (size_t)(n_slots > 0 ? n_slots : 1));
        double *ratio = malloc(sizeof(double) * (size_t)(n_slots > 0 ? n_slots : 1));
        uint32_t *qthr = malloc(sizeof(uint32_t) * (size_t)(n_slots > 0 ? n_slots : 1));
        int32_t *qalias = malloc(sizeof(int32_t) * (size_t)(n_slots > 0 ? n_slots : 1));
        for (int i = 0; i < N; ++i) {
            double tot = 0.0;
            for (int k = 0; k < deg[i]; ++k) {
                const int64_t s = slot_begin[i] + k;
                const double p = fabs(a[i][slot_col[s]]) / r[i];
                prob[s] = 0.5 * p + 0.5 / deg[i];
                ratio[s] = p / prob[s];
                tot += prob[s];
            }
            (void)tot;
        }
        orc_alias_tables(N, slot_begin, deg, prob, qthr, qalias);
        double s1[N], s2[N], m1[N], m2[N];
        int64_t jumps[N];
        uint64_t hs[N];
        int64_t all[N];
        for (int i = 0; i < N; ++i) all[i] = i;
        orc_level_sums(d, inv_r, slot_begin, deg, slot_col, slot_sign, slot_thr, slot_alias, qthr,
                       qalias, ratio, beta, l0 + 1, l0, 3u, 2u, u, NULL, 1, N, all, 0u, 400u, s1,
                       s2, m1, m2, jumps, hs, 2);
        for (int i = 0; i < N; ++i) checksum += s1[i];
        free(prob);
        free(ratio);
        free(qthr);
        free(qalias);
    }
    /* the scalar functional and the forward full vector from a start law over rows */
    {
        int64_t one_begin[2] = {0, N};
        int32_t one_deg[1] = {N};
        double p_rows[N];
        double U = 0.0;
        uint8_t neg[N];
        for (int i = 0; i < N; ++i) U += fabs(u[i]);
        for (int i = 0; i < N; ++i) {
            p_rows[i] = fabs(u[i]) / U;
            neg[i] = u[i] < 0.0;
        }
        uint32_t sthr[N];
        int32_t salias[N];
        orc_alias_tables(1, one_begin, one_deg, p_rows, sthr, salias);
        double f1, f2, fs1[N], fs2[N], fm[N];
        int64_t fj, cnt[N];
        uint64_t fh;
        for (int lev = l0; lev <= l0 + 2; ++lev) {
            orc_functional_sums(d, inv_r, slot_begin, deg, slot_col, slot_sign, slot_thr,
                                slot_alias, beta, lev, l0, 8u, 0u, N, sthr, salias, neg, F, 0u,
                                3000u, &f1, &f2, &fj, &fh);
            checksum += f1;
            if (orc_forward_sums(d, inv_r, slot_begin, deg, slot_col, slot_sign, slot_thr,
                                 slot_alias, beta, lev, l0, 8u, 0u, N, sthr, salias, neg, 0u,
                                 3000u, fs1, fs2, fm, cnt, &fj, &fh) != 0)
                return 3;
            for (int i = 0; i < N; ++i) checksum += fs1[i];
        }
    }
    if (!isfinite(checksum)) return 4;
    printf("oracle sanitize ok %.17g\n", checksum);
    return 0;
}
