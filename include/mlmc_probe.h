/*
 * mlmc_probe: measurement probes shipped with the mlmc_expv library (libmlmc_expv.so).
 *
 * They calibrate the rooflines the walk kernels are reported against and take no part in
 * a walk. The cost model of the method (section 4: time = a gather term per jump plus a
 * term per time step) has two machine rates, which these measure on the device in use:
 *   - the rate of uniformly random 16-byte gathers from a table of a given size (the
 *     memory level holding the table: L2, the MALL or HBM), the bound of the jump term;
 *   - the issue rate of plain 32-bit integer VALU instructions, the bound of the step term
 *     (the generator and the step test are integer work).
 * Both return MLMC_OK or an MLMC_ERR_* status (mlmc_last_error() has the detail), run on
 * the current device, wait for `stream`, and allocate a 1 KiB device sink on first use.
 */
#ifndef MLMC_PROBE_H
#define MLMC_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Uniformly random gathers of 16-byte records from `table` (DEVICE, caller owned, at least
 * 2^log2_records records of 16 bytes, contents arbitrary): a grid of waves_per_cu waves per
 * compute unit (4, 8, ..., 32), each lane doing iters x 8 gathers with 8 independent index
 * streams (xorshift32). One untimed launch, then one launch timed with events on `stream`.
 *   gathers: HOST, receives the gathers of the timed launch; ms: HOST, its duration. */
int mlmc_probe_gather(const void *table, int32_t log2_records, int32_t waves_per_cu,
                      int32_t iters, uint64_t *gathers, double *ms, void *stream);

/* mlmc_probe_gather with a mode (bits):
 *   MLMC_PROBE_LDS: each workgroup first copies the table's 2^log2_records records into its
 *     LDS (log2_records <= 12, 64 KB) and gathers from there (the copy is in the timed
 *     launch; it is small against iters x 8 gathers per lane);
 *   MLMC_PROBE_DEPENDENT: one index stream per lane, each next index taking in the first
 *     word of the record just read, so a lane's gathers are serial: the launch then keeps
 *     waves_per_cu x 64 gathers in flight per compute unit, and that count divided by the
 *     rate is the latency of one gather.
 * gathers counts iters x 8 per lane, or iters per lane with MLMC_PROBE_DEPENDENT. Mode 0 is
 * mlmc_probe_gather. This is what staging rows' tables in LDS could gain per gather. */
#define MLMC_PROBE_LDS 1
#define MLMC_PROBE_DEPENDENT 2
int mlmc_probe_gather_mode(const void *table, int32_t log2_records, int32_t waves_per_cu,
                           int32_t iters, int32_t mode, uint64_t *gathers, double *ms,
                           void *stream);

/* Eight chains per lane of a_j = a_j ^ a_{j+1} ^ i (one v_bitop3_b32 each), iters rounds,
 * on waves_per_cu waves per compute unit. lane_ops: HOST, lane-instructions of the timed
 * launch; ms: HOST, its duration. */
int mlmc_probe_valu(int32_t waves_per_cu, int32_t iters, uint64_t *lane_ops, double *ms,
                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MLMC_PROBE_H */
