/*
 * ptmi_probe.h -- measurement helpers beside the parallel-tempering library:
 * achievable LDS read bandwidth of the device, used as the measured peak of
 * the LDS roofline the sweep kernels are reported against, and a replay of
 * the field update alone.
 */
#ifndef PTMI_PROBE_H
#define PTMI_PROBE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif
/* Streams 16-byte LDS reads (lane-contiguous, bank-conflict free) in
 * `blocks` workgroups of `threads` threads, `iters` reads per thread per
 * pass over a 64 KB LDS buffer, timed with HIP events on the null stream.
 * *bytes_per_s receives the aggregate read bandwidth.  Returns 0, or a
 * negative value if a HIP call failed (blocks/threads/iters must be >= 1,
 * threads <= 1024). */
int ptmi_lds_read_bandwidth(int32_t blocks, int32_t threads, int32_t iters, double *bytes_per_s);
/* The field update alone (a5; the paper recomputes energies instead, sec.
 * 4.2, so the table and its update are this library's): the FP64 table
 * h[k][j] = sum_{i != j} J*(|i - j|) [s_i = k] of an L-site ring with q <= 4
 * states takes a flip sequence, window by window (64 flips at a time), in the
 * sweep kernel's own flush (h[old][j] -= J*(|j - i|), h[new][j] += J*(|j - i|)
 * for every site j), in LDS, in `workgroups` workgroups of 256 threads that
 * each replay the whole sequence `reps` times on their own copy.
 *   jstar  [L] host: J*(r), r = 0..L-1 (J*(0) = 0)
 *   h0     [q][L] host: the starting table (state-major rows)
 *   words  [nwords] host: flips, site | old << 16 | new << 20 (states 0-based;
 *          old != new; every site < L and every state < q, checked)
 *   h_out  [q][L] host: workgroup 0's table after the timed launch
 *   ms_out the timed launch (HIP events, null stream; a warm-up launch with
 *          reps = 1 runs first)
 * All buffers are the caller's; the function allocates and frees its own
 * device copies.  Returns 0, -1 on a bad argument (including a table that does
 * not fit in LDS), or another negative value if a HIP call failed. */
int ptmi_flush_replay(int32_t L, int32_t q, const double *jstar, const double *h0, const uint32_t *words,
                      int64_t nwords, int32_t workgroups, int32_t reps, double *h_out, double *ms_out);
/* Issue rate of one instruction kind (0: FP64 FMA, 1: FP32 FMA) at a given
 * occupancy: `blocks` workgroups of `threads`
 * threads (a multiple of 64, at most 1024), each thread updating 16
 * independent accumulators `iters` times (at most 2^20) with multiplier 1 and
 * addend 1, timed with HIP events on the null stream after a warm-up launch.
 * *ms_out receives the timed launch; *sum_out the sum of thread 0's
 * accumulators in workgroup 0, 120 + 16 iters exactly, which shows the
 * instructions ran.  With one workgroup of 256 threads per CU there is one
 * wave per SIMD: ms / (16 iters) is the time between two issues of the kind by
 * one wave.  Returns 0, -1 on a bad argument, or another negative value if a
 * HIP call failed. */
int ptmi_valu_issue_rate(int32_t kind, int32_t blocks, int32_t threads, int32_t iters, double *ms_out,
                         double *sum_out);
#ifdef __cplusplus
}
#endif
#endif
