/*
 * ptmi_probe.h -- measurement helpers beside the parallel-tempering library:
 * achievable LDS read bandwidth of the device, used as the measured peak of
 * the LDS roofline the sweep kernels are reported against.
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
#ifdef __cplusplus
}
#endif
#endif
