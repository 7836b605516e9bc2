/*
 * lds_probe.h - C ABI of liblds_probe.so, the LDS bandwidth probe.
 *
 * The decoder keeps every Tanner-graph message in LDS (local data share), so
 * the rate at which a compute unit can read and write LDS is the roofline its
 * message traffic is measured against. This library measures that rate on
 * the device instead of taking it from a data sheet: streaming kernels issue
 * LDS instructions of one kind and width with a bank-conflict-free pattern
 * and nothing else, on every compute unit.
 *
 * Not part of the decoder (include/bpsf.h); the benchmark calls it.
 */
#ifndef LDS_PROBE_H
#define LDS_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LDS_PROBE_READ 0    /* ds_read_b32 / b64 / b128 */
#define LDS_PROBE_WRITE 1   /* ds_write_b32 / b64 / b128 */

/*
 * Run one probe kernel on the current device and time it.
 *   kind           LDS_PROBE_READ or LDS_PROBE_WRITE
 *   width          bytes per lane per instruction: 4, 8 or 16
 *   blocks_per_cu  workgroups of 256 threads (four waves, 8 KB of LDS each)
 *                  launched per compute unit, 1..64 (the device runs as many
 *                  at once as fit)
 *   iters          groups of eight instructions every thread issues, >= 1
 *   stream         hipStream_t (NULL = default stream)
 *   bytes_per_s    host out: LDS bytes moved by the timed launch / its time
 *   ms_out         host out (may be NULL): the timed launch's duration
 * One untimed launch precedes the timed one (HIP events on `stream`); the
 * call waits for both. Allocates no device memory. Returns 0, -1 for a bad
 * argument, -4 for a failed HIP call.
 */
int lds_probe_run(int32_t kind, int32_t width, int32_t blocks_per_cu, int32_t iters, void* stream,
                  double* bytes_per_s, float* ms_out);

#ifdef __cplusplus
}
#endif

#endif /* LDS_PROBE_H */
