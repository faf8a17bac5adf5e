/*
 * tdec_probe.h -- device ceilings measured on the GPU the library runs on.
 *
 * The roofline fractions the decoder reports are taken against published
 * peaks (the packed int16 VALU rate of 256 CUs x 4 SIMDs x 16 lanes x 2
 * halves x 2.4 GHz, 8 TB/s of HBM).  These probes measure the same ceilings
 * with the decoder's own instructions and access patterns, so the fractions
 * can also be stated against what the device delivers.  They are
 * measurement tools, not part of the decoding path.
 *
 * Every probe runs synchronously on the given device, allocates and frees
 * its own device memory (hipMalloc / hipFree), and returns 0 or a
 * tdec_status error (TDEC_EINVAL for bad arguments, TDEC_ENOMEM when an
 * allocation fails, TDEC_EDEVICE for a HIP error).  Results are written
 * only on success.
 */
#ifndef TDEC_PROBE_H
#define TDEC_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Packed int16 VALU throughput.  Eight independent chains per lane of the
 * decoder's add-compare-select instructions (saturating packed add, packed
 * maximum), 256-thread work groups, eight per CU on every CU.  *tops =
 * int16 operations per second / 1e12, two per lane per instruction.
 * iters: loop trips per lane (16 instructions each), 1 .. 1e6. */
int tdec_probe_valu_int16(int device, int32_t iters, double *tops);

/* HBM streaming bandwidth over a buffer of `bytes` (16 MiB .. 16 GiB, a
 * multiple of 16): *read_gbs = bytes read per second / 1e9 by a 16-byte
 * load kernel that keeps one word per thread; *copy_gbs = (bytes read +
 * bytes written) per second / 1e9 of a 16-byte copy kernel into a second
 * buffer of the same size. */
int tdec_probe_hbm(int device, size_t bytes, double *read_gbs, double *copy_gbs);

/* Launch overheads over n empty kernels (1 .. 100000): *us_launch = device
 * time per launch when the host queues them back to back on one stream;
 * *us_graph_node = the same for a HIP graph holding the n launches,
 * replayed once. */
int tdec_probe_launch(int device, int32_t n, double *us_launch, double *us_graph_node);

#ifdef __cplusplus
}
#endif

#endif /* TDEC_PROBE_H */
