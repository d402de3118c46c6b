/*
 * kmicro.h - microbenchmarks of the gfx950 resources the decision kernels
 * are priced against (a measurement tool beside the decision library, not
 * part of its path).
 *
 * kmicro_run measures, on the current HIP device and the stream hip_stream:
 *   valu_int32_tops  int32/bitwise VALU lane-operations per second (1e12),
 *                    from independent xor/add chains in every lane;
 *   lds_tbs          LDS read bandwidth (1e12 bytes/s), 16-byte
 *                    conflict-free reads from 64 KB per workgroup;
 *   hbm_gbs          HBM read bandwidth (1e9 bytes/s), one pass of 16-byte
 *                    loads over the buffer;
 * each as the best of several timed launches (HIP events), with the kernel
 * time in ms beside it, and the device's CU count and peak clock.
 * dev_buf: device memory of buf_bytes >= 64 MiB, 16-byte aligned, owned by
 * the caller; its first 16 KB may be written, the rest is only read.
 * Returns 0, or -1 on a bad argument or a failed HIP call (then *out is
 * incomplete).  The stream is synchronised on return.
 */
#ifndef KMICRO_H
#define KMICRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double valu_int32_tops, lds_tbs, hbm_gbs;
  double valu_ms, lds_ms, hbm_ms;
  uint32_t cus, clock_mhz;
} kmicro_peaks;

int kmicro_run(const void* dev_buf, size_t buf_bytes, void* hip_stream, kmicro_peaks* out);

#ifdef __cplusplus
}
#endif
#endif /* KMICRO_H */
