/*
 * ader_probe.h -- measurement tooling beside the ADER-CG step library: the
 * peak rates the step library's code reaches on a device, the denominators
 * of its kernels' rooflines.  Built as its own library (libader_probe.so);
 * not part of the step's C ABI (ader.h) and never called by it.
 */
#ifndef ADER_PROBE_H
#define ADER_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

/* The peak rates the step library's code reaches on `device`.
 * ADER_PROBE_FP32_FMA and ADER_PROBE_FP64_FMA time independent FMA chains
 * (8 per thread, 32 waves per compute unit; FP32 as this library compiles
 * it, without packed FP32 instructions) and return TFLOP/s;
 * ADER_PROBE_HBM_COPY times a 1 GiB device-to-device copy kernel and
 * returns GB/s (bytes read plus bytes written).  Each takes the best of
 * several launches on a stream of its own and synchronises; the copy
 * allocates 2 GiB for its duration (ADER_ENOMEM if it cannot).
 * ADER_EINVAL for an unknown kind, a device out of range or a null
 * value_out. */
enum { ADER_PROBE_FP32_FMA = 0, ADER_PROBE_FP64_FMA = 1, ADER_PROBE_HBM_COPY = 2 };
int ader_probe_peak(int device, int kind, double* value_out);

#ifdef __cplusplus
}
#endif
#endif /* ADER_PROBE_H */
