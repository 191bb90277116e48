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

/* VALU against MFMA on one contraction of the predictor: the values of the
 * space-time polynomial at the side points of the face quadrature (App. D:
 * per side the barycentre and the face-average nodes; order 3: 42 points
 * from 15 modes, 390 nonzero entries; order 4: 78 points from 35 modes,
 * 1584 nonzero entries), for 4 Mi zones x 5 variables in FP32, each zone's
 * point values reduced to the sum of their squares.  The VALU kernel takes
 * one lane per zone with the nonzero entries as immediate operands (the
 * form of the predictor kernels); the MFMA kernel takes 32 zones per wave
 * through v_mfma_f32_32x32x2f32 with the matrix zero-padded to 32-point
 * tiles and an even mode count.  out[6] receives: the useful rate (2 x
 * nonzero entries per zone and variable) of the VALU and of the MFMA
 * kernel in TFLOP/s, their launch times in ms (best of 5), the MFMA
 * kernel's dense (padded) rate in TFLOP/s, and the largest relative
 * difference between the two kernels' per-zone results.  Allocates about
 * 0.6 GB (order 4) for its duration (ADER_ENOMEM if it cannot); ADER_EINVAL
 * for an order other than 3 or 4, a device out of range or a null out. */
int ader_probe_face_eval(int device, int order, double* out);

#ifdef __cplusplus
}
#endif
#endif /* ADER_PROBE_H */
