/*
 * fobf_peak.h -- instruction-rate probes for MI355X (gfx950).
 *
 * The filter kernels are built from four instruction classes: fp32 vector
 * FMA, the vector sine/cosine used for the per-pixel trigonometric terms of
 * the shiftable kernel (eq. (3)), and the 16x16 matrix instructions for the
 * Gaussian convolutions in fp32, fp16 and bf16.  fobf_peak times one
 * saturating kernel of the requested class on the current device and
 * reports its rate, so that kernel efficiencies can be quoted against a
 * measured ceiling next to the published one.  Diagnostic only: nothing in
 * the filter path calls it.
 */
#ifndef FOBF_PEAK_H
#define FOBF_PEAK_H

#include "fobf.h"

#ifdef __cplusplus
extern "C" {
#endif

enum fobf_peak_kind {
  FOBF_PEAK_VALU_FMA_F32 = 0, /* v_fma_f32, 2 flop per lane (packed fp32 off) */
  FOBF_PEAK_VALU_SIN_F32 = 1, /* v_sin_f32, 1 op per lane                     */
  FOBF_PEAK_MFMA_F32 = 2,     /* 16x16x4 fp32 matrix instruction              */
  FOBF_PEAK_MFMA_F16 = 3,     /* 16x16x32 fp16 matrix instruction, fp32 acc    */
  FOBF_PEAK_MFMA_BF16 = 4     /* 16x16x32 bf16 matrix instruction, fp32 acc    */
};

/*
 * fobf_peak -- runs the probe of class `kind` on `stream` (a hipStream_t;
 * NULL = default stream) and writes the measured rate to *rate in units of
 * 1e12 per second: flop/s for the FMA and matrix classes (a multiply-add
 * counts 2), operations/s for the sine.  Blocks until the probe finishes.
 * Allocates and frees a 2 MiB device buffer.  FOBF_EINVAL for an unknown
 * kind or NULL rate, FOBF_ENOMEM / FOBF_EHIP on device errors.
 */
fobf_status fobf_peak(int kind, void* stream, double* rate);

#ifdef __cplusplus
}
#endif

#endif /* FOBF_PEAK_H */
