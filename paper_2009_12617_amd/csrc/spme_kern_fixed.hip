// Kernels of one precision (FP32 splines/FFT/convolution with a 64-bit fixed-point charge grid):
// every grid shape, spline order and variant, instantiated from the
// templates in spme_kernels.h.
#include "spme_kernels.h"

namespace spme {
const PrecOps kOpsFixed = make_ops<PFixed>();
}  // namespace spme
