// Kernels of one precision (FP32/fixed with a bfloat16 half spectrum between launches):
// every grid shape, spline order and variant, instantiated from the
// templates in spme_kernels.h.
#include "spme_kernels.h"

namespace spme {
const PrecOps kOpsBf16 = make_ops<PBf16>();
}  // namespace spme
