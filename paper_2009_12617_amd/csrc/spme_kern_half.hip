// Kernels of one precision (FP32/fixed with a binary16 half spectrum between launches):
// every grid shape, spline order and variant, instantiated from the
// templates in spme_kernels.h.
#include "spme_kernels.h"

namespace spme {
const PrecOps kOpsHalf = make_ops<PHalf>();
}  // namespace spme
