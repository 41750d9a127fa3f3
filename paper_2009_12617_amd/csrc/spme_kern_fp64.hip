// Kernels of one precision (FP64 throughout):
// every grid shape, spline order and variant, instantiated from the
// templates in spme_kernels.h.
#include "spme_kernels.h"

namespace spme {
const PrecOps kOpsDouble = make_ops<PDouble>();
}  // namespace spme
