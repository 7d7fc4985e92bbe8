// Matvec pass kernels with float grids (see dda_passes.h).
#include "dda_passes.h"

namespace dda {
DDA_INSTANTIATE_PASSES(float)
}  // namespace dda
