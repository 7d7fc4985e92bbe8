// Matvec pass kernels with double grids (see dda_passes.h).
#include "dda_passes.h"

namespace dda {
DDA_INSTANTIATE_PASSES(double)
}  // namespace dda
