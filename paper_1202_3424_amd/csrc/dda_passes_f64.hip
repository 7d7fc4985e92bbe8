// Matvec pass kernels with double grids (see dda_passes.h).
#include "dda_passes.h"

namespace dda {
DDA_INSTANTIATE_PASSES(double)

// (one definition for both precisions, from the variant tables)
bool strided_variant_xcd(int L, bool gh, bool fp32, int v) {
    if (!gh || !ct_length(L) || v < 0 || v >= strided_variants(L, gh)) return false;
    using namespace passes;
    if (v < n_lds_variants(1)) return variant_xg(1, v);
    const int r = v - n_lds_variants(1);
    return rf_xg(1, r) && (fp32 ? rf_feasible<float>(L, 1, r) : rf_feasible<double>(L, 1, r));
}
}  // namespace dda
