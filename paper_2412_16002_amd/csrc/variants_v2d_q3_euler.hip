// Compiled variants: 2D Q^3 Euler; FP64 and mixed precision, both with the
// cooperative stage kernels (one wavefront per variable, 16 x 4 tiles):
// measured on a 512^2 RK4 wave 0.79 ms per step FP64 and 0.445 mixed,
// against 1.00 and 0.50 for the one-thread-per-cell kernels, which also run
// at the register limit in FP64 (64 FP64 values per state).
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    OpsCoop<2, 3, SYS_EULER, double, 16, 4, 1>::make(), OpsCoop<2, 3, SYS_EULER, float, 16, 4, 1>::make(),
};
int variants_v2d_q3_euler(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
