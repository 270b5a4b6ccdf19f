// Compiled variants: 2D Q^3 Euler; FP64 and mixed precision.
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    Ops<2, 3, SP_Q, SYS_EULER, double>::make(), Ops<2, 3, SP_Q, SYS_EULER, float>::make(),
};
int variants_v2d_q3_euler(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
