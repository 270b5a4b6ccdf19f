// Compiled variants: 2D Q^1, Q^2 Euler; FP64 and mixed precision.
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    Ops<2, 1, SP_Q, SYS_EULER, double>::make(), Ops<2, 1, SP_Q, SYS_EULER, float>::make(),
    Ops<2, 2, SP_Q, SYS_EULER, double>::make(), Ops<2, 2, SP_Q, SYS_EULER, float>::make(),
};
int variants_v2d_q12_euler(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
