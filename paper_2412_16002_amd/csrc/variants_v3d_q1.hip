// Compiled variants: 3D Q^1 advection / Euler; FP64 and mixed precision.
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    Ops<3, 1, SP_Q, SYS_ADV, double>::make(), Ops<3, 1, SP_Q, SYS_ADV, float>::make(),
    Ops<3, 1, SP_Q, SYS_EULER, double>::make(), Ops<3, 1, SP_Q, SYS_EULER, float>::make(),
};
int variants_v3d_q1(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
