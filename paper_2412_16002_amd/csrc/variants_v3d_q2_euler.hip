// Compiled variants: 3D Q^2 Euler (27 modes x 5 variables, rolled point
// loops); FP64 and mixed precision.
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    Ops<3, 2, SP_Q, SYS_EULER, double>::make(), Ops<3, 2, SP_Q, SYS_EULER, float>::make(),
};
int variants_v3d_q2_euler(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
