// Compiled variants: 3D P^1 (total degree) advection / Euler and P^2
// advection; FP64 and mixed precision.  (3D P^2 Euler: mixed form only, in
// its own translation unit, variants_v3d_p2_euler.hip.)
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    Ops<3, 1, SP_P, SYS_ADV, double>::make(),   Ops<3, 1, SP_P, SYS_ADV, float>::make(),
    Ops<3, 1, SP_P, SYS_EULER, double>::make(), Ops<3, 1, SP_P, SYS_EULER, float>::make(),
    Ops<3, 2, SP_P, SYS_ADV, double>::make(),   Ops<3, 2, SP_P, SYS_ADV, float>::make(),
};
int variants_v3d_p(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
