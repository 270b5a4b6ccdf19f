// Compiled variants: 2D P^1..P^3 advection; FP64 and mixed precision.
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    Ops<2, 1, SP_P, SYS_ADV, double>::make(), Ops<2, 1, SP_P, SYS_ADV, float>::make(),
    Ops<2, 2, SP_P, SYS_ADV, double>::make(), Ops<2, 2, SP_P, SYS_ADV, float>::make(),
    Ops<2, 3, SP_P, SYS_ADV, double>::make(), Ops<2, 3, SP_P, SYS_ADV, float>::make(),
};
int variants_v2d_p_adv(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
