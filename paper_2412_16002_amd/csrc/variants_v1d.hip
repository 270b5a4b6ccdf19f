// Compiled variants: 1D, P^1..P^3, advection / Burgers / Euler; FP64 and mixed precision.
#include "variants.hpp"

namespace crkdg {
static const VariantOps kOps[] = {
    Ops<1, 1, SP_Q, SYS_ADV, double>::make(), Ops<1, 1, SP_Q, SYS_ADV, float>::make(),
    Ops<1, 2, SP_Q, SYS_ADV, double>::make(), Ops<1, 2, SP_Q, SYS_ADV, float>::make(),
    Ops<1, 3, SP_Q, SYS_ADV, double>::make(), Ops<1, 3, SP_Q, SYS_ADV, float>::make(),
    Ops<1, 1, SP_Q, SYS_BURG, double>::make(), Ops<1, 1, SP_Q, SYS_BURG, float>::make(),
    Ops<1, 2, SP_Q, SYS_BURG, double>::make(), Ops<1, 2, SP_Q, SYS_BURG, float>::make(),
    Ops<1, 3, SP_Q, SYS_BURG, double>::make(), Ops<1, 3, SP_Q, SYS_BURG, float>::make(),
    Ops<1, 1, SP_Q, SYS_EULER, double>::make(), Ops<1, 1, SP_Q, SYS_EULER, float>::make(),
    Ops<1, 2, SP_Q, SYS_EULER, double>::make(), Ops<1, 2, SP_Q, SYS_EULER, float>::make(),
    Ops<1, 3, SP_Q, SYS_EULER, double>::make(), Ops<1, 3, SP_Q, SYS_EULER, float>::make(),
};
int variants_v1d(const VariantOps** out) {
  *out = kOps;
  return static_cast<int>(sizeof(kOps) / sizeof(kOps[0]));
}
}  // namespace crkdg
